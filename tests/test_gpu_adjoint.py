"""liblf's adjoint (reverse steps with checkpoints) against the FP64 oracle's
adjoint and against central finite differences of the oracle's forward map.

Initial program-unit velocities and a'(0) come from the oracle's Friedmann
initialisation and are given to both sides as inputs; the gradient is taken
with v(0), a_0, a'_0 held fixed except where their own derivatives are
checked."""
import numpy as np
import pytest
import torch

import oracle as O
from _parity import log, to_dev
from paper_0911_5692_amd import Lattice, LeapfrogLoss
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu

WEIGHTS = (0.0, 1.0, 0.0, 1.0)  # K_chi + G_chi


def _model(kind, N):
    if kind == "lphi4":
        return O.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=1.0187733)
    return O.Model(N=N, L=N * 0.05, dt=2 ** -8, beta=2, c1=1.0, G=400.0, r=1.5, s=0.0, kappa2=1.0187733)


def _state(m, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    N = m.N
    f1 = 1.0 + amp * rng.standard_normal((N, N, N))
    f2 = amp * rng.standard_normal((N, N, N))
    u1 = -0.3 + amp * rng.standard_normal((N, N, N))
    u2 = amp * rng.standard_normal((N, N, N))
    v1, v2, ad0 = O.init_physical(m, f1, f2, u1, u2, 1.0)
    return f1, f2, v1, v2, ad0


def _gpu_adjoint(m, f1, f2, v1, v2, ad0, n, K, dtype):
    lat = Lattice(N=m.N, L=m.L, dt=m.dt, beta=m.beta, c1=m.c1, G=m.G, r=m.r, s=m.s, kappa2=m.kappa2,
                  dtype=dtype)
    lat.init(to_dev(f1), to_dev(f2), to_dev(v1), to_dev(v2), 1.0, ad0)
    loss = lat.adjoint_forward(n, K, WEIGHTS)
    g = lat.adjoint_backward(1.0)
    return loss, g


def _relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("kind", ["lphi4", "m2phi2"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
def test_adjoint_matches_oracle_adjoint(kind, dtype, tol):
    m = _model(kind, 10)
    f1, f2, v1, v2, ad0 = _state(m, 3)
    n, K = 30, 7  # segments of 7 with a ragged last one
    ref = O.adjoint(m, f1, f2, v1, v2, 1.0, ad0, n, wK=WEIGHTS[:2], wG=WEIGHTS[2:])
    loss, g = _gpu_adjoint(m, f1, f2, v1, v2, ad0, n, K, dtype)
    log(f"[adj] {kind} {dtype}: loss {loss} vs {ref['E']}; dG {g['G']} vs {ref['dG']}")
    assert abs(loss - ref["E"]) <= tol * abs(ref["E"])
    assert abs(g["G"] - ref["dG"]) <= tol * abs(ref["dG"])
    assert abs(g["a0"] - ref["da0"]) <= tol * abs(ref["da0"])
    assert abs(g["ad0"] - ref["dad0"]) <= tol * abs(ref["dad0"])
    for k in ("f1", "f2", "v1", "v2"):
        err = _relmax(g[k].cpu().numpy(), ref[k])
        log(f"[adj]   d/d{k}: {err:.2e}")
        assert err <= tol, k


@pytest.mark.timeout(900)
def test_checkpoint_interval_and_repeats_on_one_context():
    """The backward pass recomputes segment s-1 on a second stream while the
    reverse steps of segment s run.  On one context: a single segment (no
    overlap), segments of 7 and 3 steps (ragged last ones, odd and even
    counts) give the same gradients up to the order of the step sums at
    segment starts, and a repeat of the first configuration gives bitwise the
    same result."""
    m = _model("lphi4", 12)
    f1, f2, v1, v2, ad0 = _state(m, 5)
    lat = Lattice(N=m.N, L=m.L, dt=m.dt, beta=m.beta, c1=m.c1, G=m.G, r=m.r, s=m.s, kappa2=m.kappa2,
                  dtype=torch.float32)
    n, res = 40, []
    for K in (40, 7, 3, 40):
        lat.init(to_dev(f1), to_dev(f2), to_dev(v1), to_dev(v2), 1.0, ad0)
        loss = lat.adjoint_forward(n, K, WEIGHTS)
        g = lat.adjoint_backward(1.0)
        res.append((K, loss, {k: (v.clone() if torch.is_tensor(v) else v) for k, v in g.items()}))
    lat.close()
    K0, loss0, g0 = res[0]
    for K, loss, g in res[1:]:
        assert loss == loss0, K
        for k, v in g.items():
            if torch.is_tensor(v):
                err = float((v - g0[k]).abs().max() / g0[k].abs().max())
                log(f"[adj] K={K} d/d{k} vs K={K0}: {err:.1e}")
                assert err <= 1e-12, (K, k)
            else:
                assert abs(v - g0[k]) <= 1e-12 * abs(g0[k]), (K, k)
    _, _, g3 = res[3]
    for k, v in g3.items():
        assert (torch.equal(v, g0[k]) if torch.is_tensor(v) else v == g0[k]), k


def test_workload5_adjoint_vs_finite_differences():
    """128^3 lambda phi^4 (G = 100), FP32 lattice, 500 steps, checkpoints every
    50: dL/dG, the derivative along 8 random directions of f_phi(0) and along
    2 random directions of f_chi(0) (directions from SeedSequence([5, 999, j]),
    unit rms) against central differences of the FP64 oracle, each within
    1e-4."""
    w = W.CFG5
    m = O.Model(**w.model())
    ic = W.make_inputs(w)
    v1, v2, ad0 = O.init_physical(m, ic["f1"], ic["f2"], ic["u1"], ic["u2"], 1.0)
    f1, f2 = ic["f1"], ic["f2"]
    n, K = w.steps, 50
    loss, g = _gpu_adjoint(m, f1, f2, v1, v2, ad0, n, K, torch.float32)
    grad = {k: g[k].cpu().numpy() for k in ("f1", "f2")}

    def oracle_loss(G=m.G, df1=None, df2=None):
        mm = m.replace(G=G)
        st = O.start(mm, f1 if df1 is None else f1 + df1, f2 if df2 is None else f2 + df2, v1, v2, 1.0, ad0)
        O.evolve(st, n)
        e = O.energies(st)
        return e["K2"] + e["G2"]

    L0 = oracle_loss()
    log(f"[adj] workload 5: loss gpu {loss:.10e} oracle {L0:.10e}")
    assert abs(loss - L0) <= 1e-5 * abs(L0)
    hG = 1e-4 * m.G
    fdG = (oracle_loss(G=m.G + hG) - oracle_loss(G=m.G - hG)) / (2 * hG)
    log(f"[adj] dL/dG adjoint {g['G']:.8e} fd {fdG:.8e} rel {abs(g['G'] - fdG) / abs(fdG):.2e}")
    assert abs(g["G"] - fdG) <= 1e-4 * abs(fdG)
    h = 1e-6
    worst = 0.0
    for j, field in [(j, "f1") for j in range(8)] + [(8, "f2"), (9, "f2")]:
        rng = np.random.default_rng(np.random.SeedSequence([5, 999, j]))
        d = rng.standard_normal(f1.shape)
        d /= np.sqrt(np.mean(d * d))
        kw = lambda sgn: {"df1" if field == "f1" else "df2": sgn * h * d}
        fdd = (oracle_loss(**kw(1.0)) - oracle_loss(**kw(-1.0))) / (2 * h)
        adj_d = float(np.sum(grad[field] * d))
        rel = abs(adj_d - fdd) / abs(fdd)
        worst = max(worst, rel)
        log(f"[adj] direction {j} of {field}(0): adjoint {adj_d:.8e} fd {fdd:.8e} rel {rel:.2e}")
        assert rel <= 1e-4, (j, field, adj_d, fdd)
    log(f"[adj] worst directional relative difference {worst:.2e}")


def test_leapfrog_loss_autograd():
    m = _model("lphi4", 8)
    f1, f2, v1, v2, ad0 = _state(m, 5)
    spec = dict(N=m.N, L=m.L, dt=m.dt, beta=m.beta, c1=m.c1, r=m.r, s=m.s, kappa2=m.kappa2,
                dtype=torch.float64, n=20, K=6, a0=1.0, ad0=ad0, weights=WEIGHTS)
    G = torch.tensor(m.G, dtype=torch.float64, requires_grad=True)
    t1 = to_dev(f1).requires_grad_(True)
    loss = LeapfrogLoss.apply(G, t1, to_dev(f2), to_dev(v1), to_dev(v2), spec)
    (2.0 * loss).backward()
    ref = O.adjoint(m, f1, f2, v1, v2, 1.0, ad0, 20, wK=WEIGHTS[:2], wG=WEIGHTS[2:])
    assert abs(loss.item() - ref["E"]) <= 1e-10 * ref["E"]
    assert abs(float(G.grad) - 2.0 * ref["dG"]) <= 1e-9 * abs(2.0 * ref["dG"])
    assert _relmax(t1.grad.cpu().numpy(), 2.0 * ref["f1"]) <= 1e-9
