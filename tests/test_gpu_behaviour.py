"""GPU behaviour of liblf beyond plain parity: every sweep variant against the
oracle, determinism, graph replay vs single steps, bitwise checkpoint/resume,
non-finite detection, the exact discrete free wave, and coupling changes."""
import numpy as np
import pytest
import torch

import oracle as O
from _parity import ARRAYS, compare_state, gpu_run, log, make_lattice, oracle_run, to_dev
from paper_0911_5692_amd import LfError
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fields(lat):
    return [x.cpu().numpy() for x in lat.fields(dtype=torch.float64)]


@pytest.mark.parametrize("tile_y,zchunk", [(1, 0), (4, 8), (4, 13), (8, 16), (8, 64), (16, 7), (16, 32)])
def test_sweep_variants_match_oracle(tile_y, zchunk):
    """Each launch shape (plain, LDS tiles of 4/8/16 rows, ragged z-chunks) on
    a ragged 48^3 lattice (48 = 0.75 x 64 columns) stays within 1e-5."""
    w = W.CFG2.resized(48)
    steps = 150
    log(f"[variant] tile_y={tile_y} zchunk={zchunk}")
    st, en, _, ic = oracle_run(w, steps)
    lat, _ = gpu_run(w, ic, steps, tile_y=tile_y, zchunk=zchunk)
    errs = compare_state(_fields(lat), st)
    assert max(errs.values()) <= 1e-5, errs
    g = lat.energies()
    assert abs(g["a"] - en["a"]) <= 1e-9 * en["a"] and abs(g["R"] - en["R"]) <= 1e-8


@pytest.mark.parametrize("tile_y", [1, 4, 16])
def test_sweep_variants_fp64(tile_y):
    w = W.CFG1.resized(40)
    st, en, _, ic = oracle_run(w, 60)
    lat, _ = gpu_run(w, ic, 60, dtype="f64", tile_y=tile_y, zchunk=16 if tile_y > 1 else 0)
    errs = compare_state(_fields(lat), st)
    assert max(errs.values()) <= 1e-11, errs


def test_deterministic_repeat_bitwise():
    w = W.CFG3.resized(64)
    ic = W.make_inputs(w)
    outs = []
    for _ in range(2):
        lat, _ = gpu_run(w, ic, 100)
        outs.append((lat.get_state()[0], lat.energies()))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert torch.equal(a, b)
    assert outs[0][1] == outs[1][1]


def test_graph_replay_equals_single_steps():
    """lf_step(n) replays multi-step graphs; n calls of lf_step(1) replay the
    one-step graphs: same kernels, same order, bitwise the same state."""
    w = W.CFG1.resized(32)
    ic = W.make_inputs(w)
    n = 2 * 32 + 5
    a, _ = gpu_run(w, ic, n, dtype="f32")
    b, _ = gpu_run(w, ic, 0, dtype="f32")
    for _ in range(n):
        b.step(1)
    sa, sca = a.get_state()
    sb, scb = b.get_state()
    for x, y in zip(sa, sb):
        assert torch.equal(x, y)
    assert sca.a_half == scb.a_half and sca.ad == scb.ad and sca.step == scb.step == n


def test_checkpoint_resume_bitwise():
    w = W.CFG2.resized(64)
    ic = W.make_inputs(w)
    n = 37
    full, _ = gpu_run(w, ic, 2 * n)
    half, _ = gpu_run(w, ic, n)
    arrays, sc = half.get_state()
    arrays = [x.clone() for x in arrays]
    fresh = make_lattice(w)
    fresh.set_state(arrays, sc)
    fresh.step(n)
    s1, c1 = full.get_state()
    s2, c2 = fresh.get_state()
    for x, y in zip(s1, s2):
        assert torch.equal(x, y)
    assert (c1.a_half, c1.ad, c1.step, tuple(c1.pend)) == (c2.a_half, c2.ad, c2.step, tuple(c2.pend))
    e1, e2 = full.energies(), fresh.energies()
    assert e1 == e2


def test_nonfinite_input_is_reported():
    w = W.CFG1.resized(16)
    ic = W.make_inputs(w)
    f1 = ic["f1"].copy()
    f1[3, 4, 5] = np.nan
    lat = make_lattice(w)
    with pytest.raises(LfError) as ei:
        lat.init_physical(to_dev(f1), to_dev(ic["f2"]), to_dev(ic["u1"]), to_dev(ic["u2"]), 1.0)
    assert ei.value.code == 3
    lat2 = make_lattice(w)
    lat2.init(to_dev(f1), to_dev(ic["f2"]), to_dev(ic["u1"]), to_dev(ic["u2"]), 1.0, 0.3)
    lat2.step(3)
    with pytest.raises(LfError) as ei:
        lat2.energies()
    assert ei.value.code == 3
    e = lat2.energies(check_finite=False)
    assert e["status"] != 0


def test_cfl_violation_blows_up_and_is_flagged():
    """dt far above the leapfrog stability bound dt sqrt(12/dx^2 + m^2) < 2: the
    fields overflow, the non-finite flag trips and stays set (sticky)."""
    w = W.CFG1.resized(16)
    from dataclasses import replace
    w = replace(w, dt=3.0 * w.dx)
    ic = W.make_inputs(w)
    lat, _ = gpu_run(w, ic, 400)
    with pytest.raises(LfError) as ei:
        lat.energies()
    assert ei.value.code == 3


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_free_wave_exact_discrete_solution_gpu(dtype, tol):
    """kappa^2 = 0, G = 0, V = c1 f^2/2: cos(k.x) evolves as cos(k Omega dt)
    with sin(Omega dt/2) = omega dt/2 (exact for the discrete leapfrog)."""
    N, dx, dt, c1 = 32, 0.5, 0.05, 2.5
    from paper_0911_5692_amd import Lattice
    lat = Lattice(N=N, L=N * dx, dt=dt, beta=2, c1=c1, G=0.0, r=1.5, s=0.0, kappa2=0.0,
                  dtype=torch.float64 if dtype == "f64" else torch.float32)
    z, y, x = np.meshgrid(*(np.arange(N) * dx,) * 3, indexing="ij")
    n = np.array([3, 5, 16])
    k = 2 * np.pi * n / (N * dx)
    shape = np.cos(k[0] * x + k[1] * y + k[2] * z)
    zero = np.zeros_like(shape)
    lat.init(to_dev(shape), to_dev(zero), to_dev(zero), to_dev(zero), 1.0, 0.0)
    steps = 300
    lat.step(steps)
    w2 = (4 / dx ** 2) * np.sum(np.sin(k * dx / 2) ** 2) + c1
    Om = 2 * np.arcsin(np.sqrt(w2) * dt / 2) / dt
    f1, f2, v1, v2 = [t.cpu().numpy() for t in lat.fields(synchronized=True, dtype=torch.float64)]
    assert np.max(np.abs(f1 - np.cos(steps * Om * dt) * shape)) <= tol
    assert np.max(np.abs(f2)) == 0.0
    e = lat.energies()
    assert e["a"] == 1.0 and e["ad"] == 0.0


def test_set_coupling_mid_run_matches_oracle():
    w = W.CFG1.resized(24)
    ic = W.make_inputs(w)
    m = O.Model(**w.model())
    st = O.start_physical(m, ic["f1"], ic["f2"], ic["u1"], ic["u2"], 1.0)
    O.evolve(st, 30)
    st.m = m.replace(G=180.0)
    O.evolve(st, 30)
    lat, _ = gpu_run(w, ic, 30, dtype="f64")
    lat.set_coupling(180.0)
    lat.step(30)
    errs = compare_state(_fields(lat), st)
    assert max(errs.values()) <= 1e-10, errs


def test_step_before_init_is_a_state_error():
    lat = make_lattice(W.CFG1.resized(8))
    with pytest.raises(LfError) as ei:
        lat.step(1)
    assert ei.value.code == 4
    with pytest.raises(LfError) as ei:
        lat.step(-1)
    assert ei.value.code == 1


SHAPES27 = [dict(tile_x=64, tile_y=4, zchunk=8), dict(tile_x=64, tile_y=8, zchunk=13),
            dict(tile_x=64, tile_y=16, zchunk=48), dict(tile_x=128, tile_y=4, zchunk=7),
            dict(tile_x=128, tile_y=8, zchunk=0)]
# the 7-point sweep also has 32-wide tiles; the plain 27-point variant sums
# its stencil in another order, so only the 7-point list holds the plain sweep
SHAPES7 = [dict(tile_y=1)] + SHAPES27 + [dict(tile_x=32, tile_y=8, zchunk=11), dict(tile_x=32, tile_y=16, zchunk=0)]


@pytest.mark.parametrize("stencil", [7, 27])
def test_tile_invariance(stencil):
    """Every launch shape computes the same per-site arithmetic: from one
    state, one step gives bitwise equal arrays; after 50 steps (step sums
    added in a shape-dependent order, so the FP64 coefficients may differ
    in their last bits) the arrays agree to a few FP32 ulp."""
    from dataclasses import replace
    w = replace(W.CFG3.resized(48), stencil=stencil)
    _, _, _, ic = oracle_run(w, 1)
    shapes = SHAPES7 if stencil == 7 else SHAPES27
    one, many = [], []
    for sh in shapes:
        lat, _ = gpu_run(w, ic, 1, **sh)
        one.append(lat.get_state()[0])
        lat.step(49)
        many.append(lat.fields(dtype=torch.float64))
        lat.close()
    for sh, arrs in zip(shapes[1:], one[1:]):
        for k, a, b in zip(ARRAYS, arrs, one[0]):
            assert torch.equal(a, b), (sh, k, "one step differs")
    worst = 0.0
    for arrs in many[1:]:
        for a, b in zip(arrs, many[0]):
            worst = max(worst, float(((a - b).abs().max() / b.abs().max()).item()))
    log(f"[tiles] stencil {stencil}: one step bitwise over {len(shapes)} shapes; 50 steps max rel {worst:.2e}")
    assert worst <= 1e-6


def test_zero_steps_leave_the_state_unchanged():
    w = W.CFG1.resized(24)
    _, _, _, ic = oracle_run(w, 5)
    lat, _ = gpu_run(w, ic, 5)
    arrays, sc = lat.get_state()
    lat.step(0)
    arrays2, sc2 = lat.get_state()
    for a, b in zip(arrays, arrays2):
        assert torch.equal(a, b)
    assert sc2.step == sc.step == 5 and sc2.a_half == sc.a_half and sc2.ad == sc.ad
    assert lat.energies()["step"] == 5


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_rho_p_matches_oracle(dtype, tol):
    """Per-site energy density and pressure (the paper's second kernel) and
    w = <p>/<rho> against the oracle, on the 512^3-model recipe at 48^3."""
    w = W.CFG3.resized(48)
    st, _, _, ic = oracle_run(w, 120)
    rho, p, avg = O.rho_p(st)
    lat, _ = gpu_run(w, ic, 120, dtype=dtype)
    grho, gp, gavg = lat.rho_p()
    assert float(np.max(np.abs(grho.cpu().numpy() - rho)) / np.max(np.abs(rho))) <= tol
    assert float(np.max(np.abs(gp.cpu().numpy() - p)) / np.max(np.abs(p))) <= tol
    for k in ("rho", "p", "w"):
        assert abs(gavg[k] - avg[k]) <= tol * abs(avg[k]), k
    _, _, only = lat.rho_p(arrays=False)
    assert only == gavg


@pytest.mark.parametrize("stencil", [7, 27])
def test_history_series_matches_oracle(stencil):
    """a(t), H, rho, R and w(t) recorded every 40 steps (the series the paper
    plots) against the oracle's at the same steps, FP64."""
    from dataclasses import replace
    w = replace(W.CFG3, stencil=stencil).resized(24)
    ic = W.make_inputs(w)
    m = O.Model(**w.model())
    st = O.start_physical(m, ic["f1"], ic["f2"], ic["u1"], ic["u2"], 1.0)
    lat = make_lattice(w, dtype="f64")
    lat.init_physical(to_dev(ic["f1"]), to_dev(ic["f2"]), to_dev(ic["u1"]), to_dev(ic["u2"]), 1.0)
    h = lat.history(200, 40)
    assert list(h["step"]) == [0, 40, 80, 120, 160, 200]
    for j in range(len(h["step"])):
        if j:
            O.evolve(st, 40)
        e = O.energies(st)
        _, _, avg = O.rho_p(st, arrays=False)
        assert abs(h["a"][j] - e["a"]) <= 1e-12 * e["a"]
        assert abs(h["hubble"][j] - e["ad"] / e["a"]) <= 1e-11 * abs(e["ad"] / e["a"])
        assert abs(h["rho"][j] - e["rho"]) <= 1e-10 * e["rho"]
        assert abs(h["R"][j] - e["R"]) <= 1e-12
        assert abs(h["w"][j] - avg["w"]) <= 1e-10 * max(1.0, abs(avg["w"]))


@pytest.mark.parametrize("stencil", [7, 27])
def test_rho_p_and_energies_full_size_512_periodic(stencil):
    """512^3 in the benchmark's launch shape with a 64^3-periodic state: the
    per-site rho and p (FP32 out) repeat bitwise with the period and equal the
    oracle's 64^3 values; the averages and the energies equal the oracle's."""
    from dataclasses import replace
    base = replace(W.CFG3, stencil=stencil)
    w = base.resized(64)
    shape = W.BENCH_SHAPES[W.CFG3_S27.name if stencil == 27 else W.CFG3.name]
    log(f"[rho_p 512] stencil={stencil} shape={shape}")
    st, en, _, ic = oracle_run(w, 40)
    rho, p, avg = O.rho_p(st)
    lat, _ = gpu_run(w, ic, 40, dtype="f32", reps=8, **shape)
    grho, gp, gavg = lat.rho_p(dtype=torch.float32)
    for name, g, ref in (("rho", grho, rho), ("p", gp, p)):
        t = g.view(8, 64, 8, 64, 8, 64)
        assert bool((t == t[0:1, :, 0:1, :, 0:1, :]).all()), f"periodic copies of {name} differ"
        first = g[:64, :64, :64].double().cpu().numpy()
        err = float(np.max(np.abs(first - ref)) / np.max(np.abs(ref)))
        log(f"[rho_p 512] {name} rel err {err:.2e}")
        assert err <= 1e-5, (name, err)
    for k in ("rho", "p", "w"):
        assert abs(gavg[k] - avg[k]) <= 1e-5 * abs(avg[k]), (k, gavg[k], avg[k])
    g = lat.energies()
    for k in ("K1", "K2", "G1", "G2", "P", "rho"):
        assert abs(g[k] - en[k]) <= 1e-5 * abs(en[k]), k
    lat.close()
