"""Pin of the oracle's hand-written adjoint against complex-step
differentiation of the oracle's own forward map (Im F(x + i h d) / h = J d to
rounding, no cancellation): the derivative of the loss in every input
direction and the dot-product identity <lambda_n, J d> = <J^T lambda_n, d>."""
import numpy as np
import pytest

H = 1e-30


def _setup(orc, model, N=4):
    if model == "lphi4":
        m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0,
                      kappa2=1.0187733)
    else:
        m = orc.Model(N=N, L=N * 0.2, dt=2 ** -7, beta=2, c1=1.0, G=400.0, r=1.5, s=0.0,
                      kappa2=1.0187733)
    rng = np.random.default_rng(7)
    f1 = 1.0 + 0.05 * rng.standard_normal((N, N, N))
    f2 = 0.05 * rng.standard_normal((N, N, N))
    u1 = -0.3 + 0.05 * rng.standard_normal((N, N, N))
    v1, v2, ad0 = orc.init_physical(m, f1, f2, u1, 0.02 * rng.standard_normal((N, N, N)), 1.0)
    return m, f1, f2, v1, v2, ad0, rng


@pytest.mark.parametrize("model", ["lphi4", "m2phi2"])
def test_adjoint_matches_complex_step(orc, model):
    m, f1, f2, v1, v2, ad0, rng = _setup(orc, model)
    n = 12
    wK, wG = (0.3, 1.0), (0.5, 1.0)
    adj = orc.adjoint(m, f1, f2, v1, v2, 1.0, ad0, n, wK=wK, wG=wG)

    def loss_imag(G=m.G, a0=1.0, ad=ad0, d=None):
        x = [f1, f2, v1, v2]
        x = [xi.astype(np.complex128) for xi in x]
        if d is not None:
            for j in range(4):
                x[j] = x[j] + 1j * H * d[j]
        out = orc.complex_run(m, G, *x, a0, ad, n)
        en = out[-1]
        E = wK[0] * en[2] + wK[1] * en[3] + wG[0] * en[4] + wG[1] * en[5]
        return E

    E = loss_imag()
    assert abs(E.real - adj["E"]) <= 1e-14 * abs(adj["E"])
    # every input direction
    d = [rng.standard_normal(f1.shape) for _ in range(4)]
    cs = loss_imag(d=d).imag / H
    ad = sum(np.sum(adj[k] * d[j]) for j, k in enumerate(("f1", "f2", "v1", "v2")))
    assert abs(cs - ad) <= 1e-10 * abs(cs)
    for j, k in enumerate(("f1", "f2", "v1", "v2")):
        dj = [np.zeros_like(f1)] * 4
        dj[j] = d[j]
        cs = loss_imag(d=dj).imag / H
        assert abs(cs - np.sum(adj[k] * d[j])) <= 1e-9 * max(abs(cs), 1e-12), k
    cs = loss_imag(G=complex(m.G, H)).imag / H
    assert abs(cs - adj["dG"]) <= 1e-10 * abs(cs)
    cs = loss_imag(a0=complex(1.0, H)).imag / H
    assert abs(cs - adj["da0"]) <= 1e-10 * abs(cs)
    cs = loss_imag(ad=complex(ad0, H)).imag / H
    assert abs(cs - adj["dad0"]) <= 1e-10 * abs(cs)


def test_adjoint_dot_product_identity(orc):
    """<lambda_n, J d> = <J^T lambda_n, d> for a random cotangent on the final
    desynchronised state (f(n+1/2), v(n), a_{n+1/2}, a'_n)."""
    m, f1, f2, v1, v2, ad0, rng = _setup(orc, "m2phi2", N=5)
    n = 9
    seed = [rng.standard_normal(f1.shape) for _ in range(4)] + [rng.standard_normal(), rng.standard_normal()]
    adj = orc.adjoint(m, f1, f2, v1, v2, 1.0, ad0, n, wK=(0, 0), wG=(0, 0), seed=seed)
    d = [rng.standard_normal(f1.shape) for _ in range(4)]
    da, dad = rng.standard_normal(), rng.standard_normal()
    x = [xi.astype(np.complex128) + 1j * H * dj for xi, dj in zip((f1, f2, v1, v2), d)]
    g1, g2, w1, w2, ah, ad, _ = orc.complex_run(m, m.G, *x, complex(1.0, H * da), complex(ad0, H * dad), n)
    Jd = [g1.imag / H, g2.imag / H, w1.imag / H, w2.imag / H, ah.imag / H, ad.imag / H]
    lhs = sum(np.sum(seed[j] * Jd[j]) for j in range(4)) + seed[4] * Jd[4] + seed[5] * Jd[5]
    rhs = (sum(np.sum(adj[k] * d[j]) for j, k in enumerate(("f1", "f2", "v1", "v2")))
           + adj["da0"] * da + adj["dad0"] * dad)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
