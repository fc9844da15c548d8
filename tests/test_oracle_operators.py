"""Pins of the oracle's lattice operators and volume averages.

Each check compares the oracle with something other than itself: the
closed-form eigenvalue of the 7-point Laplacian on plane waves, pure-Python
brute-force sums, and the rescaling of the physical potential written from
the definitions of Sec. II.B.
"""
import itertools

import numpy as np
import pytest


def _model(orc, N, dx=0.3, **kw):
    base = dict(N=N, L=N * dx, dt=0.01, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=1.0)
    base.update(kw)
    return orc.Model(**base)


def _grid(N, dx):
    z, y, x = np.meshgrid(*(np.arange(N) * dx,) * 3, indexing="ij")
    return x, y, z


@pytest.mark.parametrize("N", [8, 7])
def test_laplacian_plane_wave_eigenvalue(orc, N):
    """Lap cos(k.x + c) = -(4/dx^2) sum_i sin^2(k_i dx/2) cos(k.x + c) for every
    lattice wavevector, Nyquist included (the discrete closed form)."""
    dx = 0.37
    m = _model(orc, N, dx)
    x, y, z = _grid(N, dx)
    u = 2.0 ** -53
    ns = range(-(N // 2), N - N // 2)
    rng = np.random.default_rng(1)
    checked = 0
    for n in itertools.product(ns, ns, ns):
        if rng.random() > 0.25 and n != (N // 2, N // 2, N // 2) and n != (0, 0, N // 2):
            continue
        k = 2 * np.pi * np.array(n) / (N * dx)
        for phase in (0.0, 0.7):
            f = np.cos(k[0] * x + k[1] * y + k[2] * z + phase)
            lam = -(4.0 / dx ** 2) * np.sum(np.sin(k * dx / 2.0) ** 2)
            got = orc.laplacian(m, f)
            # bound from rounding the inputs and the 7-term sum
            assert np.max(np.abs(got - lam * f)) <= 64 * u * (1 + abs(lam) * dx ** 2) / dx ** 2
            checked += 1
    assert checked > 20


def _brute_grad2_sum(f, dx):
    N = f.shape[0]
    s = 0.0
    for z in range(N):
        for y in range(N):
            for x in range(N):
                c = f[z, y, x]
                s += ((f[z, y, (x + 1) % N] - c) ** 2 + (f[z, (y + 1) % N, x] - c) ** 2
                      + (f[(z + 1) % N, y, x] - c) ** 2)
    return s / dx ** 2


@pytest.mark.parametrize("N", [4, 5, 6])
def test_summation_by_parts(orc, N):
    """-<f Lap f> (the paper's divergence-theorem form, Sec. II.B) equals the
    brute-force <|grad+ f|^2> on a periodic lattice."""
    dx = 0.31
    m = _model(orc, N, dx)
    rng = np.random.default_rng(N)
    f1 = 1.0 + 0.1 * rng.standard_normal((N, N, N))
    f2 = 0.2 * rng.standard_normal((N, N, N))
    Sg, _ = orc.averages(m, f1, f2, 1.0)
    ref = (_brute_grad2_sum(f1, dx) + _brute_grad2_sum(f2, dx)) / N ** 3
    assert abs(Sg - ref) <= 1e-13 * ref
    g = orc.grad2(m, f2)
    assert abs(g.sum() - _brute_grad2_sum(f2, dx)) <= 1e-13 * g.sum()


@pytest.mark.parametrize("model", ["lphi4", "m2phi2", "beta6"])
def test_potential_rescaling(orc, model):
    """<V_pr> against the physical potential rescaled by the definitions of
    Sec. II.B: V_pr = (A^2/B^2) a^(-2s+2r) V(phi), phi = f/(A a^r)."""
    N = 4
    rng = np.random.default_rng(3)
    f1 = 1.0 + 0.2 * rng.standard_normal((N, N, N))
    f2 = 0.3 * rng.standard_normal((N, N, N))
    phi0, a = 1.3, 1.7
    if model == "lphi4":
        beta, cpl, g2, r, s = 4, 2.0, 5.0, 1.0, -1.0
    elif model == "m2phi2":
        beta, cpl, g2, r, s = 2, 0.8, 5.0, 1.5, 0.0
    else:
        beta, cpl, g2, r, s = 6, 0.5, 3.0, 0.75, -1.5
    A = 1.0 / phi0
    B = np.sqrt(cpl) * phi0 ** (-1 + beta / 2)   # Sec. II.B rescaling for V = cpl phi^beta/beta
    c1 = cpl * A ** (2 - beta) / B ** 2
    G = g2 * A ** -2 / B ** 2
    m = _model(orc, N, beta=beta, c1=c1, G=G, r=r, s=s)
    phi, chi = f1 / (A * a ** r), f2 / (A * a ** r)
    V = cpl * phi ** beta / beta + 0.5 * g2 * phi ** 2 * chi ** 2
    ref = np.mean((A ** 2 / B ** 2) * a ** (-2 * s + 2 * r) * V)
    _, SV = orc.averages(m, f1, f2, a)
    assert abs(SV - ref) <= 1e-13 * abs(ref)


def test_scale_quadratic_solves_midpoint_equation(orc):
    """The returned a'_{k+1} satisfies the time-centred form of eq. (scale)
    (checked by substitution), and a'' and a_{k+3/2} follow from it."""
    for r, s in ((1.0, -1.0), (1.5, 0.0), (0.75, -1.5)):
        m = _model(orc, 4, r=r, s=s, dt=0.05)
        a, w, Sg, SV = 1.3, 0.4, 0.02, 0.6
        u, adh, add, an = orc.scale_step(m, a, w, Sg, SV)
        Fa = m.kappa2 * a ** (-2 * s - 2 * r - 1) * (Sg / 3 + a ** (2 * s + 2) * SV)
        rhs = w + m.dt * ((-s - 2) * ((w + u) / 2) ** 2 / a + Fa)
        assert abs(u - rhs) <= 1e-15 * abs(u) * 4
        assert abs(adh - (w + u) / 2) <= 1e-16
        assert abs(add - (u - w) / m.dt) <= 1e-12 * abs(add)
        assert abs(an - (a + m.dt * u)) <= 1e-15
        # the other root of the quadratic is far away (no root confusion)
        c = (-s - 2) * m.dt / (4 * a)
        if c != 0:
            other = (1 - 2 * c * w) / c - u
            assert abs(other - u) > 10 * abs(u)
