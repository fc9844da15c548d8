"""Pins of the oracle's 27-point Laplacian (the stencil the paper itself uses,
Sec. II.C: all 26 neighbours of the 3x3x3 cube, second-order accurate,
fourth-order isotropic) and of everything built on it.

The weights are not printed in the paper; the reading taken is the member
(centre, face, edge, corner) = (-64/15, 7/15, 1/10, 1/30) of the family that
the stated properties leave open.  The properties themselves are checked on
the oracle's operator, independently of that choice: zero sum, second-order
consistency, and isotropy of the O(k^4) error (where the 7-point stencil is
anisotropic).  The member is then fixed by the closed-form plane-wave
eigenvalue.  The gradient energy is checked as the stencil's Dirichlet form
against a brute-force bond sum, and the time stepping against the exact
discrete free-wave solution, energy conservation and complex-step
differentiation of the adjoint.
"""
import itertools

import numpy as np
import pytest

W = (-64.0 / 15.0, 7.0 / 15.0, 1.0 / 10.0, 1.0 / 30.0)  # the reading (centre, face, edge, corner)
U = 2.0 ** -53


def _model(orc, N, dx=0.3, stencil=27, **kw):
    base = dict(N=N, L=N * dx, dt=0.01, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=1.0,
                stencil=stencil)
    base.update(kw)
    return orc.Model(**base)


def _grid(N, dx):
    z, y, x = np.meshgrid(*(np.arange(N) * dx,) * 3, indexing="ij")
    return x, y, z


def _symbol(theta):
    """dx^2 x eigenvalue of the 27-point stencil on exp(i k.x), theta = k dx."""
    c = np.cos(theta)
    pairs = c[0] * c[1] + c[0] * c[2] + c[1] * c[2]
    return W[0] + 2 * W[1] * c.sum() + 4 * W[2] * pairs + 8 * W[3] * c.prod()


def _eig(orc, N, n, stencil, dx=1.0):
    """Eigenvalue x dx^2 read off the oracle's operator for wavevector index n."""
    m = _model(orc, N, dx, stencil=stencil)
    x, y, z = _grid(N, dx)
    k = 2 * np.pi * np.array(n) / (N * dx)
    f = np.cos(k[0] * x + k[1] * y + k[2] * z)
    return orc.laplacian(m, f)[0, 0, 0] * dx * dx  # f = 1 at the origin


def test_zero_sum_and_constant_field(orc):
    m = _model(orc, 5)
    f = np.full((5, 5, 5), 3.7)
    assert np.max(np.abs(orc.laplacian(m, f))) <= 64 * U * 3.7 / 0.09
    assert np.max(np.abs(orc.grad2(m, f))) == 0.0


@pytest.mark.parametrize("n", [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0)])
def test_second_order_consistency(orc, n):
    """lambda dx^2 = -theta^2 + O(theta^4): the error falls 16x when the
    wavevector halves (doubling N at fixed mode index n)."""
    errs = []
    for N in (32, 64):
        theta2 = np.sum((2 * np.pi * np.array(n) / N) ** 2)
        errs.append(_eig(orc, N, n, 27) + theta2)
    assert 14.0 < errs[0] / errs[1] < 17.0


def test_fourth_order_isotropy(orc):
    """Wavevectors of equal length along different lattice directions:
    the 27-point eigenvalues agree up to O(k^6) (anisotropy falls 64x per
    halving of k), the 7-point ones differ at O(k^4) (16x)."""
    dirs = [(9, 0, 0), (6, 6, 3), (8, 4, 1), (7, 4, 4)]  # |n| = 9
    spread = {}
    for st in (7, 27):
        for N in (96, 192):
            lam = [_eig(orc, N, n, st) for n in dirs]
            spread[(st, N)] = max(lam) - min(lam)
    r27 = spread[(27, 96)] / spread[(27, 192)]
    r7 = spread[(7, 96)] / spread[(7, 192)]
    assert 55.0 < r27 < 70.0
    assert 14.0 < r7 < 17.5
    assert spread[(27, 96)] < 0.05 * spread[(7, 96)]


@pytest.mark.parametrize("N", [6, 7])
def test_plane_wave_eigenvalue_closed_form(orc, N):
    """Lap cos(k.x + c) = dx^-2 [w0 + 2 w1 sum c_i + 4 w2 sum c_i c_j
    + 8 w3 c_x c_y c_z] cos(k.x + c), c_i = cos(k_i dx), for sampled lattice
    wavevectors, Nyquist included: fixes the member of the family."""
    dx = 0.37
    m = _model(orc, N, dx)
    x, y, z = _grid(N, dx)
    ns = range(-(N // 2), N - N // 2)
    rng = np.random.default_rng(2)
    checked = 0
    for n in itertools.product(ns, ns, ns):
        if rng.random() > 0.3 and n != (N // 2,) * 3:
            continue
        k = 2 * np.pi * np.array(n) / (N * dx)
        for phase in (0.0, 0.9):
            f = np.cos(k[0] * x + k[1] * y + k[2] * z + phase)
            lam = _symbol(k * dx) / dx ** 2
            got = orc.laplacian(m, f)
            assert np.max(np.abs(got - lam * f)) <= 512 * U / dx ** 2
            checked += 1
    assert checked > 40


def _brute_dirichlet(f, dx):
    """1/2 sum_x sum over all 26 neighbours d of w_d (f(x+d) - f(x))^2 / dx^2."""
    N = f.shape[0]
    tot = 0.0
    for z, y, x in itertools.product(range(N), repeat=3):
        for dz, dy, dx_ in itertools.product((-1, 0, 1), repeat=3):
            nz = abs(dz) + abs(dy) + abs(dx_)
            if nz == 0:
                continue
            d = f[(z + dz) % N, (y + dy) % N, (x + dx_) % N] - f[z, y, x]
            tot += 0.5 * W[nz] * d * d
    return tot / dx ** 2


@pytest.mark.parametrize("N", [4, 5])
def test_gradient_energy_is_the_dirichlet_form(orc, N):
    """sum grad2 equals the brute-force bond sum and -sum f Lap f (so the
    semi-discrete dynamics conserves this energy), and Sg of the averages."""
    dx = 0.41
    m = _model(orc, N, dx)
    rng = np.random.default_rng(10 + N)
    f1 = 1.0 + 0.1 * rng.standard_normal((N, N, N))
    f2 = 0.2 * rng.standard_normal((N, N, N))
    b1, b2 = _brute_dirichlet(f1, dx), _brute_dirichlet(f2, dx)
    g1 = orc.grad2(m, f1).sum()
    assert abs(g1 - b1) <= 1e-13 * b1
    assert abs(-np.sum(f1 * orc.laplacian(m, f1)) - b1) <= 1e-12 * b1
    Sg, _ = orc.averages(m, f1, f2, 1.0)
    assert abs(Sg - (b1 + b2) / N ** 3) <= 1e-13 * Sg
    assert np.all(orc.grad2(m, f2) >= 0.0)


def test_gradient_density_of_a_linear_field(orc):
    """Per site, grad2 of f = g.x (at sites whose 13 bonds do not cross the
    periodic seam) is |g|^2: the density is a consistent |grad f|^2."""
    N, dx = 9, 0.5
    m = _model(orc, N, dx)
    x, y, z = _grid(N, dx)
    g = np.array([0.3, -1.1, 0.7])
    f = g[0] * x + g[1] * y + g[2] * z
    d = orc.grad2(m, f)
    inner = d[0:N - 1, 1:N - 1, 1:N - 1]  # bonds go to z, z+1; y, x within +-1
    assert np.max(np.abs(inner - g @ g)) <= 1e-12


@pytest.mark.parametrize("c1", [0.0, 2.5])
def test_free_wave_exact_discrete_solution(orc, c1):
    """Flat space, G = 0, V = c1 f^2/2: cos(k.x) evolves as cos(k Omega dt)
    cos(k.x) with sin(Omega dt/2) = omega dt/2, omega^2 = -lambda_27(k) + c1."""
    N, dx, dt = 8, 0.5, 0.05
    m = orc.Model(N=N, L=N * dx, dt=dt, beta=2, c1=c1, G=0.0, r=1.5, s=0.0, kappa2=0.0, stencil=27)
    x, y, z = _grid(N, dx)
    for n in [(1, 0, 0), (1, 2, 3), (4, 4, 4), (0, 3, 4)]:
        k = 2 * np.pi * np.array(n) / (N * dx)
        shape = np.cos(k[0] * x + k[1] * y + k[2] * z)
        w2 = -_symbol(k * dx) / dx ** 2 + c1
        Om = 2 * np.arcsin(np.sqrt(w2) * dt / 2) / dt
        zero = np.zeros_like(shape)
        st = orc.start(m, shape, zero, zero, zero, 1.0, 0.0)
        nsteps = 211
        orc.evolve(st, nsteps)
        fs, _ = orc.synchronized_fields(st)
        assert np.max(np.abs(fs - np.cos(nsteps * Om * dt) * shape)) < 1e-12


def _white(N, seed, amp):
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.standard_normal((N, N, N)), amp * rng.standard_normal((N, N, N))


def test_flat_space_energy_no_secular_drift(orc):
    """kappa^2 = 0, interacting fields: rho_pr (with the Dirichlet-form
    gradient energy) oscillates at O(dt^2) with no secular drift."""
    N = 6
    m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=0.0,
                  stencil=27)
    f1, f2 = _white(N, 11, 0.1)
    st = orc.start(m, f1, f2, np.zeros_like(f1), np.zeros_like(f1), 1.0, 0.0)
    rhos = []
    for _ in range(60):
        orc.evolve(st, 100)
        rhos.append(orc.energies(st)["rho"])
    rhos = np.array(rhos)
    band = np.ptp(rhos)
    slope = np.polyfit(np.arange(len(rhos)), rhos, 1)[0]
    assert abs(slope) * len(rhos) < 0.1 * band
    assert band < 1e-2 * rhos.mean()


def test_friedmann_residual_and_reversibility(orc):
    """Expanding lambda phi^4 lattice with the 27-point stencil: R = 0 at the
    Friedmann initialisation and O(dt^2) at t = 1 (halving dt divides it by
    ~4); synchronise, reverse the velocities and a', evolve back: the initial
    state returns."""
    N = 6
    f1, f2 = _white(N, 5, 0.05)
    u1 = np.full_like(f1, -0.3)
    Rs = []
    for dt in (0.04, 0.02, 0.01):
        m = orc.Model(N=N, L=N * 0.625, dt=dt, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0,
                      kappa2=1.0187733, stencil=27)
        st = orc.start_physical(m, f1, f2, u1, np.zeros_like(f1), 1.0)
        assert abs(orc.energies(st)["R"]) < 1e-13
        orc.evolve(st, int(round(1.0 / dt)))
        Rs.append(orc.energies(st)["R"])
    assert 3.5 < Rs[0] / Rs[1] < 4.5 and 3.5 < Rs[1] / Rs[2] < 4.5, Rs
    m = m.replace(dt=0.03125)
    v1, v2, ad0 = orc.init_physical(m, f1, f2, u1, np.zeros_like(f1), 1.0)
    st = orc.start(m, f1, f2, v1, v2, 1.0, ad0)
    orc.evolve(st, 200)
    e = orc.energies(st)
    fs1, fs2 = orc.synchronized_fields(st)
    back = orc.start(m, fs1, fs2, -st.v1, -st.v2, e["a"], -e["ad"])
    orc.evolve(back, 200)
    g1, g2 = orc.synchronized_fields(back)
    assert np.max(np.abs(g1 - f1)) < 1e-12 and np.max(np.abs(g2 - f2)) < 1e-12


H = 1e-30


def test_adjoint_matches_complex_step(orc):
    """The hand-written adjoint with the 27-point stencil against complex-step
    derivatives of the oracle's forward map in every input direction and G."""
    N = 4
    m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0,
                  kappa2=1.0187733, stencil=27)
    rng = np.random.default_rng(8)
    f1 = 1.0 + 0.05 * rng.standard_normal((N, N, N))
    f2 = 0.05 * rng.standard_normal((N, N, N))
    u1 = -0.3 + 0.05 * rng.standard_normal((N, N, N))
    v1, v2, ad0 = orc.init_physical(m, f1, f2, u1, 0.02 * rng.standard_normal((N, N, N)), 1.0)
    n = 10
    wK, wG = (0.3, 1.0), (0.5, 1.0)
    adj = orc.adjoint(m, f1, f2, v1, v2, 1.0, ad0, n, wK=wK, wG=wG)

    def loss(G=m.G, d=None):
        x = [xi.astype(np.complex128) for xi in (f1, f2, v1, v2)]
        if d is not None:
            x = [xi + 1j * H * dj for xi, dj in zip(x, d)]
        en = orc.complex_run(m, G, *x, 1.0, ad0, n)[-1]
        return wK[0] * en[2] + wK[1] * en[3] + wG[0] * en[4] + wG[1] * en[5]

    assert abs(loss().real - adj["E"]) <= 1e-14 * abs(adj["E"])
    d = [rng.standard_normal(f1.shape) for _ in range(4)]
    cs = loss(d=d).imag / H
    ad = sum(np.sum(adj[k] * d[j]) for j, k in enumerate(("f1", "f2", "v1", "v2")))
    assert abs(cs - ad) <= 1e-10 * abs(cs)
    cs = loss(G=complex(m.G, H)).imag / H
    assert abs(cs - adj["dG"]) <= 1e-10 * abs(cs)
