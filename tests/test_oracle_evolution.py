"""Pins of the oracle's time stepping (staggered leapfrog, eq. evo, applied to
eq. scalar-evo and eq. scale of Sainio, arXiv:0911.5692).

References used: the exact solution of the discrete leapfrog for free waves,
Jacobi cn for the homogeneous lambda phi^4 oscillation, a high-accuracy ODE
integration (scipy DOP853) of the homogeneous equations with expansion, the
Friedmann constraint, exact time reversibility, energy conservation in flat
space, and translation / axis-permutation equivariance.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import ellipj


def _grid(N, dx):
    z, y, x = np.meshgrid(*(np.arange(N) * dx,) * 3, indexing="ij")
    return x, y, z


def _hom(N, val):
    return np.full((N, N, N), float(val))


@pytest.mark.parametrize("c1", [0.0, 2.5])
def test_free_wave_exact_discrete_solution(orc, c1):
    """Flat space (kappa^2 = 0, a = 1), G = 0, V = c1 f^2/2: f(0) = cos(k.x),
    v(0) = 0 evolves as f(k) = cos(k Omega dt) cos(k.x) with
    sin(Omega dt/2) = omega dt/2, omega^2 = (4/dx^2) sum sin^2(k_i dx/2) + c1,
    exactly (the stored half-step value is cos(Omega dt (k+1/2))/cos(Omega dt/2))."""
    N, dx, dt = 8, 0.5, 0.05
    m = orc.Model(N=N, L=N * dx, dt=dt, beta=2, c1=c1, G=0.0, r=1.5, s=0.0, kappa2=0.0)
    x, y, z = _grid(N, dx)
    for n in [(1, 0, 0), (1, 2, 3), (4, 4, 4), (0, 3, 4)]:
        k = 2 * np.pi * np.array(n) / (N * dx)
        shape = np.cos(k[0] * x + k[1] * y + k[2] * z)
        w2 = (4 / dx ** 2) * np.sum(np.sin(k * dx / 2) ** 2) + c1
        Om = 2 * np.arcsin(np.sqrt(w2) * dt / 2) / dt
        st = orc.start(m, shape, np.zeros_like(shape), np.zeros_like(shape), np.zeros_like(shape),
                       1.0, 0.0)
        nsteps = 237
        orc.evolve(st, nsteps)
        exact_half = np.cos(Om * dt * (nsteps + 0.5)) / np.cos(Om * dt / 2) * shape
        assert np.max(np.abs(st.f1 - exact_half)) < 1e-12
        fs, _ = orc.synchronized_fields(st)
        assert np.max(np.abs(fs - np.cos(nsteps * Om * dt) * shape)) < 1e-12
        assert np.max(np.abs(st.f2)) == 0.0
        assert st.a_half == 1.0 and st.ad == 0.0


def test_homogeneous_lphi4_jacobi_cn_second_order(orc):
    """Homogeneous f'' = -f^3 (lambda phi^4, flat space) has f = f0 cn(f0 t | m=1/2);
    the leapfrog error at fixed t falls 4x per halving of dt, all sites stay equal."""
    N, f0, T = 4, 1.0, 3.0
    errs = []
    for dt in (0.02, 0.01, 0.005):
        m = orc.Model(N=N, L=N * 0.5, dt=dt, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=0.0)
        st = orc.start(m, _hom(N, f0), _hom(N, 0), _hom(N, 0), _hom(N, 0), 1.0, 0.0)
        n = int(round(T / dt))
        orc.evolve(st, n)
        fs, _ = orc.synchronized_fields(st)
        assert np.all(fs == fs.flat[0])
        exact = f0 * ellipj(f0 * T, 0.5)[1]
        errs.append(abs(fs.flat[0] - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.9 < r1 < 4.1 and 3.9 < r2 < 4.1, errs


def _ode_rhs(beta, c1, G, r, s, kappa2):
    """Homogeneous eq. (scalar-evo) and eq. (scale) as a first-order system in
    (f1, f2, f1', f2', a, a')."""
    p1, p2 = -2 * s + (2 - beta) * r, -2 * s - 2 * r

    def rhs(t, y):
        f1, f2, v1, v2, a, ad = y
        V = c1 * a ** p1 * f1 ** beta / beta + 0.5 * G * a ** p2 * f1 ** 2 * f2 ** 2
        add = (-s - 2) * ad ** 2 / a + kappa2 * a ** (-2 * s - 2 * r - 1) * a ** (2 * s + 2) * V
        b = r * (s - r + 2) * (ad / a) ** 2 + r * add / a
        d1 = c1 * a ** p1 * f1 ** (beta - 1) + G * a ** p2 * f1 * f2 ** 2
        d2 = G * a ** p2 * f1 ** 2 * f2
        return [v1, v2, b * f1 - d1, b * f2 - d2, ad, add]
    return rhs


@pytest.mark.parametrize("model", ["m2phi2", "lphi4"])
def test_homogeneous_expansion_vs_dop853(orc, model):
    """Homogeneous mode with expansion against DOP853 (rtol 1e-12): the
    synchronised f, f', a, a' converge at second order in dt."""
    if model == "m2phi2":
        kw = dict(beta=2, c1=1.0, G=50.0, r=1.5, s=0.0, kappa2=1.0187733)
        f10, f20, u10 = 1.0, 0.05, -0.7071
    else:
        kw = dict(beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=1.0187733)
        f10, f20, u10 = 1.0, 0.02, 0.1
    N, T = 4, 2.0
    errs = []
    for dt in (2 ** -5, 2 ** -6, 2 ** -7):
        m = orc.Model(N=N, L=2.0, dt=dt, **kw)
        v1, v2, ad0 = orc.init_physical(m, _hom(N, f10), _hom(N, f20), _hom(N, u10), _hom(N, 0), 1.0)
        y0 = [f10, f20, v1.flat[0], v2.flat[0], 1.0, ad0]
        sol = solve_ivp(_ode_rhs(**kw), (0, T), y0, method="DOP853", rtol=1e-12, atol=1e-14)
        st = orc.start(m, _hom(N, f10), _hom(N, f20), v1, v2, 1.0, ad0)
        orc.evolve(st, int(round(T / dt)))
        fs1, fs2 = orc.synchronized_fields(st)
        e = orc.energies(st)
        got = np.array([fs1.flat[0], fs2.flat[0], st.v1.flat[0], st.v2.flat[0], e["a"], e["ad"]])
        errs.append(np.abs(got - sol.y[:, -1]))
    e0, e1, e2 = (np.max(x) for x in errs)
    assert 3.7 < e0 / e1 < 4.3 and 3.7 < e1 / e2 < 4.3, errs
    assert e2 < 1e-3


def _white(N, seed, amp=1e-2):
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.standard_normal((N, N, N)), amp * rng.standard_normal((N, N, N))


@pytest.mark.parametrize("case", ["homog_m2phi2", "lattice_lphi4"])
def test_friedmann_residual_second_order(orc, case):
    """The Friedmann residual R vanishes at t = 0 (a'(0) from the constraint)
    and is O(dt^2) later: halving dt divides it by ~4."""
    N = 4 if case.startswith("homog") else 6
    Rs = []
    for dt in (0.04, 0.02, 0.01):
        if case == "homog_m2phi2":
            m = orc.Model(N=N, L=2.0, dt=dt, beta=2, c1=1.0, G=50.0, r=1.5, s=0.0, kappa2=1.0187733)
            f1, f2, u1 = _hom(N, 1.0), _hom(N, 0.05), _hom(N, -0.7071)
        else:
            m = orc.Model(N=N, L=N * 0.625, dt=dt, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0,
                          kappa2=1.0187733)
            f1, f2 = _white(N, 5, 0.05)
            u1 = np.zeros_like(f1)
        st = orc.start_physical(m, f1, f2, u1, np.zeros_like(f1), 1.0)
        orc.evolve(st, int(round(1.0 / dt)))
        Rs.append(orc.energies(st)["R"])
    assert 3.5 < Rs[0] / Rs[1] < 4.5 and 3.5 < Rs[1] / Rs[2] < 4.5, Rs


def test_friedmann_residual_zero_initially(orc):
    """With a'(0) from the constraint, the synchronised residual at step 0 is 0."""
    N = 5
    m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0,
                  kappa2=1.0187733)
    f1, f2 = _white(N, 9, 0.05)
    rng = np.random.default_rng(2)
    u1, u2 = 0.01 * rng.standard_normal((2, N, N, N))
    st = orc.start_physical(m, f1, f2, u1, u2, 1.0)
    assert abs(orc.energies(st)["R"]) < 1e-14


@pytest.mark.parametrize("N", [4, 6, 8])
def test_time_reversibility(orc, N):
    """Synchronise after n steps, reverse v and a', evolve n more steps: the
    initial state returns with reversed velocities (exact in exact arithmetic)."""
    for model in ("lphi4", "m2phi2"):
        if model == "lphi4":
            m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0,
                          kappa2=1.0187733)
        else:
            m = orc.Model(N=N, L=N * 0.1, dt=2 ** -8, beta=2, c1=1.0, G=300.0, r=1.5, s=0.0,
                          kappa2=1.0187733)
        f1, f2 = _white(N, N, 0.05)
        u1 = np.full_like(f1, -0.3)
        v1, v2, ad0 = orc.init_physical(m, f1, f2, u1, np.zeros_like(f1), 1.0)
        st = orc.start(m, f1, f2, v1, v2, 1.0, ad0)
        orc.evolve(st, 100)
        fs1, fs2 = orc.synchronized_fields(st)
        e = orc.energies(st)
        back = orc.start(m, fs1, fs2, -st.v1, -st.v2, e["a"], -e["ad"])
        orc.evolve(back, 100)
        g1, g2 = orc.synchronized_fields(back)
        eb = orc.energies(back)
        assert np.max(np.abs(g1 - f1)) < 1e-12 and np.max(np.abs(g2 - f2)) < 1e-12
        assert np.max(np.abs(back.v1 + v1)) < 1e-12 * max(1, np.max(np.abs(v1)))
        assert np.max(np.abs(back.v2 + v2)) < 1e-12
        assert abs(eb["a"] - 1.0) < 1e-12 and abs(eb["ad"] + ad0) < 1e-12


def test_flat_space_energy_no_secular_drift(orc):
    """kappa^2 = 0: rho_pr oscillates at O(dt^2) with no secular drift."""
    N = 6
    m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=0.0)
    f1, f2 = _white(N, 11, 0.1)
    st = orc.start(m, f1, f2, np.zeros_like(f1), np.zeros_like(f1), 1.0, 0.0)
    rhos = []
    for _ in range(100):
        orc.evolve(st, 100)
        rhos.append(orc.energies(st)["rho"])
    rhos = np.array(rhos)
    t = np.arange(len(rhos))
    band = np.ptp(rhos)
    slope = np.polyfit(t, rhos, 1)[0]  # per 100 steps
    # any linear drift over the 10^4 steps is far inside the O(dt^2) band ...
    assert abs(slope) * len(rhos) < 0.1 * band
    # ... the band does not grow ...
    half = len(rhos) // 2
    dev = np.abs(rhos - rhos.mean())
    assert dev[half:].max() < 1.5 * dev[:half].max()
    # ... and it is small
    assert band < 1e-2 * rhos.mean()


def test_equivariance_roll_and_transpose(orc):
    """Rolling or permuting the axes of the initial state rolls/permutes the
    result (up to the summation order of the volume averages)."""
    N = 6
    m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0,
                  kappa2=1.0187733)
    f1, f2 = _white(N, 13, 0.05)
    rng = np.random.default_rng(4)
    u1 = 0.02 * rng.standard_normal(f1.shape)
    base = orc.start_physical(m, f1, f2, u1, np.zeros_like(f1), 1.0)
    orc.evolve(base, 40)
    for tf in (lambda a: np.roll(a, (1, 2, 3), axis=(0, 1, 2)),
               lambda a: np.ascontiguousarray(np.transpose(a, (2, 1, 0))),
               lambda a: np.ascontiguousarray(np.transpose(a, (1, 0, 2)))):
        st = orc.start_physical(m, tf(f1), tf(f2), tf(u1), np.zeros_like(f1), 1.0)
        orc.evolve(st, 40)
        for a, b in ((st.f1, base.f1), (st.f2, base.f2), (st.v1, base.v1), (st.v2, base.v2)):
            assert np.max(np.abs(a - tf(b))) <= 1e-13 * max(1.0, np.max(np.abs(b)))
        assert abs(st.a_half - base.a_half) < 1e-14
