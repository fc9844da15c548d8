"""Pins of the oracle's energy density and pressure (eq. rho-pres, program
units) by the virial theorem and the radiation equation of state:
time-averaged w = <p>/<rho> is 0 for a homogeneous m^2 phi^2 oscillation,
1/3 for a homogeneous lambda phi^4 oscillation and 1/3 for a free massless
standing wave, all in flat space."""
import numpy as np
import pytest


def _hom(N, v):
    return np.full((N, N, N), float(v))


def _time_avg_w(orc, st, nsteps, every):
    rs, ps = [], []
    for _ in range(nsteps // every):
        orc.evolve(st, every)
        _, _, avg = orc.rho_p(st, arrays=False)
        rs.append(avg["rho"])
        ps.append(avg["p"])
    return np.mean(ps) / np.mean(rs), np.array(rs)


@pytest.mark.parametrize("beta,w_expect", [(2, 0.0), (4, 1.0 / 3.0)])
def test_virial_equation_of_state_homogeneous(orc, beta, w_expect):
    N = 4
    r, s = (1.5, 0.0) if beta == 2 else (1.0, -1.0)
    m = orc.Model(N=N, L=1.0, dt=0.005, beta=beta, c1=1.0, G=0.0, r=r, s=s, kappa2=0.0)
    st = orc.start(m, _hom(N, 1.0), _hom(N, 0.0), _hom(N, 0.0), _hom(N, 0.0), 1.0, 0.0)
    # many oscillation periods (T = 2 pi for beta 2, 7.416 for beta 4)
    w, rho = _time_avg_w(orc, st, 60000, 10)
    assert abs(w - w_expect) < 2e-3, w
    assert np.ptp(rho) < 1e-4 * rho.mean()  # conserved energy


def test_radiation_equation_of_state_standing_wave(orc):
    N, dx = 16, 0.5
    m = orc.Model(N=N, L=N * dx, dt=0.02, beta=2, c1=0.0, G=0.0, r=1.5, s=0.0, kappa2=0.0)
    z, y, x = np.meshgrid(*(np.arange(N) * dx,) * 3, indexing="ij")
    f = np.cos(2 * np.pi * 2 * x / (N * dx)) * np.cos(2 * np.pi * 3 * y / (N * dx))
    st = orc.start(m, f, 0 * f, 0 * f, 0 * f, 1.0, 0.0)
    w, _ = _time_avg_w(orc, st, 40000, 5)
    assert abs(w - 1.0 / 3.0) < 3e-3, w


def test_rho_matches_energies_and_pressure_per_site(orc):
    N = 6
    m = orc.Model(N=N, L=N * 0.625, dt=0.03125, beta=4, c1=1.0, G=100.0, r=1.0, s=-1.0, kappa2=1.0187733)
    rng = np.random.default_rng(3)
    f1 = 1.0 + 0.05 * rng.standard_normal((N, N, N))
    f2 = 0.05 * rng.standard_normal((N, N, N))
    st = orc.start_physical(m, f1, f2, 0 * f1, 0 * f1, 1.0)
    orc.evolve(st, 17)
    rho, p, avg = orc.rho_p(st)
    e = orc.energies(st)
    assert abs(avg["rho"] - e["rho"]) <= 1e-14 * e["rho"]
    # p = rho - 2 (sum G/3 ... ): rho - p = 4/3 sum G + 2 V per site, so the averages obey
    assert abs((avg["rho"] - avg["p"]) - (4.0 / 3.0 * (e["G1"] + e["G2"]) + 2.0 * e["P"])) <= 1e-13 * avg["rho"]
    assert abs(rho.mean() - avg["rho"]) <= 1e-14 * avg["rho"] and abs(avg["w"] - avg["p"] / avg["rho"]) < 1e-15
