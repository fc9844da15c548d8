"""The benchmark and parity workloads, as plain data, plus their seeded inputs.

Program units throughout (Sainio, arXiv:0911.5692, Sec. II.B).  Models:
  lambda phi^4 + g^2 phi^2 chi^2 / 2, rescaled with A = 1/phi0, B = sqrt(lambda) phi0,
      r = 1, s = -1:  c1 = 1, G = g^2/lambda, no a-dependence of V_pr;
  m^2 phi^2 / 2 + g^2 phi^2 chi^2 / 2 (the chaotic-inflation model of Sec. III),
      A = 1/phi0, B = m, r = 3/2, s = 0:  c1 = 1, G = g^2 phi0^2 / m^2, V_pr's coupling
      term carries a^-3.
kappa2 = 8 pi G_N / A^2 = phi0^2 in reduced-Planck units; with the paper's
phi0 = 1.009343 (Sec. III) that is 1.0187733, used for every workload.

Initial velocities are given as rescaled physical velocities u = (A/B) a^(r-s) dphi/dt;
the program-unit velocities and a'(0) follow from the Friedmann constraint inside
the library (and, independently, inside the oracle).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import inputs

PHI0 = 1.009343          # homogeneous inflaton, reduced Planck units (Sec. III)
HUBBLE0 = 0.50467        # initial H / m (Sec. III)
KAPPA2 = PHI0 ** 2       # 8 pi G / A^2 with A = 1/phi0 and 8 pi G = 1
# Initial inflaton velocity in program units, u0 = dphi/dt / (phi0 m): from the
# Friedmann constraint 3 H^2 = phidot^2/2 + m^2 phi0^2/2 with the paper's phi0 and H,
# phidot = -sqrt(6 H^2 - phi0^2) = -0.7137069 (the inflaton rolls down).
U0_INFLATON = -0.7071004761148857
# Vacuum-fluctuation amplitude in program units, m / phi0 with m = 5e-6 M_pl (Sec. III;
# the printed exponent sign is read as 5e-6).
EPS_VACUUM = 5e-6 / PHI0


@dataclass(frozen=True)
class Workload:
    name: str
    cfg: int            # seed namespace
    N: int
    L: float
    dt: float
    beta: int
    c1: float
    G: float
    r: float
    s: float
    kappa2: float
    steps: int
    dtype: str          # "f32" or "f64": element type of the lattice arrays
    ic: str             # "white" | "grf" | "vacuum"
    stencil: int = 7    # Laplacian: 7 or 27 points (Sec. II.C)

    @property
    def dx(self) -> float:
        return self.L / self.N

    @property
    def sites(self) -> int:
        return self.N ** 3

    def model(self) -> dict:
        """Keyword arguments accepted by both the Lattice and the oracle Model."""
        return dict(N=self.N, L=self.L, dt=self.dt, beta=self.beta, c1=self.c1, G=self.G,
                    r=self.r, s=self.s, kappa2=self.kappa2, stencil=self.stencil)

    def resized(self, N: int) -> "Workload":
        """Same model, dx and dt on an N^3 box (L scales with N)."""
        return replace(self, N=N, L=self.dx * N)


def _lphi4(name, cfg, N, steps, dtype, ic):
    L = 20.0
    return Workload(name, cfg, N, L, (L / N) / 20.0, 4, 1.0, 100.0, 1.0, -1.0, KAPPA2, steps,
                    dtype, ic)


CFG1 = _lphi4("lphi4_32c_f64", 1, 32, 200, "f64", "white")
CFG2 = _lphi4("lphi4_256c_f32", 2, 256, 1000, "f32", "grf")
CFG3 = Workload("m2phi2_512c_f32", 3, 512, 10.0, 2.0 ** -10, 2, 1.0, 2.5e5, 1.5, 0.0, KAPPA2,
                2000, "f32", "vacuum")
CFG5 = _lphi4("lphi4_128c_f32_adjoint", 5, 128, 500, "f32", "white")
# the 512^3 m^2 phi^2 run with the paper's own 27-point Laplacian (same inputs)
CFG3_S27 = replace(CFG3, name="m2phi2_512c_f32_s27", stencil=27)
# the configuration the paper times (Sec. III): 256^3, the same model and dt,
# FP32, 27-point Laplacian (box side at the benchmark's dx)
PAPER_256_S27 = replace(CFG3_S27.resized(256), name="m2phi2_256c_f32_s27")
# ensemble: 48 x 64^3 + 16 x 96^3 + 4 x 160^3 of the lambda phi^4 model, own dx and dt each
ENSEMBLE_SIZES = [64] * 48 + [96] * 16 + [160] * 4
ENSEMBLE_STEPS = 500


def ensemble_members():
    return [_lphi4(f"ens{r}_{n}c", 4, n, ENSEMBLE_STEPS, "f32", "white")
            for r, n in enumerate(ENSEMBLE_SIZES)]


WORKLOADS = {w.name: w for w in (CFG1, CFG2, CFG3, CFG5, CFG3_S27, PAPER_256_S27)}

# Sweep launch shapes used by the benchmark, measured on an MI355X (gfx950)
# with lf_autotune and sweeps of tiles and z-chunks.  Re-run the autotuner
# (bench.py --autotune) on other parts.
BENCH_SHAPES = {
    CFG3.name: dict(tile_x=128, tile_y=8, zchunk=256),
    CFG3_S27.name: dict(tile_x=128, tile_y=8, zchunk=256),
    PAPER_256_S27.name: dict(tile_x=128, tile_y=8, zchunk=32),
}


def vacuum_spec(w: Workload, seed: int) -> dict:
    """Spectrum of the vacuum workloads for the device generator
    (Lattice.init_vacuum / vacuum_fields): f = (1, 0) + fluctuations,
    u = (U0_INFLATON, 0) + fluctuations, m_eff^2 = (c1, G) at f1 = 1, f2 = 0,
    amplitude EPS_VACUUM, cut at N/4."""
    return dict(f0=(1.0, 0.0), u0=(U0_INFLATON, 0.0), m2=(w.c1, w.G), eps2=EPS_VACUUM ** 2, cutoff=0.0,
                seed=int(seed))


def make_inputs(w: Workload, realization: int = 0) -> dict:
    """Initial fields f1, f2 and rescaled physical velocities u1, u2 (float64),
    a0 = 1.  Seeds: SeedSequence([cfg, realization, field, kind])."""
    N, L = w.N, w.L
    if w.ic == "white":
        f1 = 1.0 + inputs.white_noise(N, 1e-3, inputs.rng_for(w.cfg, realization, 0, 0))
        f2 = inputs.white_noise(N, 1e-3, inputs.rng_for(w.cfg, realization, 1, 0))
        u1 = np.zeros_like(f1)
        u2 = np.zeros_like(f1)
    elif w.ic == "grf":
        # P ∝ 1/omega_k, m_eff^2 = d^2 V_pr/df_i^2 at f1 = 1, f2 = 0: 3 and G
        f1 = 1.0 + inputs.gaussian_random_field(N, L, 3.0 * w.c1, inputs.rng_for(w.cfg, realization, 0, 0),
                                                std=1e-3)
        f2 = inputs.gaussian_random_field(N, L, w.G, inputs.rng_for(w.cfg, realization, 1, 0), std=1e-3)
        u1 = np.zeros_like(f1)
        u2 = np.zeros_like(f1)
    elif w.ic == "vacuum":
        e2 = EPS_VACUUM ** 2
        m1, m2 = w.c1, w.G  # m_eff^2 at f1 = 1, f2 = 0, a = 1
        f1 = 1.0 + inputs.gaussian_random_field(N, L, m1, inputs.rng_for(w.cfg, realization, 0, 0),
                                                amplitude2=e2)
        f2 = inputs.gaussian_random_field(N, L, m2, inputs.rng_for(w.cfg, realization, 1, 0), amplitude2=e2)
        u1 = U0_INFLATON + inputs.gaussian_random_field(N, L, m1, inputs.rng_for(w.cfg, realization, 0, 1),
                                                        amplitude2=e2, kind="velocity")
        u2 = inputs.gaussian_random_field(N, L, m2, inputs.rng_for(w.cfg, realization, 1, 1),
                                          amplitude2=e2, kind="velocity")
    else:
        raise ValueError(w.ic)
    return dict(f1=f1, f2=f2, u1=u1, u2=u2, a0=1.0)


def tile_inputs(ic: dict, reps: int) -> dict:
    """Periodic repetition of an initial state reps times along each axis."""
    out = {k: (np.tile(v, (reps, reps, reps)) if isinstance(v, np.ndarray) else v)
           for k, v in ic.items()}
    return out
