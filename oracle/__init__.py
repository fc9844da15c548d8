"""FP64 CPU oracle for the FRW lattice leapfrog (Sainio, arXiv:0911.5692, Sec. II.B).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
loads it and shares no code with it.

This is a thin ctypes wrapper around ``lf_oracle.c`` (plain C, OpenMP site
loops, built with ``-ffp-contract=off``).  Arrays are float64 (complex128 for
the complex-step entry points), C-contiguous, shape (N, N, N) with x the last
(fastest) axis.  The state convention follows the staggered leapfrog,
eq. (evo): f is stored at half-integer times, v = f' and a' at integer times.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lf_oracle.c")
# LF_ORACLE_LIB selects another build of the same source (the sanitizer
# build below); by default the plain optimised one.
LIB = os.environ.get("LF_ORACLE_LIB") or os.path.join(HERE, "liblf_oracle.so")
ASAN_LIB = os.path.join(HERE, "liblf_oracle_asan.so")
CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared"]
# AddressSanitizer and UndefinedBehaviorSanitizer, every finding fatal; the
# library is loaded into an uninstrumented Python with the gcc runtimes
# preloaded (see tests/test_oracle_sanitized.py)
ASAN_CFLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (always, when force is true); sanitize=True
    builds the AddressSanitizer/UBSan variant instead."""
    out = ASAN_LIB if sanitize else LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        flags = [f for f in CFLAGS if f != "-O2"] + ASAN_CFLAGS if sanitize else CFLAGS
        subprocess.run(["gcc", *flags, "-o", tmp, SRC, "-lm"], check=True, cwd=HERE)
        os.replace(tmp, out)
    return out


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("L", ctypes.c_double), ("dt", ctypes.c_double),
                ("beta", ctypes.c_int32), ("stencil", ctypes.c_int32), ("c1", ctypes.c_double),
                ("G", ctypes.c_double), ("r", ctypes.c_double), ("s", ctypes.c_double),
                ("kappa2", ctypes.c_double)]


@dataclass
class Model:
    """Lattice and model parameters in program units (Sec. II.B).

    V_pr = c1 a^p1 f1^beta / beta + G a^p2 f1^2 f2^2 / 2 with
    p1 = -2s + (2-beta) r and p2 = -2s - 2r; the rescaling obeys s - 2r + 3 = 0.
    """
    N: int
    L: float
    dt: float
    beta: int
    c1: float
    G: float
    r: float
    s: float
    kappa2: float
    stencil: int = 7   # Laplacian: 7 or 27 points (Sec. II.C)

    def c(self) -> _Params:
        return _Params(self.N, self.L, self.dt, self.beta, self.stencil, self.c1, self.G, self.r,
                       self.s, self.kappa2)

    def replace(self, **kw) -> "Model":
        d = dict(self.__dict__)
        d.update(kw)
        return Model(**d)


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_P = ctypes.POINTER(_Params)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        d, i64, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        sig = {
            "orc_abi": ([], ctypes.c_int),
            "orc_check_params": ([_P], ctypes.c_int),
            "orc_laplacian": ([_P, vp, vp], None),
            "orc_grad2": ([_P, vp, vp], None),
            "orc_averages": ([_P, vp, vp, d, vp], None),
            "orc_scale_step": ([_P, d, d, d, d, vp], None),
            "orc_desync_state": ([_P, vp, vp, vp, vp, d, d, vp], None),
            "orc_evolve": ([_P, vp, vp, vp, vp, vp, vp, i64, vp], None),
            "orc_energy": ([_P, vp, vp, vp, vp, d, d, vp], None),
            "orc_init_physical": ([_P, vp, vp, vp, vp, d], d),
            "orc_rho_p": ([_P, vp, vp, vp, vp, d, d, vp, vp, vp], None),
            "orcz_desync_state": ([_P, vp, vp, vp, vp, vp, vp, vp], None),
            "orcz_evolve": ([_P, vp, vp, vp, vp, vp, vp, vp, i64], None),
            "orcz_energy": ([_P, vp, vp, vp, vp, vp, vp, vp, vp], None),
            "orc_adjoint": ([_P, vp, vp, vp, vp, d, d, i64, vp, vp, vp, vp, vp, vp, vp, vp],
                            ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _arr(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(m: Model):
    rc = lib().orc_check_params(ctypes.byref(m.c()))
    if rc:
        raise ValueError(f"invalid oracle parameters (code {rc}): {m}")


# ---------------------------------------------------------------- operators

def laplacian(m: Model, f):
    """The model's Laplacian (7 or 27 points) with 1/dx^2, periodic (Sec. II.C)."""
    f = _arr(f)
    out = np.empty_like(f)
    lib().orc_laplacian(ctypes.byref(m.c()), _ptr(f), _ptr(out))
    return out


def grad2(m: Model, f):
    """Gradient energy density per site (Dirichlet form of the Laplacian; for
    7 points the forward-difference |grad+ f|^2), with 1/dx^2."""
    f = _arr(f)
    out = np.empty_like(f)
    lib().orc_grad2(ctypes.byref(m.c()), _ptr(f), _ptr(out))
    return out


def averages(m: Model, f1, f2, a: float):
    """(Sg, SV): -<sum f Lap f> and <V_pr> at scale factor a (eq. scale)."""
    f1, f2 = _arr(f1), _arr(f2)
    out = np.zeros(2)
    lib().orc_averages(ctypes.byref(m.c()), _ptr(f1), _ptr(f2), a, _ptr(out))
    return float(out[0]), float(out[1])


def scale_step(m: Model, a: float, w: float, Sg: float, SV: float):
    """(a'_{k+1}, a'_{k+1/2}, a''_{k+1/2}, a_{k+3/2}) from a_{k+1/2}, a'_k."""
    out = np.zeros(4)
    lib().orc_scale_step(ctypes.byref(m.c()), a, w, Sg, SV, _ptr(out))
    return tuple(float(x) for x in out)


# ---------------------------------------------------------------- evolution

@dataclass
class State:
    """Desynchronised leapfrog state: f(k+1/2), v(k), a_{k+1/2}, a'_k."""
    m: Model
    f1: np.ndarray
    f2: np.ndarray
    v1: np.ndarray
    v2: np.ndarray
    a_half: float
    ad: float
    step: int = 0

    def copy(self) -> "State":
        return State(self.m, self.f1.copy(), self.f2.copy(), self.v1.copy(), self.v2.copy(),
                     self.a_half, self.ad, self.step)


def init_physical(m: Model, f1, f2, u1, u2, a0: float = 1.0):
    """Program-unit v(0) and a'(0) from f(0) and rescaled physical velocities.

    Returns (v1, v2, ad0): a'_0 from the Friedmann constraint, v = u + r(a'/a)f
    (Sec. II.B, conversion to program units).
    """
    _check(m)
    f1, f2 = _arr(f1), _arr(f2)
    v1, v2 = _arr(u1).copy(), _arr(u2).copy()
    ad0 = lib().orc_init_physical(ctypes.byref(m.c()), _ptr(f1), _ptr(f2), _ptr(v1), _ptr(v2), a0)
    return v1, v2, float(ad0)


def start(m: Model, f1, f2, v1, v2, a0: float, ad0: float) -> State:
    """Desynchronise a synchronised program-unit state (Sec. II.B)."""
    _check(m)
    st = State(m, _arr(f1).copy(), _arr(f2).copy(), _arr(v1).copy(), _arr(v2).copy(), 0.0, ad0)
    ah = ctypes.c_double(0.0)
    lib().orc_desync_state(ctypes.byref(m.c()), _ptr(st.f1), _ptr(st.f2), _ptr(st.v1),
                           _ptr(st.v2), a0, ad0, ctypes.byref(ah))
    st.a_half = ah.value
    return st


def start_physical(m: Model, f1, f2, u1, u2, a0: float = 1.0) -> State:
    v1, v2, ad0 = init_physical(m, f1, f2, u1, u2, a0)
    return start(m, f1, f2, v1, v2, a0, ad0)


def evolve(st: State, nsteps: int, tape: bool = False):
    """Advance the state in place by nsteps; optionally return the scalar tape
    (n, 5): a_{k+1/2}, a'_k, Sg, SV, a'_{k+1}."""
    ah = ctypes.c_double(st.a_half)
    ad = ctypes.c_double(st.ad)
    tp = np.zeros((max(nsteps, 1), 5)) if tape else None
    lib().orc_evolve(ctypes.byref(st.m.c()), _ptr(st.f1), _ptr(st.f2), _ptr(st.v1), _ptr(st.v2),
                     ctypes.byref(ah), ctypes.byref(ad), int(nsteps),
                     _ptr(tp) if tape else None)
    st.a_half, st.ad = ah.value, ad.value
    st.step += nsteps
    return tp[:nsteps] if tape else st


ENERGY_KEYS = ("a", "ad", "K1", "K2", "G1", "G2", "P", "rho", "R")


def energies(st: State) -> dict:
    """Synchronised volume averages (program units): a, a', K_i, G_i, P, rho, R."""
    out = np.zeros(9)
    lib().orc_energy(ctypes.byref(st.m.c()), _ptr(st.f1), _ptr(st.f2), _ptr(st.v1),
                     _ptr(st.v2), st.a_half, st.ad, _ptr(out))
    d = dict(zip(ENERGY_KEYS, (float(x) for x in out)))
    d["step"] = st.step
    return d


def rho_p(st: State, arrays: bool = True):
    """Energy density and pressure at the synchronised time (eq. rho-pres in
    program units): (rho, p) arrays (or None) and dict(rho, p, w) of averages."""
    out = np.zeros(3)
    rho = np.empty_like(st.f1) if arrays else None
    pr = np.empty_like(st.f1) if arrays else None
    lib().orc_rho_p(ctypes.byref(st.m.c()), _ptr(st.f1), _ptr(st.f2), _ptr(st.v1), _ptr(st.v2),
                    st.a_half, st.ad, _ptr(rho) if arrays else None, _ptr(pr) if arrays else None, _ptr(out))
    return rho, pr, dict(rho=float(out[0]), p=float(out[1]), w=float(out[2]))


def synchronized_fields(st: State):
    """f(k) = f(k+1/2) - dt/2 v(k) (never written back)."""
    h = 0.5 * st.m.dt
    return st.f1 - h * st.v1, st.f2 - h * st.v2


# ---------------------------------------------------------------- complex step

def complex_run(m: Model, G: complex, f1, f2, v1, v2, a0: complex, ad0: complex, nsteps: int):
    """The same map (desync, nsteps steps, energies) over complex numbers.

    Returns (state arrays f1, f2, v1, v2, a_half, ad, energies[9]) all complex.
    Used for complex-step differentiation: a perturbation i*h*delta of the
    input gives h * (J delta) in the imaginary part, free of cancellation.
    """
    _check(m)
    c = m.c()
    f1, f2, v1, v2 = (np.ascontiguousarray(x, dtype=np.complex128).copy() for x in (f1, f2, v1, v2))
    a0a = np.array([a0.real, a0.imag]) if isinstance(a0, complex) else np.array([a0, 0.0])
    ad0a = np.array([ad0.real, ad0.imag]) if isinstance(ad0, complex) else np.array([ad0, 0.0])
    Ga = np.array([complex(G).real, complex(G).imag])
    ah = np.zeros(2)
    lib().orcz_desync_state(ctypes.byref(c), _ptr(f1), _ptr(f2), _ptr(v1), _ptr(v2),
                            _ptr(a0a), _ptr(ad0a), _ptr(ah))
    ad = ad0a.copy()
    lib().orcz_evolve(ctypes.byref(c), _ptr(Ga), _ptr(f1), _ptr(f2), _ptr(v1), _ptr(v2),
                      _ptr(ah), _ptr(ad), int(nsteps))
    out = np.zeros(18)
    lib().orcz_energy(ctypes.byref(c), _ptr(Ga), _ptr(f1), _ptr(f2), _ptr(v1), _ptr(v2),
                      _ptr(ah), _ptr(ad), _ptr(out))
    en = out[0::2] + 1j * out[1::2]
    return f1, f2, v1, v2, complex(ah[0], ah[1]), complex(ad[0], ad[1]), en


# ---------------------------------------------------------------- adjoint

def adjoint(m: Model, f1, f2, v1, v2, a0: float, ad0: float, nsteps: int,
            wK=(0.0, 1.0), wG=(0.0, 1.0), seed=None):
    """Reverse-mode gradient of E = sum_i wK_i K_i + wG_i G_i at the final
    synchronised time (plus <seed, X_n> for a seed on the final desynchronised
    state) with respect to the synchronised initial state and G.

    Returns dict(E, dG, da0, dad0, f1, f2, v1, v2) — the last four are arrays.
    Stores every state: tiny lattices only.
    """
    _check(m)
    N3 = m.N ** 3
    f1, f2, v1, v2 = (_arr(x) for x in (f1, f2, v1, v2))
    g = [np.zeros_like(f1) for _ in range(4)]
    out = np.zeros(4)
    wKa, wGa = np.array(wK, dtype=np.float64), np.array(wG, dtype=np.float64)
    sd = None
    if seed is not None:
        sd = np.concatenate([np.ravel(seed[0]), np.ravel(seed[1]), np.ravel(seed[2]),
                             np.ravel(seed[3]), [seed[4], seed[5]]]).astype(np.float64)
        assert sd.size == 4 * N3 + 2
    rc = lib().orc_adjoint(ctypes.byref(m.c()), _ptr(f1), _ptr(f2), _ptr(v1), _ptr(v2), a0, ad0,
                           int(nsteps), _ptr(wKa), _ptr(wGa), _ptr(sd) if sd is not None else None,
                           _ptr(out), _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), _ptr(g[3]))
    if rc:
        raise MemoryError("oracle adjoint: out of memory")
    return dict(E=float(out[0]), dG=float(out[1]), da0=float(out[2]), dad0=float(out[3]),
                f1=g[0], f2=g[1], v1=g[2], v2=g[3])
