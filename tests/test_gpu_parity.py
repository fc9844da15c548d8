"""GPU (liblf, gfx950) against the FP64 oracle on the same seeded inputs.

Metric: per-array max|gpu - oracle| / max|oracle| over f1 = phi, f2 = chi
(stored at half steps) and their velocities; the scale factor, a' and the
Friedmann residual are compared directly.  Bars: FP32 lattice arrays 1e-5,
FP64 1e-10.
"""
import numpy as np
import pytest

from _parity import ARRAYS, compare_state, gpu_run, log, oracle_run, rel_err
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-10}


def _check(w, steps, dtype=None, reps=1, **kw):
    dtype = dtype or w.dtype
    log(f"[parity] {w.name} N={w.N} reps={reps} steps={steps} dtype={dtype} {kw}")
    st, en, ad0, ic = oracle_run(w, steps)
    lat, gad0 = gpu_run(w, ic, steps, dtype=dtype, reps=reps, **kw)
    assert abs(gad0 - ad0) <= 1e-12 * ad0
    import torch
    full = lat.fields(dtype=torch.float64)
    n = w.N
    if reps > 1:
        for k, x in zip(ARRAYS, full):
            t = x.view(reps, n, reps, n, reps, n)
            first = t[0:1, :, 0:1, :, 0:1, :]
            assert bool((t == first).all()), f"periodic copies of {k} differ"
    f = [x[:n, :n, :n].cpu().numpy() for x in full]
    del full
    errs = compare_state(f, st)
    g = lat.energies()
    log(f"[parity] {w.name}: {errs} a {g['a']} vs {en['a']} R {g['R']} vs {en['R']}")
    tol = TOL[dtype]
    for k in ARRAYS:
        assert errs[k] <= tol, (k, errs)
    atol = 1e-12 if dtype == "f64" else 1e-9
    assert abs(g["a"] - en["a"]) <= atol * en["a"]
    assert abs(g["ad"] - en["ad"]) <= atol * abs(en["ad"])
    assert abs(g["R"] - en["R"]) <= (1e-12 if dtype == "f64" else 1e-8)
    for k in ("K1", "K2", "G1", "G2", "P", "rho"):
        assert abs(g[k] - en[k]) <= (1e-10 if dtype == "f64" else 1e-5) * abs(en[k]) + 1e-300, k
    assert g["step"] == steps
    lat.close()


def test_cfg1_lphi4_32_fp64_200_steps():
    _check(W.CFG1, W.CFG1.steps)


def test_cfg2_recipe_64_fp32_1000_steps():
    _check(W.CFG2.resized(64), W.CFG2.steps)


def test_cfg3_recipe_64_fp32_2000_steps():
    _check(W.CFG3.resized(64), W.CFG3.steps)


def test_cfg2_full_size_256_periodic_tiles():
    """256^3 (the launch shape of the full workload) with a 64^3-periodic
    initial state: every periodic copy is bitwise identical and equals the
    oracle's 64^3 evolution."""
    _check(W.CFG2.resized(64), W.CFG2.steps, reps=4)


def test_cfg3_full_size_512_periodic_tiles():
    """512^3 FP32, 2000 steps: the benchmark's launch shape, against the oracle
    on the 64^3 period (same dx, dt)."""
    _check(W.CFG3.resized(64), W.CFG3.steps, reps=8, **W.BENCH_SHAPES[W.CFG3.name])


@pytest.mark.parametrize("stencil", [7, 27])
def test_large_1024_periodic_tiles(stencil):
    """1024^3 FP32 (34 GB of lattice arrays, 8x the benchmark's sites) in the
    automatic launch shape, 100 steps: every 64^3 periodic copy bitwise equal
    and equal to the oracle's 64^3 run."""
    from dataclasses import replace
    _check(replace(W.CFG3, stencil=stencil).resized(64), 100, reps=16)


@pytest.mark.parametrize("N", [4, 5, 7, 33, 100])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_edge_and_ragged_sizes(N, dtype):
    w = W.CFG1.resized(N)
    _check(w, 40, dtype=dtype)
