"""Helpers shared by the GPU parity tests: run a workload through liblf and
through the FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import functools
import sys

import numpy as np

import oracle as O
from paper_0911_5692_amd import workloads as W

ARRAYS = ("f1", "f2", "v1", "v2")


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dtype(w, dtype=None):
    import torch
    return torch.float64 if (dtype or w.dtype) == "f64" else torch.float32


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def make_lattice(w, dtype=None, **kw):
    from paper_0911_5692_amd import Lattice
    return Lattice(**w.model(), dtype=torch_dtype(w, dtype), **kw)


def gpu_run(w, ic, steps, dtype=None, reps=1, **kw):
    """Evolve on the GPU; ic is tiled reps times per axis on the device.
    Returns (lattice, ad0)."""
    lat = make_lattice(w if reps == 1 else w.resized(w.N * reps), dtype, **kw)
    t = [to_dev(ic[k]) for k in ("f1", "f2", "u1", "u2")]
    if reps > 1:
        t = [x.repeat(reps, reps, reps).contiguous() for x in t]
    ad0 = lat.init_physical(*t, ic["a0"])
    del t
    lat.step(steps)
    return lat, ad0


@functools.lru_cache(maxsize=8)
def oracle_run(w, steps, realization=0):
    """FP64 oracle result (cached per session): (state, energies, ad0, ic)."""
    ic = W.make_inputs(w, realization)
    m = O.Model(**w.model())
    v1, v2, ad0 = O.init_physical(m, ic["f1"], ic["f2"], ic["u1"], ic["u2"], ic["a0"])
    st = O.start(m, ic["f1"], ic["f2"], v1, v2, ic["a0"], ad0)
    O.evolve(st, steps)
    return st, O.energies(st), ad0, ic


def rel_err(got, ref) -> float:
    """max |got - ref| / max |ref| (per-array relative error)."""
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def fluct_err(got, ref) -> float:
    """max |got - ref| / max |ref - <ref>|: the error against the array's
    spatial fluctuation.  For the inflaton f1 = 1 + O(1e-4) the plain
    relative error divides by the homogeneous value and cannot see an error
    that is a sizeable part of the fluctuation; this one can.  0 when the
    reference has no fluctuation and the arrays agree, inf when it has none
    and they differ."""
    ref = np.asarray(ref)
    num = float(np.max(np.abs(got - ref)))
    den = float(np.max(np.abs(ref - ref.mean())))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def compare_state(gpu_arrays, st, crop=None):
    """Per array: the larger of the plain relative error and the error
    against the fluctuation (both must meet a test's bar)."""
    out = {}
    for k, g in zip(ARRAYS, gpu_arrays):
        r = getattr(st, k)
        if crop is not None:
            g = g[:crop, :crop, :crop]
        g = np.asarray(g)
        out[k] = max(rel_err(g, r), fluct_err(g, r))
    return out
