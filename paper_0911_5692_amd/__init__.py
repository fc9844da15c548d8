"""MI355X-native FRW lattice leapfrog (Sainio, "CUDAEASY", arXiv:0911.5692).

Two interacting scalar fields on a periodic N^3 lattice in an expanding
universe, evolved by the staggered leapfrog of Sec. II.B with hand-written
HIP kernels for gfx950 (liblf.so, C ABI in include/lf.h).  PyTorch provides
device memory and streams only.

Submodules are imported lazily so that the input generators can be used on a
machine without the built library.
"""
from __future__ import annotations

import importlib

__all__ = ["Lattice", "Ensemble", "LeapfrogLoss", "autotune", "ens_autotune", "vacuum_fields", "stream_copy",
           "LfError", "inputs", "workloads", "build"]


def __getattr__(name):
    if name in ("Lattice", "Ensemble", "LeapfrogLoss", "autotune", "ens_autotune", "vacuum_fields",
                "stream_copy"):
        return getattr(importlib.import_module(".lattice", __name__), name)
    if name == "LfError":
        return importlib.import_module("._lib", __name__).LfError
    if name in ("inputs", "workloads", "build"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
