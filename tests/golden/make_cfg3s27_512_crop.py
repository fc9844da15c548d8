"""Write the stored oracle result of the 512^3 m^2 phi^2 workload with the
27-point Laplacian.

The workload is the benchmark's 512^3 chaotic-inflation model of Sec. III
(the same program units, L = 10, dt = 2^-10, seeded vacuum initial state,
seeds [3, 0, field, kind]) with the paper's own 27-point isotropic Laplacian
of Sec. II.C, evolved 240 leapfrog steps in FP64 by the oracle.  In 240 steps
(dt/dx = 1/20) a site feels the lattice 12 sites away, so the stored
[0, 64)^3 corner reaches across the periodic wrap in x, y and z; the 16384
random sites cover the rest of the lattice, the z-chunk boundary of the
benchmark's launch shape included.  The file keeps the same items as
cfg3_512_crop.npz.

Only the oracle and the seeded input generator are called.  About an hour
and a half on 8 host cores.  Usage: python tests/golden/make_cfg3s27_512_crop.py
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from make_cfg3_512_crop import W, run  # noqa: E402

OUT = os.path.join(HERE, "cfg3s27_512_crop.npz")
STEPS = 240

if __name__ == "__main__":
    run(W.CFG3_S27, STEPS, OUT)
    sys.exit(0)
