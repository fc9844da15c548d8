"""Write the stored oracle result of the configuration the paper times, with
its own 27-point Laplacian.

The workload is the 256^3 chaotic-inflation model of Sec. III (the same
program units as the 512^3 benchmark workload, L = 5, dt = 2^-10) with the
27-point isotropic Laplacian of Sec. II.C, from the seeded vacuum initial
state (seeds [3, 0, field, kind]), evolved 600 leapfrog steps in FP64 by the
oracle.  The file keeps the same items as cfg3_512_crop.npz (the [0, 64)^3
corner, 16384 random sites, the scalars and the energies).

Only the oracle and the seeded input generator are called.  About half an
hour on 8 host cores.  Usage: python tests/golden/make_paper256_s27_crop.py
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from make_cfg3_512_crop import W, run  # noqa: E402

OUT = os.path.join(HERE, "paper256_s27_crop.npz")
STEPS = 600

if __name__ == "__main__":
    run(W.PAPER_256_S27, STEPS, OUT)
    sys.exit(0)
