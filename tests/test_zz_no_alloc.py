"""lf_slab_sweep_sums, the allocation-free variant of lf_slab_sweep: its
partial-sum rows live in the library's static device array.

Two calls in a row (the second on a smaller slab, so the array holds the
first call's rows beyond the second's) must give lf_slab_sweep's new arrays
bitwise and the totals of its partial rows; a launch shape that needs more
rows than the array holds is rejected before any device work."""
import ctypes
import math

import pytest
import torch

from paper_0911_5692_amd import Lattice
from paper_0911_5692_amd import workloads as W
from paper_0911_5692_amd._lib import lib

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64


def _lattice(w, dtype, **shape):
    lat = Lattice(**w.model(), dtype=dtype, **shape)
    ic = W.make_inputs(w)
    dev = lambda a: torch.tensor(a, dtype=F64, device="cuda")
    lat.init_physical(dev(ic["f1"]), dev(ic["f2"]), dev(ic["u1"]), dev(ic["u2"]), ic["a0"])
    lat.step(3)  # the slab sweeps reuse the coefficients of the last step
    return lat


def _slab(state, zb, ze, N):
    slab = [s[zb:ze].clone() for s in state]
    lo = [s[[(zb - 2) % N, (zb - 1) % N]].clone() for s in state[:2]]
    lo += [s[[(zb - 1) % N]].clone() for s in state[2:]]
    hi = [s[[ze % N]].clone() for s in state[:2]]
    return slab, lo, hi


@pytest.mark.parametrize("stencil,dtype,shape,slabs", [
    (7, F32, dict(tile_x=128, tile_y=8), [(0, 48, 0), (17, 30, 4)]),
    (27, F32, dict(tile_x=64, tile_y=8), [(5, 48, 8), (40, 41, 0)]),
    (7, F64, dict(tile_x=64, tile_y=4), [(0, 40, 5), (33, 40, 0)]),
])
def test_allocation_free_slab_sweep_matches_lf_slab_sweep(stencil, dtype, shape, slabs):
    from dataclasses import replace
    w = replace(W.CFG3, stencil=stencil).resized(48) if dtype == F32 else replace(W.CFG1, stencil=stencil).resized(40)
    lat = _lattice(w, dtype, **shape)
    N = lat.N
    state, _ = lat.get_state()
    for zb, ze, zchunk in slabs:
        print(f"[no-alloc] stencil {stencil} {dtype} {shape} slab [{zb}, {ze}) zchunk {zchunk}", flush=True)
        slab, lo, hi = _slab(state, zb, ze, N)
        ref_out, part = lat.slab_sweep(slab, lo, hi, zchunk=zchunk)
        torch.cuda.synchronize()
        rows = part.cpu().numpy()
        want = [math.fsum(rows[:, i]) for i in range(4)]
        out = tuple(torch.full_like(s, float("nan")) for s in slab)
        sums = torch.full((4,), float("nan"), dtype=F64, device="cuda")
        lat.slab_sweep_sums(slab, lo, hi, out, sums, zchunk=zchunk)
        torch.cuda.synchronize()
        for i, name in enumerate(("d1", "d2", "e1", "e2")):
            bad = (out[i] != ref_out[i]).sum().item()
            assert bad == 0, f"{name}: {bad} sites differ from lf_slab_sweep"
        got = sums.cpu().tolist()
        for i in range(4):
            assert abs(got[i] - want[i]) <= 1e-13 * abs(want[i]), (i, got, want)
    lat.close()


def test_allocation_free_slab_sweep_rejects_more_rows_than_the_static_array():
    """264^3 with 64 x 4 tiles and one plane per block: 5 x 66 x 264 = 87120
    rows > 65536.  The check comes before any device work."""
    w = W.CFG1.resized(264)
    lat = Lattice(**w.model(), dtype=F32, tile_x=64, tile_y=4)
    assert lat.slab_rows(264, 1) == 87120
    p = (ctypes.c_void_p * 4)(0x100000, 0x100000, 0x100000, 0x100000)
    rc = lib().lf_slab_sweep_sums(lat._ctx, 264, 1, p, p, p, p, ctypes.c_void_p(0x100000))
    assert rc == 1, rc
    assert "static scratch" in lib().lf_last_error().decode()
    lat.close()
