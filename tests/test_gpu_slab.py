"""The sweep on one GPU's share of a lattice split into z-slabs
(lf_slab_sweep): the periodic z wrap replaced by halo planes.

With the state a step started from cut into slabs, and each slab's halo
planes copied out of its neighbours (separate buffers, as a halo exchange
would deliver them), the slab sweeps must give that step's new arrays
bitwise, and their partial-sum rows together the step's sums (the same bonds
and sites, summed in another order)."""
import ctypes

import pytest
import torch

from paper_0911_5692_amd import Lattice, LfError
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64


def _lattice(w, dtype, steps=3, **shape):
    lat = Lattice(**w.model(), dtype=dtype, **shape)
    ic = W.make_inputs(w)
    dev = lambda a: torch.tensor(a, dtype=F64, device="cuda")
    lat.init_physical(dev(ic["f1"]), dev(ic["f2"]), dev(ic["u1"]), dev(ic["u2"]), ic["a0"])
    if steps:
        lat.step(steps)
    return lat


def _halos(state, zb, ze, N):
    lo = [s[[(zb - 2) % N, (zb - 1) % N]].clone() for s in state[:2]]
    lo += [s[[(zb - 1) % N]].clone() for s in state[2:]]
    hi = [s[[ze % N]].clone() for s in state[:2]]
    return lo, hi


# Bound on the relative difference of the step sums between two z-chunkings
# of the same step: the same per-site terms summed in another order (FP64).
# The 27-point sweep runs its z loop in three phase-specialised copies; its
# per-site bond sums are explicit fma chains, so every copy rounds a site's
# term the same way and the FP32 terms do not depend on where a chunk starts.
def _sum_tol(lat):
    return 1e-12


def _check_slabs(lat, bounds, zchunk):
    N = lat.N
    state, _ = lat.get_state()
    lat.step(1)
    ref, sc = lat.get_state()
    outs, tot = [], torch.zeros(4, dtype=F64, device="cuda")
    for zb, ze in zip(bounds[:-1], bounds[1:]):
        lo, hi = _halos(state, zb, ze, N)
        out, part = lat.slab_sweep([s[zb:ze] for s in state], lo, hi, zchunk=zchunk)
        assert part.shape[0] == lat.slab_rows(ze - zb, zchunk)
        outs.append(out)
        tot += part.sum(0)
    torch.cuda.synchronize()
    for i, name in enumerate(("d1", "d2", "e1", "e2")):
        got = torch.cat([o[i] for o in outs])
        bad = (got != ref[i]).sum().item()
        assert bad == 0, f"{name}: {bad} sites differ from the periodic step"
    want = torch.tensor(list(sc.pend), dtype=F64)
    rel = ((tot.cpu() - want).abs() / want.abs()).max().item()
    print(f"[slab] bounds {bounds} zchunk {zchunk}: arrays bitwise, sums rel {rel:.2e}", flush=True)
    assert rel < _sum_tol(lat)


CFG3_48 = W.CFG3.resized(48)
CASES = [
    # model, dtype, launch shape, slab bounds (ragged, one-plane slabs), z-chunk
    (7, W.CFG1.resized(48), F32, dict(tile_x=64, tile_y=8), [0, 20, 33, 48], 8),
    (27, W.CFG1.resized(48), F32, dict(tile_x=64, tile_y=8), [0, 20, 33, 48], 8),
    (7, CFG3_48, F32, dict(tile_x=128, tile_y=8), [0, 1, 2, 25, 48], 0),
    (27, CFG3_48, F32, dict(tile_x=128, tile_y=8), [0, 1, 2, 25, 48], 0),
    (7, W.CFG1.resized(40), F64, dict(tile_x=64, tile_y=4), [0, 13, 14, 40], 5),
    (27, W.CFG1.resized(40), F64, dict(tile_x=64, tile_y=16), [0, 13, 14, 40], 0),
    # one slab holding the whole lattice: every halo plane is one of its own
    (7, W.CFG1.resized(48), F32, dict(tile_x=64, tile_y=8), [0, 48], 0),
    (27, W.CFG1.resized(48), F32, dict(tile_x=64, tile_y=8), [0, 48], 16),
    # 128-wide tiles in FP64 (a tile wider than the lattice: ragged in x)
    (7, W.CFG1.resized(40), F64, dict(tile_x=128, tile_y=4), [0, 7, 40], 6),
    (27, W.CFG1.resized(40), F64, dict(tile_x=128, tile_y=8), [0, 7, 40], 0),
]


@pytest.mark.parametrize("stencil,w,dtype,shape,bounds,zchunk", CASES)
def test_slabs_reproduce_the_periodic_step(stencil, w, dtype, shape, bounds, zchunk):
    from dataclasses import replace
    print(f"[slab] stencil {stencil} {w.name} N={w.N} {dtype} {shape}", flush=True)
    lat = _lattice(replace(w, stencil=stencil), dtype, **shape)
    _check_slabs(lat, bounds, zchunk)


@pytest.mark.parametrize("stencil,dtype", [(7, F32), (27, F32), (27, F64)])
def test_periodic_chunkings_agree(stencil, dtype):
    """The same periodic step with z-chunks of 8 and of 9 planes: new arrays
    bitwise equal, step sums within _sum_tol (no slabs involved)."""
    from dataclasses import replace
    w = replace(W.CFG1.resized(48), stencil=stencil)
    res = []
    for zc in (8, 9):
        lat = _lattice(w, dtype, tile_x=64, tile_y=8, zchunk=zc)
        res.append(lat.get_state())
        tol = _sum_tol(lat)
        lat.close()
    for i in range(4):
        assert torch.equal(res[0][0][i], res[1][0][i])
    a, b = (torch.tensor(list(r[1].pend), dtype=F64) for r in res)
    rel = ((a - b).abs() / a.abs()).max().item()
    print(f"[slab] periodic stencil {stencil} {dtype}: z-chunks 8 vs 9, sums rel {rel:.2e}", flush=True)
    assert rel < tol


def test_slab_share_of_the_512_lattice():
    """One GPU's share of the 512^3 benchmark lattice split over 8 GPUs:
    planes [192, 256) with halos, bitwise against the periodic step, in the
    benchmark's launch shape with the automatic slab z-chunk."""
    w = W.CFG3
    lat = Lattice(**w.model(), dtype=F32, **W.BENCH_SHAPES[w.name])
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    N = w.N
    f = [1 + 1e-4 * torch.randn((N, N, N), dtype=F64, device="cuda", generator=g),
         1e-5 * torch.randn((N, N, N), dtype=F64, device="cuda", generator=g),
         -0.7 + 1e-4 * torch.randn((N, N, N), dtype=F64, device="cuda", generator=g),
         1e-3 * torch.randn((N, N, N), dtype=F64, device="cuda", generator=g)]
    lat.init_physical(*f, 1.0)
    del f
    lat.step(2)
    state, _ = lat.get_state()
    lat.step(1)
    ref, _ = lat.get_state()
    zb, ze = 192, 256
    lo, hi = _halos(state, zb, ze, N)
    out, part = lat.slab_sweep([s[zb:ze] for s in state], lo, hi)
    torch.cuda.synchronize()
    print(f"[slab] 512^3 share [{zb}, {ze}): rows {part.shape[0]}", flush=True)
    for i in range(4):
        assert torch.equal(out[i], ref[i][zb:ze])
    assert torch.isfinite(part).all()


def test_slab_sweep_errors():
    w = W.CFG1.resized(16)
    lat = _lattice(w, F32, steps=0, tile_x=64, tile_y=4)
    N = lat.N
    state = [torch.zeros((4, N, N), device="cuda") for _ in range(4)]
    lo = [torch.zeros((2, N, N), device="cuda") for _ in range(2)] + [torch.zeros((1, N, N), device="cuda")
                                                                       for _ in range(2)]
    hi = [torch.zeros((1, N, N), device="cuda") for _ in range(2)]
    with pytest.raises(LfError, match="take a step"):
        lat.slab_sweep(state, lo, hi)
    lat.step(1)
    with pytest.raises(LfError, match="nz=0"):
        lat.slab_rows(0)
    with pytest.raises(LfError, match="nz=17"):
        lat.slab_rows(17)
    with pytest.raises(LfError, match="zchunk"):
        lat.slab_rows(4, -1)
    # an output that overlaps an input
    with pytest.raises(LfError, match="overlaps"):
        lat.slab_sweep(state, lo, hi, out=(state[0], *[torch.zeros_like(s) for s in state[1:]]))
    # partials too small, through the C entry point
    from paper_0911_5692_amd._lib import lib
    arr = lambda ts: (ctypes.c_void_p * len(ts))(*(t.data_ptr() for t in ts))
    out = [torch.zeros_like(s) for s in state]
    part = torch.zeros(4, dtype=F64, device="cuda")
    rc = lib().lf_slab_sweep(lat._ctx, 4, 0, arr(state), arr(lo), arr(hi), arr(out),
                             ctypes.c_void_p(part.data_ptr()), 0)
    assert rc != 0 and "rows" in lib().lf_last_error().decode()
    # the plain sweep has no slab form
    plain = _lattice(w, F32, steps=1, tile_y=1)
    with pytest.raises(LfError, match="LDS launch shape"):
        plain.slab_rows(4)
