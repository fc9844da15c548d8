"""Host models of two kernels' tile index maps (no GPU).

Each model restates, in Python, how a kernel assigns lattice cells to
threads, LDS slots and z-planes, and checks the invariants the kernel relies
on.  The GPU parity tests check the kernels themselves; these catch an
indexing mistake on the CPU, before any launch, at sizes (ragged tiles, N
below the tile width, grids smaller than the item list) that are cheap here.

* The XCD-contiguous order in which the grid-stride kernels walk their
  items visits every item exactly once.
* k_diag_march (energies, rho/p): 64 x 4 KI tiles (KI sites per thread)
  marching z with three LDS planes and a one-cell ring.  Every LDS index is in range, every gathered
  neighbour of an evaluated site is its periodic neighbour, and every site is
  evaluated exactly once.
* sweep_tile27 (27-point sweep): the staged plane covers the tile, its ring
  and halo exactly once; every LDS read is in range; and the gradient energy's
  13 forward bonds of every site are counted exactly once over all tiles and
  z-chunks (the bond-ownership rule).
"""
import itertools
from collections import Counter

import numpy as np
import pytest


# ---- k_diag_march: tile 64 x 4 KI (KI sites per thread, rows ly, ly+4, ...),
# LDS planes of (64 + 2) x (4 KI + 2) doubles
DX = 64
LW = DX + 2
DIAG_KI = {7: 2, 27: 1}  # diag_ki<ST>() in lf_kernels.hip
BONDS = {7: [(1,0,0),(0,1,0),(0,0,1)],
         27: [(1,0,0),(0,1,0),(0,0,1),(-1,1,0),(1,1,0),(0,-1,1),(0,1,1),(-1,0,1),(1,0,1),
              (-1,-1,1),(1,-1,1),(-1,1,1),(1,1,1)]}


def ring(ST, DY):
    return 2*LW + 2*DY if ST == 27 else DX + DY


def ring_cell(ST, c, DY):
    if ST == 27:
        if c < LW: return c-1, -1
        if c < 2*LW: return c-LW-1, DY
        if c < 2*LW+DY: return -1, c-2*LW
        return DX, c-2*LW-DY
    if c < DY: return DX, c
    return c-DY, DY


def xcd_remap(b, nb):
    """Block b's logical tile when each XCD (b mod 8) takes a contiguous range."""
    q = nb // 8
    return b if b >= q * 8 else (b % 8) * q + b // 8


def xcd_items(blk, items, grid):
    """Items block blk walks (xcd_item in lf_internal.h): XCD-contiguous
    ranges in every full round, the plain order in the last partial round."""
    base = 0
    while base + blk < items:
        yield base + (xcd_remap(blk, grid) if base + grid <= items else blk)
        base += grid


@pytest.mark.parametrize("items,grid", [(512, 512), (1000, 512), (1024, 512), (13, 5), (64, 64), (70, 9),
                                        (2048, 2048), (7, 7), (100, 1)])
def test_xcd_item_order_visits_every_item_once(items, grid):
    seen = Counter(i for b in range(grid) for i in xcd_items(b, items, grid))
    assert sorted(seen) == list(range(items)) and set(seen.values()) == {1}


def shape(N, rows, DY):
    ntx = (N+DX-1)//DX; nty = (N+DY-1)//DY; tiles = ntx*nty
    nz = max(1, min(N, rows//tiles)); zc = (N+nz-1)//nz; nz = (N+zc-1)//zc
    items = tiles*nz
    return ntx, nty, zc, items, min(items, rows)


def check_diag(N, ST, rows=2048, KI=None):
    KI = KI or DIAG_KI[ST]
    DY = 4 * KI
    PL = LW * (DY + 2)
    rng = np.random.default_rng(N*100+ST)
    f = rng.standard_normal((N, N, N))   # [z, y, x]
    ntx, nty, zc, items, grid = shape(N, rows, DY)
    seen = np.zeros((N, N, N), int)
    # a thread's KI sites as KI x 256 lanes
    t = np.tile(np.arange(256), KI); lx = t & 63; ly = (t >> 6) + 4 * np.repeat(np.arange(KI), 256)
    slot = (ly+1)*LW + lx + 1
    assert len(set(slot)) == len(slot)
    t = np.arange(256)
    NR = ring(ST, DY); hasr = t < NR
    assert NR <= 256
    rc = [ring_cell(ST, int(c), DY) if c < NR else (0, 0) for c in t]
    rx = np.array([a for a, b in rc]); ry = np.array([b for a, b in rc])
    rslot = (ry+1)*LW + rx + 1
    assert slot.min() >= 0 and slot.max() < PL and rslot.min() >= 0 and rslot.max() < PL
    # interior and ring slots never collide
    assert not set(slot) & set(rslot[hasr])
    for blk in range(grid):
        for item in xcd_items(blk, items, grid):
            tx = item % ntx; rest = item // ntx; ty = rest % nty; tz = rest // nty
            x0, y0, z0 = tx*DX, ty*DY, tz*zc; z1 = min(z0+zc, N)
            assert z0 < N
            act = (x0+lx < N) & (y0+ly < N)
            xi, yi = (x0+lx) % N, (y0+ly) % N
            xr, yr = (x0+rx) % N, (y0+ry) % N
            off = yi*N + xi; roff = yr*N + xr
            assert off.max() < N*N and roff.max() < N*N
            buf = {}
            def stage(b, z):
                assert 0 <= z <= N
                zw = z - N if z >= N else z
                assert 0 <= zw < N
                p = np.full(PL, np.nan)
                p[slot] = f[zw, yi, xi]
                p[rslot[hasr]] = f[zw, yr[hasr], xr[hasr]]
                buf[b] = (z, p)
            stage(0, z0); stage(1, z0+1)
            b0 = 0
            for z in range(z0, z1):
                b1 = (b0+1) % 3; b2 = (b1+1) % 3
                zb0, P0 = buf[b0]; zb1, P1 = buf[b1]
                assert zb0 == z and zb1 == z+1
                a = act
                for dx, dy, dz in BONDS[ST]:
                    idx = slot + dy*LW + dx
                    assert idx[a].min() >= 0 and idx[a].max() < PL
                    got = (P1 if dz else P0)[idx[a]]
                    want = f[(z+dz) % N, (y0+ly[a]+dy) % N, (x0+lx[a]+dx) % N]
                    assert np.array_equal(got, want), (N, ST, item, z, dx, dy, dz)
                seen[z, (y0+ly[a]) % N, (x0+lx[a]) % N] += 1
                if z+1 < z1:
                    stage(b2, z+2)
                b0 = b1
    assert (seen == 1).all(), (N, ST, seen.min(), seen.max())
    return ntx, nty, zc, items, grid


# ---- sweep_tile27: forward bonds of the 27-point Dirichlet form
H = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
     if (dz, dy, dx) != (0, 0, 0) and [v for v in (dz, dy, dx) if v != 0][0] == 1]
assert len(H) == 13


def check_sweep27(N, TX, TY, ZC):
    RPR = 256 // TX; KI = TY // RPR
    LW, LH = TX + 4, TY + 3
    NW, NHT = TX + 2, TY + 1
    NRING = TX + 2 + TY
    NHALO = 2 * (TX + 4) + 3 * TY + 2
    ntx, nty, nzc = -(-N // TX), -(-N // TY), -(-N // ZC)
    cnt = Counter()
    for tz in range(nzc):
        z0 = tz * ZC; z1 = min(z0 + ZC, N)
        for ty in range(nty):
            for tx in range(ntx):
                x0, y0 = tx * TX, ty * TY
                wv, hv = min(TX, N - x0), min(TY, N - y0)
                # staged coverage
                staged = set()
                for t in range(256):
                    cx, cy = t % TX, t // TX
                    for k in range(KI):
                        staged.add((cx, cy + RPR * k))
                    if t < NRING:
                        staged.add((t - 1, -1) if t < TX + 2 else (-1, t - (TX + 2)))
                for t in range(256):
                    for m in range(2):
                        hc = t + 256 * m
                        if hc >= NHALO: continue
                        if hc < TX + 4: p = (hc - 2, -2)
                        elif hc < 2 * (TX + 4): p = (hc - (TX + 4) - 2, TY)
                        elif hc < 2 * (TX + 4) + TY + 1: p = (-2, hc - 2 * (TX + 4) - 1)
                        elif hc < 2 * (TX + 4) + 2 * (TY + 1): p = (TX + 1, hc - 2 * (TX + 4) - (TY + 1) - 1)
                        else: p = (TX, hc - 2 * (TX + 4) - 2 * (TY + 1))
                        assert p not in staged, ("dup halo", p)
                        staged.add(p)
                full = {(x, y) for x in range(-2, TX + 2) for y in range(-2, TY + 1)}
                assert staged == full, (len(staged), len(full))
                assert all(0 <= (y + 2) * LW + x + 2 < LH * LW for x, y in staged)
                # stencil reads of computed sites stay in the staged plane
                comp = [(cx, yl) for cx in range(TX) for yl in range(TY)] + \
                       [(x, -1) for x in range(-1, TX + 1)] + [(-1, y) for y in range(TY)]
                for (x, y) in comp:
                    for dx, dy in itertools.product((-1, 0, 1), repeat=2):
                        assert (x + dx, y + dy) in full
                def g(lx, ly, z):  # global site
                    return ((x0 + lx) % N, (y0 + ly) % N, z % N)
                def nidx(lx, ly):
                    i = (ly + 1) * NW + lx + 1
                    assert 0 <= i < NHT * NW, (lx, ly)
                    return i
                def add(p, q, z_p, z_q):
                    o = (q[0] - p[0], q[1] - p[1], z_q - z_p)
                    a = g(*p, z_p); b = g(*q, z_q)
                    if o in H: key = (a, o)
                    else:
                        assert (-o[0], -o[1], -o[2]) in H
                        key = (b, (-o[0], -o[1], -o[2]))
                    cnt[key] += 1
                for z in range(z0, z1):
                    for t in range(256):
                        cx, cy = t % TX, t // TX
                        for k in range(KI):
                            yl = cy + RPR * k
                            act = x0 + cx < N and y0 + yl < N
                            if not act: continue
                            okx = cx + 1 < wv; oky = yl + 1 < hv; ok4 = yl == 0 or okx
                            p = (cx, yl)
                            l = nidx(cx, yl)
                            # in-plane
                            for (dx, dy, ok) in ((-1, 0, True), (0, -1, True), (-1, -1, True), (1, -1, ok4)):
                                if ok:
                                    nidx(cx + dx, yl + dy); add(p, (cx + dx, yl + dy), z, z)
                            for dx, dy in itertools.product((-1, 0, 1), repeat=2):
                                ok = {(1, -1): ok4, (1, 0): okx, (1, 1): okx and oky, (0, 1): oky, (-1, 1): oky}.get((dx, dy), True)
                                if ok:
                                    nidx(cx + dx, yl + dy); add(p, (cx + dx, yl + dy), z, z - 1)
                        if t < NRING:
                            rrow = t < TX + 2
                            rlx, rly = (t - 1, -1) if rrow else (-1, t - (TX + 2))
                            nidx(rlx, rly)
                            for j in range(3):
                                if rrow:
                                    x = rlx + j - 1
                                    if 0 <= x < wv: nidx(x, 0); add((rlx, rly), (x, 0), z, z - 1)
                                else:
                                    y = rly + j - 1
                                    if rly < hv and 0 <= y < hv: nidx(0, y); add((rlx, rly), (0, y), z, z - 1)
                            if not rrow and 1 <= rly < hv:
                                nidx(0, rly - 1); add((rlx, rly), (0, rly - 1), z, z)
    want = Counter({((x, y, z), o): 1 for x in range(N) for y in range(N) for z in range(N) for o in H})
    bad = [(k, cnt[k]) for k in set(cnt) | set(want) if cnt[k] != want[k]]
    assert not bad, (N, TX, TY, ZC, len(bad), bad[:5])
    return len(cnt)


@pytest.mark.parametrize("KI", [1, 2, 4])
@pytest.mark.parametrize("N", [4, 5, 9, 33, 67])
@pytest.mark.parametrize("ST", [7, 27])
def test_diag_march_indexing(N, ST, KI):
    check_diag(N, ST, KI=KI)


@pytest.mark.parametrize("KI", [1, 2, 4])
@pytest.mark.parametrize("N,rows", [(17, 5), (40, 3), (9, 1)])
def test_diag_march_items_beyond_grid(N, rows, KI):
    check_diag(N, 7, rows, KI=KI)
    check_diag(N, 27, rows, KI=KI)


@pytest.mark.parametrize("case", [(4, 64, 8, 4), (5, 64, 4, 3), (7, 64, 16, 8), (12, 64, 8, 5),
                                  (9, 128, 4, 9), (20, 64, 16, 7)])


def test_sweep27_staging_and_bond_ownership(case):
    check_sweep27(*case)


# ---- k_adj_fields: tile 64 x 4, four LDS planes of (64 + 2) x (4 + 2), full ring
AX, AY = 64, 4
ALW, ALH = AX + 2, AY + 2
APL = ALW * ALH
ARING = 2 * ALW + 2 * AY


def adj_ring_cell(c):
    if c < ALW:
        return c - 1, -1
    if c < 2 * ALW:
        return c - ALW - 1, AY
    if c < 2 * ALW + AY:
        return -1, c - 2 * ALW
    return AX, c - 2 * ALW - AY


def adj_grid(N, rows):
    ntx = (N + AX - 1) // AX
    nty = (N + AY - 1) // AY
    nz = max(1, min(N, rows // (ntx * nty)))
    zc = (N + nz - 1) // nz
    nz = (N + zc - 1) // zc
    items = ntx * nty * nz
    return ntx, nty, zc, items, min(items, rows)


def check_adj(N, rows=512):
    """Every LDS index in range, every gathered value of planes z-1, z, z+1
    the periodic neighbour, each site evaluated once, and the buffer a plane
    is staged into last read two iterations earlier (one barrier apart)."""
    rng = np.random.default_rng(N)
    f = rng.standard_normal((N, N, N))
    ntx, nty, zc, items, grid = adj_grid(N, rows)
    seen = np.zeros((N, N, N), int)
    t = np.arange(256)
    lx, ly = t & 63, t >> 6
    slot = (ly + 1) * ALW + lx + 1
    hasr = t < ARING
    rc = [adj_ring_cell(int(c)) if c < ARING else (0, 0) for c in t]
    rx = np.array([a for a, _ in rc])
    ry = np.array([b for _, b in rc])
    rslot = (ry + 1) * ALW + rx + 1
    assert slot.max() < APL and rslot.min() >= 0 and rslot.max() < APL
    assert not set(slot) & set(rslot[hasr])
    for blk in range(grid):
        for item in xcd_items(blk, items, grid):
            tx = item % ntx
            rest = item // ntx
            ty, tz = rest % nty, rest // nty
            x0, y0, z0 = tx * AX, ty * AY, tz * zc
            z1 = min(z0 + zc, N)
            act = (x0 + lx < N) & (y0 + ly < N)
            xi, yi = (x0 + lx) % N, (y0 + ly) % N
            xr, yr = (x0 + rx) % N, (y0 + ry) % N
            buf, last_read = {}, {}

            def stage(b, z, it):
                assert -1 <= z <= N
                # the buffer's previous plane was last read at least two
                # iterations ago (a barrier lies between)
                assert last_read.get(b, -10) <= it - 2, (b, last_read.get(b), it)
                p = np.full(APL, np.nan)
                p[slot] = f[z % N, yi, xi]
                p[rslot[hasr]] = f[z % N, yr[hasr], xr[hasr]]
                buf[b] = (z, p)

            stage(0, z0 - 1, -5)
            stage(1, z0, -5)
            for z in range(z0, z1):
                it = z - z0
                bp, bc, bn = (z - z0) & 3, (z - z0 + 1) & 3, (z - z0 + 2) & 3
                stage(bn, z + 1, it)
                for b in (bp, bc, bn):
                    last_read[b] = it
                assert buf[bp][0] == z - 1 and buf[bc][0] == z and buf[bn][0] == z + 1
                a = act
                for dz, b in ((-1, bp), (0, bc), (1, bn)):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            idx = slot[a] + dy * ALW + dx
                            assert idx.min() >= 0 and idx.max() < APL
                            got = buf[b][1][idx]
                            want = f[(z + dz) % N, (y0 + ly[a] + dy) % N, (x0 + lx[a] + dx) % N]
                            assert np.array_equal(got, want), (N, item, z, dx, dy, dz)
                seen[z, (y0 + ly[a]) % N, (x0 + lx[a]) % N] += 1
    assert (seen == 1).all()
    return grid


@pytest.mark.parametrize("N,rows", [(4, 512), (5, 512), (9, 512), (33, 512), (67, 512), (128, 512), (20, 7), (12, 1)])
def test_adj_fields_march_indexing(N, rows):
    grid = check_adj(N, rows)
    assert grid <= rows
