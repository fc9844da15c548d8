// The fused sweep on a z-slab of a lattice split along z (one GPU's share):
// the same per-site arithmetic and partial sums as the periodic sweeps
// (lf_sweep.hip, lf_sweep27.hip), with the planes outside the slab read from
// halo buffers through ZPlanes (lf_sweep_common.h) instead of the periodic
// wrap.  Separate instantiations, so that the periodic kernels keep their
// own plane addressing.  7-point kernel here; the 27-point one is in
// lf_slab27.hip.
#include "lf_sweep_tile.h"

namespace lf {

// One block per (tile, z-chunk) of the slab, XCD-aware tile order.
template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP_MIN_WAVES) k_sweep_slab(
    const T *__restrict__ d1, const T *__restrict__ d2, const T *__restrict__ e1, const T *__restrict__ e2,
    T *__restrict__ d1n, T *__restrict__ d2n, T *__restrict__ e1n, T *__restrict__ e2n, const int N,
    const ZPlanes<T> zp, const int zchunk, const int ntx, const int nty, const CoefPair *__restrict__ C,
    double *__restrict__ part)
{
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, b = tile / ntx;
    const int ty = b % nty;
    const int tz = b / nty;
    const int z0 = tz * zchunk;
    sweep_tile<T, NH, TX, TY, LF_SWEEP_PREFETCH, true>(d1, d2, e1, e2, d1n, d2n, e1n, e2n, N, zp, tx * TX,
                                                       ty * TY, z0, min(z0 + zchunk, zp.nz), C,
                                                       part + (size_t)tile * kNPart);
}

namespace {

template <typename T, int NH, int TX, int TY>
void slab_t(const SweepIO &io, int N, int zchunk, const CoefPair *C, double *part, hipStream_t st)
{
    const int ntx = (N + TX - 1) / TX, nty = (N + TY - 1) / TY, nzc = (io.nz + zchunk - 1) / zchunk;
    hipLaunchKernelGGL((k_sweep_slab<T, NH, TX, TY>), dim3(ntx * nty * nzc), dim3(256), 0, st,
                       (const T *)io.in[0], (const T *)io.in[1], (const T *)io.in[2], (const T *)io.in[3],
                       (T *)io.out[0], (T *)io.out[1], (T *)io.out[2], (T *)io.out[3], N, planes_of<T>(io),
                       zchunk, ntx, nty, C, part);
}

template <typename T, int TX, int TY>
void slab_b(int beta, const SweepIO &io, int N, int zchunk, const CoefPair *C, double *part, hipStream_t st)
{
    switch (beta) {
    case 2: slab_t<T, 1, TX, TY>(io, N, zchunk, C, part, st); break;
    case 3: slab_t<T, 2, TX, TY>(io, N, zchunk, C, part, st); break;
    case 4: slab_t<T, 3, TX, TY>(io, N, zchunk, C, part, st); break;
    case 5: slab_t<T, 4, TX, TY>(io, N, zchunk, C, part, st); break;
    default: slab_t<T, 5, TX, TY>(io, N, zchunk, C, part, st); break;
    }
}

// Supported tiles (x by y): 32x8, 32x16, 64x4, 64x8, 64x16, 128x4, 128x8.
template <typename T>
void slab_y(int tile_x, int tile_y, int beta, const SweepIO &io, int N, int zchunk, const CoefPair *C,
            double *part, hipStream_t st)
{
    if (tile_x == 128) {
        if (tile_y == 4) slab_b<T, 128, 4>(beta, io, N, zchunk, C, part, st);
        else slab_b<T, 128, 8>(beta, io, N, zchunk, C, part, st);
        return;
    }
    if (tile_x == 32) {
        if (tile_y == 8) slab_b<T, 32, 8>(beta, io, N, zchunk, C, part, st);
        else slab_b<T, 32, 16>(beta, io, N, zchunk, C, part, st);
        return;
    }
    switch (tile_y) {
    case 4: slab_b<T, 64, 4>(beta, io, N, zchunk, C, part, st); break;
    case 8: slab_b<T, 64, 8>(beta, io, N, zchunk, C, part, st); break;
    default: slab_b<T, 64, 16>(beta, io, N, zchunk, C, part, st); break;
    }
}

}  // namespace

void launch_sweep_slab(int stencil, int dtype, int tile_x, int tile_y, int beta, const SweepIO &io, int N,
                       int zchunk, const CoefPair *C, double *part, hipStream_t st)
{
    if (stencil == 27) launch_sweep_slab27(dtype, tile_x, tile_y, beta, io, N, zchunk, C, part, st);
    else if (dtype == 0) slab_y<float>(tile_x, tile_y, beta, io, N, zchunk, C, part, st);
    else slab_y<double>(tile_x, tile_y, beta, io, N, zchunk, C, part, st);
}

}  // namespace lf
