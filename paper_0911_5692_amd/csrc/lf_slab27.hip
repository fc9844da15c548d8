// The 27-point sweep on a z-slab with halo planes (one GPU's share of a
// lattice split along z); see lf_slab7.hip.  Separate instantiations of
// sweep_tile27 (lf_sweep27_tile.h) with SLAB = true.
#include "lf_sweep27_tile.h"

namespace lf {

template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP27_WAVES(T)) k_sweep_slab27(
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
    sweep_tile27<T, NH, TX, TY, true>(d1, d2, e1, e2, d1n, d2n, e1n, e2n, N, zp, tx * TX, ty * TY, z0,
                                      min(z0 + zchunk, zp.nz), C, part + (size_t)tile * kNPart);
}

namespace {

template <typename T>
void slab27_t(int tile_x, int tile_y, int beta, const SweepIO &io, int N, int zchunk, const CoefPair *C,
              double *part, hipStream_t st)
{
    with_tile(tile_x, tile_y, [&](auto tx, auto ty) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
        with_nh(beta, [&](auto nh) {
            constexpr int NH = decltype(nh)::value;
            const int ntx = (N + TX - 1) / TX, nty = (N + TY - 1) / TY, nzc = (io.nz + zchunk - 1) / zchunk;
            hipLaunchKernelGGL((k_sweep_slab27<T, NH, TX, TY>), dim3(ntx * nty * nzc), dim3(256), 0, st,
                               (const T *)io.in[0], (const T *)io.in[1], (const T *)io.in[2],
                               (const T *)io.in[3], (T *)io.out[0], (T *)io.out[1], (T *)io.out[2],
                               (T *)io.out[3], N, planes_of<T>(io), zchunk, ntx, nty, C, part);
        });
    });
}

}  // namespace

void launch_sweep_slab27(int dtype, int tile_x, int tile_y, int beta, const SweepIO &io, int N, int zchunk,
                         const CoefPair *C, double *part, hipStream_t st)
{
    if (dtype == 0) slab27_t<float>(tile_x, tile_y, beta, io, N, zchunk, C, part, st);
    else slab27_t<double>(tile_x, tile_y, beta, io, N, zchunk, C, part, st);
}

}  // namespace lf
