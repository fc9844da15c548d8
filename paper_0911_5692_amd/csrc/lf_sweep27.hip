// Fused kick-drift sweep with the 27-point Laplacian (Sainio,
// arXiv:0911.5692, Sec. II.C: second-order accurate, fourth-order isotropic;
// weights (centre, face, edge, corner) = (-128, 14, 3, 1)/30), gfx950.
//
// Same per-site update as the 7-point sweep (lf_sweep.hip), with the raw
// stencil sum in place of S6.  The 3x3x3 neighbourhood is never held in LDS
// at once: for every plane p and site, two in-plane partial sums are formed
// while p is staged,
//   A(p) = 14 c + 3 S4 + S4d      (what p contributes to the planes p-1, p+1)
//   B(p) = -128 c + 14 S4 + 3 S4d (what p contributes to itself)
// with c the site, S4 its 4 in-plane face neighbours and S4d its 4 in-plane
// diagonal neighbours, so that raw Lap(z) = B(z) + A(z-1) + A(z+1).  A block
// keeps A(z-1), A(z), B(z) per site in registers; one staged plane (z+1) per
// iteration completes the Laplacian of plane z.
//
// Reductions for the next a'': the gradient energy of the 27-point stencil is
// its Dirichlet form, a sum over lattice bonds of w_b (f(p) - f(q))^2.  Each
// bond is counted by exactly one (tile, plane):
//   * a bond between two z-planes is counted at the upper plane;
//   * a bond whose xy-projection crosses a tile border is counted by the tile
//     whose "lower ring" (row y0-1 from x0-1 to x0+TX, column x0-1 from y0 to
//     y0+TY-1) holds the other end; among the 8 xy-neighbour relations of two
//     tiles exactly one of them has that property.
// So a block needs the new values on its interior and its lower ring for the
// planes z and z-1: the ring values are computed redundantly (never stored),
// as is the plane z0-1 below the chunk, and the bonds counted are
//   interior(z) - {interior, ring}(z) through the 4 in-plane offsets
//     (-1,0), (0,-1), (-1,-1), (+1,-1);
//   interior(z) - {interior, ring}(z-1) through the 9 offsets below;
//   ring(z) - interior(z-1), and the ring column's in-plane (+1,-1) bond
//   into the interior.
// Per site the squared differences are summed by bond type in the working
// precision and the weighted site sum 14 F + 3 E + C is accumulated in FP64.
//
// LDS per block: three staged planes of (TX+4)(TY+3) and three new-value
// planes of (TX+2)(TY+1), both fields, each padded to 256 bytes (FP32: 33 KB
// for the 64 x 8 tile, 63 KB for 128 x 8).  With three buffers each, the
// loop is written out per phase of the rotation, so LDS addresses are
// loop-invariant registers plus immediate offsets and the register queues
// need no moves inside a period (17% fewer VALU instructions per site than
// a runtime buffer index).
//
// The tile function (sweep_tile27) is in lf_sweep27_tile.h; this file holds
// the periodic and ensemble kernels and their launchers, lf_slab27.hip the
// z-slab kernel.
#include "lf_sweep27_tile.h"

namespace lf {

template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP27_WAVES(T)) k_sweep_lds27(
    const T *__restrict__ d1, const T *__restrict__ d2, const T *__restrict__ e1, const T *__restrict__ e2,
    T *__restrict__ d1n, T *__restrict__ d2n, T *__restrict__ e1n, T *__restrict__ e2n, const int N,
    const int zchunk, const int ntx, const int nty, const CoefPair *__restrict__ C, double *__restrict__ part)
{
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, b = tile / ntx;
    const int ty = b % nty;
    const int tz = b / nty;
    const int z0 = tz * zchunk;
    sweep_tile27<T, NH, TX, TY, false>(d1, d2, e1, e2, d1n, d2n, e1n, e2n, N, ZPlanes<T>{}, tx * TX, ty * TY,
                                       z0, min(z0 + zchunk, N), C, part + (size_t)tile * kNPart);
}

template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP27_WAVES(T)) k_sweep_ens27(
    const EnsEntry *__restrict__ tab, const int4 *__restrict__ items, const int nitems, int *queue,
    const int parity)
{
    for_each_item(queue, nitems, [&](int i) {
        const int4 it = items[i];  // x: realization, y: tile index within it, z: partial row
        const EnsEntry &e = tab[it.x];
        const int tx = it.y % e.ntx, r2 = it.y / e.ntx, ty = r2 % e.nty, tz = r2 / e.nty;
        const int z0 = tz * e.zchunk;
        const T *const *in = (const T *const *)e.buf[parity];
        T *const *out = (T *const *)e.buf[parity ^ 1];
        sweep_tile27<T, NH, TX, TY, false>(in[0], in[1], in[2], in[3], out[0], out[1], out[2], out[3], e.N,
                                           ZPlanes<T>{}, tx * TX, ty * TY, z0, min(z0 + e.zchunk, e.N), e.C,
                                           e.part + (size_t)it.z * kNPart);
    });
}

// ------------------------------------------------------------ launchers

namespace {

template <typename T>
void lds27_t(int tile_x, int tile_y, int beta, const void *const in[4], void *const out[4], int N,
             int zchunk, const CoefPair *C, double *part, hipStream_t st)
{
    with_tile(tile_x, tile_y, [&](auto tx, auto ty) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
        with_nh(beta, [&](auto nh) {
            constexpr int NH = decltype(nh)::value;
            const int ntx = (N + TX - 1) / TX, nty = (N + TY - 1) / TY, nzc = (N + zchunk - 1) / zchunk;
            hipLaunchKernelGGL((k_sweep_lds27<T, NH, TX, TY>), dim3(ntx * nty * nzc), dim3(256), 0, st,
                               (const T *)in[0], (const T *)in[1], (const T *)in[2], (const T *)in[3],
                               (T *)out[0], (T *)out[1], (T *)out[2], (T *)out[3], N, zchunk, ntx, nty, C,
                               part);
        });
    });
}

template <typename T>
void ens27_t(int tile_x, int tile_y, int beta, const EnsEntry *tab, const int4 *items, int nitems, int *queue,
             int grid, int parity, hipStream_t st)
{
    with_tile(tile_x, tile_y, [&](auto tx, auto ty) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
        with_nh(beta, [&](auto nh) {
            constexpr int NH = decltype(nh)::value;
            hipLaunchKernelGGL((k_sweep_ens27<T, NH, TX, TY>), dim3(grid), dim3(256), 0, st, tab, items, nitems,
                               queue, parity);
        });
    });
}

template <typename T>
int occ27_t(int tile_x, int tile_y, int beta)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    with_tile(tile_x, tile_y, [&](auto tx, auto ty) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
        with_nh(beta, [&](auto nh) {
            constexpr int NH = decltype(nh)::value;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep_lds27<T, NH, TX, TY>, 256, 0);
        });
    });
    return e == hipSuccess ? nb : 0;
}

}  // namespace

void launch_sweep_lds27(int dtype, int tile_x, int tile_y, int beta, const void *const in[4],
                        void *const out[4], int N, int zchunk, const CoefPair *C, double *part,
                        hipStream_t st)
{
    if (dtype == 0) lds27_t<float>(tile_x, tile_y, beta, in, out, N, zchunk, C, part, st);
    else lds27_t<double>(tile_x, tile_y, beta, in, out, N, zchunk, C, part, st);
}

void launch_sweep_ens27(int dtype, int tile_x, int tile_y, int beta, const EnsEntry *tab,
                        const int4 *items, int nitems, int *queue, int grid, int parity, hipStream_t st)
{
    if (dtype == 0) ens27_t<float>(tile_x, tile_y, beta, tab, items, nitems, queue, grid, parity, st);
    else ens27_t<double>(tile_x, tile_y, beta, tab, items, nitems, queue, grid, parity, st);
}

int sweep_lds27_blocks_per_cu(int dtype, int tile_x, int tile_y, int beta)
{
    return dtype == 0 ? occ27_t<float>(tile_x, tile_y, beta) : occ27_t<double>(tile_x, tile_y, beta);
}

}  // namespace lf
