// Fused kick-drift sweep of the staggered leapfrog (Sainio, arXiv:0911.5692,
// eq. evo applied to eq. scalar-evo), gfx950.
//
// The lattice arrays hold deviations d_i = f_i - f_bar_i and e_i = v_i - v_bar_i
// from the FP64 homogeneous mode, so per site and field
//   e_i(k+1)   = e_i(k) + [Cl * S6(d_i) + Cf * d_i - dt (dV_pr/df_i(f_bar + d) - dV_pr/df_i(f_bar))]
//   d_i(k+3/2) = d_i(k+1/2) + dt * e_i(k+1)
// with S6(d) = sum of the 6 neighbours - 6 d, Cl = dt a^(-2s-2)/dx^2 and
// Cf = dt [r(s-r+2)(a'/a)^2 + r a''/a] (coefficients from the FP64 scale-factor
// kernel).  The potential difference is expanded around f_bar so that no
// O(1) quantity is rounded into an O(deviation) result:
//   c1 a^p1 [(g+d)^(beta-1) - g^(beta-1)] = d * Horner(h, d)
//   G a^p2 [f1 f2^2 - g1 g2^2] = C2 [d1 (g2+d2)^2 + g1 d2 (2 g2 + d2)]
//   G a^p2 [f1^2 f2 - g1^2 g2] = C2 [d1 (2 g1 + d1)(g2 + d2) + g1^2 d2]
//
// Two implementations of the same per-site arithmetic (identical rounding):
//
// k_sweep_lds — the production kernel.  A block of 256 threads owns a
//   TX (x, 64 or 128) x TY (y) column tile and marches a chunk of z planes.
//   Each plane of d1, d2 is staged in LDS with its halo (the paper's "three
//   shared planes" become one LDS plane plus a register queue d(z-1), d(z),
//   d(z+1) per site); x rows are TX consecutive elements, so every global
//   access is a coalesced 256- or 512-byte row.  The sums the next scale-factor update needs
//   (sum |grad d_new|^2 per field, sum f1^beta, sum f1^2 f2^2 of the new
//   fields) are formed in the same sweep: gradients use backward differences,
//   and the block also computes d_new on a one-sided ring (row y0-1, column
//   x0-1, and the plane z0-1 before its chunk) without storing it, so no
//   second pass over the lattice is needed.  That keeps HBM traffic at the
//   algorithmic 32 B per site in FP32 (f and v read, v and f written, two
//   fields); halo and ring re-reads are served from L2.  Per-block FP64
//   partial sums (wave butterfly, then waves in order) go to part[block];
//   the scale-factor kernel adds them in a fixed order.
//
// k_sweep_plain — one thread per site, neighbours straight from global
//   memory, followed by the separate reduction k_reduce.  Kept as the simple
//   reference variant (tile_y = 1); it also implements the 27-point stencil
//   (ST = 27, the paper's own Laplacian, Sec. II.C).
//
// The LDS z-march itself (sweep_tile) is in lf_sweep_tile.h; the 27-point
// stencil's is k_sweep_lds27 (lf_sweep27.hip), and the launchers here
// dispatch to it.  The z-slab variants are in lf_slab7.hip / lf_slab27.hip.
#include "lf_sweep_tile.h"

namespace lf {

// ------------------------------------------------------------ plain variant

template <typename T, int NH, int ST>
__global__ void __launch_bounds__(256) k_sweep_plain(const T *__restrict__ d1, const T *__restrict__ d2,
                                                     const T *__restrict__ e1, const T *__restrict__ e2,
                                                     T *__restrict__ d1n, T *__restrict__ d2n,
                                                     T *__restrict__ e1n, T *__restrict__ e2n, int N,
                                                     const CoefPair *__restrict__ C)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= N || y >= N) return;
    Coefs<T, NH> c;
    c.load(coef_of<T>(C));
    const int64_t NN = (int64_t)N * N;
    const int64_t i = (int64_t)z * NN + (int64_t)y * N + x;
    const int64_t xm = (x == 0) ? i + (N - 1) : i - 1;
    const int64_t xp = (x == N - 1) ? i - (N - 1) : i + 1;
    const int64_t ym = (y == 0) ? i + (int64_t)(N - 1) * N : i - N;
    const int64_t yp = (y == N - 1) ? i - (int64_t)(N - 1) * N : i + N;
    const int64_t zm = (z == 0) ? i + (int64_t)(N - 1) * NN : i - NN;
    const int64_t zp = (z == N - 1) ? i - (int64_t)(N - 1) * NN : i + NN;
    const T a = d1[i], b = d2[i];
    T la, lb;
    if constexpr (ST == 7) {
        la = six_sum(d1[xm], d1[xp], d1[ym], d1[yp], d1[zm], d1[zp], a);
        lb = six_sum(d2[xm], d2[xp], d2[ym], d2[yp], d2[zm], d2[zp], b);
    } else {
        auto idx = [&](int dx, int dy, int dz) {
            const int64_t ox = dx < 0 ? xm - i : (dx > 0 ? xp - i : 0);
            const int64_t oy = dy < 0 ? ym - i : (dy > 0 ? yp - i : 0);
            const int64_t oz = dz < 0 ? zm - i : (dz > 0 ? zp - i : 0);
            return i + ox + oy + oz;
        };
        la = lap_raw<27, T>([&](int dx, int dy, int dz) { return d1[idx(dx, dy, dz)]; }, a);
        lb = lap_raw<27, T>([&](int dx, int dy, int dz) { return d2[idx(dx, dy, dz)]; }, b);
    }
    T ia, ib;
    c.force(a, b, la, lb, ia, ib);
    const T ea = e1[i] + ia, eb = e2[i] + ib;
    e1n[i] = ea;
    e2n[i] = eb;
    d1n[i] = a + c.dt * ea;
    d2n[i] = b + c.dt * eb;
}

// Single lattice: one block per (tile, z-chunk), XCD-aware tile order.
template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP_MIN_WAVES) k_sweep_lds(
    const T *__restrict__ d1, const T *__restrict__ d2, const T *__restrict__ e1, const T *__restrict__ e2,
    T *__restrict__ d1n, T *__restrict__ d2n, T *__restrict__ e1n, T *__restrict__ e2n, const int N,
    const int zchunk, const int ntx, const int nty, const CoefPair *__restrict__ C, double *__restrict__ part)
{
    // partial row = logical tile index (the ensemble kernel uses the same rows)
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, b = tile / ntx;
    const int ty = b % nty;
    const int tz = b / nty;
    const int z0 = tz * zchunk;
    sweep_tile<T, NH, TX, TY, LF_SWEEP_PREFETCH, false>(d1, d2, e1, e2, d1n, d2n, e1n, e2n, N, ZPlanes<T>{},
                                                        tx * TX, ty * TY, z0, min(z0 + zchunk, N), C,
                                                        part + (size_t)tile * kNPart);
}

// Ensemble: a persistent grid takes the work items (realization, tile,
// z-chunk) of a static list from per-XCD segments (for_each_item); each item
// writes its own partial row of its realization.  All realizations advance
// one step per launch.
template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP_MIN_WAVES) k_sweep_ens(
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
        sweep_tile<T, NH, TX, TY, LF_SWEEP_PREFETCH, false>(in[0], in[1], in[2], in[3], out[0], out[1], out[2],
                                                            out[3], e.N, ZPlanes<T>{}, tx * TX, ty * TY, z0,
                                                            min(z0 + e.zchunk, e.N), e.C,
                                                            e.part + (size_t)it.z * kNPart);
    });
}

// ------------------------------------------------------------ launchers

template <typename T, int NH, int ST>
static void sweep_plain_t(const void *const in[4], void *const out[4], int N, const CoefPair *C,
                          hipStream_t st)
{
    dim3 grid((N + 63) / 64, (N + 3) / 4, N), block(64, 4);
    hipLaunchKernelGGL((k_sweep_plain<T, NH, ST>), grid, block, 0, st, (const T *)in[0], (const T *)in[1],
                       (const T *)in[2], (const T *)in[3], (T *)out[0], (T *)out[1], (T *)out[2],
                       (T *)out[3], N, C);
}

template <typename T, int ST>
static void sweep_plain_b(int beta, const void *const in[4], void *const out[4], int N,
                          const CoefPair *C, hipStream_t st)
{
    switch (beta) {
    case 2: sweep_plain_t<T, 1, ST>(in, out, N, C, st); break;
    case 3: sweep_plain_t<T, 2, ST>(in, out, N, C, st); break;
    case 4: sweep_plain_t<T, 3, ST>(in, out, N, C, st); break;
    case 5: sweep_plain_t<T, 4, ST>(in, out, N, C, st); break;
    default: sweep_plain_t<T, 5, ST>(in, out, N, C, st); break;
    }
}

void launch_sweep_plain(int stencil, int dtype, int beta, const void *const in[4], void *const out[4],
                        int N, const CoefPair *C, hipStream_t st)
{
    if (stencil == 27) {
        if (dtype == 0) sweep_plain_b<float, 27>(beta, in, out, N, C, st);
        else sweep_plain_b<double, 27>(beta, in, out, N, C, st);
    } else {
        if (dtype == 0) sweep_plain_b<float, 7>(beta, in, out, N, C, st);
        else sweep_plain_b<double, 7>(beta, in, out, N, C, st);
    }
}

int sweep_lds_blocks(int N, int tile_x, int tile_y, int zchunk)
{
    return sweep_io_blocks(N, N, tile_x, tile_y, zchunk);
}

int sweep_io_blocks(int N, int nz, int tile_x, int tile_y, int zchunk)
{
    return ((N + tile_x - 1) / tile_x) * ((N + tile_y - 1) / tile_y) * ((nz + zchunk - 1) / zchunk);
}

template <typename T, int NH, int TX, int TY>
static void sweep_lds_t(const void *const in[4], void *const out[4], int N, int zchunk,
                        const CoefPair *C, double *part, hipStream_t st)
{
    const int ntx = (N + TX - 1) / TX, nty = (N + TY - 1) / TY, nzc = (N + zchunk - 1) / zchunk;
    hipLaunchKernelGGL((k_sweep_lds<T, NH, TX, TY>), dim3(ntx * nty * nzc), dim3(256), 0, st,
                       (const T *)in[0], (const T *)in[1], (const T *)in[2], (const T *)in[3],
                       (T *)out[0], (T *)out[1], (T *)out[2], (T *)out[3], N, zchunk, ntx, nty, C, part);
}

template <typename T, int TX, int TY>
static void sweep_lds_b(int beta, const void *const in[4], void *const out[4], int N, int zchunk,
                        const CoefPair *C, double *part, hipStream_t st)
{
    switch (beta) {
    case 2: sweep_lds_t<T, 1, TX, TY>(in, out, N, zchunk, C, part, st); break;
    case 3: sweep_lds_t<T, 2, TX, TY>(in, out, N, zchunk, C, part, st); break;
    case 4: sweep_lds_t<T, 3, TX, TY>(in, out, N, zchunk, C, part, st); break;
    case 5: sweep_lds_t<T, 4, TX, TY>(in, out, N, zchunk, C, part, st); break;
    default: sweep_lds_t<T, 5, TX, TY>(in, out, N, zchunk, C, part, st); break;
    }
}

// Supported tiles (x by y): 32x8, 32x16, 64x4, 64x8, 64x16, 128x4, 128x8.
template <typename T>
static void sweep_lds_y(int tile_x, int tile_y, int beta, const void *const in[4], void *const out[4],
                        int N, int zchunk, const CoefPair *C, double *part, hipStream_t st)
{
    if (tile_x == 128) {
        if (tile_y == 4) sweep_lds_b<T, 128, 4>(beta, in, out, N, zchunk, C, part, st);
        else sweep_lds_b<T, 128, 8>(beta, in, out, N, zchunk, C, part, st);
        return;
    }
    if (tile_x == 32) {
        if (tile_y == 8) sweep_lds_b<T, 32, 8>(beta, in, out, N, zchunk, C, part, st);
        else sweep_lds_b<T, 32, 16>(beta, in, out, N, zchunk, C, part, st);
        return;
    }
    switch (tile_y) {
    case 4: sweep_lds_b<T, 64, 4>(beta, in, out, N, zchunk, C, part, st); break;
    case 8: sweep_lds_b<T, 64, 8>(beta, in, out, N, zchunk, C, part, st); break;
    default: sweep_lds_b<T, 64, 16>(beta, in, out, N, zchunk, C, part, st); break;
    }
}

template <typename T, int TX, int TY>
static int occ_b(int beta)
{
    int nb = 0;
    hipError_t e;
    switch (beta) {
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep_lds<T, 1, TX, TY>, 256, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep_lds<T, 2, TX, TY>, 256, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep_lds<T, 3, TX, TY>, 256, 0); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep_lds<T, 4, TX, TY>, 256, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep_lds<T, 5, TX, TY>, 256, 0); break;
    }
    return e == hipSuccess ? nb : 0;
}

template <typename T>
static int occ_y(int tile_x, int tile_y, int beta)
{
    if (tile_x == 128) return tile_y == 4 ? occ_b<T, 128, 4>(beta) : occ_b<T, 128, 8>(beta);
    if (tile_x == 32) return tile_y == 8 ? occ_b<T, 32, 8>(beta) : occ_b<T, 32, 16>(beta);
    switch (tile_y) {
    case 4: return occ_b<T, 64, 4>(beta);
    case 8: return occ_b<T, 64, 8>(beta);
    default: return occ_b<T, 64, 16>(beta);
    }
}

int sweep_lds_blocks_per_cu(int stencil, int dtype, int tile_x, int tile_y, int beta)
{
    if (stencil == 27) return sweep_lds27_blocks_per_cu(dtype, tile_x, tile_y, beta);
    return dtype == 0 ? occ_y<float>(tile_x, tile_y, beta) : occ_y<double>(tile_x, tile_y, beta);
}

template <typename T, int NH, int TX, int TY>
static void sweep_ens_t(const EnsEntry *tab, const int4 *items, int nitems, int *queue, int grid, int parity,
                        hipStream_t st)
{
    hipLaunchKernelGGL((k_sweep_ens<T, NH, TX, TY>), dim3(grid), dim3(256), 0, st, tab, items, nitems, queue,
                       parity);
}

template <typename T, int TX, int TY>
static void sweep_ens_b(int beta, const EnsEntry *tab, const int4 *items, int nitems, int *queue, int grid,
                        int parity, hipStream_t st)
{
    switch (beta) {
    case 2: sweep_ens_t<T, 1, TX, TY>(tab, items, nitems, queue, grid, parity, st); break;
    case 3: sweep_ens_t<T, 2, TX, TY>(tab, items, nitems, queue, grid, parity, st); break;
    case 4: sweep_ens_t<T, 3, TX, TY>(tab, items, nitems, queue, grid, parity, st); break;
    case 5: sweep_ens_t<T, 4, TX, TY>(tab, items, nitems, queue, grid, parity, st); break;
    default: sweep_ens_t<T, 5, TX, TY>(tab, items, nitems, queue, grid, parity, st); break;
    }
}

// Supported tiles (x by y): 32x8, 32x16, 64x4, 64x8, 64x16, 128x4, 128x8.
template <typename T>
static void sweep_ens_y(int tile_x, int tile_y, int beta, const EnsEntry *tab, const int4 *items,
                        int nitems, int *queue, int grid, int parity, hipStream_t st)
{
    if (tile_x == 128) {
        if (tile_y == 4) sweep_ens_b<T, 128, 4>(beta, tab, items, nitems, queue, grid, parity, st);
        else sweep_ens_b<T, 128, 8>(beta, tab, items, nitems, queue, grid, parity, st);
        return;
    }
    if (tile_x == 32) {
        if (tile_y == 8) sweep_ens_b<T, 32, 8>(beta, tab, items, nitems, queue, grid, parity, st);
        else sweep_ens_b<T, 32, 16>(beta, tab, items, nitems, queue, grid, parity, st);
        return;
    }
    switch (tile_y) {
    case 4: sweep_ens_b<T, 64, 4>(beta, tab, items, nitems, queue, grid, parity, st); break;
    case 8: sweep_ens_b<T, 64, 8>(beta, tab, items, nitems, queue, grid, parity, st); break;
    default: sweep_ens_b<T, 64, 16>(beta, tab, items, nitems, queue, grid, parity, st); break;
    }
}

void launch_sweep_ens(int stencil, int dtype, int tile_x, int tile_y, int beta, const EnsEntry *tab,
                      const int4 *items, int nitems, int *queue, int grid, int parity, hipStream_t st)
{
    if (stencil == 27) launch_sweep_ens27(dtype, tile_x, tile_y, beta, tab, items, nitems, queue, grid, parity, st);
    else if (dtype == 0) sweep_ens_y<float>(tile_x, tile_y, beta, tab, items, nitems, queue, grid, parity, st);
    else sweep_ens_y<double>(tile_x, tile_y, beta, tab, items, nitems, queue, grid, parity, st);
}

void launch_sweep_lds(int stencil, int dtype, int tile_x, int tile_y, int beta, const void *const in[4],
                      void *const out[4], int N, int zchunk, const CoefPair *C, double *part,
                      hipStream_t st)
{
    if (stencil == 27) launch_sweep_lds27(dtype, tile_x, tile_y, beta, in, out, N, zchunk, C, part, st);
    else if (dtype == 0) sweep_lds_y<float>(tile_x, tile_y, beta, in, out, N, zchunk, C, part, st);
    else sweep_lds_y<double>(tile_x, tile_y, beta, in, out, N, zchunk, C, part, st);
}

}  // namespace lf
