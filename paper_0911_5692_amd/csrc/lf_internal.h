// Internal declarations shared by the kernels and the C-ABI layer of liblf.
// Equation references: Sainio, "CUDAEASY", arXiv:0911.5692, Sec. II.B.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lf_stencil.h"

namespace lf {

constexpr int kMaxBeta = 6;
constexpr int kNPart = 4;   // step reduction: sum|d+ f1|^2, sum|d+ f2|^2, sum f1^beta, sum f1^2 f2^2
constexpr int kNMom = 10;   // input moments (see k_input_moments)
constexpr int kNEn = 6;     // energy sums (see k_diag_march)
constexpr int kStage2Threads = 256;

// Model parameters in device memory (read by the scale-factor kernel, so a
// captured graph picks up lf_set_coupling without re-capture).
struct DevParams {
    double L, dx, dt, c1, G, r, s, kappa2;
    double p1, p2;      // powers of a of the degree-beta and degree-4 terms of V_pr
    int N, beta;
    double N3;          // N^3 as a double
    double gw;          // stencil weight: 1 (7-point) or 1/30 (27-point); multiplies
                        // every raw Laplacian and gradient sum with 1/dx^2
    int stencil, pad;   // 7 or 27
};

// FP64 scalar state of the evolution (device resident).
struct DevScalars {
    double a_half;      // a_{k+1/2}
    double ad;          // a'_k
    double bg_f[2];     // homogeneous mode f_bar_i(k+1/2)
    double bg_v[2];     // homogeneous mode v_bar_i(k)
    double pend[kNPart];// totals of the last step reduction (over the stored f)
    long long step;
    unsigned int status;// bit 0: non-finite average / quadratic
    unsigned int pad;
    // initialisation scratch
    double mean_f[2], mean_u[2], conv, ad0;
};

// Per-step coefficients of the fused kick-drift, written by the scale-factor
// kernel in both precisions (the sweep reads its own).
template <typename T>
struct Coef {
    T Cl;        // dt a^(-2s-2) gw / dx^2  (multiplies the raw stencil sum)
    T Cf;        // dt [r(s-r+2)(a'/a)^2 + r a''/a]
    T dt;
    T C2;        // dt G a^p2
    T g1, g2;    // background f_bar at k+1/2
    T two_g1, two_g2, g1sq;
    T h[kMaxBeta];  // dt c1 a^p1 C(beta-1, j) g1^(beta-1-j), j = 1..beta-1 (h[j-1])
    int nh;         // beta - 1
    int pad;
};

struct CoefPair {
    Coef<float> f;
    Coef<double> d;
    double g1n, g2n;    // background at k+3/2 (FP64), for the reduction of f_new
};

// Hardware places block b on XCD (b mod 8).  Give each XCD a contiguous range
// of logical tiles, so that tiles sharing halo rows run on the same L2.
__device__ inline int xcd_remap(int b, int nb)
{
    constexpr int kXcd = 8;
    const int q = nb / kXcd;
    if (b >= q * kXcd) return b;
    return (b % kXcd) * q + b / kXcd;
}

// The same order for a grid-stride walk over nitems items: in every round
// where the whole grid has an item, the blocks of each XCD take a contiguous
// range of them; the last, partial round keeps the plain order.
__device__ inline int xcd_item(int round_base, int nitems)
{
    return round_base + (round_base + (int)gridDim.x <= nitems ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x);
}

// One realization of an ensemble, as the batched kernels see it.
struct EnsEntry {
    void *buf[2][4];        // ping/pong deviation arrays d1, d2, e1, e2
    double *part;           // partial-sum rows of this realization
    const CoefPair *C;      // its per-step coefficients
    const DevParams *P;
    DevScalars *S;
    CoefPair *Cw;           // same as C, writable (scale-factor kernel)
    int N, zchunk, ntx, nty, rows, pad;
};

// Launch helpers (lf_kernels.hip, lf_sweep.hip).  All enqueue on `st`.
void launch_input_moments(int stencil, int in_dtype, const void *f1, const void *f2, const void *v1,
                          const void *v2, int N, int beta, double *part, int nblk, hipStream_t st);
void launch_init_scalars(const double *part, int nblk, const DevParams *P, DevScalars *S,
                         int physical, double a0, double ad0, hipStream_t st);
void launch_init_fields(int dtype, int in_dtype, const void *f1, const void *f2, const void *v1,
                        const void *v2, void *d1, void *d2, void *e1, void *e2, int N,
                        const DevParams *P, const DevScalars *S, hipStream_t st);
void launch_reduce(int stencil, int dtype, const void *d1, const void *d2, int N, const double *bg_f,
                   int beta, double *part, int nblk, hipStream_t st);
// tape (may be NULL): receives a copy of *S as it was before the update
void launch_aupdate(const double *part, int nblk, const DevParams *P, DevScalars *S,
                    CoefPair *C, hipStream_t st, DevScalars *tape = nullptr);
// queue: the ensemble sweep's work counters (8, 32 ints apart), reset to 0
// by this kernel, followed by the 9 segment bounds of the item list
void launch_aupdate_ens(const EnsEntry *tab, int R, int *queue, hipStream_t st);
void launch_sweep_ens(int stencil, int dtype, int tile_x, int tile_y, int beta, const EnsEntry *tab,
                      const int4 *items, int nitems, int *queue, int grid, int parity, hipStream_t st);
void launch_sweep_plain(int stencil, int dtype, int beta, const void *const in[4], void *const out[4], int N,
                        const CoefPair *C, hipStream_t st);
// Arrays of one sweep over planes [0, nz) of an N x N x nz z-slab: the
// inputs d1, d2, e1, e2, their halo bases (lo: plane -2, hi: plane nz; see
// ZPlanes in lf_sweep_common.h) and the outputs.
struct SweepIO {
    const void *in[4];
    const void *lo[4];
    const void *hi[4];
    void *out[4];
    int nz;
};
void launch_sweep_lds(int stencil, int dtype, int tile_x, int tile_y, int beta, const void *const in[4],
                      void *const out[4], int N, int zchunk, const CoefPair *C, double *part,
                      hipStream_t st);
// z-slab sweeps (lf_slab7.hip, lf_slab27.hip); launch_sweep_slab dispatches
// to launch_sweep_slab27 for stencil 27
void launch_sweep_slab(int stencil, int dtype, int tile_x, int tile_y, int beta, const SweepIO &io, int N,
                       int zchunk, const CoefPair *C, double *part, hipStream_t st);
void launch_sweep_slab27(int dtype, int tile_x, int tile_y, int beta, const SweepIO &io, int N, int zchunk,
                         const CoefPair *C, double *part, hipStream_t st);
int sweep_lds_blocks(int N, int tile_x, int tile_y, int zchunk);
// blocks (= partial rows) of a sweep over nz planes of an N x N x nz block
int sweep_io_blocks(int N, int nz, int tile_x, int tile_y, int zchunk);
// 27-point LDS sweep (lf_sweep27.hip); launch_sweep_lds / launch_sweep_ens /
// sweep_lds_blocks_per_cu dispatch to these for stencil 27.
void launch_sweep_lds27(int dtype, int tile_x, int tile_y, int beta, const void *const in[4],
                        void *const out[4], int N, int zchunk, const CoefPair *C, double *part,
                        hipStream_t st);
void launch_sweep_ens27(int dtype, int tile_x, int tile_y, int beta, const EnsEntry *tab,
                        const int4 *items, int nitems, int *queue, int grid, int parity, hipStream_t st);
int sweep_lds27_blocks_per_cu(int dtype, int tile_x, int tile_y, int beta);
// Resident blocks per CU of the LDS sweep instantiation (0 if unknown, e.g.
// no device).
int sweep_lds_blocks_per_cu(int stencil, int dtype, int tile_x, int tile_y, int beta);
void launch_energy(int stencil, int dtype, const void *const st4[4], int N, const DevParams *P,
                   const DevScalars *S, double *part, int nblk, double *out_dev, hipStream_t st);
void launch_rho_p(int stencil, int dtype, int out_dtype, const void *const s4[4], void *rho, void *pr, int N,
                  const DevParams *P, const DevScalars *S, double *part, int nblk, double *out_dev,
                  hipStream_t st);
void launch_get_fields(int dtype, int out_dtype, const void *const st4[4], void *const out[4],
                       int N, const DevParams *P, const DevScalars *S, int synchronized,
                       hipStream_t st);
void launch_stream_copy(const float *const a[4], float *const b[4], int64_t n, hipStream_t st);
void launch_sync_deviation(int dtype, const void *d, const void *e, double *out, int N, double h, int velocity,
                           hipStream_t st);
void launch_sum_partials(const double *part, int nblk, int nv, double *out, hipStream_t st);
void launch_fill_synthetic(int dtype, void *const s4[4], int N, DevScalars *S, hipStream_t st);
// adjoint (lf_adjoint.hip)
constexpr int kNAdjPart = 7;
void launch_adj_seed(int stencil, int dtype, const void *const s4[4], int N, const DevParams *P, const DevScalars *S,
                     const double *w, double *const lam[4], double *part, int nblk, double *A,
                     hipStream_t st);
// One reverse step: stored fields d1, d2 and scalars tape of X_k, cotangents
// lin (of X_{k+1}) -> lout (of X_k).  have_sums: part already holds the
// step's sums (formed by the previous step's fields pass).  next_*: when set,
// the fields pass also forms the sums of the next reverse step (X_{k-1}).
struct AdjStep {
    const void *d1, *d2;
    const DevScalars *tape;
    double *const *lin;
    double *const *lout;
    bool have_sums;
    const void *next_d1, *next_d2;
    const DevScalars *next_tape;
};
void launch_adj_step(int stencil, int dtype, const AdjStep &a, int N, int beta, const DevParams *P, double dt,
                     double *part, int nblk, double *A, double *cf, hipStream_t st);
void launch_adj_desync(int N, double dt, double *const lam[4], double *A, hipStream_t st);
void launch_set_pending(double *part, int nblk, const double *totals, hipStream_t st);
}  // namespace lf

// FFT-based parts (lf_fft.hip): vacuum initial state and power spectra;
// nonzero return = failure, message in msg
struct lf_vacuum;
namespace lf {
size_t vacuum_spectrum_bytes(int N);
int vacuum_workspace(int N, size_t *bytes, char *msg, size_t len);
int vacuum_generate(int N, double L, const struct ::lf_vacuum *v, hipStream_t st, void *ws, size_t ws_bytes,
                    double *const out[4], char *msg, size_t len);
int spectrum_bins(int N);
int spectrum_workspace_bytes(int N, size_t *bytes, char *msg, size_t len);
// power, count: host arrays of nbins; dev: FP64 device array N^3 holding the
// deviation from the homogeneous value bg (device scalar), which enters shell 0
int spectrum_compute(int N, double L, double *dev, const double *bg, int nbins, hipStream_t st, void *ws,
                     size_t ws_bytes, double *power, double *count, char *msg, size_t len);

}  // namespace lf
