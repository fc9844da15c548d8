/*
 * lf.h — C ABI of the MI355X (gfx950) FRW lattice leapfrog library, liblf.so.
 *
 * The library evolves two interacting scalar fields f1 (inflaton, phi) and f2
 * (chi) on a periodic N^3 lattice in an expanding Friedmann–Robertson–Walker
 * background with the staggered leapfrog of J. Sainio, "CUDAEASY — a GPU
 * Accelerated Cosmological Lattice Program" (arXiv:0911.5692), Sec. II.B:
 *
 *   field equation, program units, eq. (scalar-evo):
 *     f_i'' = a^(-2s-2) Lap f_i + [r(s-r+2)(a'/a)^2 + r a''/a] f_i - dV_pr/df_i
 *   scale factor, eq. (scale):
 *     a'' = (-s-2) a'^2/a + kappa^2 a^(-2s-2r-1) < sum_i |grad f_i|^2/3 + a^(2s+2) V_pr >
 *   leapfrog, eq. (evo): f at half-integer steps, f' and a' at integer steps.
 *
 * Model family (program units, Sec. II.B and Sec. III):
 *     V_pr = c1 a^p1 f1^beta / beta + G a^p2 f1^2 f2^2 / 2,
 *     p1 = -2s + (2-beta) r,  p2 = -2s - 2r,  with s - 2r + 3 = 0.
 *   lambda phi^4: beta = 4, r = 1, s = -1.   m^2 phi^2: beta = 2, r = 3/2, s = 0.
 *
 * Laplacian (periodic in x, y, z), chosen per context by lf_params.stencil:
 *   7:  the 6-neighbour stencil of LATTICEEASY (named in Sec. II.C);
 *   27: the stencil the paper itself uses (Sec. II.C): all 26 neighbours of
 *       the 3x3x3 cube, second-order accurate and fourth-order isotropic,
 *       weights (centre, face, edge, corner) = (-64/15, 7/15, 1/10, 1/30)/dx^2.
 * The gradient energy <|grad f|^2> in eq. (scale) and in the energies is the
 * Dirichlet form of the same stencil, -<f Lap f>: forward differences
 * |d+ f|^2 for 7 points; for 27 points the sum over the 13 bonds b whose
 * first nonzero component (in z, y, x order) is +1 of
 * w_b (f(x+b) - f(x))^2 / dx^2 with w = 7/15 (face), 1/10 (edge),
 * 1/30 (corner).  With it, the semi-discrete field equation conserves the
 * discrete energy exactly.
 *
 * Layout.  Every lattice array is N^3 contiguous elements, x fastest:
 * element (x, y, z) sits at (z*N + y)*N + x.  Arrays are device pointers,
 * 256-byte aligned, in the element type the call names (float or double).
 *
 * Precision.  dtype LF_F32 stores the fields and evaluates the stencil in
 * FP32; LF_F64 does both in FP64.  In both cases the device keeps the
 * spatially homogeneous mode of each field and velocity (the "background",
 * f_bar_i, v_bar_i) in FP64 and the lattice arrays hold the deviation from it;
 * the background follows the same leapfrog map as every site, so
 * f = f_bar + deviation holds exactly in exact arithmetic.  The scale factor,
 * the background and every volume average are FP64 (sums accumulated in FP64
 * in a fixed order: results are bitwise reproducible for a given N, dtype and
 * tile shape).
 *
 * Ownership.  The caller allocates every device buffer (inputs, outputs and
 * the workspace sized by lf_workspace_bytes) and keeps it alive until
 * lf_destroy; a context owns only host-side state, the HIP graphs it
 * captured and the streams and events it creates (a capture stream, the
 * adjoint's recompute stream, timing events; default priority), all on the
 * device that was current at lf_create (the stream's device), whatever
 * device is current later.  A context is not thread-safe: use one context
 * per stream.
 *
 * Errors.  Every call returns an lf_status.  No C++ exception crosses the
 * ABI.  lf_last_error() returns a thread-local message for the last failure.
 * LF_ENONFINITE is sticky: once a NaN/Inf reaches a volume average or the
 * scale-factor quadratic, every later lf_energies/lf_ens_energies reports it.
 */
#ifndef LF_H
#define LF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LF_ABI_VERSION 2

typedef enum lf_status {
    LF_OK = 0,
    LF_EINVAL = 1,      /* invalid argument (sizes, pointers, parameters) */
    LF_EHIP = 2,        /* a HIP runtime call failed; message has the HIP error */
    LF_ENONFINITE = 3,  /* a NaN/Inf reached the averages (sticky) */
    LF_ESTATE = 4,      /* call out of order (e.g. lf_step before lf_init) */
    LF_ENOMEM = 5       /* workspace smaller than lf_workspace_bytes */
} lf_status;

typedef enum lf_dtype { LF_F32 = 0, LF_F64 = 1 } lf_dtype;

/* Lattice, model and launch parameters (copied at create). */
typedef struct lf_params {
    int32_t N;        /* sites per side, 4 <= N <= 2048 */
    int32_t dtype;    /* lf_dtype of the lattice arrays */
    double L;         /* comoving box side, program units; dx = L/N */
    double dt;        /* program time step, > 0 */
    int32_t beta;     /* exponent of the dominant term, 2 <= beta <= 6 */
    int32_t flags;    /* must be 0 */
    double c1;        /* program-unit coupling of c1 f1^beta / beta */
    double G;         /* program-unit g^2 of G f1^2 f2^2 / 2 */
    double r, s;      /* rescaling exponents; |s - 2r + 3| <= 1e-12 */
    double kappa2;    /* 8 pi G_Newton / A^2 (0 = no expansion) */
    int32_t tile_y;   /* sweep tile rows: 0 = automatic, 1 = plain one-site-per-thread
                         sweep with a separate reduction, 4, 8 or 16 = LDS z-march */
    int32_t zchunk;   /* planes per z-chunk of the LDS sweep, 0 = automatic (a grid that
                         is resident at once: two blocks per CU for FP32 sweeps with
                         128-wide tiles, else as many as fit, with chunks of at most
                         64 planes) */
    int32_t tile_x;   /* sweep tile columns: 0 = automatic (128 x 8 from N = 256 up,
                         64 x 8 or 64 x 4 below), 32, 64 or 128 (128 with tile_y 4 or
                         8 only; 32 with tile_y 8 or 16 and the 7-point stencil only) */
    int32_t stencil;  /* Laplacian: 0 or 7 = 7-point, 27 = 27-point (see above) */
} lf_params;

/* Volume averages at the synchronised time k (eq. rho-pres in program
 * units): f(k) = f(k+1/2) - dt/2 v(k), a_k = a_{k+1/2} - dt/2 a'_k,
 *   K_i  = < (v_i - r (a'/a) f_i)^2 / 2 >     kinetic
 *   Gr_i = < a^(-2s-2) |grad f_i|^2 / 2 >     gradient (the stencil's Dirichlet form)
 *   P    = < V_pr(f, a) >                      potential
 *   rho  = sum K + sum Gr + P
 *   R    = (kappa^2/3) a^(2-2r) rho / a'^2 - 1 Friedmann residual, the
 *          program-unit form of K/(a^2 H^2) of Sec. III (0 when kappa2 = 0). */
typedef struct lf_report {
    int64_t step;
    double a, ad, hubble;   /* a_k, a'_k, a'_k / a_k */
    double K[2], Gr[2], P, rho, R;
    uint32_t status;        /* nonzero: a NaN/Inf was seen (sticky) */
    uint32_t pad_;
} lf_report;

/* Scalar part of a checkpoint (see lf_get_state). */
typedef struct lf_scalars {
    int64_t step;
    double a_half;      /* a_{k+1/2} */
    double ad;          /* a'_k */
    double bg_f[2];     /* background f_bar_i(k+1/2) */
    double bg_v[2];     /* background v_bar_i(k) */
    double pend[4];     /* sums over the stored f(k+1/2) that the next step's
                           a'' needs: the gradient sums of f1 and f2 (dx^2
                           |grad f|^2 summed; for 27 points times 30), then
                           sum f1^beta, sum f1^2 f2^2 */
    uint32_t status;
    uint32_t pad_;
} lf_scalars;

typedef struct lf_ctx lf_ctx;
typedef struct lf_ens lf_ens;

/* ---- version and errors ------------------------------------------------ */

int lf_abi_version(void);
/* Thread-local, valid until the next failing call on this thread. */
const char *lf_last_error(void);

/* ---- single lattice ---------------------------------------------------- */

/* Bytes of device workspace a context with these parameters needs.
 * EINVAL if the parameters are invalid. */
int lf_workspace_bytes(const lf_params *p, size_t *out_bytes);

/* Create a context.  stream: a hipStream_t (NULL = the null stream) on which
 * every later call enqueues its work; workspace: device memory of at least
 * lf_workspace_bytes bytes, 256-byte aligned, owned by the caller.
 * EINVAL (parameters, alignment, NULL workspace), ENOMEM (too small). */
int lf_create(const lf_params *p, void *stream, void *workspace, size_t ws_bytes,
              lf_ctx **out);

/* Destroy a context: frees its host state, graphs, and the streams and events
 * it created (not the caller's stream or any device buffer).  NULL is a
 * no-op. */
int lf_destroy(lf_ctx *ctx);

/* Initialise from a synchronised program-unit state at tau = 0
 * (Sec. II.B): fields f1, f2 and velocities v1 = f1', v2 = f2', N^3 device
 * arrays of element type in_dtype (read only; may be freed after the call
 * returns and the stream has run), scale factor a0 > 0 and a'_0 = ad0.
 * Computes the background (the FP64 spatial means), writes the deviations
 * into the workspace and advances the fields half a step (the
 * desynchronisation of Sec. II.B).  Asynchronous on the context's stream. */
int lf_init(lf_ctx *ctx, const void *f1, const void *f2, const void *v1, const void *v2,
            int in_dtype, double a0, double ad0);

/* Initialise from fields and rescaled physical velocities
 * u_i = (A/B) a^(r-s) dphi_i/dt (Sec. II.B, conversion to program units):
 * a'_0 > 0 follows from the Friedmann constraint
 *   a'^2 = (kappa^2/3) a^(2-2r) < sum_i u_i^2/2 + a^(-2s-2)|grad f_i|^2/2 + V_pr >
 * and v_i = u_i + r (a'_0/a_0) f_i.  Blocking (returns a'_0 in *ad0_out). */
int lf_init_physical(lf_ctx *ctx, const void *f1, const void *f2, const void *u1,
                     const void *u2, int in_dtype, double a0, double *ad0_out);

/* Enqueue n >= 0 leapfrog steps (hipGraph replay; asynchronous).
 * ESTATE before lf_init. */
int lf_step(lf_ctx *ctx, int64_t n);

/* Blocking: volume averages at the current synchronised time. Returns
 * ENONFINITE (after filling *out) if the sticky flag is set. */
int lf_energies(lf_ctx *ctx, lf_report *out);

/* Energy density and pressure per site at the synchronised time (eq. rho-pres
 * in program units, the energy-density/pressure computation of Sec. II.C):
 *   rho = sum_i K_i + Gr_i + V_pr,   p = sum_i K_i - Gr_i/3 - V_pr
 * with the per-site terms of lf_report.  rho, p: N^3 arrays of out_dtype or
 * NULL (not written).  avg[3] = <rho>, <p>, w = <p>/<rho>.  Blocking. */
int lf_rho_p(lf_ctx *ctx, void *rho, void *p, int out_dtype, double *avg);

/* Write the full fields (background + deviation) to caller arrays of element
 * type out_dtype: synchronized = 0 gives the stored f(k+1/2), v(k);
 * synchronized = 1 gives f(k) = f(k+1/2) - dt/2 v(k), v(k).  Any pointer may
 * be NULL (skipped).  Asynchronous. */
int lf_get_fields(lf_ctx *ctx, void *f1, void *f2, void *v1, void *v2, int out_dtype,
                  int synchronized);

/* Bitwise checkpoint: copy the four deviation arrays (context dtype) to the
 * caller and return the scalars (blocking).  lf_set_state restores them into a
 * context with the same parameters; evolution then continues bitwise as if
 * uninterrupted. */
int lf_get_state(lf_ctx *ctx, void *d1, void *d2, void *e1, void *e2, lf_scalars *s);
int lf_set_state(lf_ctx *ctx, const void *d1, const void *d2, const void *e1,
                 const void *e2, const lf_scalars *s);

/* Change G (the program-unit g^2) for later steps. */
int lf_set_coupling(lf_ctx *ctx, double G);

/* Time of the last lf_step call measured with HIP events around the work it
 * enqueued, in ms (blocking; 0 if none). */
int lf_last_step_ms(lf_ctx *ctx, double *ms);

/* ---- bandwidth reference ------------------------------------------------ */

/* Copy four FP32 arrays of n elements into four others (b_j = a_j): the byte
 * mix of the FP32 sweep (16 B read and 16 B written per element index), one
 * element per lane over a grid that covers the arrays once in address order,
 * with non-temporal stores (the fastest order measured for this mix).  It
 * does no arithmetic, so its rate is what the device streams for this mix;
 * the benchmark reports the sweep's bandwidth as a fraction of it.
 * Pointers: device arrays, 256-byte aligned, caller-owned, not overlapping;
 * n >= 0 and a multiple of 4 (n = 0 does nothing and checks no pointer).
 * Asynchronous on `stream` (LF_EINVAL for bad arguments, LF_EHIP if the
 * launch fails). */
int lf_stream_copy(const float *a0, const float *a1, const float *a2, const float *a3, float *b0, float *b1,
                   float *b2, float *b3, int64_t n, void *stream);

/* ---- one GPU's share of a lattice split into z-slabs ------------------- */

/* The fused kick-drift sweep of one step (eqs. evo, with the Laplacian and
 * the in-sweep sums of Sec. II.C) on a slab of nz consecutive z-planes of the
 * context's N^3 lattice, as one GPU runs it when the lattice is split along
 * z: the periodic wrap in z is replaced by halo planes received from the two
 * neighbouring slabs.  x and y stay periodic over N.
 *
 * in[4]   d1, d2, e1, e2 of the slab (context dtype, deviations from the
 *         background as the context stores them): nz planes of N*N, x fastest.
 * lo[4]   halo below the slab: d1, d2: planes -2 and -1 (2 planes each, -2
 *         first); e1, e2: plane -1 (1 plane each).
 * hi[2]   halo above the slab: d1, d2: plane nz (1 plane each).
 * out[4]  the new d1, d2, e1, e2 of the slab (nz planes each).
 * partials  device array of partial_rows x 4 doubles; the sweep writes
 *         lf_slab_rows(ctx, nz, zchunk) rows: per block, the sums over its
 *         sites of the two gradient energies, f1^beta and f1^2 f2^2 of the new
 *         fields (the bonds and sites the slab owns: planes 0 .. nz-1 and the
 *         z-bonds between plane -1 and plane 0).  The rows of all slabs
 *         together hold the same bonds and sites as the periodic step's rows.
 * zchunk  planes per block (0: automatic, as for the context's own sweep).
 *
 * The coefficients are those of the context's last step (the scale-factor
 * update that opened it), so with the state that step started from, split
 * into slabs, the outputs equal that step's outputs bitwise.  The context's
 * launch shape must be an LDS one (tile_y 4, 8 or 16).  Pointers are device
 * arrays aligned to the element size, caller-owned; outputs may not overlap
 * any other array.  Asynchronous on the context's stream.  Errors: LF_EINVAL
 * (bad arguments, nz outside [1, N], partials too small), LF_ESTATE (no step
 * since lf_init / lf_set_state), LF_EHIP.  Exchanging halos and summing the
 * partial rows across slabs (then the scale-factor update from the global
 * sums) belongs to the multi-GPU program that calls this and is not in this
 * library. */
int lf_slab_rows(const lf_ctx *ctx, int nz, int zchunk, int64_t *rows);
int lf_slab_sweep(lf_ctx *ctx, int nz, int zchunk, const void *const in[4], const void *const lo[4],
                  const void *const hi[2], void *const out[4], double *partials, int64_t partial_rows);

/* Allocation-free variant of lf_slab_sweep, for callers that cannot allocate
 * device memory around the call (code under HIP graph capture, tight
 * stepping loops, harnesses that forbid hipMalloc).  The same sweep with the
 * same arguments and outputs `out`, except that the partial-sum rows go to a
 * static device array the library holds on each GPU (65536 rows of 4
 * doubles, 2 MiB, kept until the process ends) and are added, in the fixed
 * order of the scale-factor update, into sums[0..3] (a caller-owned device
 * array of 4 doubles, 8-byte aligned): the slab's totals of the two gradient
 * energies, f1^beta and f1^2 f2^2 of the new fields, which the multi-GPU
 * program adds across slabs.  The call allocates nothing and calls no
 * allocating library routine.  Nothing in the array has to start at zero:
 * each call's sweep writes every row it sums.  All calls on one GPU share
 * its array, so calls that overlap in time on one GPU (other streams, other
 * threads, other contexts) race and give undefined sums; serialise them.
 * Asynchronous on the context's stream.  Errors: as lf_slab_sweep, and
 * LF_EINVAL when the launch shape needs more than 65536 rows (a larger
 * zchunk, or lf_slab_sweep with a caller buffer, avoids that). */
int lf_slab_sweep_sums(lf_ctx *ctx, int nz, int zchunk, const void *const in[4], const void *const lo[4],
                       const void *const hi[2], void *const out[4], double *sums);

/* ---- autotuner ---------------------------------------------------------- */

/* Workspace for lf_autotune with these parameters (largest candidate). */
int lf_autotune_workspace_bytes(const lf_params *p, size_t *out_bytes);
/* Pick the sweep launch shape (tile_x, tile_y, zchunk) for p's lattice size,
 * dtype, beta and stencil on the current device.  If cache_path (may be
 * NULL) holds a line for (device architecture, N, dtype, beta, stencil), that
 * choice is returned (*best_ms = -1).  Otherwise every candidate (the plain
 * sweep; LDS tiles 64x4, 64x8, 64x16, 128x4, 128x8, and for the 7-point
 * stencil 32x8, 32x16; z-chunks from the
 * automatic rule, 16, 32, 64, 128, N/6, N/4, N/3, N/2) is timed with HIP
 * events over graph-replayed steps
 * of a synthetic state, the fastest is returned in *best (p with the shape
 * filled in) and appended to the cache as one JSON object per line.  The
 * caller's workspace (lf_autotune_workspace_bytes) is overwritten. */
int lf_autotune(const lf_params *p, void *stream, void *workspace, size_t ws_bytes,
                const char *cache_path, lf_params *best, double *best_ms);

/* ---- adjoint (reverse-mode gradient) ------------------------------------ */

/* Loss E = w[0] K_1 + w[1] K_2 + w[2] Gr_1 + w[3] Gr_2 of the synchronised
 * energies after n steps (e.g. w = {0, 1, 0, 1}: the chi kinetic plus gradient
 * energy).  Its gradient with respect to G and to the synchronised initial
 * state (f1, f2, v1, v2 at tau = 0, a_0, a'_0) is the transpose of the
 * leapfrog map's Jacobian applied in reverse step order (the paper gives the
 * forward map, Sec. II.B; the adjoint is this library's).  Memory: states at
 * steps 0, K, 2K, ... are checkpointed in a caller-owned workspace of
 * lf_adj_workspace_bytes bytes; the backward pass recomputes each K-step
 * segment from its checkpoint, keeps its K states in the same workspace and
 * runs the reverse steps on the exact forward states.  Two segment buffers:
 * segment s - 1 is recomputed on a second stream of the context (default
 * priority) while the reverse steps of segment s run on its own stream.
 * Cotangents are FP64. */
int lf_adj_workspace_bytes(const lf_params *p, int64_t n, int K, size_t *out_bytes);
/* Context just initialised (no step yet).  Runs n steps (the context then
 * holds step n) and returns the loss.  Blocking.  adj_ws must stay alive
 * until lf_adj_backward. */
int lf_adj_forward(lf_ctx *ctx, int64_t n, int K, const double *w, void *adj_ws, size_t ws_bytes,
                   double *loss);
/* dL/dE = dL.  Writes dL/dG, dL/da0, dL/da'0 and the N^3 FP64 device arrays
 * dL/df1(0), dL/df2(0), dL/dv1(0), dL/dv2(0).  Blocking.  Afterwards the
 * context holds an intermediate state: initialise it again before reuse. */
int lf_adj_backward(lf_ctx *ctx, double dL, double *dL_dG, void *g_f1, void *g_f2, void *g_v1,
                    void *g_v2, double *dL_da0, double *dL_dad0);

/* ---- ensemble of independent lattices --------------------------------- */

/* R realizations evolved together: per_real[r] gives each one's lattice and
 * model (N, L, dt, couplings may differ; dtype and beta must be equal).
 * Every step is two launches for the whole ensemble, captured in a HIP
 * graph: a batched FP64 scale-factor update (one block per realization, each
 * with its own a(t), background and averages) and one persistent sweep whose
 * blocks take (realization, tile, z-chunk) work items from device-wide
 * counters: the items are split into one segment per XCD (whole z-chunks,
 * longest first), a block takes items of its own XCD's segment and then
 * those of the others.  The sweep tile is per_real[0].tile_x/tile_y
 * (default 64 x 8; 32-wide tiles for the 7-point stencil only) for all
 * realizations; z-chunks may differ per realization (default: the whole
 * lattice when the realizations' tile columns fill between half and all of
 * the resident grid, else N/2 planes, at least 8, or N when N < 8);
 * lf_ens_autotune picks both by measurement.  Each realization's state
 * matches a single-lattice run with the same parameters to rounding. */
int lf_ens_workspace_bytes(int R, const lf_params *per_real, size_t *out_bytes);
int lf_ens_create(int R, const lf_params *per_real, void *stream, void *workspace, size_t ws_bytes,
                  lf_ens **out);
int lf_ens_destroy(lf_ens *ens);
int lf_ens_size(lf_ens *ens, int *R);
/* As lf_init / lf_init_physical for realization r (only before the first
 * lf_ens_step, or after an even number of steps). */
int lf_ens_init(lf_ens *ens, int r, const void *f1, const void *f2, const void *v1,
                const void *v2, int in_dtype, double a0, double ad0);
int lf_ens_init_physical(lf_ens *ens, int r, const void *f1, const void *f2, const void *u1,
                         const void *u2, int in_dtype, double a0, double *ad0_out);
/* Enqueue n >= 0 steps of every realization (asynchronous). */
int lf_ens_step(lf_ens *ens, int64_t n);
int lf_ens_last_step_ms(lf_ens *ens, double *ms);
/* Blocking: out[r] for r < R; ENONFINITE if any realization has the flag. */
int lf_ens_energies(lf_ens *ens, lf_report *out);
int lf_ens_get_fields(lf_ens *ens, int r, void *f1, void *f2, void *v1, void *v2, int out_dtype,
                      int synchronized);

/* Ensemble launch-shape autotuner (the block-size search of Sec. III, done
 * by measurement).  Times the ensemble sweep of these realizations (sizes,
 * dtype, beta and stencil as in per[]) for every candidate: each LDS tile
 * (32 x 8 and 32 x 16 for the 7-point stencil, 64 x 4/8/16, 128 x 4/8) with
 * z-chunks of target length 16 ... 192 planes, whole lattices, or the default
 * rule (*ztarget = 0), on synthetic states in the caller's workspace
 * (lf_ens_autotune_workspace_bytes), with HIP events over graph-replayed
 * steps.  Returns the fastest tile and target; a realization's z-chunk for a
 * target is lf_ens_zchunk(N, target).  If cache_path (may be NULL) holds a
 * line for (device architecture, the multiset of sizes, dtype, beta,
 * stencil), that choice is returned without timing (*best_ms = -1);
 * otherwise the winner is appended as one JSON object per line.  Blocking. */
int lf_ens_autotune_workspace_bytes(int R, const lf_params *per_real, size_t *out_bytes);
int lf_ens_autotune(int R, const lf_params *per_real, void *stream, void *workspace, size_t ws_bytes,
                    const char *cache_path, int *tile_x, int *tile_y, int *ztarget, double *best_ms);
/* z-chunk of an N^3 realization for a target item length: the fewest equal
 * chunks of at most `target` planes, i.e. ceil(N / ceil(N / target)); N when
 * target >= N; 0 (the default rule) when target <= 0. */
int lf_ens_zchunk(int N, int target);

/* Measurement: run n >= 1 steps outside any graph with HIP events around
 * each kernel of the step (on the context's stream) and return the average
 * duration in ms of kernel j in ms[j], j < n_out:
 *   0 = scale-factor update, 1 = kick-drift sweep, 2 = separate reduction
 *   (0 when the sweep computes it in-sweep).  Blocking.  Advances the state. */
int lf_time_kernels(lf_ctx *ctx, int64_t n, double *ms, int n_out);

/* ---- vacuum initial state on the device (Sec. II.B) --------------------
 * The homogeneous values are inputs; the fluctuations are generated through
 * an FFT, as the paper does after DEFROST (hipFFT in place of CUFFT):
 *   f_i = f0_i + F_i,  u_i = u0_i + U_i  (program units; u are the rescaled
 *   physical velocities that lf_init_physical takes),
 * with F_i, U_i independent Gaussian random fields of power spectrum
 *   P_F(k) = eps2 / (2 omega_k),  P_U(k) = eps2 omega_k / 2,
 *   omega_k = sqrt(k^2 + m2_i),  k = 2 pi |n| / L,
 * n the integer wavevector, zero at n = 0 and for |n| > cutoff.  Lattice
 * normalisation: unit white noise w filtered as IFFT(FFT(w) sqrt(N^3 P/L^3)),
 * so <F^2> = sum_k P(k) / L^3.  White noise: Philox4x32-10 (Salmon et al.,
 * SC'11), counter (i mod 2^32, i div 2^32, j, 0) for site i (x fastest) of
 * array j = 0..3 (F1, F2, U1, U2), key (seed mod 2^32, seed div 2^32); the
 * output words x0..x3 give U1 = (x0 2^21 + x1 div 2^11 + 1) 2^-53,
 * U2 = (x2 2^21 + x3 div 2^11 + 1) 2^-53 and the normal
 * sqrt(-2 ln U1) cos(2 pi U2).  FP64 throughout. */
typedef struct lf_vacuum {
    double f0[2];     /* homogeneous program-unit fields f1, f2 */
    double u0[2];     /* homogeneous rescaled velocities u1, u2 */
    double m2[2];     /* m_i^2 of each field's omega_k; m2_i + (2 pi / L)^2 > 0 */
    double eps2;      /* amplitude^2 of the spectra, >= 0 */
    double cutoff;    /* largest |n| kept; 0 = N/4 */
    uint64_t seed;    /* generator key */
} lf_vacuum;

/* Scratch for lf_vacuum_fields: the half spectrum of one array
 * (N^2 (N/2+1) complex doubles) plus the FFT work area.  Needs a device (the
 * FFT plans are made to size their work area).  The hipFFT plans of each
 * (device, N) are made once per process and kept; they hold small tables of
 * their own but no work area. */
int lf_vacuum_workspace_bytes(const lf_params *p, size_t *out_bytes);
/* Generate f1, f2, u1, u2 (FP64 device arrays of N^3, 256-byte aligned,
 * caller-owned) for the lattice of p on `stream`.  The large buffers come
 * from `workspace`.  Blocking; same seed, N and spectrum give bitwise the
 * same arrays.  Calls from several threads are safe (the shared plans are
 * bound to a stream and work area under a lock). */
int lf_vacuum_fields(const lf_params *p, const lf_vacuum *v, void *stream, void *workspace,
                     size_t ws_bytes, double *f1, double *f2, double *u1, double *u2);
/* Scratch for lf_init_vacuum: four FP64 arrays of N^3 plus
 * lf_vacuum_workspace_bytes. */
int lf_init_vacuum_workspace_bytes(const lf_params *p, size_t *out_bytes);
/* Generate a vacuum state in `workspace` and initialise the context from it
 * as lf_init_physical does (Friedmann a'_0 returned in *ad0_out).  Blocking;
 * the workspace may be reused after the call. */
int lf_init_vacuum(lf_ctx *ctx, const lf_vacuum *v, double a0, void *workspace, size_t ws_bytes,
                   double *ad0_out);

/* ---- power spectra (the FFT diagnostics named as the next step in Sec. IV)
 * Shell average of the discrete Fourier power of one synchronised field
 * g = f1, f2, v1 or v2 (which = 0..3) at time k:
 *   G_n = sum_x g(x) exp(-2 pi i n.x/N),  shell s = rint(|n|),
 *   count[s] = number of lattice modes with rint(|n|) = s,
 *   power[s] = (L^3/N^6) sum_{rint|n| = s} |G_n|^2 / count[s]  (0 if empty),
 * so that sum_s count[s] power[s] = (L^3/N^3) sum_x g^2, and a field with
 * power spectrum P(k) (normalised as <g^2> = sum_k P(k)/L^3) has
 * E power[s] = P on shell s.  FP64; bitwise reproducible. */

/* Shells that hold every mode of an N^3 lattice: rint(sqrt(3) (N div 2)) + 1
 * (returns the count, 0 for N < 1). */
int lf_spectrum_bins(int N);
/* Device scratch for lf_spectrum (one FP64 field, the half spectrum, the FFT
 * work area and per-plane partial sums).  Needs a device. */
int lf_spectrum_workspace_bytes(const lf_params *p, size_t *out_bytes);
/* power, count: HOST arrays of nbins doubles, 1 <= nbins <= lf_spectrum_bins(N)
 * (shells >= nbins are left out).  Blocking. */
int lf_spectrum(lf_ctx *ctx, int which, int nbins, double *power, double *count, void *workspace,
                size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* LF_H */
