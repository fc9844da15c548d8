// C-ABI layer of liblf: parameter validation, workspace layout, the step
// sequence and its HIP-graph capture.  Declarations and semantics: include/lf.h.
#include "lf_internal.h"
#include "../../include/lf.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

using namespace lf;

namespace {

thread_local std::string g_err;

// A named host range for profilers (rocTX; visible under rocprofv3
// --marker-trace) around each entry point that enqueues or waits for device
// work.  It costs a few host instructions when no profiler is attached.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(LF_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxLogK = 5;          // longest step graph: 32 steps
constexpr int kRedBlocks = 2048;     // grid of the grid-stride reductions

// Sweep variant and launch shape.  tile_y: 1 = plain one-site-per-thread
// sweep plus a separate reduction; 4, 8, 16 = LDS z-march with in-sweep
// reductions (rows per tile); 0 = automatic.  zchunk: planes per block.
struct Shape {
    int tile_x, tile_y, zchunk, rows;  // rows: partial-sum rows the step reduction writes
};

// Automatic launch shape.  Tiles of 128 x 8 from N = 256 (both stencils),
// narrower ones below.  The z-chunk is chosen so that the whole grid is
// resident at once (resident blocks = blocks per CU from the occupancy
// calculator x CU count): all tiles then march their chunks in lockstep and
// the halo rows a tile shares with its neighbours are still in L2 when they
// are needed (see auto_zchunk).  The resident count is only queried on a
// machine with a GPU; elsewhere (and for the workspace size) 3 blocks on 256
// CUs is assumed, which only changes the partial-sum row count.
// 7 or 27 (lf_params.stencil 0 means 7).
int stencil_of(const lf_params *p) { return p->stencil == 27 ? 27 : 7; }

int cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    (void)hipGetLastError();
    return cus > 0 ? cus : 256;
}

int resident_blocks(const lf_params *p, int tile_x, int tile_y)
{
    int per_cu = sweep_lds_blocks_per_cu(stencil_of(p), p->dtype, tile_x, tile_y, p->beta);
    (void)hipGetLastError();
    if (per_cu <= 0) per_cu = 3;
    return per_cu * cu_count();
}

// Automatic z-chunk of an LDS sweep over nz planes of N x N (N = p->N).
// The whole grid resident at once (tiles march in lockstep and find their
// neighbours' halo lines in L2).  The FP32 sweeps with 128-wide tiles do best
// with two blocks per CU: a smaller L2 working set per XCD and long chunks
// (7 points at 512^3: 256 planes, fetch 1.03x the algorithmic reads against
// 1.16x with three blocks per CU and 64 planes; 256^3: 32 planes; 27 points:
// 6% faster at 512^3 and 11% at 256^3 than 64-wide tiles filling the CUs).
// The other sweeps fill the CUs and keep chunks of at most 64 planes.
int auto_zchunk(const lf_params *p, int tile_x, int tile_y, int nz)
{
    const int N = p->N;
    const bool two_per_cu = p->dtype == LF_F32 && tile_x == 128;
    const int per_slab = ((N + tile_x - 1) / tile_x) * ((N + tile_y - 1) / tile_y);
    const int res = resident_blocks(p, tile_x, tile_y);
    const int target = two_per_cu && 2 * cu_count() < res ? 2 * cu_count() : res;
    int nzc = target / per_slab;
    nzc = nzc < 1 ? 1 : nzc;
    int dz = (nz + nzc - 1) / nzc;
    const int dz_max = two_per_cu ? nz : 64;
    dz = dz < 8 ? 8 : (dz > dz_max ? dz_max : dz);
    return dz < nz ? dz : nz;
}

Shape shape_of(const lf_params *p)
{
    Shape sh{};
    const int N = p->N;
    if (p->tile_y) {
        sh.tile_y = p->tile_y;
        sh.tile_x = p->tile_x ? p->tile_x : 64;
    } else if (N >= 256) {
        sh.tile_x = 128;
        sh.tile_y = 8;
    } else {
        sh.tile_x = 64;
        sh.tile_y = N >= 96 ? 8 : 4;
    }
    if (sh.tile_y == 1) {
        sh.tile_x = 0;
        sh.zchunk = 0;
        sh.rows = kRedBlocks;
        return sh;
    }
    sh.zchunk = p->zchunk ? (p->zchunk < N ? p->zchunk : N) : auto_zchunk(p, sh.tile_x, sh.tile_y, N);
    sh.rows = sweep_lds_blocks(N, sh.tile_x, sh.tile_y, sh.zchunk);
    return sh;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t state[2][4];
    size_t part, mom, enp, enout, tot, P, S, C;
    size_t total;
};

size_t esize(int dtype) { return dtype == LF_F64 ? 8 : 4; }

Layout layout_of(const lf_params *p)
{
    Layout L{};
    const size_t n3 = (size_t)p->N * p->N * p->N;
    size_t off = 0;
    for (int b = 0; b < 2; ++b)
        for (int j = 0; j < 4; ++j) {
            L.state[b][j] = off;
            off = align_up(off + n3 * esize(p->dtype));
        }
    L.part = off; off = align_up(off + (size_t)shape_of(p).rows * kNPart * sizeof(double));
    L.mom = off; off = align_up(off + (size_t)kRedBlocks * kNMom * sizeof(double));
    L.enp = off; off = align_up(off + (size_t)kRedBlocks * kNEn * sizeof(double));
    L.enout = off; off = align_up(off + 16 * sizeof(double));
    L.tot = off; off = align_up(off + 8 * sizeof(double));
    L.P = off; off = align_up(off + sizeof(DevParams));
    L.S = off; off = align_up(off + sizeof(DevScalars));
    L.C = off; off = align_up(off + sizeof(CoefPair));
    L.total = off;
    return L;
}

int validate(const lf_params *p)
{
    if (!p) return fail(LF_EINVAL, "params is NULL");
    if (p->N < 4 || p->N > 2048) return fail(LF_EINVAL, "N=%d out of range [4, 2048]", p->N);
    if (p->dtype != LF_F32 && p->dtype != LF_F64) return fail(LF_EINVAL, "dtype=%d", p->dtype);
    if (!(p->L > 0.0) || !isfinite(p->L)) return fail(LF_EINVAL, "L must be finite and > 0");
    if (!(p->dt > 0.0) || !isfinite(p->dt)) return fail(LF_EINVAL, "dt must be finite and > 0");
    if (p->beta < 2 || p->beta > kMaxBeta) return fail(LF_EINVAL, "beta=%d out of range [2, 6]", p->beta);
    if (p->flags != 0) return fail(LF_EINVAL, "flags must be 0");
    if (!isfinite(p->c1) || !isfinite(p->G) || !isfinite(p->r) || !isfinite(p->s))
        return fail(LF_EINVAL, "non-finite model parameter");
    if (fabs(p->s - 2.0 * p->r + 3.0) > 1e-12)
        return fail(LF_EINVAL, "rescaling exponents violate s - 2r + 3 = 0 (r=%g, s=%g)", p->r, p->s);
    if (!(p->kappa2 >= 0.0) || !isfinite(p->kappa2)) return fail(LF_EINVAL, "kappa2 must be >= 0");
    if (p->tile_y != 0 && p->tile_y != 1 && p->tile_y != 4 && p->tile_y != 8 && p->tile_y != 16)
        return fail(LF_EINVAL, "tile_y=%d: must be 0 (auto), 1 (plain), 4, 8 or 16", p->tile_y);
    if (p->zchunk < 0 || p->zchunk > 4096) return fail(LF_EINVAL, "zchunk=%d out of range", p->zchunk);
    if (p->tile_x != 0 && p->tile_x != 32 && p->tile_x != 64 && p->tile_x != 128)
        return fail(LF_EINVAL, "tile_x=%d: must be 0 (auto), 32, 64 or 128", p->tile_x);
    if (p->tile_x == 128 && p->tile_y != 4 && p->tile_y != 8)
        return fail(LF_EINVAL, "tile_x=128 needs tile_y 4 or 8");
    if (p->tile_x == 32 && ((p->tile_y != 8 && p->tile_y != 16) || p->stencil == 27))
        return fail(LF_EINVAL, "tile_x=32 needs tile_y 8 or 16 and the 7-point stencil");
    if (p->stencil != 0 && p->stencil != 7 && p->stencil != 27)
        return fail(LF_EINVAL, "stencil=%d: must be 0 or 7 (7-point) or 27 (27-point)", p->stencil);
    return LF_OK;
}

}  // namespace

struct lf_ctx {
    lf_params p;
    Layout L;
    Shape sh;
    hipStream_t stream;
    hipStream_t cap;
    hipStream_t aux;    // the adjoint backward's recompute stream (default priority)
    int device;         // current device at lf_create (the stream's device)
    char *ws;
    void *buf[2][4];
    int cur;
    double *part, *mom, *enp, *enout, *tot;
    DevParams *P;
    DevScalars *S;
    CoefPair *C;
    int inited;
    // g[j][p]: 2^j steps from buffer parity p, j = 0 .. logK (K = 2^logK
    // steps per long graph).  An n-step call launches n div K long graphs and
    // one graph per set bit of n mod K.
    hipGraphExec_t g[kMaxLogK + 1][2];
    int logK;
    int graphs_ready;   // every g[j][p] instantiated and uploaded
    int ens_member;     // stepped by an ensemble: its own graphs are never used
    hipEvent_t ev0, ev1;
    int timed;
    int64_t hstep;  // steps since lf_init / lf_set_state, as enqueued by the host
    // adjoint bookkeeping (lf_adj_forward / lf_adj_backward)
    char *adj_ws;
    int64_t adj_n;
    int adj_K, adj_ready;
    double adj_w[4];
};

namespace {

// One leapfrog step: FP64 scale-factor update from the pending partial sums,
// then the fused kick-drift sweep from the arrays `in` into `out`, which
// leaves the partial sums of the new fields for the next step.
void enqueue_step_io(lf_ctx *c, const void *const in[4], void *const out[4], hipStream_t st, hipEvent_t *ev,
                     DevScalars *tape = nullptr)
{
    if (ev) (void)hipEventRecord(ev[0], st);
    launch_aupdate(c->part, c->sh.rows, c->P, c->S, c->C, st, tape);
    if (ev) (void)hipEventRecord(ev[1], st);
    if (c->sh.tile_y == 1) {
        launch_sweep_plain(stencil_of(&c->p), c->p.dtype, c->p.beta, in, out, c->p.N, c->C, st);
        if (ev) (void)hipEventRecord(ev[2], st);
        launch_reduce(stencil_of(&c->p), c->p.dtype, out[0], out[1], c->p.N, c->S->bg_f, c->p.beta, c->part,
                      c->sh.rows, st);
    } else {
        launch_sweep_lds(stencil_of(&c->p), c->p.dtype, c->sh.tile_x, c->sh.tile_y, c->p.beta, in, out, c->p.N,
                         c->sh.zchunk, c->C, c->part, st);
        if (ev) (void)hipEventRecord(ev[2], st);
    }
    if (ev) (void)hipEventRecord(ev[3], st);
}

// The step from the context's buffer `cur` into `cur ^ 1`.
void enqueue_step(lf_ctx *c, int cur, hipStream_t st, hipEvent_t *ev)
{
    const void *in[4] = {c->buf[cur][0], c->buf[cur][1], c->buf[cur][2], c->buf[cur][3]};
    void *out[4] = {c->buf[cur ^ 1][0], c->buf[cur ^ 1][1], c->buf[cur ^ 1][2], c->buf[cur ^ 1][3]};
    enqueue_step_io(c, in, out, st, ev);
}

// Makes dev the current device for the scope and restores the caller's on
// exit.  Streams and events belong to the device current when they are
// created, so the ones a context creates after lf_create (capture streams,
// events, the adjoint's second stream) are created inside such a scope on
// the context's device, whatever device the caller has made current since.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess) prev = cur;
    }
    ~DeviceScope()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceScope(const DeviceScope &) = delete;
    DeviceScope &operator=(const DeviceScope &) = delete;
};

int ensure_events(int dev, hipEvent_t *ev0, hipEvent_t *ev1)
{
    if (*ev0 && *ev1) return LF_OK;
    DeviceScope scope(dev);
    if (!*ev0) HIPCHK(hipEventCreate(ev0));
    if (!*ev1) HIPCHK(hipEventCreate(ev1));
    return LF_OK;
}

int capture(lf_ctx *c, int nsteps, int start, hipGraphExec_t *exec)
{
    DeviceScope scope(c->device);
    if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int cur = start;
    for (int k = 0; k < nsteps; ++k) {
        enqueue_step(c, cur, c->cap, nullptr);
        cur ^= 1;
    }
    hipGraph_t g = nullptr;
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    if (e1 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LF_EHIP, "kernel launch during capture: %s", hipGetErrorString(e1));
    }
    if (e2 != hipSuccess) return fail(LF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return fail(LF_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
    return LF_OK;
}

// The graph of 2^j steps from parity p, captured on first use.
int ensure_graph(lf_ctx *c, int j, int p)
{
    if (c->g[j][p]) return LF_OK;
    return capture(c, 1 << j, p, &c->g[j][p]);
}

// Instantiate and upload every graph lf_step can launch, so that no call
// pays for a capture or for a graph's first upload.  Runs at lf_init /
// lf_set_state, once per context (the graphs depend only on the buffers).
int prepare_graphs(lf_ctx *c)
{
    if (c->graphs_ready || c->ens_member) return LF_OK;
    int rc;
    for (int j = 0; j <= c->logK; ++j)
        for (int p = 0; p < 2; ++p) {
            if ((rc = ensure_graph(c, j, p))) return rc;
            HIPCHK(hipGraphUpload(c->g[j][p], c->stream));
        }
    c->graphs_ready = 1;
    return LF_OK;
}

void fill_dev_params(const lf_params *p, DevParams *d)
{
    d->L = p->L;
    d->dx = p->L / p->N;
    d->dt = p->dt;
    d->c1 = p->c1;
    d->G = p->G;
    d->r = p->r;
    d->s = p->s;
    d->kappa2 = p->kappa2;
    d->p1 = -2.0 * p->s + (2.0 - p->beta) * p->r;
    d->p2 = -2.0 * p->s - 2.0 * p->r;
    d->N = p->N;
    d->beta = p->beta;
    d->N3 = (double)p->N * p->N * p->N;
    d->stencil = stencil_of(p);
    d->gw = d->stencil == 27 ? 1.0 / 30.0 : 1.0;
    d->pad = 0;
}

int check_ptr(const void *ptr, const char *name)
{
    if (!ptr) return fail(LF_EINVAL, "%s is NULL", name);
    if ((uintptr_t)ptr % kAlign) return fail(LF_EINVAL, "%s is not 256-byte aligned", name);
    return LF_OK;
}

// Allocation-free slab sweep (lf_slab_sweep_sums): the partial-sum rows of
// one call live in this array, which the library holds on every GPU it runs
// on until the process ends (kScratchRows rows of kNPart doubles, 2 MiB).
// Host code never passes the array's name to a kernel or a copy: on the host
// it is only a stand-in for the symbol.  Its device address is looked up once
// per device (scratch_rows) and that address is what the kernels receive.
constexpr int kScratchRows = 65536;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchRows * kNPart];

std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices];

// Device address of `scratch` on device dev (looked up with dev current on
// the first call for that device, then kept).
int scratch_rows(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(LF_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int prev = 0;
        HIPCHK(hipGetDevice(&prev));
        if (prev != dev) HIPCHK(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess || !ptr)
            return fail(LF_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return LF_OK;
}

}  // namespace

extern "C" {

int lf_abi_version(void) { return LF_ABI_VERSION; }

const char *lf_last_error(void) { return g_err.c_str(); }

int lf_workspace_bytes(const lf_params *p, size_t *out_bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!out_bytes) return fail(LF_EINVAL, "out_bytes is NULL");
    *out_bytes = layout_of(p).total;
    return LF_OK;
}

int lf_create(const lf_params *p, void *stream, void *workspace, size_t ws_bytes, lf_ctx **out)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!out) return fail(LF_EINVAL, "out is NULL");
    *out = nullptr;
    if ((rc = check_ptr(workspace, "workspace"))) return rc;
    Layout L = layout_of(p);
    if (ws_bytes < L.total)
        return fail(LF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    lf_ctx *c = new (std::nothrow) lf_ctx();
    if (!c) return fail(LF_ENOMEM, "host allocation failed");
    c->p = *p;
    c->L = L;
    c->sh = shape_of(p);
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(LF_EHIP, "hipGetDevice failed");
    }
    c->ws = (char *)workspace;
    for (int b = 0; b < 2; ++b)
        for (int j = 0; j < 4; ++j) c->buf[b][j] = c->ws + L.state[b][j];
    c->part = (double *)(c->ws + L.part);
    c->mom = (double *)(c->ws + L.mom);
    c->enp = (double *)(c->ws + L.enp);
    c->enout = (double *)(c->ws + L.enout);
    c->tot = (double *)(c->ws + L.tot);
    c->P = (DevParams *)(c->ws + L.P);
    c->S = (DevScalars *)(c->ws + L.S);
    c->C = (CoefPair *)(c->ws + L.C);
    c->logK = (p->N >= 256) ? 3 : 5;
    hipError_t e;
    DevParams dp;
    fill_dev_params(p, &dp);
    e = hipMemcpyAsync(c->P, &dp, sizeof dp, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        lf_destroy(c);
        return fail(LF_EHIP, "uploading parameters: %s", hipGetErrorString(e));
    }
    *out = c;
    return LF_OK;
}

int lf_destroy(lf_ctx *c)
{
    if (!c) return LF_OK;
    for (int j = 0; j <= kMaxLogK; ++j)
        for (int b = 0; b < 2; ++b)
            if (c->g[j][b]) (void)hipGraphExecDestroy(c->g[j][b]);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return LF_OK;
}

static int init_common(lf_ctx *c, const void *f1, const void *f2, const void *v1, const void *v2,
                       int in_dtype, double a0, double ad0, int physical)
{
    TraceRange range_("lf_init");
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    int rc;
    if ((rc = check_ptr(f1, "f1")) || (rc = check_ptr(f2, "f2")) || (rc = check_ptr(v1, "v1")) ||
        (rc = check_ptr(v2, "v2")))
        return rc;
    if (in_dtype != LF_F32 && in_dtype != LF_F64) return fail(LF_EINVAL, "in_dtype=%d", in_dtype);
    if (!(a0 > 0.0) || !isfinite(a0)) return fail(LF_EINVAL, "a0 must be finite and > 0");
    if (!isfinite(ad0)) return fail(LF_EINVAL, "ad0 must be finite");
    const int N = c->p.N;
    launch_input_moments(stencil_of(&c->p), in_dtype, f1, f2, v1, v2, N, c->p.beta, c->mom, kRedBlocks, c->stream);
    launch_init_scalars(c->mom, kRedBlocks, c->P, c->S, physical, a0, ad0, c->stream);
    launch_init_fields(c->p.dtype, in_dtype, f1, f2, v1, v2, c->buf[0][0], c->buf[0][1],
                       c->buf[0][2], c->buf[0][3], N, c->P, c->S, c->stream);
    launch_reduce(stencil_of(&c->p), c->p.dtype, c->buf[0][0], c->buf[0][1], N, c->S->bg_f, c->p.beta, c->part,
                  c->sh.rows, c->stream);
    HIPCHK(hipGetLastError());
    c->cur = 0;
    c->inited = 1;
    c->timed = 0;
    c->hstep = 0;
    c->adj_ready = 0;
    return prepare_graphs(c);
}

int lf_init(lf_ctx *c, const void *f1, const void *f2, const void *v1, const void *v2, int in_dtype,
            double a0, double ad0)
{
    return init_common(c, f1, f2, v1, v2, in_dtype, a0, ad0, 0);
}

int lf_init_physical(lf_ctx *c, const void *f1, const void *f2, const void *u1, const void *u2,
                     int in_dtype, double a0, double *ad0_out)
{
    if (!ad0_out) return fail(LF_EINVAL, "ad0_out is NULL");
    int rc = init_common(c, f1, f2, u1, u2, in_dtype, a0, 0.0, 1);
    if (rc) return rc;
    DevScalars hs;
    HIPCHK(hipMemcpyAsync(&hs, c->S, sizeof hs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *ad0_out = hs.ad0;
    if (hs.status) return fail(LF_ENONFINITE, "non-finite initial state or Friedmann constraint");
    return LF_OK;
}

int lf_step(lf_ctx *c, int64_t n)
{
    TraceRange range_("lf_step");
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    if (n < 0) return fail(LF_EINVAL, "n=%lld < 0", (long long)n);
    if (!c->inited) return fail(LF_ESTATE, "lf_step before lf_init");
    if (n == 0) return LF_OK;
    const int64_t n0 = n, K = (int64_t)1 << c->logK;
    int rc;
    // every graph this call launches exists before the first event
    if (n >= K && (rc = ensure_graph(c, c->logK, c->cur))) return rc;
    for (int j = c->logK - 1, p = c->cur; j >= 0; --j)
        if (n % K & ((int64_t)1 << j)) {
            if ((rc = ensure_graph(c, j, p))) return rc;
            if (j == 0) p ^= 1;
        }
    if ((rc = ensure_events(c->device, &c->ev0, &c->ev1))) return rc;
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    for (; n >= K; n -= K) HIPCHK(hipGraphLaunch(c->g[c->logK][c->cur], c->stream));
    for (int j = c->logK - 1; j >= 0; --j)
        if (n & ((int64_t)1 << j)) {
            HIPCHK(hipGraphLaunch(c->g[j][c->cur], c->stream));
            if (j == 0) c->cur ^= 1;  // an odd step count swaps the buffers
        }
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    c->timed = 1;
    c->hstep += n0;
    return LF_OK;
}

int lf_last_step_ms(lf_ctx *c, double *ms)
{
    if (!c || !ms) return fail(LF_EINVAL, "NULL argument");
    *ms = 0.0;
    if (!c->timed) return LF_OK;
    HIPCHK(hipEventSynchronize(c->ev1));
    float f = 0.0f;
    HIPCHK(hipEventElapsedTime(&f, c->ev0, c->ev1));
    *ms = f;
    return LF_OK;
}

int lf_energies(lf_ctx *c, lf_report *out)
{
    TraceRange range_("lf_energies");
    if (!c || !out) return fail(LF_EINVAL, "NULL argument");
    if (!c->inited) return fail(LF_ESTATE, "lf_energies before lf_init");
    const void *s4[4] = {c->buf[c->cur][0], c->buf[c->cur][1], c->buf[c->cur][2], c->buf[c->cur][3]};
    launch_energy(stencil_of(&c->p), c->p.dtype, s4, c->p.N, c->P, c->S, c->enp, kRedBlocks, c->enout, c->stream);
    HIPCHK(hipGetLastError());
    double h[12];
    HIPCHK(hipMemcpyAsync(h, c->enout, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    memset(out, 0, sizeof *out);
    out->step = (int64_t)h[0];
    out->a = h[1];
    out->ad = h[2];
    out->hubble = h[3];
    out->K[0] = h[4];
    out->K[1] = h[5];
    out->Gr[0] = h[6];
    out->Gr[1] = h[7];
    out->P = h[8];
    out->rho = h[9];
    out->R = h[10];
    out->status = (uint32_t)h[11];
    if (out->status) return fail(LF_ENONFINITE, "non-finite value reached the volume averages");
    return LF_OK;
}

int lf_rho_p(lf_ctx *c, void *rho, void *p, int out_dtype, double *avg)
{
    TraceRange range_("lf_rho_p");
    if (!c || !avg) return fail(LF_EINVAL, "NULL argument");
    if (!c->inited) return fail(LF_ESTATE, "lf_rho_p before lf_init");
    if (out_dtype != LF_F32 && out_dtype != LF_F64) return fail(LF_EINVAL, "out_dtype=%d", out_dtype);
    if ((rho && (uintptr_t)rho % kAlign) || (p && (uintptr_t)p % kAlign))
        return fail(LF_EINVAL, "output arrays must be 256-byte aligned");
    const void *s4[4] = {c->buf[c->cur][0], c->buf[c->cur][1], c->buf[c->cur][2], c->buf[c->cur][3]};
    // the energy partial rows (kRedBlocks x kNEn doubles) hold the 2 sums here
    launch_rho_p(stencil_of(&c->p), c->p.dtype, out_dtype, s4, rho, p, c->p.N, c->P, c->S, c->enp, kRedBlocks, c->enout, c->stream);
    HIPCHK(hipGetLastError());
    double h[3];
    HIPCHK(hipMemcpyAsync(h, c->enout, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < 3; ++i) avg[i] = h[i];
    return LF_OK;
}

int lf_get_fields(lf_ctx *c, void *f1, void *f2, void *v1, void *v2, int out_dtype, int synchronized)
{
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    if (!c->inited) return fail(LF_ESTATE, "lf_get_fields before lf_init");
    if (out_dtype != LF_F32 && out_dtype != LF_F64) return fail(LF_EINVAL, "out_dtype=%d", out_dtype);
    void *o[4] = {f1, f2, v1, v2};
    for (int j = 0; j < 4; ++j)
        if (o[j] && (uintptr_t)o[j] % kAlign) return fail(LF_EINVAL, "output %d not 256-byte aligned", j);
    const void *s4[4] = {c->buf[c->cur][0], c->buf[c->cur][1], c->buf[c->cur][2], c->buf[c->cur][3]};
    launch_get_fields(c->p.dtype, out_dtype, s4, o, c->p.N, c->P, c->S, synchronized ? 1 : 0, c->stream);
    HIPCHK(hipGetLastError());
    return LF_OK;
}

int lf_get_state(lf_ctx *c, void *d1, void *d2, void *e1, void *e2, lf_scalars *s)
{
    if (!c || !s) return fail(LF_EINVAL, "NULL argument");
    if (!c->inited) return fail(LF_ESTATE, "lf_get_state before lf_init");
    void *o[4] = {d1, d2, e1, e2};
    int rc;
    for (int j = 0; j < 4; ++j)
        if ((rc = check_ptr(o[j], "state array"))) return rc;
    const size_t bytes = (size_t)c->p.N * c->p.N * c->p.N * esize(c->p.dtype);
    for (int j = 0; j < 4; ++j)
        HIPCHK(hipMemcpyAsync(o[j], c->buf[c->cur][j], bytes, hipMemcpyDeviceToDevice, c->stream));
    launch_sum_partials(c->part, c->sh.rows, kNPart, c->tot, c->stream);
    HIPCHK(hipGetLastError());
    DevScalars hs;
    double tot[kNPart];
    HIPCHK(hipMemcpyAsync(&hs, c->S, sizeof hs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(tot, c->tot, sizeof tot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    memset(s, 0, sizeof *s);
    s->step = hs.step;
    s->a_half = hs.a_half;
    s->ad = hs.ad;
    for (int i = 0; i < 2; ++i) {
        s->bg_f[i] = hs.bg_f[i];
        s->bg_v[i] = hs.bg_v[i];
    }
    for (int i = 0; i < kNPart; ++i) s->pend[i] = tot[i];
    s->status = hs.status;
    return LF_OK;
}

int lf_set_state(lf_ctx *c, const void *d1, const void *d2, const void *e1, const void *e2,
                 const lf_scalars *s)
{
    if (!c || !s) return fail(LF_EINVAL, "NULL argument");
    const void *in[4] = {d1, d2, e1, e2};
    int rc;
    for (int j = 0; j < 4; ++j)
        if ((rc = check_ptr(in[j], "state array"))) return rc;
    if (!(s->a_half > 0.0)) return fail(LF_EINVAL, "a_half must be > 0");
    const size_t bytes = (size_t)c->p.N * c->p.N * c->p.N * esize(c->p.dtype);
    for (int j = 0; j < 4; ++j)
        HIPCHK(hipMemcpyAsync(c->buf[0][j], in[j], bytes, hipMemcpyDeviceToDevice, c->stream));
    DevScalars hs;
    memset(&hs, 0, sizeof hs);
    hs.a_half = s->a_half;
    hs.ad = s->ad;
    for (int i = 0; i < 2; ++i) {
        hs.bg_f[i] = s->bg_f[i];
        hs.bg_v[i] = s->bg_v[i];
    }
    for (int i = 0; i < kNPart; ++i) hs.pend[i] = s->pend[i];
    hs.step = s->step;
    hs.status = s->status;
    double tot[8] = {0};
    for (int i = 0; i < kNPart; ++i) tot[i] = s->pend[i];
    HIPCHK(hipMemcpyAsync(c->S, &hs, sizeof hs, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->tot, tot, sizeof tot, hipMemcpyHostToDevice, c->stream));
    launch_set_pending(c->part, c->sh.rows, c->tot, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->cur = 0;
    c->inited = 1;
    c->hstep = s->step;
    c->adj_ready = 0;
    return prepare_graphs(c);
}

int lf_set_coupling(lf_ctx *c, double G)
{
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    if (!isfinite(G)) return fail(LF_EINVAL, "G must be finite");
    c->p.G = G;
    DevParams dp;
    fill_dev_params(&c->p, &dp);
    HIPCHK(hipMemcpyAsync(c->P, &dp, sizeof dp, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LF_OK;
}

int lf_stream_copy(const float *a0, const float *a1, const float *a2, const float *a3, float *b0, float *b1,
                   float *b2, float *b3, int64_t n, void *stream)
{
    if (n < 0 || n % 4) return fail(LF_EINVAL, "n=%lld: must be >= 0 and a multiple of 4", (long long)n);
    if (n == 0) return LF_OK;
    const float *a[4] = {a0, a1, a2, a3};
    float *b[4] = {b0, b1, b2, b3};
    const char *an[4] = {"a0", "a1", "a2", "a3"}, *bn[4] = {"b0", "b1", "b2", "b3"};
    int rc;
    for (int j = 0; j < 4; ++j)
        if ((rc = check_ptr(a[j], an[j])) || (rc = check_ptr(b[j], bn[j]))) return rc;
    launch_stream_copy(a, b, n, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return LF_OK;
}

// z-slab sweep: launch shape (the context's tiles, z-chunk zchunk or
// automatic over nz planes) after the argument checks common to both calls.
static int slab_shape(const lf_ctx *c, int nz, int zchunk, int *zeff, int64_t *rows)
{
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    if (nz < 1 || nz > c->p.N) return fail(LF_EINVAL, "nz=%d: must be in [1, N=%d]", nz, c->p.N);
    if (zchunk < 0) return fail(LF_EINVAL, "zchunk=%d: must be >= 0 (0 = automatic)", zchunk);
    if (c->sh.tile_y == 1)
        return fail(LF_EINVAL, "the slab sweep needs an LDS launch shape (tile_y 4, 8 or 16), not tile_y=1");
    const int z = zchunk ? (zchunk < nz ? zchunk : nz) : auto_zchunk(&c->p, c->sh.tile_x, c->sh.tile_y, nz);
    *zeff = z;
    *rows = sweep_io_blocks(c->p.N, nz, c->sh.tile_x, c->sh.tile_y, z);
    return LF_OK;
}

int lf_slab_rows(const lf_ctx *c, int nz, int zchunk, int64_t *rows)
{
    if (!rows) return fail(LF_EINVAL, "rows is NULL");
    int z;
    return slab_shape(c, nz, zchunk, &z, rows);
}

static int slab_sweep_impl(lf_ctx *c, int nz, int zchunk, const void *const in[4], const void *const lo[4],
                           const void *const hi[2], void *const out[4], double *partials, int64_t partial_rows)
{
    int z;
    int64_t rows;
    int rc = slab_shape(c, nz, zchunk, &z, &rows);
    if (rc) return rc;
    if (!in || !lo || !hi || !out) return fail(LF_EINVAL, "NULL pointer array");
    if (!c->inited || c->hstep < 1)
        return fail(LF_ESTATE, "lf_slab_sweep reuses the coefficients of the context's last step: "
                               "take a step after lf_init / lf_set_state first");
    if (!partials) return fail(LF_EINVAL, "partials is NULL");
    if (partial_rows < rows)
        return fail(LF_EINVAL, "partials holds %lld rows, the sweep writes %lld", (long long)partial_rows,
                    (long long)rows);
    const size_t es = esize(c->p.dtype), plane = (size_t)c->p.N * c->p.N * es;
    // byte ranges: slab arrays nz planes, lower halo 2 planes (d) or 1 (e),
    // upper halo 1 plane (d)
    struct Range { const char *p; size_t n; const char *name; };
    const char *names[14] = {"in[0]", "in[1]", "in[2]", "in[3]", "lo[0]", "lo[1]", "lo[2]", "lo[3]",
                             "hi[0]", "hi[1]", "out[0]", "out[1]", "out[2]", "out[3]"};
    Range r[14];
    for (int i = 0; i < 4; ++i) {
        r[i] = {(const char *)in[i], nz * plane, names[i]};
        r[4 + i] = {(const char *)lo[i], (i < 2 ? 2 : 1) * plane, names[4 + i]};
        r[10 + i] = {(const char *)out[i], nz * plane, names[10 + i]};
    }
    for (int i = 0; i < 2; ++i) r[8 + i] = {(const char *)hi[i], plane, names[8 + i]};
    for (int i = 0; i < 14; ++i) {
        if (!r[i].p) return fail(LF_EINVAL, "%s is NULL", r[i].name);
        if ((uintptr_t)r[i].p % es) return fail(LF_EINVAL, "%s is not aligned to its element size", r[i].name);
    }
    // the outputs are written while neighbouring planes are still read: no
    // output may overlap an input, a halo plane or another output
    for (int i = 10; i < 14; ++i)
        for (int j = 0; j < 14; ++j) {
            const uintptr_t a = (uintptr_t)r[i].p, b = (uintptr_t)r[j].p;
            if (j != i && a < b + r[j].n && b < a + r[i].n)
                return fail(LF_EINVAL, "%s overlaps %s", r[i].name, r[j].name);
        }
    SweepIO io{};
    for (int i = 0; i < 4; ++i) {
        io.in[i] = in[i];
        io.out[i] = out[i];
    }
    // halo bases: the sweep addresses plane z < 0 of input i at lo + (z + 2)
    // planes and plane z >= nz at hi + (z - nz) planes.  e's lower halo holds
    // plane -1 only, so its base sits one plane below (plane -2 of e is never
    // read); e is never read above the slab
    io.lo[0] = lo[0];
    io.lo[1] = lo[1];
    io.lo[2] = (const char *)lo[2] - plane;
    io.lo[3] = (const char *)lo[3] - plane;
    io.hi[0] = hi[0];
    io.hi[1] = hi[1];
    io.hi[2] = in[2];
    io.hi[3] = in[3];
    io.nz = nz;
    launch_sweep_slab(stencil_of(&c->p), c->p.dtype, c->sh.tile_x, c->sh.tile_y, c->p.beta, io, c->p.N, z,
                      c->C, partials, c->stream);
    HIPCHK(hipGetLastError());
    return LF_OK;
}

int lf_slab_sweep(lf_ctx *c, int nz, int zchunk, const void *const in[4], const void *const lo[4],
                  const void *const hi[2], void *const out[4], double *partials, int64_t partial_rows)
{
    TraceRange range_("lf_slab_sweep");
    return slab_sweep_impl(c, nz, zchunk, in, lo, hi, out, partials, partial_rows);
}

int lf_slab_sweep_sums(lf_ctx *c, int nz, int zchunk, const void *const in[4], const void *const lo[4],
                       const void *const hi[2], void *const out[4], double *sums)
{
    int z;
    int64_t rows;
    int rc = slab_shape(c, nz, zchunk, &z, &rows);
    if (rc) return rc;
    if (!sums) return fail(LF_EINVAL, "sums is NULL");
    if ((uintptr_t)sums % sizeof(double)) return fail(LF_EINVAL, "sums is not 8-byte aligned");
    if (rows > kScratchRows)
        return fail(LF_EINVAL,
                    "the sweep writes %lld partial rows, the library's static scratch holds %d: use a larger "
                    "zchunk, or lf_slab_sweep with a caller buffer",
                    (long long)rows, kScratchRows);
    double *rows_dev = nullptr;
    if ((rc = scratch_rows(c->device, &rows_dev))) return rc;
    if ((rc = slab_sweep_impl(c, nz, zchunk, in, lo, hi, out, rows_dev, kScratchRows))) return rc;
    // every row the sweep's blocks write is read, in the fixed order of the
    // scale-factor kernel's stage 2; rows beyond them are not read
    launch_sum_partials(rows_dev, (int)rows, kNPart, sums, c->stream);
    HIPCHK(hipGetLastError());
    return LF_OK;
}

int lf_time_kernels(lf_ctx *c, int64_t n, double *ms, int n_out)
{
    if (!c || !ms) return fail(LF_EINVAL, "NULL argument");
    if (n < 1 || n_out < 1) return fail(LF_EINVAL, "n and n_out must be >= 1");
    if (!c->inited) return fail(LF_ESTATE, "lf_time_kernels before lf_init");
    DeviceScope scope(c->device);
    hipEvent_t ev[4] = {};
    int rc = LF_OK;
    for (int i = 0; i < 4 && rc == LF_OK; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) rc = fail(LF_EHIP, "hipEventCreate failed");
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < n && rc == LF_OK; ++k) {
        enqueue_step(c, c->cur, c->stream, ev);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
        float t;
        for (int j = 0; j < 3 && e == hipSuccess; ++j) {
            e = hipEventElapsedTime(&t, ev[j], ev[j + 1]);
            acc[j] += t;
        }
        if (e != hipSuccess) rc = fail(LF_EHIP, "timing step: %s", hipGetErrorString(e));
        c->cur ^= 1;
        c->hstep += 1;
    }
    for (int i = 0; i < 4; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (rc) return rc;
    for (int j = 0; j < n_out; ++j) ms[j] = (j < 3) ? acc[j] / (double)n : 0.0;
    return LF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- adjoint

namespace {

struct AdjLayout {
    int64_t nck;            // checkpoint slots (state at steps 0, K, 2K, ...)
    size_t slot_bytes;      // one checkpoint: 4 arrays + scalars + pending sums
    size_t arr_bytes;       // one lattice array of the context dtype
    size_t ck, seg, tape, lam, part, A, cf, w, total;
};

AdjLayout adj_layout(const lf_params *p, int64_t n, int K)
{
    AdjLayout L{};
    const size_t n3 = (size_t)p->N * p->N * p->N;
    L.arr_bytes = align_up(n3 * esize(p->dtype));
    L.nck = (n + K - 1) / K;
    L.slot_bytes = 4 * L.arr_bytes + align_up(sizeof(DevScalars)) + align_up(8 * sizeof(double));
    size_t off = 0;
    L.ck = off; off += (size_t)L.nck * L.slot_bytes;
    // two segment buffers and tapes: the backward pass recomputes segment
    // s - 1 into one while the reverse steps of segment s read the other
    L.seg = off; off += 2 * (size_t)K * 4 * L.arr_bytes;
    L.tape = off; off = align_up(off + 2 * (size_t)K * sizeof(DevScalars));
    L.lam = off; off += 8 * align_up(n3 * sizeof(double));
    L.part = off; off = align_up(off + (size_t)kRedBlocks * kNAdjPart * sizeof(double));
    L.A = off; off = align_up(off + 8 * sizeof(double));
    L.cf = off; off = align_up(off + 8 * sizeof(double));
    L.w = off; off = align_up(off + 8 * sizeof(double));
    L.total = off;
    return L;
}

int save_slot(lf_ctx *c, char *slot, const AdjLayout &L)
{
    const size_t bytes = (size_t)c->p.N * c->p.N * c->p.N * esize(c->p.dtype);
    for (int j = 0; j < 4; ++j)
        HIPCHK(hipMemcpyAsync(slot + j * L.arr_bytes, c->buf[c->cur][j], bytes, hipMemcpyDeviceToDevice, c->stream));
    char *sc = slot + 4 * L.arr_bytes;
    HIPCHK(hipMemcpyAsync(sc, c->S, sizeof(DevScalars), hipMemcpyDeviceToDevice, c->stream));
    launch_sum_partials(c->part, c->sh.rows, kNPart, (double *)(sc + align_up(sizeof(DevScalars))), c->stream);
    HIPCHK(hipGetLastError());
    return LF_OK;
}

// Checkpoint `slot` back: its four arrays into `arrays` (4 x arr_bytes apart),
// its scalars and pending sums into the context.
int restore_slot(lf_ctx *c, const char *slot, char *arrays, const AdjLayout &L, hipStream_t st)
{
    const size_t bytes = (size_t)c->p.N * c->p.N * c->p.N * esize(c->p.dtype);
    for (int j = 0; j < 4; ++j)
        HIPCHK(hipMemcpyAsync(arrays + j * L.arr_bytes, slot + j * L.arr_bytes, bytes, hipMemcpyDeviceToDevice,
                              st));
    const char *sc = slot + 4 * L.arr_bytes;
    HIPCHK(hipMemcpyAsync(c->S, sc, sizeof(DevScalars), hipMemcpyDeviceToDevice, st));
    launch_set_pending(c->part, c->sh.rows, (const double *)(sc + align_up(sizeof(DevScalars))), st);
    HIPCHK(hipGetLastError());
    return LF_OK;
}

// Recompute segment s into segment buffer b on stream st: buffer slot j
// receives the state before step j (the sweep of step j - 1 writes it there
// directly) and the tape entry j the scalars before step j; the segment's
// last step is not needed.  Uses the context's scalars, coefficients and
// partial rows (and nothing the reverse steps read).
int recompute_segment(lf_ctx *c, char *ws, const AdjLayout &L, int64_t s, int b, hipStream_t st)
{
    const int64_t n = c->adj_n;
    const int K = c->adj_K;
    char *seg = ws + L.seg + (size_t)b * K * 4 * L.arr_bytes;
    DevScalars *tape = (DevScalars *)(ws + L.tape) + (size_t)b * K;
    int rc;
    if ((rc = restore_slot(c, ws + L.ck + s * L.slot_bytes, seg, L, st))) return rc;
    const int64_t m = (n - s * K) < K ? (n - s * K) : K;
    for (int64_t j = 0; j < m; ++j) {
        if (j + 1 < m) {
            char *a = seg + (size_t)j * 4 * L.arr_bytes, *nb = a + 4 * L.arr_bytes;
            const void *in[4] = {a, a + L.arr_bytes, a + 2 * L.arr_bytes, a + 3 * L.arr_bytes};
            void *out[4] = {nb, nb + L.arr_bytes, nb + 2 * L.arr_bytes, nb + 3 * L.arr_bytes};
            enqueue_step_io(c, in, out, st, nullptr, tape + j);
        } else {
            HIPCHK(hipMemcpyAsync(tape + j, c->S, sizeof(DevScalars), hipMemcpyDeviceToDevice, st));
        }
    }
    HIPCHK(hipGetLastError());
    return LF_OK;
}

}  // namespace

extern "C" {

int lf_adj_workspace_bytes(const lf_params *p, int64_t n, int K, size_t *out_bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (n < 1 || K < 1) return fail(LF_EINVAL, "n and K must be >= 1");
    if (!out_bytes) return fail(LF_EINVAL, "out_bytes is NULL");
    *out_bytes = adj_layout(p, n, K).total;
    return LF_OK;
}

int lf_adj_forward(lf_ctx *c, int64_t n, int K, const double *w, void *adj_ws, size_t ws_bytes,
                   double *loss)
{
    TraceRange range_("lf_adj_forward");
    if (!c || !w || !loss) return fail(LF_EINVAL, "NULL argument");
    if (!c->inited || c->hstep != 0) return fail(LF_ESTATE, "lf_adj_forward needs a context just initialised");
    if (n < 1 || K < 1) return fail(LF_EINVAL, "n and K must be >= 1");
    int rc;
    if ((rc = check_ptr(adj_ws, "adjoint workspace"))) return rc;
    AdjLayout L = adj_layout(&c->p, n, K);
    if (ws_bytes < L.total) return fail(LF_ENOMEM, "adjoint workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    char *ws = (char *)adj_ws;
    c->adj_ws = ws;
    c->adj_n = n;
    c->adj_K = K;
    for (int i = 0; i < 4; ++i) c->adj_w[i] = w[i];
    for (int64_t s = 0; s < L.nck; ++s) {
        if ((rc = save_slot(c, ws + L.ck + s * L.slot_bytes, L))) return rc;
        const int64_t m = (n - s * K) < K ? (n - s * K) : K;
        if ((rc = lf_step(c, m))) return rc;
    }
    lf_report rep;
    if ((rc = lf_energies(c, &rep))) return rc;
    *loss = w[0] * rep.K[0] + w[1] * rep.K[1] + w[2] * rep.Gr[0] + w[3] * rep.Gr[1];
    c->adj_ready = 1;
    return LF_OK;
}

int lf_adj_backward(lf_ctx *c, double dL, double *dL_dG, void *g_f1, void *g_f2, void *g_v1, void *g_v2,
                    double *dL_da0, double *dL_dad0)
{
    TraceRange range_("lf_adj_backward");
    if (!c || !dL_dG || !dL_da0 || !dL_dad0) return fail(LF_EINVAL, "NULL argument");
    if (!c->adj_ready) return fail(LF_ESTATE, "lf_adj_backward needs a preceding lf_adj_forward");
    void *go[4] = {g_f1, g_f2, g_v1, g_v2};
    int rc;
    for (int j = 0; j < 4; ++j)
        if ((rc = check_ptr(go[j], "gradient array"))) return rc;
    const int64_t n = c->adj_n;
    const int K = c->adj_K;
    AdjLayout L = adj_layout(&c->p, n, K);
    char *ws = c->adj_ws;
    const size_t n3 = (size_t)c->p.N * c->p.N * c->p.N;
    const size_t lam_bytes = align_up(n3 * sizeof(double));
    double *lam[2][4];
    for (int b = 0; b < 2; ++b)
        for (int j = 0; j < 4; ++j) lam[b][j] = (double *)(ws + L.lam + (b * 4 + j) * lam_bytes);
    double *part = (double *)(ws + L.part), *A = (double *)(ws + L.A), *cf = (double *)(ws + L.cf);
    double *wd = (double *)(ws + L.w);
    double hw[8] = {0};
    for (int i = 0; i < 4; ++i) hw[i] = dL * c->adj_w[i];
    HIPCHK(hipMemcpyAsync(wd, hw, sizeof hw, hipMemcpyHostToDevice, c->stream));
    // seed: cotangent of the final state
    const void *s4[4] = {c->buf[c->cur][0], c->buf[c->cur][1], c->buf[c->cur][2], c->buf[c->cur][3]};
    launch_adj_seed(stencil_of(&c->p), c->p.dtype, s4, c->p.N, c->P, c->S, wd, lam[0], part, kRedBlocks, A, c->stream);
    HIPCHK(hipGetLastError());
    // The reverse steps of segment s run on the context's stream while the
    // recompute of segment s - 1 runs on the auxiliary stream, into the other
    // segment buffer.  Events: seg_ready[b] after a recompute into buffer b,
    // seg_free[b] after the reverse steps that read buffer b; the first
    // recompute waits for the seed, which reads the context's final state.
    DeviceScope scope(c->device);
    if (!c->aux) HIPCHK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    hipEvent_t ev[5] = {};
    for (int i = 0; i < 5 && rc == LF_OK; ++i)
        if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess)
            rc = fail(LF_EHIP, "hipEventCreateWithFlags failed");
    hipEvent_t seeded = ev[0], seg_ready[2] = {ev[1], ev[2]}, seg_free[2] = {ev[3], ev[4]};
    auto check = [&](hipError_t e, const char *what) {
        if (rc == LF_OK && e != hipSuccess) rc = fail(LF_EHIP, "%s: %s", what, hipGetErrorString(e));
    };
    if (rc == LF_OK) {
        check(hipEventRecord(seeded, c->stream), "hipEventRecord");
        check(hipStreamWaitEvent(c->aux, seeded, 0), "hipStreamWaitEvent");
    }
    int li = 0;
    const int64_t last = L.nck - 1;
    if (rc == LF_OK && (rc = recompute_segment(c, ws, L, last, (int)(last & 1), c->aux)) == LF_OK)
        check(hipEventRecord(seg_ready[last & 1], c->aux), "hipEventRecord");
    for (int64_t s = last; s >= 0 && rc == LF_OK; --s) {
        const int b = (int)(s & 1);
        // the next segment down goes into the other buffer once the reverse
        // steps of segment s + 1, which read it, are done
        if (s > 0) {
            if (s + 1 <= last) check(hipStreamWaitEvent(c->aux, seg_free[b ^ 1], 0), "hipStreamWaitEvent");
            if (rc == LF_OK && (rc = recompute_segment(c, ws, L, s - 1, b ^ 1, c->aux)) == LF_OK)
                check(hipEventRecord(seg_ready[b ^ 1], c->aux), "hipEventRecord");
        }
        check(hipStreamWaitEvent(c->stream, seg_ready[b], 0), "hipStreamWaitEvent");
        if (rc) break;
        // reverse steps; inside a segment the fields pass of step j also
        // forms the sums of step j - 1 (its stored state is at hand)
        const int64_t m = (n - s * K) < K ? (n - s * K) : K;
        const char *seg = ws + L.seg + (size_t)b * K * 4 * L.arr_bytes;
        const DevScalars *tape = (const DevScalars *)(ws + L.tape) + (size_t)b * K;
        for (int64_t j = m - 1; j >= 0; --j) {
            const char *src = seg + (size_t)j * 4 * L.arr_bytes;
            AdjStep a{};
            a.d1 = src;
            a.d2 = src + L.arr_bytes;
            a.tape = tape + j;
            a.lin = lam[li];
            a.lout = lam[li ^ 1];
            a.have_sums = j < m - 1;
            if (j > 0) {
                a.next_d1 = src - 4 * L.arr_bytes;
                a.next_d2 = src - 3 * L.arr_bytes;
                a.next_tape = tape + j - 1;
            }
            launch_adj_step(stencil_of(&c->p), c->p.dtype, a, c->p.N, c->p.beta, c->P, c->p.dt, part, kRedBlocks, A,
                            cf, c->stream);
            li ^= 1;
        }
        check(hipGetLastError(), "reverse step launch");
        check(hipEventRecord(seg_free[b], c->stream), "hipEventRecord");
    }
    if (c->aux) check(hipStreamSynchronize(c->aux), "hipStreamSynchronize");
    for (int i = 0; i < 5; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (rc) return rc;
    launch_adj_desync(c->p.N, c->p.dt, lam[li], A, c->stream);
    for (int j = 0; j < 4; ++j)
        HIPCHK(hipMemcpyAsync(go[j], lam[li][j], n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    double hA[4];
    HIPCHK(hipMemcpyAsync(hA, A, sizeof hA, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *dL_da0 = hA[0];
    *dL_dad0 = hA[1];
    *dL_dG = hA[2];
    c->adj_ready = 0;
    c->hstep = -1;  // the state is no longer the forward's: re-initialise before reuse
    return LF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- vacuum initial state

namespace {

int validate_vacuum(const lf_params *p, const lf_vacuum *v)
{
    if (!v) return fail(LF_EINVAL, "vacuum spec is NULL");
    const double kmin2 = (2.0 * M_PI / p->L) * (2.0 * M_PI / p->L);
    for (int i = 0; i < 2; ++i) {
        if (!isfinite(v->f0[i]) || !isfinite(v->u0[i]) || !isfinite(v->m2[i]))
            return fail(LF_EINVAL, "vacuum spec: non-finite homogeneous value or m2");
        if (!(v->m2[i] + kmin2 > 0.0))
            return fail(LF_EINVAL, "vacuum spec: m2[%d] = %g leaves omega_k imaginary", i, v->m2[i]);
    }
    if (!(v->eps2 >= 0.0) || !isfinite(v->eps2)) return fail(LF_EINVAL, "vacuum spec: eps2 must be >= 0");
    if (!(v->cutoff >= 0.0) || !isfinite(v->cutoff)) return fail(LF_EINVAL, "vacuum spec: cutoff must be >= 0");
    return LF_OK;
}

size_t vac_array_bytes(int N) { return align_up((size_t)N * N * N * sizeof(double)); }

}  // namespace

extern "C" {

int lf_vacuum_workspace_bytes(const lf_params *p, size_t *out_bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!out_bytes) return fail(LF_EINVAL, "out_bytes is NULL");
    char msg[256];
    if (vacuum_workspace(p->N, out_bytes, msg, sizeof msg)) return fail(LF_EHIP, "%s", msg);
    return LF_OK;
}

int lf_vacuum_fields(const lf_params *p, const lf_vacuum *v, void *stream, void *workspace, size_t ws_bytes,
                     double *f1, double *f2, double *u1, double *u2)
{
    int rc = validate(p);
    if (rc || (rc = validate_vacuum(p, v))) return rc;
    if ((rc = check_ptr(workspace, "workspace")) || (rc = check_ptr(f1, "f1")) || (rc = check_ptr(f2, "f2")) ||
        (rc = check_ptr(u1, "u1")) || (rc = check_ptr(u2, "u2")))
        return rc;
    double *const out[4] = {f1, f2, u1, u2};
    char msg[256];
    const int e = vacuum_generate(p->N, p->L, v, (hipStream_t)stream, workspace, ws_bytes, out, msg, sizeof msg);
    if (e) return fail(e == 2 ? LF_ENOMEM : LF_EHIP, "%s", msg);
    return LF_OK;
}

int lf_init_vacuum_workspace_bytes(const lf_params *p, size_t *out_bytes)
{
    int rc = lf_vacuum_workspace_bytes(p, out_bytes);
    if (rc) return rc;
    *out_bytes += 4 * vac_array_bytes(p->N);
    return LF_OK;
}

int lf_init_vacuum(lf_ctx *c, const lf_vacuum *v, double a0, void *workspace, size_t ws_bytes, double *ad0_out)
{
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    if (!ad0_out) return fail(LF_EINVAL, "ad0_out is NULL");
    int rc;
    if ((rc = check_ptr(workspace, "workspace"))) return rc;
    const size_t arr = vac_array_bytes(c->p.N);
    if (ws_bytes < 4 * arr) return fail(LF_ENOMEM, "workspace of %zu bytes is smaller than four arrays", ws_bytes);
    char *w = (char *)workspace;
    double *f[4] = {(double *)w, (double *)(w + arr), (double *)(w + 2 * arr), (double *)(w + 3 * arr)};
    if ((rc = lf_vacuum_fields(&c->p, v, (void *)c->stream, w + 4 * arr, ws_bytes - 4 * arr, f[0], f[1], f[2],
                               f[3])))
        return rc;
    return lf_init_physical(c, f[0], f[1], f[2], f[3], LF_F64, a0, ad0_out);
}

int lf_spectrum_bins(int N) { return N >= 1 ? spectrum_bins(N) : 0; }

int lf_spectrum_workspace_bytes(const lf_params *p, size_t *out_bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!out_bytes) return fail(LF_EINVAL, "out_bytes is NULL");
    char msg[256];
    size_t b = 0;
    if (spectrum_workspace_bytes(p->N, &b, msg, sizeof msg)) return fail(LF_EHIP, "%s", msg);
    *out_bytes = vac_array_bytes(p->N) + b;
    return LF_OK;
}

int lf_spectrum(lf_ctx *c, int which, int nbins, double *power, double *count, void *workspace, size_t ws_bytes)
{
    TraceRange range_("lf_spectrum");
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    if (which < 0 || which > 3) return fail(LF_EINVAL, "which=%d: 0..3 = f1, f2, v1, v2", which);
    const int nmax = spectrum_bins(c->p.N);
    if (nbins < 1 || nbins > nmax) return fail(LF_EINVAL, "nbins=%d out of range [1, %d]", nbins, nmax);
    if (!power || !count) return fail(LF_EINVAL, "power and count must be host arrays");
    int rc;
    if ((rc = check_ptr(workspace, "workspace"))) return rc;
    if (!c->inited) return fail(LF_ESTATE, "lf_spectrum before lf_init");
    const size_t arr = vac_array_bytes(c->p.N);
    if (ws_bytes < arr) return fail(LF_ENOMEM, "workspace of %zu bytes is smaller than one array", ws_bytes);
    // the synchronised deviation of field `which` and, in the scalar slot,
    // its homogeneous value (background at time k)
    double *dev = (double *)workspace;
    const int fld = which & 1, vel = which >> 1;
    const double h = 0.5 * c->p.dt;
    launch_sync_deviation(c->p.dtype, c->buf[c->cur][fld], c->buf[c->cur][2 + fld], dev, c->p.N, h, vel,
                          c->stream);
    HIPCHK(hipGetLastError());
    DevScalars hs;
    HIPCHK(hipMemcpyAsync(&hs, c->S, sizeof hs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const double bg = vel ? hs.bg_v[fld] : hs.bg_f[fld] - h * hs.bg_v[fld];
    HIPCHK(hipMemcpyAsync(c->tot, &bg, sizeof bg, hipMemcpyHostToDevice, c->stream));
    char msg[256];
    const int e = spectrum_compute(c->p.N, c->p.L, dev, c->tot, nbins, c->stream, (char *)workspace + arr,
                                   ws_bytes - arr, power, count, msg, sizeof msg);
    if (e) return fail(e == 2 ? LF_ENOMEM : LF_EHIP, "%s", msg);
    return LF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner

namespace {

struct TuneKey {
    char arch[64];
    int N, dtype, beta, stencil;
};

int current_arch(char *arch, size_t n)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LF_EHIP, "no HIP device for the autotuner");
    }
    snprintf(arch, n, "%s", prop.gcnArchName);
    for (char *c = arch; *c; ++c)
        if (*c == ':') { *c = 0; break; }
    return LF_OK;
}

// Cache: one JSON object per line,
// {"arch": "gfx950", "N": 512, "dtype": 0, "beta": 2, "stencil": 7, "tile_x": 128, "tile_y": 8,
//  "zchunk": 256, "ms": 0.87}
int cache_lookup(const char *path, const TuneKey &k, lf_params *best)
{
    if (!path) return 0;
    FILE *f = fopen(path, "r");
    if (!f) return 0;
    char line[512];
    int found = 0;
    while (fgets(line, sizeof line, f)) {
        char arch[64] = {0};
        int N, dt, beta, st, tx, ty, zc;
        double ms;
        if (sscanf(line, " {\"arch\": \"%63[^\"]\", \"N\": %d, \"dtype\": %d, \"beta\": %d, \"stencil\": %d, "
                         "\"tile_x\": %d, \"tile_y\": %d, \"zchunk\": %d, \"ms\": %lf",
                   arch, &N, &dt, &beta, &st, &tx, &ty, &zc, &ms) == 9 &&
            !strcmp(arch, k.arch) && N == k.N && dt == k.dtype && beta == k.beta && st == k.stencil) {
            best->tile_x = tx;
            best->tile_y = ty;
            best->zchunk = zc;
            found = 1;  // the last matching line wins
        }
    }
    fclose(f);
    return found;
}

void cache_append(const char *path, const TuneKey &k, const lf_params *b, double ms)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"arch\": \"%s\", \"N\": %d, \"dtype\": %d, \"beta\": %d, \"stencil\": %d, \"tile_x\": %d, "
               "\"tile_y\": %d, \"zchunk\": %d, \"ms\": %.6f}\n",
            k.arch, k.N, k.dtype, k.beta, k.stencil, b->tile_x, b->tile_y, b->zchunk, ms);
    fclose(f);
}

// Candidate launch shapes: the plain sweep, every LDS tile, and z-chunks from
// the resident-grid choice, fixed depths and fractions of N (up to 46).
int candidates(const lf_params *p, lf_params *out, int cap)
{
    int n = 0;
    lf_params q = *p;
    q.tile_x = 0; q.tile_y = 1; q.zchunk = 0;
    out[n++] = q;
    const int tiles[7][2] = {{64, 4}, {64, 8}, {64, 16}, {128, 4}, {128, 8}, {32, 8}, {32, 16}};
    const int ntiles = stencil_of(p) == 27 ? 5 : 7;  // 32-wide tiles: 7-point sweep only
    for (int t = 0; t < ntiles; ++t) {
        const int zs[9] = {0, 16, 32, 64, 128, p->N / 6, p->N / 4, p->N / 3, p->N / 2};
        int seen[9], ns = 0;
        for (int j = 0; j < 9; ++j) {
            q = *p;
            q.tile_x = tiles[t][0];
            q.tile_y = tiles[t][1];
            q.zchunk = zs[j];
            if (zs[j] != 0 && (zs[j] < 8 || zs[j] > p->N)) continue;
            const int eff = shape_of(&q).zchunk;
            int dup = 0;
            for (int i = 0; i < ns; ++i) dup |= seen[i] == eff;
            if (dup || n >= cap) continue;
            seen[ns++] = eff;
            q.zchunk = eff;
            out[n++] = q;
        }
    }
    return n;
}

}  // namespace

extern "C" {

int lf_autotune_workspace_bytes(const lf_params *p, size_t *out_bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!out_bytes) return fail(LF_EINVAL, "out_bytes is NULL");
    lf_params cand[64];
    const int n = candidates(p, cand, 64);
    size_t m = 0;
    for (int i = 0; i < n; ++i) {
        const size_t b = layout_of(&cand[i]).total;
        m = b > m ? b : m;
    }
    *out_bytes = m;
    return LF_OK;
}

int lf_autotune(const lf_params *p, void *stream, void *workspace, size_t ws_bytes, const char *cache_path,
                lf_params *best, double *best_ms)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!best) return fail(LF_EINVAL, "best is NULL");
    TuneKey k{};
    if ((rc = current_arch(k.arch, sizeof k.arch))) return rc;
    k.N = p->N;
    k.dtype = p->dtype;
    k.beta = p->beta;
    k.stencil = stencil_of(p);
    *best = *p;
    if (cache_lookup(cache_path, k, best)) {
        if (best_ms) *best_ms = -1.0;
        return validate(best);
    }
    size_t need = 0;
    if ((rc = lf_autotune_workspace_bytes(p, &need))) return rc;
    if ((rc = check_ptr(workspace, "workspace"))) return rc;
    if (ws_bytes < need) return fail(LF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    lf_params cand[64];
    const int n = candidates(p, cand, 64);
    double bms = 1e300;
    int bi = -1;
    const int steps = p->N >= 256 ? 10 : 40;
    for (int i = 0; i < n; ++i) {
        lf_ctx *c = nullptr;
        if ((rc = lf_create(&cand[i], stream, workspace, ws_bytes, &c))) return rc;
        void *s4[4] = {c->buf[0][0], c->buf[0][1], c->buf[0][2], c->buf[0][3]};
        launch_fill_synthetic(c->p.dtype, s4, c->p.N, c->S, c->stream);
        launch_reduce(stencil_of(&c->p), c->p.dtype, s4[0], s4[1], c->p.N, c->S->bg_f, c->p.beta, c->part,
                      c->sh.rows, c->stream);
        c->inited = 1;
        c->cur = 0;
        double ms = 0.0;
        rc = lf_step(c, 3);
        if (!rc) rc = lf_step(c, steps);
        if (!rc) rc = lf_last_step_ms(c, &ms);
        lf_destroy(c);
        if (rc) return rc;
        ms /= steps;
        if (ms < bms) {
            bms = ms;
            bi = i;
        }
    }
    *best = cand[bi];
    if (best_ms) *best_ms = bms;
    cache_append(cache_path, k, best, bms);
    return LF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- ensemble

struct lf_ens {
    int R;
    int dtype, beta, stencil, tile_x, tile_y;
    hipStream_t stream, cap;
    int device;          // current device at lf_ens_create (the stream's device)
    lf_ctx **sub;        // one context per realization, on slices of the workspace
    EnsEntry *tab;       // device table (workspace)
    int4 *items;         // device work list (workspace)
    int *queue;          // device work counter of the persistent sweep (workspace)
    int nitems, grid;
    int cur;
    hipGraphExec_t g2, g1[2];
    hipEvent_t ev0, ev1;
    int timed;
};

namespace {

struct EnsLayout {
    size_t *sub_off;  // R + 1 offsets
    size_t tab, items, total;
    int nitems;
};

// the sweep's work counters (8, 32 ints apart) and the 9 segment bounds
constexpr int kXcdCount = 8;
constexpr int kEnsQueueInts = kXcdCount * 32 + kXcdCount + 1;

int ens_tile_y(const lf_params *p0) { return p0->tile_y ? p0->tile_y : 8; }
int ens_tile_x(const lf_params *p0) { return p0->tile_x ? p0->tile_x : 64; }

// Parameters of realization r as its sub-context sees them: the ensemble's
// common tile, and unless given a z-chunk of half the lattice (at least 8
// planes): two chunks per tile column.  On gfx950 that beat 16-64-plane
// chunks for the mixed 64^3..160^3 ensemble by 5-8%, the fewer chunk-boundary
// planes outweighing the smaller work list.
// Default z-chunk of a realization: the whole lattice (one item per tile
// column) when the ensemble's tile columns fill between half and all of the
// resident grid, so that every item runs in a single round; otherwise half
// the lattice (at least 8 planes).
lf_params ens_sub_params(const lf_params *pr, const lf_params *p0, bool full_z)
{
    lf_params q = *pr;
    q.tile_x = ens_tile_x(p0);
    q.tile_y = ens_tile_y(p0);
    if (!q.zchunk) q.zchunk = full_z ? pr->N : (pr->N / 2 > 8 ? pr->N / 2 : (pr->N < 8 ? pr->N : 8));
    return q;
}

bool ens_full_z(int R, const lf_params *per)
{
    const int tx = ens_tile_x(&per[0]), ty = ens_tile_y(&per[0]);
    long long cols = 0;
    for (int r = 0; r < R; ++r) cols += (long long)((per[r].N + tx - 1) / tx) * ((per[r].N + ty - 1) / ty);
    const lf_params q0 = ens_sub_params(&per[0], &per[0], false);
    const long long grid = resident_blocks(&q0, tx, ty);
    return 2 * cols >= grid && cols <= grid;
}

int ens_validate(int R, const lf_params *per)
{
    if (R < 1 || R > 4096) return fail(LF_EINVAL, "R=%d out of range [1, 4096]", R);
    if (!per) return fail(LF_EINVAL, "per-realization params is NULL");
    for (int r = 0; r < R; ++r) {
        int rc = validate(&per[r]);
        if (rc) return rc;
        if (per[r].dtype != per[0].dtype || per[r].beta != per[0].beta ||
            stencil_of(&per[r]) != stencil_of(&per[0]))
            return fail(LF_EINVAL, "realization %d: dtype, beta and stencil must match realization 0", r);
        if (per[r].tile_y == 1) return fail(LF_EINVAL, "the ensemble needs an LDS sweep tile (tile_y != 1)");
    }
    const int ty = ens_tile_y(&per[0]), tx = ens_tile_x(&per[0]);
    if (ty == 1 || (tx == 128 && ty != 4 && ty != 8)) return fail(LF_EINVAL, "unsupported ensemble tile");
    return LF_OK;
}

size_t ens_layout(int R, const lf_params *per, size_t *sub_off, int *nitems)
{
    size_t off = 0;
    int items = 0;
    const bool full_z = ens_full_z(R, per);
    for (int r = 0; r < R; ++r) {
        lf_params q = ens_sub_params(&per[r], &per[0], full_z);
        sub_off[r] = off;
        off = align_up(off + layout_of(&q).total);
        Shape sh = shape_of(&q);
        items += sh.rows;
    }
    sub_off[R] = off;
    *nitems = items;
    return off;
}

}  // namespace

namespace {
int ens_prepare_graphs(lf_ens *e);
}

extern "C" {

int lf_ens_workspace_bytes(int R, const lf_params *per, size_t *out_bytes)
{
    int rc = ens_validate(R, per);
    if (rc) return rc;
    if (!out_bytes) return fail(LF_EINVAL, "out_bytes is NULL");
    size_t *so = new size_t[R + 1];
    int nitems = 0;
    size_t off = ens_layout(R, per, so, &nitems);
    delete[] so;
    off = align_up(off + (size_t)R * sizeof(EnsEntry));
    off = align_up(off + (size_t)nitems * sizeof(int4));
    off = align_up(off + kEnsQueueInts * sizeof(int));
    *out_bytes = off;
    return LF_OK;
}

int lf_ens_destroy(lf_ens *e)
{
    if (!e) return LF_OK;
    if (e->sub)
        for (int r = 0; r < e->R; ++r) lf_destroy(e->sub[r]);
    delete[] e->sub;
    if (e->g2) (void)hipGraphExecDestroy(e->g2);
    for (int b = 0; b < 2; ++b)
        if (e->g1[b]) (void)hipGraphExecDestroy(e->g1[b]);
    if (e->cap) (void)hipStreamDestroy(e->cap);
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    delete e;
    return LF_OK;
}

int lf_ens_create(int R, const lf_params *per, void *stream, void *workspace, size_t ws_bytes,
                  lf_ens **out)
{
    int rc = ens_validate(R, per);
    if (rc) return rc;
    if (!out) return fail(LF_EINVAL, "out is NULL");
    *out = nullptr;
    if ((rc = check_ptr(workspace, "workspace"))) return rc;
    size_t need = 0;
    if ((rc = lf_ens_workspace_bytes(R, per, &need))) return rc;
    if (ws_bytes < need) return fail(LF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    lf_ens *e = new (std::nothrow) lf_ens();
    if (!e) return fail(LF_ENOMEM, "host allocation failed");
    e->R = R;
    e->dtype = per[0].dtype;
    e->beta = per[0].beta;
    e->stencil = stencil_of(&per[0]);
    e->tile_x = ens_tile_x(&per[0]);
    e->tile_y = ens_tile_y(&per[0]);
    e->stream = (hipStream_t)stream;
    if (hipGetDevice(&e->device) != hipSuccess) {
        delete e;
        return fail(LF_EHIP, "hipGetDevice failed");
    }
    e->sub = new (std::nothrow) lf_ctx *[R]();
    size_t *so = new size_t[R + 1];
    int nitems = 0;
    size_t off = ens_layout(R, per, so, &nitems);
    char *ws = (char *)workspace;
    e->tab = (EnsEntry *)(ws + off);
    off = align_up(off + (size_t)R * sizeof(EnsEntry));
    e->items = (int4 *)(ws + off);
    off = align_up(off + (size_t)nitems * sizeof(int4));
    e->queue = (int *)(ws + off);
    e->nitems = nitems;
    EnsEntry *htab = new EnsEntry[R];
    int4 *hitems = new int4[nitems > 0 ? nitems : 1];
    int k = 0;
    const bool full_z = ens_full_z(R, per);
    for (int r = 0; r < R && rc == LF_OK; ++r) {
        lf_params q = ens_sub_params(&per[r], &per[0], full_z);
        rc = lf_create(&q, stream, ws + so[r], so[r + 1] - so[r], &e->sub[r]);
        if (rc) break;
        lf_ctx *c = e->sub[r];
        c->ens_member = 1;
        EnsEntry &t = htab[r];
        memset(&t, 0, sizeof t);
        for (int b = 0; b < 2; ++b)
            for (int j = 0; j < 4; ++j) t.buf[b][j] = c->buf[b][j];
        t.part = c->part;
        t.C = c->C;
        t.Cw = c->C;
        t.P = c->P;
        t.S = c->S;
        t.N = q.N;
        t.zchunk = c->sh.zchunk;
        t.ntx = (q.N + c->sh.tile_x - 1) / c->sh.tile_x;
        t.nty = (q.N + c->sh.tile_y - 1) / c->sh.tile_y;
        t.rows = c->sh.rows;
        for (int j = 0; j < c->sh.rows; ++j) hitems[k++] = make_int4(r, j, j, 0);
    }
    delete[] so;
    if (rc == LF_OK) {
        // Split the items into one segment per XCD: whole z-chunks of a
        // realization (all their tiles) go to one segment, assigned longest
        // first to the segment with the least work so far; inside a segment
        // the items with the most planes come first, a chunk's tiles in tile
        // order (each item keeps its partial row, so no order changes a sum).
        auto planes = [&](const int4 &it) {
            const EnsEntry &t = htab[it.x];
            const int z0 = it.y / (t.ntx * t.nty) * t.zchunk;
            return t.N - z0 < t.zchunk ? t.N - z0 : t.zchunk;
        };
        auto chunk_of = [&](const int4 &it) { return it.y / (htab[it.x].ntx * htab[it.x].nty); };
        struct Unit { int r, c, first, count, planes; };
        std::vector<Unit> units;
        for (int i = 0; i < nitems;) {
            int j = i;
            while (j < nitems && hitems[j].x == hitems[i].x && chunk_of(hitems[j]) == chunk_of(hitems[i])) ++j;
            units.push_back(Unit{hitems[i].x, chunk_of(hitems[i]), i, j - i, planes(hitems[i])});
            i = j;
        }
        std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) {
            return (long long)a.count * a.planes > (long long)b.count * b.planes;
        });
        std::vector<int> bin(units.size());
        long long load[kXcdCount] = {0};
        for (size_t u = 0; u < units.size(); ++u) {
            int best = 0;
            for (int x = 1; x < kXcdCount; ++x)
                if (load[x] < load[best]) best = x;
            bin[u] = best;
            load[best] += (long long)units[u].count * units[u].planes;
        }
        std::vector<int4> sorted;
        sorted.reserve(nitems);
        int seg[kXcdCount + 1];
        for (int x = 0; x < kXcdCount; ++x) {
            seg[x] = (int)sorted.size();
            std::vector<size_t> mine;
            for (size_t u = 0; u < units.size(); ++u)
                if (bin[u] == x) mine.push_back(u);
            std::stable_sort(mine.begin(), mine.end(), [&](size_t a, size_t b) {
                if (units[a].planes != units[b].planes) return units[a].planes > units[b].planes;
                return units[a].r != units[b].r ? units[a].r < units[b].r : units[a].c < units[b].c;
            });
            for (size_t u : mine)
                for (int k = 0; k < units[u].count; ++k) sorted.push_back(hitems[units[u].first + k]);
        }
        seg[kXcdCount] = (int)sorted.size();
        for (int i = 0; i < nitems; ++i) hitems[i] = sorted[i];
        int hq[kEnsQueueInts] = {0};
        for (int x = 0; x <= kXcdCount; ++x) hq[8 * 32 + x] = seg[x];
        hipError_t he = hipMemcpyAsync(e->tab, htab, (size_t)R * sizeof(EnsEntry), hipMemcpyHostToDevice, e->stream);
        if (he == hipSuccess)
            he = hipMemcpyAsync(e->items, hitems, (size_t)nitems * sizeof(int4), hipMemcpyHostToDevice, e->stream);
        if (he == hipSuccess)
            he = hipMemcpyAsync(e->queue, hq, sizeof hq, hipMemcpyHostToDevice, e->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
        if (he != hipSuccess) rc = fail(LF_EHIP, "uploading the ensemble tables: %s", hipGetErrorString(he));
    }
    delete[] htab;
    delete[] hitems;
    if (rc) {
        lf_ens_destroy(e);
        return rc;
    }
    // persistent grid: as many blocks as fit on the device at once
    const lf_params q0 = ens_sub_params(&per[0], &per[0], false);
    int res = resident_blocks(&q0, e->tile_x, e->tile_y);
    e->grid = nitems < res ? nitems : res;
    if ((rc = ens_prepare_graphs(e))) {
        lf_ens_destroy(e);
        return rc;
    }
    *out = e;
    return LF_OK;
}

}  // extern "C"

namespace {

void ens_enqueue_step(lf_ens *e, int parity, hipStream_t st)
{
    launch_aupdate_ens(e->tab, e->R, e->queue, st);
    launch_sweep_ens(e->stencil, e->dtype, e->tile_x, e->tile_y, e->beta, e->tab, e->items, e->nitems, e->queue,
                     e->grid, parity, st);
}

int ens_capture(lf_ens *e, int nsteps, int start, hipGraphExec_t *exec)
{
    DeviceScope scope(e->device);
    if (!e->cap) HIPCHK(hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal));
    int par = start;
    for (int k = 0; k < nsteps; ++k, par ^= 1) ens_enqueue_step(e, par, e->cap);
    hipGraph_t g = nullptr;
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamEndCapture(e->cap, &g);
    if (e1 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LF_EHIP, "kernel launch during capture: %s", hipGetErrorString(e1));
    }
    if (e2 != hipSuccess) return fail(LF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return fail(LF_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
    return LF_OK;
}

// Instantiate and upload the ensemble's step graphs (two steps from parity
// 0, one step from either parity) at create, outside any timed call.
int ens_prepare_graphs(lf_ens *e)
{
    int rc;
    if ((rc = ens_capture(e, 2, 0, &e->g2))) return rc;
    HIPCHK(hipGraphUpload(e->g2, e->stream));
    for (int p = 0; p < 2; ++p) {
        if ((rc = ens_capture(e, 1, p, &e->g1[p]))) return rc;
        HIPCHK(hipGraphUpload(e->g1[p], e->stream));
    }
    return LF_OK;
}

int ens_check_inited(lf_ens *e)
{
    for (int r = 0; r < e->R; ++r)
        if (!e->sub[r]->inited) return fail(LF_ESTATE, "realization %d is not initialised", r);
    return LF_OK;
}

}  // namespace

extern "C" {

int lf_ens_size(lf_ens *e, int *R) {
    if (!e || !R) return fail(LF_EINVAL, "NULL argument");
    *R = e->R;
    return LF_OK;
}

int lf_ens_init(lf_ens *e, int r, const void *f1, const void *f2, const void *v1, const void *v2,
                int in_dtype, double a0, double ad0)
{
    if (!e) return fail(LF_EINVAL, "ensemble is NULL");
    if (r < 0 || r >= e->R) return fail(LF_EINVAL, "realization %d out of range", r);
    if (e->cur != 0) return fail(LF_ESTATE, "initialise every realization before stepping");
    return lf_init(e->sub[r], f1, f2, v1, v2, in_dtype, a0, ad0);
}

int lf_ens_init_physical(lf_ens *e, int r, const void *f1, const void *f2, const void *u1,
                         const void *u2, int in_dtype, double a0, double *ad0_out)
{
    if (!e) return fail(LF_EINVAL, "ensemble is NULL");
    if (r < 0 || r >= e->R) return fail(LF_EINVAL, "realization %d out of range", r);
    if (e->cur != 0) return fail(LF_ESTATE, "initialise every realization before stepping");
    return lf_init_physical(e->sub[r], f1, f2, u1, u2, in_dtype, a0, ad0_out);
}

int lf_ens_step(lf_ens *e, int64_t n)
{
    TraceRange range_("lf_ens_step");
    if (!e) return fail(LF_EINVAL, "ensemble is NULL");
    if (n < 0) return fail(LF_EINVAL, "n=%lld < 0", (long long)n);
    int rc = ens_check_inited(e);
    if (rc) return rc;
    if (n == 0) return LF_OK;
    if (n >= 2 && !e->g2 && (rc = ens_capture(e, 2, 0, &e->g2))) return rc;
    if ((rc = ensure_events(e->device, &e->ev0, &e->ev1))) return rc;
    HIPCHK(hipEventRecord(e->ev0, e->stream));
    while (n > 0) {
        if (n >= 2 && e->cur == 0) {
            HIPCHK(hipGraphLaunch(e->g2, e->stream));
            n -= 2;
        } else {
            if (!e->g1[e->cur] && (rc = ens_capture(e, 1, e->cur, &e->g1[e->cur]))) return rc;
            HIPCHK(hipGraphLaunch(e->g1[e->cur], e->stream));
            e->cur ^= 1;
            --n;
        }
    }
    HIPCHK(hipEventRecord(e->ev1, e->stream));
    e->timed = 1;
    for (int r = 0; r < e->R; ++r) e->sub[r]->cur = e->cur;
    return LF_OK;
}

int lf_ens_last_step_ms(lf_ens *e, double *ms)
{
    if (!e || !ms) return fail(LF_EINVAL, "NULL argument");
    *ms = 0.0;
    if (!e->timed) return LF_OK;
    HIPCHK(hipEventSynchronize(e->ev1));
    float f = 0.0f;
    HIPCHK(hipEventElapsedTime(&f, e->ev0, e->ev1));
    *ms = f;
    return LF_OK;
}

int lf_ens_energies(lf_ens *e, lf_report *out)
{
    if (!e || !out) return fail(LF_EINVAL, "NULL argument");
    int worst = LF_OK;
    for (int r = 0; r < e->R; ++r) {
        int rc = lf_energies(e->sub[r], &out[r]);
        if (rc == LF_ENONFINITE) worst = rc;
        else if (rc) return rc;
    }
    if (worst) return fail(worst, "non-finite value in at least one realization");
    return LF_OK;
}

int lf_ens_get_fields(lf_ens *e, int r, void *f1, void *f2, void *v1, void *v2, int out_dtype,
                      int synchronized)
{
    if (!e) return fail(LF_EINVAL, "ensemble is NULL");
    if (r < 0 || r >= e->R) return fail(LF_EINVAL, "realization %d out of range", r);
    return lf_get_fields(e->sub[r], f1, f2, v1, v2, out_dtype, synchronized);
}

}  // extern "C"

// ---------------------------------------------------------------- ensemble autotuner

namespace {

// z-chunk of an N-plane lattice for a target item length: the fewest equal
// chunks of at most `target` planes (0 = the ensemble's default rule).
int ens_zchunk_for(int N, int target)
{
    if (target <= 0 || target >= N) return target <= 0 ? 0 : N;
    const int n = (N + target - 1) / target;
    return (N + n - 1) / n;
}

// Cache key of an ensemble: the multiset of lattice sizes, "N:count,..." in
// increasing N.  Returns 0 if it does not fit in `len` characters.
int ens_key(int R, const lf_params *per, char *key, size_t len)
{
    int *ns = new int[R];
    for (int r = 0; r < R; ++r) ns[r] = per[r].N;
    std::sort(ns, ns + R);
    size_t off = 0;
    int ok = 1;
    key[0] = 0;
    for (int i = 0; i < R && ok;) {
        int j = i;
        while (j < R && ns[j] == ns[i]) ++j;
        const int w = snprintf(key + off, len - off, "%s%d:%d", off ? "," : "", ns[i], j - i);
        if (w < 0 || (size_t)w >= len - off) ok = 0;
        else off += (size_t)w;
        i = j;
    }
    delete[] ns;
    return ok;
}

// Ensemble cache lines:
// {"arch": "gfx950", "ensemble": "64:48,96:16,160:4", "dtype": 0, "beta": 4, "stencil": 7,
//  "tile_x": 64, "tile_y": 8, "ztarget": 64, "ms": 0.25}
int ens_cache_lookup(const char *path, const char *arch, const char *key, int dtype, int beta, int stencil,
                     int *tx, int *ty, int *zt)
{
    if (!path) return 0;
    FILE *f = fopen(path, "r");
    if (!f) return 0;
    char line[2048];
    int found = 0;
    while (fgets(line, sizeof line, f)) {
        char a[64] = {0}, k[1200] = {0};
        int dt, b, st, x, y, z;
        double ms;
        if (sscanf(line, " {\"arch\": \"%63[^\"]\", \"ensemble\": \"%1199[^\"]\", \"dtype\": %d, \"beta\": %d, "
                         "\"stencil\": %d, \"tile_x\": %d, \"tile_y\": %d, \"ztarget\": %d, \"ms\": %lf",
                   a, k, &dt, &b, &st, &x, &y, &z, &ms) == 9 &&
            !strcmp(a, arch) && !strcmp(k, key) && dt == dtype && b == beta && st == stencil) {
            *tx = x;
            *ty = y;
            *zt = z;
            found = 1;  // the last matching line wins
        }
    }
    fclose(f);
    return found;
}

void ens_cache_append(const char *path, const char *arch, const char *key, int dtype, int beta, int stencil,
                      int tx, int ty, int zt, double ms)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"arch\": \"%s\", \"ensemble\": \"%s\", \"dtype\": %d, \"beta\": %d, \"stencil\": %d, "
               "\"tile_x\": %d, \"tile_y\": %d, \"ztarget\": %d, \"ms\": %.6f}\n",
            arch, key, dtype, beta, stencil, tx, ty, zt, ms);
    fclose(f);
}

struct EnsCand {
    int tx, ty, zt;
};

// Candidates: every LDS tile (32-wide ones for the 7-point sweep only) with
// target item lengths from 16 planes to whole lattices, plus the default
// z-chunk rule; candidates giving the same chunks for every lattice as an
// earlier one are dropped.
int ens_candidates(int R, const lf_params *per, EnsCand *out, int cap)
{
    const int tiles[7][2] = {{64, 8}, {64, 4}, {64, 16}, {128, 4}, {128, 8}, {32, 8}, {32, 16}};
    const int ntiles = stencil_of(&per[0]) == 27 ? 5 : 7;
    const int targets[10] = {0, 16, 24, 32, 48, 64, 96, 128, 192, 1 << 20};
    int n = 0;
    for (int t = 0; t < ntiles; ++t)
        for (int j = 0; j < 10 && n < cap; ++j) {
            int dup = 0;
            for (int i = 0; i < n && !dup; ++i) {
                if (out[i].tx != tiles[t][0] || out[i].ty != tiles[t][1] || out[i].zt == 0 || targets[j] == 0)
                    continue;
                int same = 1;
                for (int r = 0; r < R && same; ++r)
                    same = ens_zchunk_for(per[r].N, out[i].zt) == ens_zchunk_for(per[r].N, targets[j]);
                dup = same;
            }
            if (!dup) out[n++] = EnsCand{tiles[t][0], tiles[t][1], targets[j]};
        }
    return n;
}

// per with candidate c's tile and z-chunks (a realization's own zchunk wins)
void ens_apply(int R, const lf_params *per, const EnsCand &c, lf_params *q)
{
    for (int r = 0; r < R; ++r) {
        q[r] = per[r];
        q[r].tile_x = c.tx;
        q[r].tile_y = c.ty;
        if (!per[r].zchunk) q[r].zchunk = ens_zchunk_for(per[r].N, c.zt);
    }
}

}  // namespace

extern "C" {

int lf_ens_zchunk(int N, int target) { return N >= 1 ? ens_zchunk_for(N, target) : 0; }

int lf_ens_autotune_workspace_bytes(int R, const lf_params *per, size_t *out_bytes)
{
    int rc = ens_validate(R, per);
    if (rc) return rc;
    if (!out_bytes) return fail(LF_EINVAL, "out_bytes is NULL");
    EnsCand cand[80];
    const int n = ens_candidates(R, per, cand, 80);
    lf_params *q = new lf_params[R];
    size_t m = 0;
    for (int i = 0; i < n && rc == LF_OK; ++i) {
        ens_apply(R, per, cand[i], q);
        size_t b = 0;
        rc = lf_ens_workspace_bytes(R, q, &b);
        m = b > m ? b : m;
    }
    delete[] q;
    if (rc) return rc;
    *out_bytes = m;
    return LF_OK;
}

int lf_ens_autotune(int R, const lf_params *per, void *stream, void *workspace, size_t ws_bytes,
                    const char *cache_path, int *tile_x, int *tile_y, int *ztarget, double *best_ms)
{
    int rc = ens_validate(R, per);
    if (rc) return rc;
    if (!tile_x || !tile_y || !ztarget) return fail(LF_EINVAL, "NULL output");
    char arch[64], key[1200];
    if ((rc = current_arch(arch, sizeof arch))) return rc;
    const int have_key = ens_key(R, per, key, sizeof key);
    const int dtype = per[0].dtype, beta = per[0].beta, stencil = stencil_of(&per[0]);
    if (have_key && ens_cache_lookup(cache_path, arch, key, dtype, beta, stencil, tile_x, tile_y, ztarget)) {
        if (best_ms) *best_ms = -1.0;
        return LF_OK;
    }
    size_t need = 0;
    if ((rc = lf_ens_autotune_workspace_bytes(R, per, &need))) return rc;
    if ((rc = check_ptr(workspace, "workspace"))) return rc;
    if (ws_bytes < need) return fail(LF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    EnsCand cand[80];
    const int n = ens_candidates(R, per, cand, 80);
    lf_params *q = new lf_params[R];
    double bms = 1e300;
    int bi = -1;
    for (int i = 0; i < n && rc == LF_OK; ++i) {
        ens_apply(R, per, cand[i], q);
        lf_ens *e = nullptr;
        if ((rc = lf_ens_create(R, q, stream, workspace, ws_bytes, &e))) break;
        for (int r = 0; r < R; ++r) {
            lf_ctx *c = e->sub[r];
            void *s4[4] = {c->buf[0][0], c->buf[0][1], c->buf[0][2], c->buf[0][3]};
            launch_fill_synthetic(c->p.dtype, s4, c->p.N, c->S, c->stream);
            launch_reduce(stencil_of(&c->p), c->p.dtype, s4[0], s4[1], c->p.N, c->S->bg_f, c->p.beta, c->part,
                          c->sh.rows, c->stream);
            c->inited = 1;
            c->cur = 0;
        }
        double ms = 0.0;
        const int steps = 40;
        rc = lf_ens_step(e, 4);
        if (!rc) rc = lf_ens_step(e, steps);
        if (!rc) rc = lf_ens_last_step_ms(e, &ms);
        lf_ens_destroy(e);
        ms /= steps;
        if (!rc && ms < bms) {
            bms = ms;
            bi = i;
        }
    }
    delete[] q;
    if (rc) return rc;
    *tile_x = cand[bi].tx;
    *tile_y = cand[bi].ty;
    *ztarget = cand[bi].zt;
    if (best_ms) *best_ms = bms;
    if (have_key) ens_cache_append(cache_path, arch, key, dtype, beta, stencil, cand[bi].tx, cand[bi].ty,
                                   cand[bi].zt, bms);
    return LF_OK;
}

}  // extern "C"
