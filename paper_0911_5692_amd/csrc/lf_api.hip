// C-ABI layer of liblf: parameter validation, workspace layout, the step
// sequence and its HIP-graph capture.  Declarations and semantics: include/lf.h.
#include "lf_internal.h"
#include "../../include/lf.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

using namespace lf;

namespace {

thread_local std::string g_err;

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
constexpr int kRedBlocks = 2048;     // grid of the grid-stride reductions
constexpr int kMaxPartRows = 65536;  // partial rows reserved for any sweep variant

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
    L.part = off; off = align_up(off + (size_t)kMaxPartRows * kNPart * sizeof(double));
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
    if (p->tile_y < 0 || p->zchunk < 0) return fail(LF_EINVAL, "tile_y/zchunk must be >= 0");
    return LF_OK;
}

}  // namespace

struct lf_ctx {
    lf_params p;
    Layout L;
    hipStream_t stream;
    hipStream_t cap;
    char *ws;
    void *buf[2][4];
    int cur;
    double *part, *mom, *enp, *enout, *tot;
    DevParams *P;
    DevScalars *S;
    CoefPair *C;
    int inited;
    hipGraphExec_t g1[2];
    hipGraphExec_t gK[2];
    int K;
    hipEvent_t ev0, ev1;
    int timed;
};

namespace {

int enqueue_step(lf_ctx *c, int cur, hipStream_t st)
{
    const void *in[4] = {c->buf[cur][0], c->buf[cur][1], c->buf[cur][2], c->buf[cur][3]};
    void *out[4] = {c->buf[cur ^ 1][0], c->buf[cur ^ 1][1], c->buf[cur ^ 1][2], c->buf[cur ^ 1][3]};
    launch_aupdate(c->part, kRedBlocks, c->P, c->S, c->C, st);
    launch_sweep_plain(c->p.dtype, in, out, c->p.N, c->C, st);
    launch_reduce(c->p.dtype, out[0], out[1], c->p.N, c->S->bg_f, c->p.beta, c->part, kRedBlocks, st);
    return LF_OK;
}

int capture(lf_ctx *c, int nsteps, int start, hipGraphExec_t *exec)
{
    HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int cur = start;
    for (int k = 0; k < nsteps; ++k) {
        enqueue_step(c, cur, c->cap);
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
}

int check_ptr(const void *ptr, const char *name)
{
    if (!ptr) return fail(LF_EINVAL, "%s is NULL", name);
    if ((uintptr_t)ptr % kAlign) return fail(LF_EINVAL, "%s is not 256-byte aligned", name);
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
    c->stream = (hipStream_t)stream;
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
    c->K = (p->N >= 256) ? 8 : 32;
    hipError_t e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return fail(LF_EHIP, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        (void)hipStreamDestroy(c->cap);
        delete c;
        return fail(LF_EHIP, "hipEventCreate failed");
    }
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
    for (int b = 0; b < 2; ++b) {
        if (c->g1[b]) (void)hipGraphExecDestroy(c->g1[b]);
        if (c->gK[b]) (void)hipGraphExecDestroy(c->gK[b]);
    }
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return LF_OK;
}

static int init_common(lf_ctx *c, const void *f1, const void *f2, const void *v1, const void *v2,
                       int in_dtype, double a0, double ad0, int physical)
{
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    int rc;
    if ((rc = check_ptr(f1, "f1")) || (rc = check_ptr(f2, "f2")) || (rc = check_ptr(v1, "v1")) ||
        (rc = check_ptr(v2, "v2")))
        return rc;
    if (in_dtype != LF_F32 && in_dtype != LF_F64) return fail(LF_EINVAL, "in_dtype=%d", in_dtype);
    if (!(a0 > 0.0) || !isfinite(a0)) return fail(LF_EINVAL, "a0 must be finite and > 0");
    if (!isfinite(ad0)) return fail(LF_EINVAL, "ad0 must be finite");
    const int N = c->p.N;
    launch_input_moments(in_dtype, f1, f2, v1, v2, N, c->p.beta, c->mom, kRedBlocks, c->stream);
    launch_init_scalars(c->mom, kRedBlocks, c->P, c->S, physical, a0, ad0, c->stream);
    launch_init_fields(c->p.dtype, in_dtype, f1, f2, v1, v2, c->buf[0][0], c->buf[0][1],
                       c->buf[0][2], c->buf[0][3], N, c->P, c->S, c->stream);
    launch_reduce(c->p.dtype, c->buf[0][0], c->buf[0][1], N, c->S->bg_f, c->p.beta, c->part,
                  kRedBlocks, c->stream);
    HIPCHK(hipGetLastError());
    c->cur = 0;
    c->inited = 1;
    c->timed = 0;
    return LF_OK;
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
    if (!c) return fail(LF_EINVAL, "ctx is NULL");
    if (n < 0) return fail(LF_EINVAL, "n=%lld < 0", (long long)n);
    if (!c->inited) return fail(LF_ESTATE, "lf_step before lf_init");
    if (n == 0) return LF_OK;
    int rc;
    if (n >= c->K && !c->gK[c->cur] && (rc = capture(c, c->K, c->cur, &c->gK[c->cur]))) return rc;
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    while (n >= c->K) {
        HIPCHK(hipGraphLaunch(c->gK[c->cur], c->stream));
        n -= c->K;
    }
    while (n > 0) {
        if (!c->g1[c->cur] && (rc = capture(c, 1, c->cur, &c->g1[c->cur]))) return rc;
        HIPCHK(hipGraphLaunch(c->g1[c->cur], c->stream));
        c->cur ^= 1;
        --n;
    }
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    c->timed = 1;
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
    if (!c || !out) return fail(LF_EINVAL, "NULL argument");
    if (!c->inited) return fail(LF_ESTATE, "lf_energies before lf_init");
    const void *s4[4] = {c->buf[c->cur][0], c->buf[c->cur][1], c->buf[c->cur][2], c->buf[c->cur][3]};
    launch_energy(c->p.dtype, s4, c->p.N, c->P, c->S, c->enp, kRedBlocks, c->enout, c->stream);
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
    launch_sum_partials(c->part, kRedBlocks, kNPart, c->tot, c->stream);
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
    launch_set_pending(c->part, kRedBlocks, c->tot, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->cur = 0;
    c->inited = 1;
    return LF_OK;
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

int lf_time_kernels(lf_ctx *c, int64_t n, double *ms, int n_out)
{
    if (!c || !ms) return fail(LF_EINVAL, "NULL argument");
    if (n < 1 || n_out < 1) return fail(LF_EINVAL, "n and n_out must be >= 1");
    if (!c->inited) return fail(LF_ESTATE, "lf_time_kernels before lf_init");
    hipEvent_t ev[4];
    for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
    double acc[3] = {0.0, 0.0, 0.0};
    int rc = LF_OK;
    for (int64_t k = 0; k < n && rc == LF_OK; ++k) {
        const int cur = c->cur;
        const void *in[4] = {c->buf[cur][0], c->buf[cur][1], c->buf[cur][2], c->buf[cur][3]};
        void *out[4] = {c->buf[cur ^ 1][0], c->buf[cur ^ 1][1], c->buf[cur ^ 1][2], c->buf[cur ^ 1][3]};
        hipError_t e = hipEventRecord(ev[0], c->stream);
        launch_aupdate(c->part, kRedBlocks, c->P, c->S, c->C, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
        launch_sweep_plain(c->p.dtype, in, out, c->p.N, c->C, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[2], c->stream);
        launch_reduce(c->p.dtype, out[0], out[1], c->p.N, c->S->bg_f, c->p.beta, c->part, kRedBlocks,
                      c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[3], c->stream);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
        float t;
        for (int j = 0; j < 3 && e == hipSuccess; ++j) {
            e = hipEventElapsedTime(&t, ev[j], ev[j + 1]);
            acc[j] += t;
        }
        if (e != hipSuccess) rc = fail(LF_EHIP, "timing step: %s", hipGetErrorString(e));
        c->cur ^= 1;
    }
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
    if (rc) return rc;
    for (int j = 0; j < n_out; ++j) ms[j] = (j < 3) ? acc[j] / (double)n : 0.0;
    return LF_OK;
}

}  // extern "C"
