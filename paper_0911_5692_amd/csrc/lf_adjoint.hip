// Reverse-mode (adjoint) kernels of the leapfrog map, gfx950.
//
// The forward step X_k -> X_{k+1} (Sainio, arXiv:0911.5692, eq. evo applied
// to eq. scalar-evo and eq. scale; X = f(k+1/2), v(k), a_{k+1/2}, a'_k) is
// differentiated by hand; its transpose is applied here step by step in
// reverse order.  Per reverse step:
//   pass A  (k_adj_reduce): volume sums of the incoming cotangent against the
//           stored fields (the global a'' coupling) and of the fields themselves;
//   scalar  (k_adj_scalar): the chain through a'', the time-centred a' update,
//           F_a and the a-powers of V_pr, in FP64, one thread (the powers on
//           parallel lanes);
//   pass B  (k_adj_fields): the field cotangents: the Laplacian (7 or 27
//           points) of mu = lambda_v' + dt lambda_f' (both stencils are
//           symmetric), the local 2x2 Hessian of V_pr, and the rank-one terms
//           from Sg and SV (the derivative of the gradient energy is -2 Lap f,
//           since it is the Dirichlet form of the same Laplacian); inside a
//           segment of stored states it also forms pass A of the next
//           reverse step.
// Cotangent arrays are FP64 whatever the state precision; stored states are
// deviations from the FP64 background and are turned back into full fields
// f = f_bar + d in FP64 on the fly.
#include "lf_internal.h"

#include <math.h>

namespace lf {

namespace {

template <int NV>
__device__ inline void bsum(double (&v)[NV], double *out)
{
    __shared__ double sm[NV][4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[i] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sm[i][wave] = v[i];
    }
    __syncthreads();
    if (t < NV) out[t] = ((sm[t][0] + sm[t][1]) + sm[t][2]) + sm[t][3];
}

template <int NV>
__device__ inline void stage2(const double *part, int nblk, double (&tot)[NV])
{
    __shared__ double res[NV];
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int j = threadIdx.x; j < nblk; j += blockDim.x) {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += part[(size_t)j * NV + i];
    }
    bsum<NV>(acc, res);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) tot[i] = res[i];
}

__device__ inline double ipw(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

}  // namespace

// ------------------------------------------------------------ loss seed

// Cotangent of E = sum_i wK_i K_i + wG_i G_i at the synchronised time of
// the state (d, e; background and scale factor in S), written to lam[0..3]
// (lambda_f1, lambda_f2, lambda_v1, lambda_v2), plus the per-block sums the
// scalar part needs: sum q1^2, sum q2^2, the raw gradient sums of fs1 and fs2,
// sum_i wK_i q_i fs_i.
template <typename T, int ST>
__global__ void __launch_bounds__(256) k_adj_seed(const T *__restrict__ d1, const T *__restrict__ d2,
                                                  const T *__restrict__ e1, const T *__restrict__ e2,
                                                  int N, const DevParams *__restrict__ P,
                                                  const DevScalars *__restrict__ S, const double *__restrict__ w,
                                                  double *lf1, double *lf2, double *lv1, double *lv2,
                                                  double *part)
{
    const int64_t N3 = (int64_t)N * N * N;
    const double h = 0.5 * P->dt, r = P->r, s = P->s, inv_dx2 = P->gw / (P->dx * P->dx);
    const double a = S->a_half - h * S->ad, hub = S->ad / a;
    const double gfac = 0.5 * pow(a, -2.0 * s - 2.0);
    const double gs1 = S->bg_f[0] - h * S->bg_v[0], gs2 = S->bg_f[1] - h * S->bg_v[1];
    const double wK1 = w[0], wK2 = w[1], wG1 = w[2], wG2 = w[3];
    const double n3 = (double)N3;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N3;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Wrap wr(i, N);
        auto sy1 = [&](int dx, int dy, int dz) {
            const int64_t j = wr(dx, dy, dz);
            return (double)d1[j] - h * (double)e1[j];
        };
        auto sy2 = [&](int dx, int dy, int dz) {
            const int64_t j = wr(dx, dy, dz);
            return (double)d2[j] - h * (double)e2[j];
        };
        const double c1v = (double)d1[i] - h * (double)e1[i], c2v = (double)d2[i] - h * (double)e2[i];
        const double fs1 = gs1 + c1v, fs2 = gs2 + c2v;
        const double q1 = (S->bg_v[0] + (double)e1[i]) - r * hub * fs1;
        const double q2 = (S->bg_v[1] + (double)e2[i]) - r * hub * fs2;
        const double lap1 = lap_raw<ST, double>(sy1, c1v) * inv_dx2;
        const double lap2 = lap_raw<ST, double>(sy2, c2v) * inv_dx2;
        const double dq1 = wK1 * q1 / n3, dq2 = wK2 * q2 / n3;
        const double dfs1 = -r * hub * dq1 - 2.0 * wG1 * gfac * lap1 / n3;
        const double dfs2 = -r * hub * dq2 - 2.0 * wG2 * gfac * lap2 / n3;
        lf1[i] = dfs1;
        lf2[i] = dfs2;
        lv1[i] = dq1 - h * dfs1;
        lv2[i] = dq2 - h * dfs2;
        acc[0] += q1 * q1;
        acc[1] += q2 * q2;
        acc[2] += grad_raw<ST>(sy1, c1v);
        acc[3] += grad_raw<ST>(sy2, c2v);
        acc[4] += wK1 * q1 * fs1 + wK2 * q2 * fs2;
    }
    bsum<5>(acc, part + (size_t)blockIdx.x * 5);
}

// Scalar part of the seed and the loss value.  A: [la, lw, gG, E, ...].
__global__ void __launch_bounds__(256) k_adj_seed_scalar(const double *part, int nblk,
                                                         const DevParams *__restrict__ P,
                                                         const DevScalars *__restrict__ S,
                                                         const double *__restrict__ w, double *A)
{
    double t[5];
    stage2<5>(part, nblk, t);
    if (threadIdx.x != 0) return;
    const double h = 0.5 * P->dt, r = P->r, s = P->s, n3 = P->N3;
    const double a = S->a_half - h * S->ad, ad = S->ad;
    const double gfac = 0.5 * pow(a, -2.0 * s - 2.0) * P->gw / (P->dx * P->dx);
    const double K1 = 0.5 * t[0] / n3, K2 = 0.5 * t[1] / n3;
    const double G1 = gfac * t[2] / n3, G2 = gfac * t[3] / n3;
    const double E = w[0] * K1 + w[1] * K2 + w[2] * G1 + w[3] * G2;
    const double dhub = -r * t[4] / n3;
    const double dEda = dhub * (-ad / (a * a)) + (w[2] * G1 + w[3] * G2) * (-2.0 * s - 2.0) / a;
    const double dEdad = dhub / a;
    A[0] = dEda;              // lambda of a_{n+1/2}
    A[1] = dEdad - h * dEda;  // lambda of a'_n
    A[2] = 0.0;               // dE/dG accumulator
    A[3] = E;
}

// ------------------------------------------------------------ reverse step

// Pass A: sums over the stored fields f = f_bar + d at k+1/2 and
// mu = lambda_v' + dt lambda_f' (cotangent of v(k+1)):
//  0: sum mu_i S(f_i)   1: sum mu_i f_i   2: sum mu1 f1 f2^2 + mu2 f1^2 f2
//  3: sum mu1 f1^(beta-1)   4: sum f1^beta   5: sum f1^2 f2^2
//  6: raw gradient sums of f_1 plus f_2
// (S: the raw stencil sum lap_raw<ST>; no 1/dx^2, no stencil weight)
template <typename T, int ST>
__global__ void __launch_bounds__(256) k_adj_reduce(const T *__restrict__ d1, const T *__restrict__ d2,
                                                    int N, int beta, const DevScalars *__restrict__ tape,
                                                    const double *__restrict__ lf1, const double *__restrict__ lf2,
                                                    const double *__restrict__ lv1, const double *__restrict__ lv2,
                                                    double dt, double *part)
{
    const int64_t N3 = (int64_t)N * N * N;
    const double g1 = tape->bg_f[0], g2 = tape->bg_f[1];
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N3;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Wrap wr(i, N);
        auto v1 = [&](int dx, int dy, int dz) { return (double)d1[wr(dx, dy, dz)]; };
        auto v2 = [&](int dx, int dy, int dz) { return (double)d2[wr(dx, dy, dz)]; };
        const double a1 = (double)d1[i], a2 = (double)d2[i];
        const double f1 = g1 + a1, f2 = g2 + a2;
        const double s1 = lap_raw<ST, double>(v1, a1);
        const double s2 = lap_raw<ST, double>(v2, a2);
        const double mu1 = lv1[i] + dt * lf1[i], mu2 = lv2[i] + dt * lf2[i];
        acc[0] += mu1 * s1 + mu2 * s2;
        acc[1] += mu1 * f1 + mu2 * f2;
        acc[2] += mu1 * f1 * f2 * f2 + mu2 * f1 * f1 * f2;
        acc[3] += mu1 * ipw(f1, beta - 1);
        acc[4] += ipw(f1, beta);
        acc[5] += f1 * f1 * f2 * f2;
        acc[6] += grad_raw<ST>(v1, a1) + grad_raw<ST>(v2, a2);
    }
    bsum<7>(acc, part + (size_t)blockIdx.x * 7);
}

// Scalar chain of one reverse step.  A: [la, lw, gG, E]; writes the field
// coefficients to cf: [dt a^(-2s-2) gw/dx^2, dt bcoef, c1 a^p1, G a^p2, cSg, cSV, dt].
__global__ void __launch_bounds__(256) k_adj_scalar(const double *part, int nblk,
                                                    const DevParams *__restrict__ P,
                                                    const DevScalars *__restrict__ tape, double *A,
                                                    double *cf)
{
    double R[7];
    stage2<7>(part, nblk, R);
    if (threadIdx.x >= 64) return;
    const double n3 = P->N3, dx = P->dx, dt = P->dt, r = P->r, s = P->s, c1 = P->c1, G = P->G;
    const int beta = P->beta;
    const double a = tape->a_half, w = tape->ad;
    const double p1 = P->p1, p2 = P->p2;
    const double e1 = -2.0 * s - 2.0 * r - 1.0;
    // the eleven powers of a, one per lane of the first wave, side by side
    const int l = threadIdx.x;
    double ex;
    switch (l) {
    case 0: ex = p1; break;
    case 1: ex = p2; break;
    case 2: ex = p1 - 1.0; break;
    case 3: ex = p2 - 1.0; break;
    case 4: ex = e1; break;
    case 5: ex = 2.0 * s + 2.0; break;
    case 6: ex = -2.0 * s - 2.0; break;
    case 7: ex = -2.0 * s - 3.0; break;
    case 8: ex = e1 + 2.0 * s + 2.0; break;
    case 9: ex = e1 - 1.0; break;
    default: ex = e1 + 2.0 * s + 1.0; break;
    }
    const double pw = pow(a, ex);
    const double ap1 = __shfl(pw, 0, 64), ap2 = __shfl(pw, 1, 64);
    const double pa_p1m = __shfl(pw, 2, 64), pa_p2m = __shfl(pw, 3, 64), pa_e1 = __shfl(pw, 4, 64);
    const double pa_2s2 = __shfl(pw, 5, 64), alpha = __shfl(pw, 6, 64), pa_m2s3 = __shfl(pw, 7, 64);
    const double pa_e1s = __shfl(pw, 8, 64), pa_e1m = __shfl(pw, 9, 64), pa_e1s1 = __shfl(pw, 10, 64);
    if (l != 0) return;
    const double dap1 = p1 * pa_p1m, dap2 = p2 * pa_p2m;
    // forward scalars of this step
    const double gw = P->gw;
    const double Sg = gw * R[6] / (dx * dx * n3);
    const double SV = (c1 * ap1 * R[4] / (double)beta + 0.5 * G * ap2 * R[5]) / n3;
    const double Fa = P->kappa2 * pa_e1 * (Sg / 3.0 + pa_2s2 * SV);
    const double c = (-s - 2.0) * dt / (4.0 * a);
    const double disc = 1.0 - 8.0 * c * w - 4.0 * c * dt * Fa;
    const double u = 2.0 * (c * w * w + w + dt * Fa) / ((1.0 - 2.0 * c * w) + sqrt(disc));
    const double adh = 0.5 * (w + u), add = (u - w) / dt;
    const double rr = r * (s - r + 2.0);
    const double bc = rr * (adh / a) * (adh / a) + r * add / a;
    // kick sensitivities
    const double galpha = dt * gw * R[0] / (dx * dx);
    const double gbeta = dt * R[1];
    const double gGk = -dt * ap2 * R[2];
    const double gak = -dt * (c1 * dap1 * R[3] + G * dap2 * R[2]);
    const double sdVda = c1 * dap1 * R[4] / (double)beta + 0.5 * G * dap2 * R[5];
    const double sdVdG = 0.5 * ap2 * R[5];
    const double la = A[0], lw = A[1];
    double ga = la + gak;
    ga += galpha * (-2.0 * s - 2.0) * pa_m2s3;
    const double g_adh = gbeta * 2.0 * rr * adh / (a * a);
    const double g_add = gbeta * r / a;
    ga += gbeta * (-2.0 * rr * adh * adh / (a * a * a) - r * add / (a * a));
    const double g_u = lw + dt * la + 0.5 * g_adh + g_add / dt;
    double g_w = 0.5 * g_adh - g_add / dt;
    const double q = dt * (-s - 2.0) * (w + u) / (2.0 * a);
    const double hu = 1.0 - q;
    g_w += g_u * (1.0 + q) / hu;
    ga += g_u * (-(dt * (-s - 2.0) * (w + u) * (w + u) / (4.0 * a * a)) / hu);
    const double gF = g_u * dt / hu;
    const double gSg = gF * P->kappa2 * pa_e1 / 3.0;
    const double gSV = gF * P->kappa2 * pa_e1s;
    ga += gF * P->kappa2 * (e1 * pa_e1m * Sg / 3.0 + (e1 + 2.0 * s + 2.0) * pa_e1s1 * SV);
    ga += gSV * sdVda / n3;
    A[0] = ga;
    A[1] = g_w;
    A[2] += gGk + gSV * sdVdG / n3;
    cf[0] = dt * alpha * gw / (dx * dx);
    cf[1] = dt * bc;
    cf[2] = c1 * ap1;
    cf[3] = G * ap2;
    cf[4] = -2.0 * gSg * gw / (n3 * dx * dx);  // multiplies the raw stencil sum of f
    cf[5] = gSV / n3;
    cf[6] = dt;
}

// Pass B: field cotangents of X_k from those of X_{k+1} (in -> out), with
// NEXT also pass A of the next reverse step (X_{k-1}: stored fields n1, n2,
// scalars tape_n) over the cotangents just written, into part.
//
// It needs, per site, mu = lambda_v' + dt lambda_f' and the stored d (and n)
// at every stencil neighbour in planes z-1, z, z+1.  A block owns a 64 x 4
// column tile and marches z over a chunk: the three planes sit in LDS with a
// one-cell ring (four buffers, so one barrier per plane), and plane z+2 is
// loaded into registers while plane z is evaluated.  The grid walks a static
// list of (tile, chunk) items.  The per-site arithmetic is that of the
// generic one-site-per-thread formulation.
constexpr int kAX = 64, kAY = 4;
constexpr int kALW = kAX + 2, kALH = kAY + 2, kAPL = kALW * kALH;  // plane with its ring
constexpr int kARing = 2 * kALW + 2 * kAY;

__device__ inline void adj_ring_cell(int c, int &lx, int &ly)
{
    if (c < kALW) { lx = c - 1; ly = -1; }
    else if (c < 2 * kALW) { lx = c - kALW - 1; ly = kAY; }
    else if (c < 2 * kALW + kAY) { lx = -1; ly = c - 2 * kALW; }
    else { lx = kAX; ly = c - 2 * kALW - kAY; }
}

// LDS bytes of k_adj_fields: four planes of mu1, mu2 (FP64) and the stored
// fields d1, d2 (and n1, n2 with NEXT) in their own type.
template <typename T, bool NEXT>
constexpr size_t adj_fields_lds()
{
    return (size_t)4 * kAPL * (2 * sizeof(double) + (NEXT ? 4 : 2) * sizeof(T));
}

template <typename T, int ST, bool NEXT>
__global__ void __launch_bounds__(256) k_adj_fields(const T *__restrict__ d1, const T *__restrict__ d2,
                                                    int N, int beta, const DevScalars *__restrict__ tape,
                                                    const double *__restrict__ cf,
                                                    const double *__restrict__ lf1, const double *__restrict__ lf2,
                                                    const double *__restrict__ lv1, const double *__restrict__ lv2,
                                                    double *of1, double *of2, double *ov1, double *ov2,
                                                    const T *__restrict__ n1, const T *__restrict__ n2,
                                                    const DevScalars *__restrict__ tape_n, double *part,
                                                    int zchunk, int ntx, int nty, int nitems)
{
    extern __shared__ double lds[];
    // buffer b: mu1, mu2 (doubles) at lds + b * 2 * kAPL; fields in type T after all mu planes
    double *smu = lds;
    T *sfl = (T *)(lds + 4 * 2 * kAPL);
    constexpr int NF = NEXT ? 4 : 2;  // d1, d2 [, n1, n2]
    auto MU = [&](int b, int q) { return smu + (b * 2 + q) * kAPL; };
    auto FL = [&](int b, int q) { return sfl + (b * NF + q) * kAPL; };

    const int64_t NN = (int64_t)N * N;
    const double g1 = tape->bg_f[0], g2 = tape->bg_f[1];
    const double cl = cf[0], cb = cf[1], c1a = cf[2], Ga = cf[3], cSg = cf[4], cSV = cf[5], dt = cf[6];
    const double gn1 = NEXT ? tape_n->bg_f[0] : 0.0, gn2 = NEXT ? tape_n->bg_f[1] : 0.0;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};

    const int t = threadIdx.x, lx = t & 63, ly = t >> 6;
    const int slot = (ly + 1) * kALW + lx + 1;
    const bool hasr = t < kARing;
    int rx = 0, ry = 0;
    if (hasr) adj_ring_cell(t, rx, ry);
    const int rslot = (ry + 1) * kALW + rx + 1;
    auto wrap = [N](int v) { return ((v % N) + N) % N; };
    // plane z in [-1, N]: one wrap suffices
    auto zoff = [&](int z) { return (int64_t)(z < 0 ? z + N : (z >= N ? z - N : z)) * NN; };

    for (int base = 0; base + (int)blockIdx.x < nitems; base += gridDim.x) {
        const int item = xcd_item(base, nitems);  // XCD-contiguous tiles share halo rows in L2
        const int tx = item % ntx, rest = item / ntx, ty = rest % nty, tz = rest / nty;
        const int x0 = tx * kAX, y0 = ty * kAY, z0 = tz * zchunk;
        const int z1 = min(z0 + zchunk, N);
        const bool act = (x0 + lx < N) && (y0 + ly < N);
        const int off = wrap(y0 + ly) * N + wrap(x0 + lx);
        const int roff = wrap(y0 + ry) * N + wrap(x0 + rx);

        // the plane in flight, site and ring cell
        double pf1, pf2, pv1, pv2, hf1 = 0, hf2 = 0, hv1 = 0, hv2 = 0;
        T pd1, pd2, hd1 = 0, hd2 = 0, pn1 = 0, pn2 = 0, hn1 = 0, hn2 = 0;
        auto load = [&](int z) {
            const int64_t o = zoff(z) + off;
            pf1 = lf1[o]; pf2 = lf2[o]; pv1 = lv1[o]; pv2 = lv2[o];
            pd1 = d1[o]; pd2 = d2[o];
            if (NEXT) { pn1 = n1[o]; pn2 = n2[o]; }
            if (hasr) {
                const int64_t h = zoff(z) + roff;
                hf1 = lf1[h]; hf2 = lf2[h]; hv1 = lv1[h]; hv2 = lv2[h];
                hd1 = d1[h]; hd2 = d2[h];
                if (NEXT) { hn1 = n1[h]; hn2 = n2[h]; }
            }
        };
        auto stage = [&](int b) {
            MU(b, 0)[slot] = pv1 + dt * pf1;
            MU(b, 1)[slot] = pv2 + dt * pf2;
            FL(b, 0)[slot] = pd1;
            FL(b, 1)[slot] = pd2;
            if (NEXT) { FL(b, 2)[slot] = pn1; FL(b, 3)[slot] = pn2; }
            if (hasr) {
                MU(b, 0)[rslot] = hv1 + dt * hf1;
                MU(b, 1)[rslot] = hv2 + dt * hf2;
                FL(b, 0)[rslot] = hd1;
                FL(b, 1)[rslot] = hd2;
                if (NEXT) { FL(b, 2)[rslot] = hn1; FL(b, 3)[rslot] = hn2; }
            }
        };
        // plane p lives in buffer (p - z0 + 1) & 3; own lambda_f of planes z, z+1
        double lc1, lc2, ln1, ln2;
        load(z0 - 1);
        stage(0);
        load(z0);
        stage(1);
        lc1 = pf1; lc2 = pf2;
        load(z0 + 1);
        for (int z = z0; z < z1; ++z) {
            const int bp = (z - z0) & 3, bc = (z - z0 + 1) & 3, bn = (z - z0 + 2) & 3;
            // plane z+1 into the buffer last read for plane z-3
            stage(bn);
            ln1 = pf1; ln2 = pf2;
            if (z + 2 <= z1) load(z + 2);
            __syncthreads();
            if (act) {
                auto pick = [&](int dz) { return dz < 0 ? bp : (dz > 0 ? bn : bc); };
                auto mu1 = [&](int dx, int dy, int dz) { return MU(pick(dz), 0)[slot + dy * kALW + dx]; };
                auto mu2 = [&](int dx, int dy, int dz) { return MU(pick(dz), 1)[slot + dy * kALW + dx]; };
                auto v1 = [&](int dx, int dy, int dz) { return (double)FL(pick(dz), 0)[slot + dy * kALW + dx]; };
                auto v2 = [&](int dx, int dy, int dz) { return (double)FL(pick(dz), 1)[slot + dy * kALW + dx]; };
                const double m1 = MU(bc, 0)[slot], m2 = MU(bc, 1)[slot];
                const double lm1 = lap_raw<ST, double>(mu1, m1);
                const double lm2 = lap_raw<ST, double>(mu2, m2);
                const double a1 = (double)FL(bc, 0)[slot], a2 = (double)FL(bc, 1)[slot];
                const double s1 = lap_raw<ST, double>(v1, a1);
                const double s2 = lap_raw<ST, double>(v2, a2);
                const double f1 = g1 + a1, f2 = g2 + a2;
                const double h11 = c1a * (double)(beta - 1) * ipw(f1, beta - 2) + Ga * f2 * f2;
                const double h12 = 2.0 * Ga * f1 * f2;
                const double h22 = Ga * f1 * f1;
                const double dv1 = c1a * ipw(f1, beta - 1) + Ga * f1 * f2 * f2;
                const double dv2 = Ga * f1 * f1 * f2;
                const double o1 = lc1 + cl * lm1 + cb * m1 - dt * (h11 * m1 + h12 * m2) + cSg * s1 + cSV * dv1;
                const double o2 = lc2 + cl * lm2 + cb * m2 - dt * (h12 * m1 + h22 * m2) + cSg * s2 + cSV * dv2;
                const int64_t i = (int64_t)z * NN + off;
                of1[i] = o1;
                of2[i] = o2;
                ov1[i] = m1;
                ov2[i] = m2;
                if (NEXT) {
                    // the terms of k_adj_reduce for X_{k-1}, with lambda = (o, m)
                    auto w1 = [&](int dx, int dy, int dz) { return (double)FL(pick(dz), 2)[slot + dy * kALW + dx]; };
                    auto w2 = [&](int dx, int dy, int dz) { return (double)FL(pick(dz), 3)[slot + dy * kALW + dx]; };
                    const double b1 = (double)FL(bc, 2)[slot], b2 = (double)FL(bc, 3)[slot];
                    const double f1n = gn1 + b1, f2n = gn2 + b2;
                    const double t1 = lap_raw<ST, double>(w1, b1);
                    const double t2 = lap_raw<ST, double>(w2, b2);
                    const double nu1 = m1 + dt * o1, nu2 = m2 + dt * o2;
                    acc[0] += nu1 * t1 + nu2 * t2;
                    acc[1] += nu1 * f1n + nu2 * f2n;
                    acc[2] += nu1 * f1n * f2n * f2n + nu2 * f1n * f1n * f2n;
                    acc[3] += nu1 * ipw(f1n, beta - 1);
                    acc[4] += ipw(f1n, beta);
                    acc[5] += f1n * f1n * f2n * f2n;
                    acc[6] += grad_raw<ST>(w1, b1) + grad_raw<ST>(w2, b2);
                }
            }
            lc1 = ln1; lc2 = ln2;
        }
        __syncthreads();  // the next item restages buffers 0 and 1
    }
    if (NEXT) bsum<7>(acc, part + (size_t)blockIdx.x * 7);
}

// Transpose of the desynchronisation f(1/2) = f(0) + dt/2 v(0) (in place on
// the v cotangents) and of a_{1/2} = a0 + dt/2 a'0 (A[1] += dt/2 A[0]).
__global__ void __launch_bounds__(256) k_adj_desync(int64_t N3, double h, const double *lf1,
                                                    const double *lf2, double *lv1, double *lv2, double *A)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N3;
         i += (int64_t)gridDim.x * blockDim.x) {
        lv1[i] += h * lf1[i];
        lv2[i] += h * lf2[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) A[1] += h * A[0];
}

// ------------------------------------------------------------ launchers

template <typename T, int ST>
static void adj_seed_t(const void *const s4[4], int N, const DevParams *P, const DevScalars *S,
                       const double *w, double *const lam[4], double *part, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL((k_adj_seed<T, ST>), dim3(nblk), dim3(256), 0, st, (const T *)s4[0], (const T *)s4[1],
                       (const T *)s4[2], (const T *)s4[3], N, P, S, w, lam[0], lam[1], lam[2], lam[3], part);
}

void launch_adj_seed(int stencil, int dtype, const void *const s4[4], int N, const DevParams *P,
                     const DevScalars *S, const double *w, double *const lam[4], double *part, int nblk,
                     double *A, hipStream_t st)
{
    if (stencil == 27) {
        if (dtype == 0) adj_seed_t<float, 27>(s4, N, P, S, w, lam, part, nblk, st);
        else adj_seed_t<double, 27>(s4, N, P, S, w, lam, part, nblk, st);
    } else {
        if (dtype == 0) adj_seed_t<float, 7>(s4, N, P, S, w, lam, part, nblk, st);
        else adj_seed_t<double, 7>(s4, N, P, S, w, lam, part, nblk, st);
    }
    hipLaunchKernelGGL(k_adj_seed_scalar, dim3(1), dim3(256), 0, st, part, nblk, P, S, w, A);
}

// Items and grid of the marching field pass: z-chunks chosen so that the
// (tile, chunk) items fill about `rows` blocks; grid = min(items, rows), which
// is also the number of partial rows the fused sums fill.
struct AdjGrid {
    int ntx, nty, zchunk, items, grid;
};

static AdjGrid adj_grid(int N, int rows)
{
    AdjGrid g;
    g.ntx = (N + kAX - 1) / kAX;
    g.nty = (N + kAY - 1) / kAY;
    int nz = rows / (g.ntx * g.nty);
    nz = nz < 1 ? 1 : (nz > N ? N : nz);
    g.zchunk = (N + nz - 1) / nz;
    nz = (N + g.zchunk - 1) / g.zchunk;
    g.items = g.ntx * g.nty * nz;
    g.grid = g.items < rows ? g.items : rows;
    return g;
}

// Target number of field-pass items: two blocks per CU of the 256-CU part,
// so that chunks are long next to the two planes each chunk stages first
// (128^3: 16-plane chunks; 2048 items of 4 planes took 20% longer).
constexpr int kAdjItems = 512;

template <typename T, int ST>
static void adj_step_t(const AdjStep &a, int N, int beta, const DevParams *P, double dt, double *part, int nblk,
                       double *A, double *cf, hipStream_t st)
{
    const AdjGrid g = adj_grid(N, nblk < kAdjItems ? nblk : kAdjItems);
    // the step's sums: from the previous field pass (g.grid rows) or from a
    // reduction pass of their own (nblk rows)
    int rows = g.grid;
    if (!a.have_sums) {
        hipLaunchKernelGGL((k_adj_reduce<T, ST>), dim3(nblk), dim3(256), 0, st, (const T *)a.d1, (const T *)a.d2,
                           N, beta, a.tape, a.lin[0], a.lin[1], a.lin[2], a.lin[3], dt, part);
        rows = nblk;
    }
    hipLaunchKernelGGL(k_adj_scalar, dim3(1), dim3(256), 0, st, part, rows, P, a.tape, A, cf);
    if (a.next_d1) {
        constexpr size_t lds = adj_fields_lds<T, true>();
        (void)hipFuncSetAttribute((const void *)k_adj_fields<T, ST, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_adj_fields<T, ST, true>), dim3(g.grid), dim3(256), lds, st, (const T *)a.d1,
                           (const T *)a.d2, N, beta, a.tape, cf, a.lin[0], a.lin[1], a.lin[2], a.lin[3], a.lout[0],
                           a.lout[1], a.lout[2], a.lout[3], (const T *)a.next_d1, (const T *)a.next_d2,
                           a.next_tape, part, g.zchunk, g.ntx, g.nty, g.items);
    } else {
        constexpr size_t lds = adj_fields_lds<T, false>();
        (void)hipFuncSetAttribute((const void *)k_adj_fields<T, ST, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_adj_fields<T, ST, false>), dim3(g.grid), dim3(256), lds, st, (const T *)a.d1,
                           (const T *)a.d2, N, beta, a.tape, cf, a.lin[0], a.lin[1], a.lin[2], a.lin[3], a.lout[0],
                           a.lout[1], a.lout[2], a.lout[3], (const T *)nullptr, (const T *)nullptr,
                           (const DevScalars *)nullptr, (double *)nullptr, g.zchunk, g.ntx, g.nty, g.items);
    }
}

void launch_adj_step(int stencil, int dtype, const AdjStep &a, int N, int beta, const DevParams *P, double dt,
                     double *part, int nblk, double *A, double *cf, hipStream_t st)
{
    if (stencil == 27) {
        if (dtype == 0) adj_step_t<float, 27>(a, N, beta, P, dt, part, nblk, A, cf, st);
        else adj_step_t<double, 27>(a, N, beta, P, dt, part, nblk, A, cf, st);
    } else {
        if (dtype == 0) adj_step_t<float, 7>(a, N, beta, P, dt, part, nblk, A, cf, st);
        else adj_step_t<double, 7>(a, N, beta, P, dt, part, nblk, A, cf, st);
    }
}

void launch_adj_desync(int N, double dt, double *const lam[4], double *A, hipStream_t st)
{
    const int64_t N3 = (int64_t)N * N * N;
    int64_t g = (N3 + 255) / 256;
    hipLaunchKernelGGL(k_adj_desync, dim3((int)(g > 65536 ? 65536 : g)), dim3(256), 0, st, N3, 0.5 * dt,
                       lam[0], lam[1], lam[2], lam[3], A);
}

}  // namespace lf
