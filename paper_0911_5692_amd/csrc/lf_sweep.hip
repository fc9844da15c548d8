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
// The LDS z-march of the 27-point stencil is k_sweep_lds27 (lf_sweep27.hip);
// the launchers here dispatch to it.
#include "lf_sweep_common.h"

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

// ------------------------------------------------------------ LDS z-march

// One block's work: the tile x0.., y0.. of an N x N x zp.nz block over
// planes [z0, z1), writing its four partial sums to part_row[0..3].
template <typename T, int NH, int TX, int TY, int PF>
__device__ __forceinline__ void sweep_tile(const T *__restrict__ d1, const T *__restrict__ d2,
                                           const T *__restrict__ e1, const T *__restrict__ e2,
                                           T *__restrict__ d1n, T *__restrict__ d2n,
                                           T *__restrict__ e1n, T *__restrict__ e2n, const int N,
                                           const ZPlanes<T> &zp,
                                           const int x0, const int y0, const int z0, const int z1,
                                           const CoefPair *__restrict__ C, double *__restrict__ part_row)
{
    constexpr int RPR = 256 / TX;               // rows per round of 256 threads
    constexpr int KI = TY / RPR;                // interior sites per thread per plane
    constexpr int LW = TX + 3, LH = TY + 3;     // staged plane: x0-2 .. x0+TX, y0-2 .. y0+TY
    constexpr int NW = TX + 1, NHT = TY + 1;    // new-value plane: x0-1 .. , y0-1 ..
    constexpr int NRING = TX + 1 + TY;          // row y0-1 (TX), corner, column x0-1 (TY)
    constexpr int NHALO = 2 * (TX + 1) + 2 * (TY + 1);
    static_assert(256 % TX == 0 && TY % RPR == 0 && NRING <= 256 && NHALO <= 512, "tile shape");
    // double-buffered: plane z is read from buffer (z - z0 + 1) & 1 while
    // plane z+1 is staged into the other one; one barrier per plane
    __shared__ T sd[2][2][LH * LW];
    __shared__ T sn[2][2][NHT * NW];

    Coefs<T, NH> c;
    c.load(coef_of<T>(C));
    const double g1n = C->g1n, g2n = C->g2n;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t NN = (int64_t)N * N;
    auto wrapc = [N](int v) { return ((v % N) + N) % N; };

    // interior sites (x0 + t % TX, y0 + t / TX + RPR k): in-plane offsets and LDS slots
    int goff[KI], lsd[KI], lsn[KI];
    bool act[KI];
    const int cx = t % TX, cy = t / TX;
    const int xi = x0 + cx;
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int yl = cy + RPR * k;
        const int y = y0 + yl;
        act[k] = (xi < N) && (y < N);
        goff[k] = (y % N) * N + (xi % N);  // in-bounds even when inactive
        lsd[k] = (yl + 2) * LW + cx + 2;
        lsn[k] = (yl + 1) * NW + cx + 1;
    }
    // ring site of this thread (t < NRING): d_new only, never stored
    const bool hasr = t < NRING;
    int rlx, rly;  // LDS coordinates, staged plane frame
    if (t < TX) { rlx = t + 2; rly = 1; }
    else if (t == TX) { rlx = 1; rly = 1; }
    else { rlx = 1; rly = t - TX - 1 + 2; }
    const int roff = wrapc(y0 + rly - 2) * N + wrapc(x0 + rlx - 2);
    const int rlsd = rly * LW + rlx, rlsn = (rly - 1) * NW + (rlx - 1);
    // halo cells of this thread (t and t + 256 below NHALO): staged-plane border
    // that no computed site covers
    bool hash[2];
    int hoff[2], hlsd[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int hc = t + 256 * m;
        hash[m] = hc < NHALO;
        int hlx, hly;
        if (hc < TX + 1) { hlx = hc + 1; hly = 0; }
        else if (hc < 2 * (TX + 1)) { hlx = hc - (TX + 1) + 1; hly = TY + 2; }
        else if (hc < 2 * (TX + 1) + TY + 1) { hlx = 0; hly = hc - 2 * (TX + 1) + 1; }
        else { hlx = TX + 2; hly = hc - 2 * (TX + 1) - (TY + 1) + 1; }
        if (!hash[m]) { hlx = 0; hly = 0; }
        hoff[m] = wrapc(y0 + hly - 2) * N + wrapc(x0 + hlx - 2);
        hlsd[m] = hly * LW + hlx;
    }
    // plane base pointers (uniform): global address = plane base + 32-bit
    // offset.  Input i: z stays within [z0 - 2, z1 + 1] (planes past z1 are
    // addressed but not read); outputs: planes [z0, z1)
    auto plane = [&](int i, const T *p, int z) { return zp.at(i, p, z, NN); };
    auto oplane = [&](T *p, int z) { return p + (int64_t)z * NN; };

    // register queues: d at z-1, z, z+1 and e at z, for both fields; PF
    // prefetch slots: slot j holds d(z+2+j), e(z+1+j) and the halo of plane
    // z+2+j at the start of iteration z
    T qm1[KI], qc1[KI], qp1[KI], qm2[KI], qc2[KI], qp2[KI], ev1[KI], ev2[KI], dn1[KI], dn2[KI];
    T rqm1 = 0, rqc1 = 0, rqp1 = 0, rqm2 = 0, rqc2 = 0, rqp2 = 0, rev1 = 0, rev2 = 0;
    T hv1[2] = {0, 0}, hv2[2] = {0, 0};  // halo of the plane staged next
    T sd1[PF][KI], sd2[PF][KI], se1[PF][KI], se2[PF][KI];
    T srd1[PF], srd2[PF], sre1[PF], sre2[PF], sh1[PF][2], sh2[PF][2];
    // load prefetch slot j with d(pz), e(pz - 1), halo(pz); planes beyond the
    // chunk's needs are skipped
    auto fill = [&](int j, int pz) {
        const bool need_d = pz <= z1, need_e = pz - 1 <= z1 - 1, need_h = pz <= z1 - 1;
        const T *a1 = plane(0, d1, pz), *a2 = plane(1, d2, pz);
        const T *b1 = plane(2, e1, pz - 1), *b2 = plane(3, e2, pz - 1);
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            sd1[j][k] = need_d ? a1[goff[k]] : T(0);
            sd2[j][k] = need_d ? a2[goff[k]] : T(0);
            se1[j][k] = need_e ? b1[goff[k]] : T(0);
            se2[j][k] = need_e ? b2[goff[k]] : T(0);
        }
        srd1[j] = (hasr && need_d) ? a1[roff] : T(0);
        srd2[j] = (hasr && need_d) ? a2[roff] : T(0);
        sre1[j] = (hasr && need_e) ? b1[roff] : T(0);
        sre2[j] = (hasr && need_e) ? b2[roff] : T(0);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            sh1[j][m] = (hash[m] && need_h) ? a1[hoff[m]] : T(0);
            sh2[j][m] = (hash[m] && need_h) ? a2[hoff[m]] : T(0);
        }
    };
    {
        const T *m1 = plane(0, d1, z0 - 2), *m2 = plane(1, d2, z0 - 2);
        const T *c1p = plane(0, d1, z0 - 1), *c2p = plane(1, d2, z0 - 1);
        const T *p1 = plane(0, d1, z0), *p2 = plane(1, d2, z0);
        const T *f1 = plane(2, e1, z0 - 1), *f2 = plane(3, e2, z0 - 1);
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            qm1[k] = m1[goff[k]]; qm2[k] = m2[goff[k]];
            qc1[k] = c1p[goff[k]]; qc2[k] = c2p[goff[k]];
            qp1[k] = p1[goff[k]]; qp2[k] = p2[goff[k]];
            ev1[k] = f1[goff[k]]; ev2[k] = f2[goff[k]];
            dn1[k] = 0; dn2[k] = 0;
        }
        if (hasr) {
            rqm1 = m1[roff]; rqm2 = m2[roff];
            rqc1 = c1p[roff]; rqc2 = c2p[roff];
            rqp1 = p1[roff]; rqp2 = p2[roff];
            rev1 = f1[roff]; rev2 = f2[roff];
        }
#pragma unroll
        for (int j = 0; j + 1 < PF; ++j) fill(j, z0 + 1 + j);
        // stage plane z0-1 (buffer 0); the halo of plane z0 is staged next
#pragma unroll
        for (int k = 0; k < KI; ++k) { sd[0][0][lsd[k]] = qc1[k]; sd[0][1][lsd[k]] = qc2[k]; }
        if (hasr) { sd[0][0][rlsd] = rqc1; sd[0][1][rlsd] = rqc2; }
#pragma unroll
        for (int m = 0; m < 2; ++m)
            if (hash[m]) {
                sd[0][0][hlsd[m]] = c1p[hoff[m]];
                sd[0][1][hlsd[m]] = c2p[hoff[m]];
                hv1[m] = p1[hoff[m]];
                hv2[m] = p2[hoff[m]];
            }
        __syncthreads();
    }

    // The new values of plane z are stored at the top of iteration z+1, just
    // before its loads.  The memory counter retires in issue order, so a wait
    // for those loads then finds stores that have had a whole iteration to
    // drain.  Stores stream once: non-temporal, so L2 keeps the halo rows.
    T pe1[KI], pe2[KI], pd1[KI], pd2[KI];
    bool pend = false;
    int pz_st = 0;
    auto flush = [&]() {
        if (pend) {
            T *o_e1 = oplane(e1n, pz_st), *o_e2 = oplane(e2n, pz_st);
            T *o_d1 = oplane(d1n, pz_st), *o_d2 = oplane(d2n, pz_st);
#pragma unroll
            for (int k = 0; k < KI; ++k)
                if (act[k]) {
                    __builtin_nontemporal_store(pe1[k], o_e1 + goff[k]);
                    __builtin_nontemporal_store(pe2[k], o_e2 + goff[k]);
                    __builtin_nontemporal_store(pd1[k], o_d1 + goff[k]);
                    __builtin_nontemporal_store(pd2[k], o_d2 + goff[k]);
                }
        }
    };
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    int cur = 0;
    for (int z = z0 - 1; z < z1; ++z, cur ^= 1) {
        flush();
        // newest prefetch slot: d(z+1+PF), e(z+PF), halo(z+1+PF)
        fill(PF - 1, z + 1 + PF);

        const bool live = (z >= z0);
        const bool more = (z + 1 < z1);
        const T *s0 = sd[cur][0], *s1 = sd[cur][1];
        T *n0 = sn[cur][0], *n1 = sn[cur][1];
        T zd1[KI], zd2[KI];
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int l = lsd[k];
            const T sa = six_sum(s0[l - 1], s0[l + 1], s0[l - LW], s0[l + LW], qm1[k], qp1[k], qc1[k]);
            const T sb = six_sum(s1[l - 1], s1[l + 1], s1[l - LW], s1[l + LW], qm2[k], qp2[k], qc2[k]);
            T ia, ib;
            c.force(qc1[k], qc2[k], sa, sb, ia, ib);
            const T ea = ev1[k] + ia, eb = ev2[k] + ib;
            const T na = qc1[k] + c.dt * ea, nb = qc2[k] + c.dt * eb;
            pe1[k] = ea; pe2[k] = eb; pd1[k] = na; pd2[k] = nb;
            n0[lsn[k]] = na;
            n1[lsn[k]] = nb;
            zd1[k] = na - dn1[k];
            zd2[k] = nb - dn2[k];
            dn1[k] = na;
            dn2[k] = nb;
        }
        if (hasr) {
            const int l = rlsd;
            const T sa = six_sum(s0[l - 1], s0[l + 1], s0[l - LW], s0[l + LW], rqm1, rqp1, rqc1);
            const T sb = six_sum(s1[l - 1], s1[l + 1], s1[l - LW], s1[l + LW], rqm2, rqp2, rqc2);
            T ia, ib;
            c.force(rqc1, rqc2, sa, sb, ia, ib);
            n0[rlsn] = rqc1 + c.dt * (rev1 + ia);
            n1[rlsn] = rqc2 + c.dt * (rev2 + ib);
        }
        // stage plane z+1 into the other buffer (data loaded earlier)
        if (more) {
            T *t0 = sd[cur ^ 1][0], *t1 = sd[cur ^ 1][1];
#pragma unroll
            for (int k = 0; k < KI; ++k) { t0[lsd[k]] = qp1[k]; t1[lsd[k]] = qp2[k]; }
            if (hasr) { t0[rlsd] = rqp1; t1[rlsd] = rqp2; }
#pragma unroll
            for (int m = 0; m < 2; ++m)
                if (hash[m]) { t0[hlsd[m]] = hv1[m]; t1[hlsd[m]] = hv2[m]; }
        }
        __syncthreads();

        if (live) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                if (!act[k]) continue;
                const int l = lsn[k];
                const T na = n0[l], nb = n1[l];
                const double ax = (double)(na - n0[l - 1]), ay = (double)(na - n0[l - NW]);
                const double bx = (double)(nb - n1[l - 1]), by = (double)(nb - n1[l - NW]);
                const double az = (double)zd1[k], bz = (double)zd2[k];
                acc0 += ax * ax + ay * ay + az * az;
                acc1 += bx * bx + by * by + bz * bz;
                const double x1 = g1n + (double)na, x2 = g2n + (double)nb;
                acc2 += potential_pow<NH>(x1);
                acc3 += x1 * x1 * x2 * x2;
            }
        }

        pend = live;
        pz_st = z;
        // rotate the queues and the prefetch slots
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            qm1[k] = qc1[k]; qc1[k] = qp1[k]; qp1[k] = sd1[0][k];
            qm2[k] = qc2[k]; qc2[k] = qp2[k]; qp2[k] = sd2[0][k];
            ev1[k] = se1[0][k]; ev2[k] = se2[0][k];
        }
        rqm1 = rqc1; rqc1 = rqp1; rqp1 = srd1[0];
        rqm2 = rqc2; rqc2 = rqp2; rqp2 = srd2[0];
        rev1 = sre1[0]; rev2 = sre2[0];
        hv1[0] = sh1[0][0]; hv1[1] = sh1[0][1];
        hv2[0] = sh2[0][0]; hv2[1] = sh2[0][1];
#pragma unroll
        for (int j = 0; j + 1 < PF; ++j) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                sd1[j][k] = sd1[j + 1][k]; sd2[j][k] = sd2[j + 1][k];
                se1[j][k] = se1[j + 1][k]; se2[j][k] = se2[j + 1][k];
            }
            srd1[j] = srd1[j + 1]; srd2[j] = srd2[j + 1];
            sre1[j] = sre1[j + 1]; sre2[j] = sre2[j + 1];
            sh1[j][0] = sh1[j + 1][0]; sh1[j][1] = sh1[j + 1][1];
            sh2[j][0] = sh2[j + 1][0]; sh2[j][1] = sh2[j + 1][1];
        }
    }

    flush();
    // block partial sums, fixed order
    double v[4] = {acc0, acc1, acc2, acc3};
    __shared__ double red[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[i] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) red[i][w] = v[i];
    }
    __syncthreads();
    if (t < 4) part_row[t] = ((red[t][0] + red[t][1]) + red[t][2]) + red[t][3];
}

#ifndef LF_SWEEP_MIN_WAVES
#define LF_SWEEP_MIN_WAVES 4
#endif
// planes of loads in flight ahead of the plane being computed (1 or 2)
#ifndef LF_SWEEP_PREFETCH
#define LF_SWEEP_PREFETCH 1
#endif

// Single lattice (or z-slab of one: zp): one block per (tile, z-chunk),
// XCD-aware tile order.
template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP_MIN_WAVES) k_sweep_lds(
    const T *__restrict__ d1, const T *__restrict__ d2, const T *__restrict__ e1, const T *__restrict__ e2,
    T *__restrict__ d1n, T *__restrict__ d2n, T *__restrict__ e1n, T *__restrict__ e2n, const int N,
    const ZPlanes<T> zp, const int zchunk, const int ntx, const int nty, const CoefPair *__restrict__ C,
    double *__restrict__ part)
{
    // partial row = logical tile index (the ensemble kernel uses the same rows)
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, b = tile / ntx;
    const int ty = b % nty;
    const int tz = b / nty;
    const int z0 = tz * zchunk;
    sweep_tile<T, NH, TX, TY, LF_SWEEP_PREFETCH>(d1, d2, e1, e2, d1n, d2n, e1n, e2n, N, zp, tx * TX, ty * TY,
                                                 z0, min(z0 + zchunk, zp.nz), C, part + (size_t)tile * kNPart);
}

// Ensemble: a persistent grid walks a static list of work items
// (realization, tile, z-chunk); item i writes partial row i of its
// realization's row range.  All realizations advance one step per launch.
template <typename T, int NH, int TX, int TY>
__global__ void __launch_bounds__(256, LF_SWEEP_MIN_WAVES) k_sweep_ens(
    const EnsEntry *__restrict__ tab, const int4 *__restrict__ items, const int nitems, const int parity)
{
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int4 it = items[i];  // x: realization, y: tile index within it, z: partial row
        const EnsEntry &e = tab[it.x];
        const int tx = it.y % e.ntx, r2 = it.y / e.ntx, ty = r2 % e.nty, tz = r2 / e.nty;
        const int z0 = tz * e.zchunk;
        const T *const *in = (const T *const *)e.buf[parity];
        T *const *out = (T *const *)e.buf[parity ^ 1];
        const ZPlanes<T> zp = periodic_planes<T>(in, e.N);
        sweep_tile<T, NH, TX, TY, LF_SWEEP_PREFETCH>(in[0], in[1], in[2], in[3], out[0], out[1], out[2], out[3], e.N,
                                                     zp, tx * TX, ty * TY, z0, min(z0 + e.zchunk, e.N), e.C,
                                                     e.part + (size_t)it.z * kNPart);
        __syncthreads();  // LDS is reused by the next item
    }
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

SweepIO periodic_io(int dtype, const void *const in[4], void *const out[4], int N)
{
    SweepIO io{};
    const int64_t plane_bytes = (int64_t)N * N * (dtype == 0 ? 4 : 8);
    for (int i = 0; i < 4; ++i) {
        io.in[i] = in[i];
        io.lo[i] = (const char *)in[i] + (N - 2) * plane_bytes;
        io.hi[i] = in[i];
        io.out[i] = out[i];
    }
    io.nz = N;
    return io;
}

template <typename T, int NH, int TX, int TY>
static void sweep_lds_t(const SweepIO &io, int N, int zchunk, const CoefPair *C, double *part, hipStream_t st)
{
    const int ntx = (N + TX - 1) / TX, nty = (N + TY - 1) / TY, nzc = (io.nz + zchunk - 1) / zchunk;
    hipLaunchKernelGGL((k_sweep_lds<T, NH, TX, TY>), dim3(ntx * nty * nzc), dim3(256), 0, st,
                       (const T *)io.in[0], (const T *)io.in[1], (const T *)io.in[2], (const T *)io.in[3],
                       (T *)io.out[0], (T *)io.out[1], (T *)io.out[2], (T *)io.out[3], N, planes_of<T>(io),
                       zchunk, ntx, nty, C, part);
}

template <typename T, int TX, int TY>
static void sweep_lds_b(int beta, const SweepIO &io, int N, int zchunk, const CoefPair *C, double *part,
                        hipStream_t st)
{
    switch (beta) {
    case 2: sweep_lds_t<T, 1, TX, TY>(io, N, zchunk, C, part, st); break;
    case 3: sweep_lds_t<T, 2, TX, TY>(io, N, zchunk, C, part, st); break;
    case 4: sweep_lds_t<T, 3, TX, TY>(io, N, zchunk, C, part, st); break;
    case 5: sweep_lds_t<T, 4, TX, TY>(io, N, zchunk, C, part, st); break;
    default: sweep_lds_t<T, 5, TX, TY>(io, N, zchunk, C, part, st); break;
    }
}

// Supported tiles (x by y): 64x4, 64x8, 64x16, 128x4, 128x8.
template <typename T>
static void sweep_lds_y(int tile_x, int tile_y, int beta, const SweepIO &io, int N, int zchunk,
                        const CoefPair *C, double *part, hipStream_t st)
{
    if (tile_x == 128) {
        if (tile_y == 4) sweep_lds_b<T, 128, 4>(beta, io, N, zchunk, C, part, st);
        else sweep_lds_b<T, 128, 8>(beta, io, N, zchunk, C, part, st);
        return;
    }
    switch (tile_y) {
    case 4: sweep_lds_b<T, 64, 4>(beta, io, N, zchunk, C, part, st); break;
    case 8: sweep_lds_b<T, 64, 8>(beta, io, N, zchunk, C, part, st); break;
    default: sweep_lds_b<T, 64, 16>(beta, io, N, zchunk, C, part, st); break;
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
static void sweep_ens_t(const EnsEntry *tab, const int4 *items, int nitems, int grid, int parity,
                        hipStream_t st)
{
    hipLaunchKernelGGL((k_sweep_ens<T, NH, TX, TY>), dim3(grid), dim3(256), 0, st, tab, items, nitems, parity);
}

template <typename T, int TX, int TY>
static void sweep_ens_b(int beta, const EnsEntry *tab, const int4 *items, int nitems, int grid,
                        int parity, hipStream_t st)
{
    switch (beta) {
    case 2: sweep_ens_t<T, 1, TX, TY>(tab, items, nitems, grid, parity, st); break;
    case 3: sweep_ens_t<T, 2, TX, TY>(tab, items, nitems, grid, parity, st); break;
    case 4: sweep_ens_t<T, 3, TX, TY>(tab, items, nitems, grid, parity, st); break;
    case 5: sweep_ens_t<T, 4, TX, TY>(tab, items, nitems, grid, parity, st); break;
    default: sweep_ens_t<T, 5, TX, TY>(tab, items, nitems, grid, parity, st); break;
    }
}

template <typename T>
static void sweep_ens_y(int tile_x, int tile_y, int beta, const EnsEntry *tab, const int4 *items,
                        int nitems, int grid, int parity, hipStream_t st)
{
    if (tile_x == 128) {
        if (tile_y == 4) sweep_ens_b<T, 128, 4>(beta, tab, items, nitems, grid, parity, st);
        else sweep_ens_b<T, 128, 8>(beta, tab, items, nitems, grid, parity, st);
        return;
    }
    switch (tile_y) {
    case 4: sweep_ens_b<T, 64, 4>(beta, tab, items, nitems, grid, parity, st); break;
    case 8: sweep_ens_b<T, 64, 8>(beta, tab, items, nitems, grid, parity, st); break;
    default: sweep_ens_b<T, 64, 16>(beta, tab, items, nitems, grid, parity, st); break;
    }
}

void launch_sweep_ens(int stencil, int dtype, int tile_x, int tile_y, int beta, const EnsEntry *tab,
                      const int4 *items, int nitems, int grid, int parity, hipStream_t st)
{
    if (stencil == 27) launch_sweep_ens27(dtype, tile_x, tile_y, beta, tab, items, nitems, grid, parity, st);
    else if (dtype == 0) sweep_ens_y<float>(tile_x, tile_y, beta, tab, items, nitems, grid, parity, st);
    else sweep_ens_y<double>(tile_x, tile_y, beta, tab, items, nitems, grid, parity, st);
}

void launch_sweep_io(int stencil, int dtype, int tile_x, int tile_y, int beta, const SweepIO &io, int N,
                     int zchunk, const CoefPair *C, double *part, hipStream_t st)
{
    if (stencil == 27) launch_sweep_lds27(dtype, tile_x, tile_y, beta, io, N, zchunk, C, part, st);
    else if (dtype == 0) sweep_lds_y<float>(tile_x, tile_y, beta, io, N, zchunk, C, part, st);
    else sweep_lds_y<double>(tile_x, tile_y, beta, io, N, zchunk, C, part, st);
}

void launch_sweep_lds(int stencil, int dtype, int tile_x, int tile_y, int beta, const void *const in[4],
                      void *const out[4], int N, int zchunk, const CoefPair *C, double *part,
                      hipStream_t st)
{
    launch_sweep_io(stencil, dtype, tile_x, tile_y, beta, periodic_io(dtype, in, out, N), N, zchunk, C, part,
                    st);
}

}  // namespace lf
