// The LDS z-march of the 7-point sweep: one block's tile over a chunk of
// z-planes (Sainio, arXiv:0911.5692, eq. evo with the 6-neighbour Laplacian;
// the design is described at the top of lf_sweep.hip).  Included by
// lf_sweep.hip (periodic lattice, ensemble) and lf_slab7.hip (z-slab with
// halo planes).
#pragma once
#include "lf_sweep_common.h"

#ifndef LF_SWEEP_MIN_WAVES
#define LF_SWEEP_MIN_WAVES 4
#endif
// planes of loads in flight ahead of the plane being computed (1 or 2)
#ifndef LF_SWEEP_PREFETCH
#define LF_SWEEP_PREFETCH 1
#endif

namespace lf {

// One block's work: the tile x0.., y0.. of an N^3 lattice (SLAB = false,
// periodic in z) or of an N x N x zp.nz slab whose outside planes come from
// halo buffers (SLAB = true) over planes [z0, z1), writing its four partial
// sums to part_row[0..3].
template <typename T, int NH, int TX, int TY, int PF, bool SLAB>
__device__ __forceinline__ void sweep_tile(const T *__restrict__ d1, const T *__restrict__ d2,
                                           const T *__restrict__ e1, const T *__restrict__ e2,
                                           T *__restrict__ d1n, T *__restrict__ d2n,
                                           T *__restrict__ e1n, T *__restrict__ e2n, const int N,
                                           const ZPlanes<T> zp,
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
    // addressed but not read), so on the periodic lattice one conditional
    // wrap suffices; outputs: planes [z0, z1)
    auto plane = [&](int i, const T *p, int z) {
        if constexpr (SLAB) {
            return zp.at(i, p, z, NN);
        } else {
            const int zw = z < 0 ? z + N : (z >= N ? z - N : z);
            return p + (int64_t)zw * NN;
        }
    };
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

}  // namespace lf
