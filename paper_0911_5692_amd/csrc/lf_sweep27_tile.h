// The LDS z-march of the 27-point sweep: one block's tile over a chunk of
// z-planes (Sainio, arXiv:0911.5692, Sec. II.C; the design is described at
// the top of lf_sweep27.hip), the occupancy rule of its kernels and the
// launch-shape dispatch helpers.  Included by lf_sweep27.hip (periodic
// lattice, ensemble) and lf_slab27.hip (z-slab with halo planes).
#pragma once
#include "lf_sweep_common.h"

#include <type_traits>

namespace lf {

namespace {

// Element at a 32-bit unsigned byte offset from a uniform base: lets the
// compiler address global memory as SGPR base + VGPR offset.
template <typename T>
__device__ inline T ld_at(const T *base, unsigned boff)
{
    return *(const T *)((const char *)base + boff);
}
template <typename T>
__device__ inline void st_nt(T v, T *base, unsigned boff)
{
    __builtin_nontemporal_store(v, (T *)((char *)base + boff));
}

// Elements of an LDS plane of n elements padded to a multiple of 256 bytes.
template <typename T>
constexpr int lds_plane(int n)
{
    return (n * (int)sizeof(T) + 255) / 256 * 256 / (int)sizeof(T);
}

// One block's work: tile (x0, y0) of an N^3 lattice (SLAB = false, periodic
// in z) or of an N x N x zp.nz slab whose outside planes come from halo
// buffers (SLAB = true) over planes [z0, z1), writing its four partial sums
// to part_row[0..3].
template <typename T, int NH, int TX, int TY, bool SLAB>
__device__ __forceinline__ void sweep_tile27(const T *__restrict__ d1, const T *__restrict__ d2,
                                             const T *__restrict__ e1, const T *__restrict__ e2,
                                             T *__restrict__ d1n, T *__restrict__ d2n,
                                             T *__restrict__ e1n, T *__restrict__ e2n, const int N,
                                             const ZPlanes<T> zp,
                                             const int x0, const int y0, const int z0, const int z1,
                                             const CoefPair *__restrict__ C, double *__restrict__ part_row)
{
    constexpr int RPR = 256 / TX;                // rows per round of 256 threads
    constexpr int KI = TY / RPR;                 // interior sites per thread per plane
    constexpr int LW = TX + 4, LH = TY + 3;      // staged plane: x0-2 .. x0+TX+1, y0-2 .. y0+TY
    constexpr int NW = TX + 2, NHT = TY + 1;     // new values: x0-1 .. x0+TX, y0-1 .. y0+TY-1
    constexpr int NRING = TX + 2 + TY;           // row y0-1 (x0-1 .. x0+TX), column x0-1 (y0 ..)
    constexpr int NHALO = 2 * (TX + 4) + 3 * TY + 2;
    static_assert(256 % TX == 0 && TY % RPR == 0 && NRING <= 256 && NHALO <= 512, "tile shape");
    // staged planes: plane z+1 is read from one buffer while z+2 is written
    // to the next; new values: plane z written, z-1 read after the barrier.
    // Both rotate over three buffers, so that three iterations bring every
    // buffer index back (see step below)
    // Each plane is padded to a multiple of 256 bytes, so that a slot of one
    // plane lies a multiple of 64 elements from the same slot of any other:
    // reads of one site in both fields or in planes z and z-1 then pair into
    // ds_read2st64 from one address (28% fewer LDS instructions)
    __shared__ T sd[3][2][lds_plane<T>(LH * LW)];
    __shared__ T sn[3][2][lds_plane<T>(NHT * NW)];

    Coefs<T, NH> c;
    c.load(coef_of<T>(C));
    const double g1n = C->g1n, g2n = C->g2n;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t NN = (int64_t)N * N;
    auto wrapc = [N](int v) { return ((v % N) + N) % N; };
    const int wv = min(TX, N - x0), hv = min(TY, N - y0);  // valid interior extent

    // interior sites (x0 + t % TX, y0 + t / TX + RPR k)
    unsigned goff[KI];  // byte offsets within a plane
    int lsd[KI], lsn[KI];
    bool act[KI];
    // bonds that may leave the interior and ring: (+1,-1) in planes z and
    // z-1, (+1,0), (0,+1), (-1,+1), (+1,+1) in plane z-1.  Index of the
    // neighbour's slot, or of the site's own slot when the bond is not this
    // block's, and a 0/1 multiplier of the difference
    int ix4[KI], ixx[KI], ixy[KI], ixyl[KI], ixxy[KI];
    T m4[KI], mx[KI], my[KI], mxy[KI];
    const int cx = t % TX, cy = t / TX;
    const int xi = x0 + cx;
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int yl = cy + RPR * k;
        const int y = y0 + yl;
        act[k] = (xi < N) && (y < N);
        goff[k] = (unsigned)((y % N) * N + (xi % N)) * sizeof(T);  // in-bounds even when inactive
        lsd[k] = (yl + 2) * LW + cx + 2;
        lsn[k] = (yl + 1) * NW + cx + 1;
        const bool okx = cx + 1 < wv;        // (cx+1, yl) is interior
        const bool oky = yl + 1 < hv;        // (cx, yl+1) is interior
        const bool ok4 = (yl == 0) || okx;   // (cx+1, yl-1) is interior or ring
        const int l = lsn[k];
        ix4[k] = ok4 ? l - NW + 1 : l;
        ixx[k] = okx ? l + 1 : l;
        ixy[k] = oky ? l + NW : l;
        ixyl[k] = oky ? l + NW - 1 : l;
        ixxy[k] = (okx && oky) ? l + NW + 1 : l;
        m4[k] = ok4 ? T(1) : T(0);
        mx[k] = okx ? T(1) : T(0);
        my[k] = oky ? T(1) : T(0);
        mxy[k] = (okx && oky) ? T(1) : T(0);
    }
    // ring site of this thread (t < NRING): new value only, never stored
    const bool hasr = t < NRING;
    const bool rrow = t < TX + 2;
    const int rlx = rrow ? t - 1 : -1, rly = rrow ? -1 : t - (TX + 2);
    unsigned roff = hasr ? (unsigned)(wrapc(y0 + rly) * N + wrapc(x0 + rlx)) * sizeof(T) : 0u;
    const int rlsd = hasr ? (rly + 2) * LW + rlx + 2 : 0;
    const int rlsn = hasr ? (rly + 1) * NW + rlx + 1 : 0;
    // the ring's bonds into the interior: three to plane z-1 (index rq,
    // validity rv; the middle one an edge, the outer two corners) and, for
    // the ring column, one in-plane edge (rqi, rvi)
    int rq[3], rqi = rlsn;
    T rv[3], rvi = T(0);  // 0/1 multipliers
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        bool ok;
        if (rrow) {
            const int x = rlx + j - 1;  // interior (x, 0)
            ok = hasr && x >= 0 && x < wv;
            rq[j] = ok ? NW + x + 1 : rlsn;
        } else {
            const int y = rly + j - 1;  // interior (0, y)
            ok = hasr && rly < hv && y >= 0 && y < hv;
            rq[j] = ok ? (y + 1) * NW + 1 : rlsn;
        }
        rv[j] = ok ? T(1) : T(0);
    }
    if (hasr && !rrow && rly >= 1 && rly < hv) {
        rvi = T(1);
        rqi = rly * NW + 1;  // interior (0, rly - 1)
    }
    // halo cells of this thread (t and t + 256 below NHALO): staged-plane
    // border that no computed site covers
    bool hash[2];
    unsigned hoff[2];
    int hlsd[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int hc = t + 256 * m;
        hash[m] = hc < NHALO;
        int hlx, hly;  // local coordinates
        if (hc < TX + 4) { hlx = hc - 2; hly = -2; }
        else if (hc < 2 * (TX + 4)) { hlx = hc - (TX + 4) - 2; hly = TY; }
        else if (hc < 2 * (TX + 4) + TY + 1) { hlx = -2; hly = hc - 2 * (TX + 4) - 1; }
        else if (hc < 2 * (TX + 4) + 2 * (TY + 1)) { hlx = TX + 1; hly = hc - 2 * (TX + 4) - (TY + 1) - 1; }
        else { hlx = TX; hly = hc - 2 * (TX + 4) - 2 * (TY + 1); }
        if (!hash[m]) { hlx = 0; hly = 0; }
        hoff[m] = (unsigned)(wrapc(y0 + hly) * N + wrapc(x0 + hlx)) * sizeof(T);
        hlsd[m] = (hly + 2) * LW + hlx + 2;
    }
    // plane base pointers (uniform).  Inputs: d is read on planes
    // [z0 - 2, z1], e on [z0 - 1, z1 - 1], so on the periodic lattice one
    // conditional wrap suffices; outputs: planes [z0, z1)
    auto plane = [&](int i, const T *p, int z) {
        if constexpr (SLAB) {
            return zp.at(i, p, z, NN);
        } else {
            const int zw = z < 0 ? z + N : (z >= N ? z - N : z);
            return p + (int64_t)zw * NN;
        }
    };
    auto oplane = [&](T *p, int z) { return p + (int64_t)z * NN; };

    // Registers per site and field: d(z) qc, d(z+1) qp, d(z+2) nd (staged this
    // iteration), e(z) ev, partial sums A(z-1) am, A(z) ac, B(z) bc; loads in
    // flight for the next iteration: d(z+3) ld, e(z+1) le, halo(z+3) lh.
    T qc1[KI], qp1[KI], nd1[KI], ld1[KI], ev1[KI], le1[KI], am1[KI], ac1[KI], bc1[KI];
    T qc2[KI], qp2[KI], nd2[KI], ld2[KI], ev2[KI], le2[KI], am2[KI], ac2[KI], bc2[KI];
    T rqc1 = 0, rqp1 = 0, rnd1 = 0, rld1 = 0, rev1 = 0, rle1 = 0, ram1 = 0, rac1 = 0, rbc1 = 0;
    T rqc2 = 0, rqp2 = 0, rnd2 = 0, rld2 = 0, rev2 = 0, rle2 = 0, ram2 = 0, rac2 = 0, rbc2 = 0;
    T hv1[2] = {0, 0}, hv2[2] = {0, 0}, lh1[2] = {0, 0}, lh2[2] = {0, 0};

    const int zs = z0 - 3;  // first iteration: plane z0-2 staged
    {
        const T *a1 = plane(0, d1, z0 - 2), *a2 = plane(1, d2, z0 - 2);
        const T *b1 = plane(0, d1, z0 - 1), *b2 = plane(1, d2, z0 - 1);
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            qp1[k] = ld_at(a1, goff[k]); qp2[k] = ld_at(a2, goff[k]);
            nd1[k] = ld_at(b1, goff[k]); nd2[k] = ld_at(b2, goff[k]);
            qc1[k] = 0; qc2[k] = 0; ev1[k] = 0; ev2[k] = 0;
            am1[k] = 0; am2[k] = 0; ac1[k] = 0; ac2[k] = 0; bc1[k] = 0; bc2[k] = 0;
            sd[0][0][lsd[k]] = qp1[k];
            sd[0][1][lsd[k]] = qp2[k];
        }
        if (hasr) {
            rqp1 = ld_at(a1, roff); rqp2 = ld_at(a2, roff);
            rnd1 = ld_at(b1, roff); rnd2 = ld_at(b2, roff);
            sd[0][0][rlsd] = rqp1;
            sd[0][1][rlsd] = rqp2;
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
            if (hash[m]) {
                sd[0][0][hlsd[m]] = ld_at(a1, hoff[m]);
                sd[0][1][hlsd[m]] = ld_at(a2, hoff[m]);
                hv1[m] = ld_at(b1, hoff[m]);
                hv2[m] = ld_at(b2, hoff[m]);
            }
        __syncthreads();
    }

    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    // The new values of plane z are stored at the top of iteration z+1, just
    // before its loads.  The memory counter retires in issue order, so the
    // wait for those loads at the end of the iteration then finds stores that
    // have had a whole iteration to drain, not ones issued a moment before.
    // Stores stream once: non-temporal, so L2 keeps the halo rows instead.
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
                    st_nt(pe1[k], o_e1, goff[k]);
                    st_nt(pe2[k], o_e2, goff[k]);
                    st_nt(pd1[k], o_d1, goff[k]);
                    st_nt(pd2[k], o_d2, goff[k]);
                }
        }
    };
    // One iteration at phase PH of the buffer rotation: staged plane sd[PH]
    // (plane z+2 goes to sd[(PH + 1) % 3]), new-value planes sn[PH] (plane z)
    // and sn[(PH + 2) % 3] (plane z-1).
    // The phase is a compile-time constant, so every LDS address is a
    // loop-invariant register plus an immediate offset.
    auto step = [&](auto phase, const int z) __attribute__((always_inline)) {
        constexpr int PH = decltype(phase)::value;
        constexpr int cur = PH, nxt = (PH + 1) % 3, nb_cur = PH, nb_prev = (PH + 2) % 3;
        // the byte offsets pass through an empty asm once per iteration, so
        // the compiler forms each address as SGPR plane base + this VGPR
        // (no 64-bit address arithmetic per access)
#pragma unroll
        for (int k = 0; k < KI; ++k) asm volatile("" : "+v"(goff[k]));
        asm volatile("" : "+v"(roff));
        asm volatile("" : "+v"(hoff[0]), "+v"(hoff[1]));
        flush();
        // loads for the next iteration: d(z+3), halo(z+3), e(z+1)
        {
            // unconditional loads (no branch to delay their issue): the plane
            // index is clamped into the chunk's range, and values of planes the
            // chunk does not need are never used
            const int pz = min(z + 3, z1);
            const int pe = min(max(z + 1, z0 - 1), z1 - 1);
            const T *a1 = plane(0, d1, pz), *a2 = plane(1, d2, pz);
            const T *b1 = plane(2, e1, pe), *b2 = plane(3, e2, pe);
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                ld1[k] = ld_at(a1, goff[k]);
                ld2[k] = ld_at(a2, goff[k]);
                le1[k] = ld_at(b1, goff[k]);
                le2[k] = ld_at(b2, goff[k]);
            }
            rld1 = ld_at(a1, roff);
            rld2 = ld_at(a2, roff);
            rle1 = ld_at(b1, roff);
            rle2 = ld_at(b2, roff);
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                lh1[m] = ld_at(a1, hoff[m]);
                lh2[m] = ld_at(a2, hoff[m]);
            }
        }

        const bool live = z >= z0;  // plane z is stored and reduced (z0-1 only feeds the reductions)
        const T *s0 = sd[cur][0], *s1 = sd[cur][1];
        T *n0 = sn[nb_cur][0], *n1 = sn[nb_cur][1];
        T an1[KI], an2[KI], bn1[KI], bn2[KI], na1[KI], na2[KI];
        // partial sums of the staged plane z+1 (explicit fma: the ring
        // sites below repeat the same expression, so a ring value equals the
        // neighbouring tile's stored value bitwise), and the update of plane z
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int l = lsd[k];
            const T f1 = (s0[l - 1] + s0[l + 1]) + (s0[l - LW] + s0[l + LW]);
            const T g1 = (s0[l - LW - 1] + s0[l - LW + 1]) + (s0[l + LW - 1] + s0[l + LW + 1]);
            const T f2 = (s1[l - 1] + s1[l + 1]) + (s1[l - LW] + s1[l + LW]);
            const T g2 = (s1[l - LW - 1] + s1[l - LW + 1]) + (s1[l + LW - 1] + s1[l + LW + 1]);
            an1[k] = fma(T(14), qp1[k], fma(T(3), f1, g1));
            bn1[k] = fma(T(-128), qp1[k], fma(T(14), f1, T(3) * g1));
            an2[k] = fma(T(14), qp2[k], fma(T(3), f2, g2));
            bn2[k] = fma(T(-128), qp2[k], fma(T(14), f2, T(3) * g2));
            T ia, ib;
            c.force_fma(qc1[k], qc2[k], (bc1[k] + am1[k]) + an1[k], (bc2[k] + am2[k]) + an2[k], ia, ib);
            const T ea = ev1[k] + ia, eb = ev2[k] + ib;
            na1[k] = fma(c.dt, ea, qc1[k]);
            na2[k] = fma(c.dt, eb, qc2[k]);
            pe1[k] = ea; pe2[k] = eb; pd1[k] = na1[k]; pd2[k] = na2[k];
            // planes below z0-1 are written too: their slots are rewritten
            // before the first read
            n0[lsn[k]] = na1[k];
            n1[lsn[k]] = na2[k];
        }
        T rna1 = 0, rna2 = 0, ran1 = 0, ran2 = 0, rbn1 = 0, rbn2 = 0;
        if (hasr) {
            const int l = rlsd;
            const T f1 = (s0[l - 1] + s0[l + 1]) + (s0[l - LW] + s0[l + LW]);
            const T g1 = (s0[l - LW - 1] + s0[l - LW + 1]) + (s0[l + LW - 1] + s0[l + LW + 1]);
            const T f2 = (s1[l - 1] + s1[l + 1]) + (s1[l - LW] + s1[l + LW]);
            const T g2 = (s1[l - LW - 1] + s1[l - LW + 1]) + (s1[l + LW - 1] + s1[l + LW + 1]);
            ran1 = fma(T(14), rqp1, fma(T(3), f1, g1));
            rbn1 = fma(T(-128), rqp1, fma(T(14), f1, T(3) * g1));
            ran2 = fma(T(14), rqp2, fma(T(3), f2, g2));
            rbn2 = fma(T(-128), rqp2, fma(T(14), f2, T(3) * g2));
            T ia, ib;
            c.force_fma(rqc1, rqc2, (rbc1 + ram1) + ran1, (rbc2 + ram2) + ran2, ia, ib);
            rna1 = fma(c.dt, rev1 + ia, rqc1);
            rna2 = fma(c.dt, rev2 + ib, rqc2);
            n0[rlsn] = rna1;
            n1[rlsn] = rna2;
        }
        // stage plane z+2 into the other buffer (loaded one iteration ago;
        // past z1 the registers repeat a clamped plane and the buffer is not
        // read again)
        {
            T *t0 = sd[nxt][0], *t1 = sd[nxt][1];
#pragma unroll
            for (int k = 0; k < KI; ++k) { t0[lsd[k]] = nd1[k]; t1[lsd[k]] = nd2[k]; }
            if (hasr) { t0[rlsd] = rnd1; t1[rlsd] = rnd2; }
#pragma unroll
            for (int m = 0; m < 2; ++m)
                if (hash[m]) { t0[hlsd[m]] = hv1[m]; t1[hlsd[m]] = hv2[m]; }
        }
        __syncthreads();

        if (live) {
            const T *p0 = sn[nb_cur][0], *p1 = sn[nb_cur][1];      // plane z
            const T *m0 = sn[nb_prev][0], *m1 = sn[nb_prev][1];    // plane z-1
            // bonds of interior site k; a bond that is not this block's
            // reads the site's own slot and is multiplied by 0 (no branch)
            // The sums of squares are written as explicit fma chains: the
            // three phase copies of this loop then round a site's term
            // identically, so the step sums do not depend on where a chunk
            // starts (left to contraction, they differed in FP32 in the
            // last bits).
            auto bonds = [&](const T *P, const T *M, const int l, const T v, const int k) {
                auto df = [&](T u) { return v - u; };
                auto dm = [&](T u, T msk) { return (v - u) * msk; };
                const T f0 = df(P[l - 1]), f1 = df(P[l - NW]), f2 = df(M[l]);
                const T F = fma(f0, f0, fma(f1, f1, f2 * f2));
                // a (+1,-1) bond that is not the block's reads the site's own
                // slot of plane z, which holds v: its difference is exactly 0
                const T e0 = df(P[l - NW - 1]), e1 = df(P[ix4[k]]), e2 = df(M[l - 1]), e3 = df(M[l - NW]);
                const T e4 = dm(M[ixx[k]], mx[k]), e5 = dm(M[ixy[k]], my[k]);
                const T E = fma(e0, e0, fma(e1, e1, fma(e2, e2, fma(e3, e3, fma(e4, e4, e5 * e5)))));
                const T c0 = df(M[l - NW - 1]), c1 = dm(M[ix4[k]], m4[k]);
                const T c2 = dm(M[ixyl[k]], my[k]), c3 = dm(M[ixxy[k]], mxy[k]);
                const T Cn = fma(c0, c0, fma(c1, c1, fma(c2, c2, c3 * c3)));
                return (double)fma(T(14), F, fma(T(3), E, Cn));
            };
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                if (!act[k]) continue;
                const int l = lsn[k];
                acc0 += bonds(p0, m0, l, na1[k], k);
                acc1 += bonds(p1, m1, l, na2[k], k);
                const double x1 = g1n + (double)na1[k], x2 = g2n + (double)na2[k];
                acc2 += potential_pow<NH>(x1);
                acc3 += x1 * x1 * x2 * x2;
            }
            if (hasr) {
                // bonds that are not this block's read the ring's own slot
                // (rq, rqi = rlsn) and are multiplied by 0
                auto rb = [&](const T *P, const T *M, const T v) {
                    auto dm = [&](T u, T msk) { return (v - u) * msk; };
                    const T e0 = dm(M[rq[1]], rv[1]), e1 = dm(P[rqi], rvi);
                    const T c0 = dm(M[rq[0]], rv[0]), c1 = dm(M[rq[2]], rv[2]);
                    const T E = fma(e0, e0, e1 * e1), Cn = fma(c0, c0, c1 * c1);
                    return (double)fma(T(3), E, Cn);
                };
                acc0 += rb(p0, m0, rna1);
                acc1 += rb(p1, m1, rna2);
            }
        }

        // rotate the queues
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            am1[k] = ac1[k]; ac1[k] = an1[k]; bc1[k] = bn1[k];
            am2[k] = ac2[k]; ac2[k] = an2[k]; bc2[k] = bn2[k];
            qc1[k] = qp1[k]; qp1[k] = nd1[k]; nd1[k] = ld1[k];
            qc2[k] = qp2[k]; qp2[k] = nd2[k]; nd2[k] = ld2[k];
            ev1[k] = le1[k]; ev2[k] = le2[k];
        }
        ram1 = rac1; rac1 = ran1; rbc1 = rbn1;
        ram2 = rac2; rac2 = ran2; rbc2 = rbn2;
        rqc1 = rqp1; rqp1 = rnd1; rnd1 = rld1;
        rqc2 = rqp2; rqp2 = rnd2; rnd2 = rld2;
        rev1 = rle1; rev2 = rle2;
#pragma unroll
        for (int m = 0; m < 2; ++m) { hv1[m] = lh1[m]; hv2[m] = lh2[m]; }
        pend = live;
        pz_st = z;
    };
    // three iterations (a full rotation period) per trip, then up to two more
    using std::integral_constant;
    int z = zs;
    for (; z + 3 <= z1; z += 3) {
        step(integral_constant<int, 0>{}, z);
        step(integral_constant<int, 1>{}, z + 1);
        step(integral_constant<int, 2>{}, z + 2);
    }
    if (z < z1) {
        step(integral_constant<int, 0>{}, z);
        if (z + 1 < z1) step(integral_constant<int, 1>{}, z + 1);
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

// Calls f.template operator()<NH>() for the beta of the model.
template <typename F>
void with_nh(int beta, F &&f)
{
    switch (beta) {
    case 2: f(std::integral_constant<int, 1>{}); break;
    case 3: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 3>{}); break;
    case 5: f(std::integral_constant<int, 4>{}); break;
    default: f(std::integral_constant<int, 5>{}); break;
    }
}

// Calls f(TX, TY) as integral constants for the supported tiles
// 64x4, 64x8, 64x16, 128x4, 128x8.
template <typename F>
void with_tile(int tile_x, int tile_y, F &&f)
{
    using std::integral_constant;
    if (tile_x == 128) {
        if (tile_y == 4) f(integral_constant<int, 128>{}, integral_constant<int, 4>{});
        else f(integral_constant<int, 128>{}, integral_constant<int, 8>{});
        return;
    }
    switch (tile_y) {
    case 4: f(integral_constant<int, 64>{}, integral_constant<int, 4>{}); break;
    case 8: f(integral_constant<int, 64>{}, integral_constant<int, 8>{}); break;
    default: f(integral_constant<int, 64>{}, integral_constant<int, 16>{}); break;
    }
}

}  // namespace

// Waves per SIMD to compile for: as many blocks as the LDS of a CU (160 KB)
// holds, each block one wave per SIMD, at most LF_SWEEP27_MIN_WAVES in FP32
// and 2 in FP64 (which needs more registers).
#ifndef LF_SWEEP27_MIN_WAVES
#define LF_SWEEP27_MIN_WAVES 3
#endif
template <typename T, int TX, int TY>
constexpr int sweep27_waves()
{
    constexpr int lds = (int)sizeof(T) * 3 * 2 * (lds_plane<T>((TY + 3) * (TX + 4)) + lds_plane<T>((TY + 1) * (TX + 2)));
    constexpr int by_lds = 160 * 1024 / lds;
    constexpr int by_regs = sizeof(T) == 4 ? LF_SWEEP27_MIN_WAVES : 2;
    return by_lds < by_regs ? (by_lds < 1 ? 1 : by_lds) : by_regs;
}
#define LF_SWEEP27_WAVES(T) (sweep27_waves<T, TX, TY>())

}  // namespace lf
