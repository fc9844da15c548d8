// Per-site arithmetic shared by the LDS sweeps of liblf (7-point in
// lf_sweep.hip, 27-point in lf_sweep27.hip): the uniform kick coefficients,
// the force with the potential difference expanded around the FP64
// background, and the XCD-aware block order.
#pragma once
#include "lf_internal.h"

namespace lf {

template <typename T>
__device__ inline const Coef<T> &coef_of(const CoefPair *C);
template <>
__device__ inline const Coef<float> &coef_of<float>(const CoefPair *C) { return C->f; }
template <>
__device__ inline const Coef<double> &coef_of<double>(const CoefPair *C) { return C->d; }

// Uniform per-step coefficients, read once per block (scalar loads).
template <typename T, int NH>
struct Coefs {
    T Cl, Cf, dt, C2, g1, g2, two_g1, two_g2, g1sq;
    T h[NH];
    __device__ inline void load(const Coef<T> &c)
    {
        Cl = c.Cl; Cf = c.Cf; dt = c.dt; C2 = c.C2; g1 = c.g1; g2 = c.g2;
        two_g1 = c.two_g1; two_g2 = c.two_g2; g1sq = c.g1sq;
#pragma unroll
        for (int j = 0; j < NH; ++j) h[j] = c.h[j];
    }
    // Velocity increments of both fields at one site from the raw stencil
    // sums (s6a, s6b: the integer-weighted neighbour sum including the centre
    // term; Cl carries 1/dx^2 and the stencil weight) and the deviations
    // a = d1, b = d2.
    __device__ inline void force(T a, T b, T s6a, T s6b, T &inc_a, T &inc_b) const
    {
        T hor = h[NH - 1];
#pragma unroll
        for (int j = NH - 2; j >= 0; --j) hor = hor * a + h[j];
        const T t2 = g2 + b;
        const T dv1 = hor * a + C2 * (a * t2 * t2 + g1 * b * (two_g2 + b));
        const T dv2 = C2 * (a * (two_g1 + a) * t2 + g1sq * b);
        inc_a = (Cl * s6a + Cf * a) - dv1;
        inc_b = (Cl * s6b + Cf * b) - dv2;
    }
    // The same increments with every multiply-add an explicit fma, so that
    // each inlined copy rounds alike whatever the compiler would contract
    // (the 27-point sweep computes a site in several copies of its loop and,
    // redundantly, as another tile's ring site).
    __device__ inline void force_fma(T a, T b, T s6a, T s6b, T &inc_a, T &inc_b) const
    {
        T hor = h[NH - 1];
#pragma unroll
        for (int j = NH - 2; j >= 0; --j) hor = fma(hor, a, h[j]);
        const T t2 = g2 + b;
        const T dv1 = fma(hor, a, C2 * fma(a * t2, t2, (g1 * b) * (two_g2 + b)));
        const T dv2 = C2 * fma(a * (two_g1 + a), t2, g1sq * b);
        inc_a = fma(Cl, s6a, fma(Cf, a, -dv1));
        inc_b = fma(Cl, s6b, fma(Cf, b, -dv2));
    }
};

template <typename T>
__device__ inline T six_sum(T xm, T xp, T ym, T yp, T zm, T zp, T c)
{
    return (((xm + xp) + (ym + yp)) + (zm + zp)) - T(6) * c;
}

template <int NH>
__device__ inline double potential_pow(double x)
{
    double r = x;
#pragma unroll
    for (int j = 0; j < NH; ++j) r *= x;  // x^(NH+1) = x^beta
    return r;
}

// Where the z-planes of the four input arrays (d1, d2, e1, e2) of a z-slab
// sweep lie.  A sweep reads d on planes [z0-2, z1] and e on [z0-1, z1-1] of
// a chunk [z0, z1) of [0, nz).  Planes 0 .. nz-1 are the arrays' own; plane
// z < 0 lies at lo[i] + (z+2) N^2 and plane z >= nz at hi[i] + (z-nz) N^2,
// in the slab's halo buffers (e is never read above the slab).  Only the
// slab kernels use this; the periodic ones wrap the plane index.
template <typename T>
struct ZPlanes {
    const T *lo[4];
    const T *hi[4];
    int nz;
    __device__ inline const T *at(int i, const T *p, int z, int64_t NN) const
    {
        return z < 0 ? lo[i] + (int64_t)(z + 2) * NN
                     : (z >= nz ? hi[i] + (int64_t)(z - nz) * NN : p + (int64_t)z * NN);
    }
};

template <typename T>
inline ZPlanes<T> planes_of(const SweepIO &io)
{
    ZPlanes<T> zp;
    for (int i = 0; i < 4; ++i) {
        zp.lo[i] = (const T *)io.lo[i];
        zp.hi[i] = (const T *)io.hi[i];
    }
    zp.nz = io.nz;
    return zp;
}

// Work item loop of the persistent ensemble sweeps.  The items are split
// into one segment per XCD (items seg[x] .. seg[x+1] - 1), each holding whole z-chunks
// of some realizations, longest first; a block takes the next item of its own
// XCD's segment (hardware places block b on XCD b mod 8) from that segment's
// counter, so the tiles of one chunk run together on one L2 and find their
// neighbours' halo rows there.  When its segment is used up it takes items of
// the other segments in turn.  queue holds the counters (queue[32 x], 128
// bytes apart), reset to 0 by the batched scale-factor kernel that runs
// before every sweep, followed by seg[0..8].  Every thread of the block sees the same index; fn(i) runs for
// each item.
constexpr int kEnsXcd = 8, kEnsQueueStride = 32;

template <typename F>
__device__ inline void for_each_item(int *queue, int nitems, F &&fn)
{
    const int *seg = queue + kEnsXcd * kEnsQueueStride;  // segment bounds follow the counters
    __shared__ int s_item;
    const int home = blockIdx.x % kEnsXcd;
    int k = 0;  // thread 0: segments used up so far, own segment first
    for (;;) {
        if (threadIdx.x == 0) {
            int item = -1;
            while (k < kEnsXcd) {
                const int x = (home + k) % kEnsXcd;
                const int j = seg[x] + atomicAdd(queue + x * kEnsQueueStride, 1);
                if (j < seg[x + 1] && j < nitems) {
                    item = j;
                    break;
                }
                ++k;
            }
            s_item = item;
        }
        __syncthreads();
        const int i = s_item;
        if (i < 0) break;
        fn(i);
        __syncthreads();  // LDS (and s_item) are reused by the next item
    }
}

}  // namespace lf
