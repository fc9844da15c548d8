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
#include "lf_internal.h"

namespace lf {

template <typename T>
struct SiteForce {
    // Returns the velocity increments of both fields at one site.
    __device__ static inline void eval(const Coef<T> &c, T a, T b, T lap_a, T lap_b, T &inc_a,
                                       T &inc_b)
    {
        T hor = c.h[c.nh - 1];
        for (int j = c.nh - 2; j >= 0; --j) hor = hor * a + c.h[j];
        const T t2 = c.g2 + b;
        const T dv1 = hor * a + c.C2 * (a * t2 * t2 + c.g1 * b * (c.two_g2 + b));
        const T dv2 = c.C2 * (a * (c.two_g1 + a) * t2 + c.g1sq * b);
        inc_a = (c.Cl * lap_a + c.Cf * a) - dv1;
        inc_b = (c.Cl * lap_b + c.Cf * b) - dv2;
    }
};

// Plain reference sweep: one thread per site, all 7 stencil points loaded
// from global memory (served by the caches).  Block (64, 4), grid
// (ceil(N/64), ceil(N/4), N).
template <typename T>
__global__ void __launch_bounds__(256) k_sweep_plain(const T *__restrict__ d1, const T *__restrict__ d2,
                                                     const T *__restrict__ e1, const T *__restrict__ e2,
                                                     T *__restrict__ d1n, T *__restrict__ d2n,
                                                     T *__restrict__ e1n, T *__restrict__ e2n, int N,
                                                     const Coef<T> *__restrict__ cp)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= N || y >= N) return;
    const Coef<T> c = *cp;
    const int64_t NN = (int64_t)N * N;
    const int64_t i = (int64_t)z * NN + (int64_t)y * N + x;
    const int64_t xm = (x == 0) ? i + (N - 1) : i - 1;
    const int64_t xp = (x == N - 1) ? i - (N - 1) : i + 1;
    const int64_t ym = (y == 0) ? i + (int64_t)(N - 1) * N : i - N;
    const int64_t yp = (y == N - 1) ? i - (int64_t)(N - 1) * N : i + N;
    const int64_t zm = (z == 0) ? i + (int64_t)(N - 1) * NN : i - NN;
    const int64_t zp = (z == N - 1) ? i - (int64_t)(N - 1) * NN : i + NN;
    const T a = d1[i], b = d2[i];
    const T la = (((d1[xm] + d1[xp]) + (d1[ym] + d1[yp])) + (d1[zm] + d1[zp])) - T(6) * a;
    const T lb = (((d2[xm] + d2[xp]) + (d2[ym] + d2[yp])) + (d2[zm] + d2[zp])) - T(6) * b;
    T ia, ib;
    SiteForce<T>::eval(c, a, b, la, lb, ia, ib);
    const T ea = e1[i] + ia, eb = e2[i] + ib;
    e1n[i] = ea;
    e2n[i] = eb;
    d1n[i] = a + c.dt * ea;
    d2n[i] = b + c.dt * eb;
}

void launch_sweep_plain(int dtype, const void *const in[4], void *const out[4], int N,
                        const CoefPair *C, hipStream_t st)
{
    dim3 grid((N + 63) / 64, (N + 3) / 4, N), block(64, 4);
    if (dtype == 0)
        hipLaunchKernelGGL(k_sweep_plain<float>, grid, block, 0, st, (const float *)in[0],
                           (const float *)in[1], (const float *)in[2], (const float *)in[3],
                           (float *)out[0], (float *)out[1], (float *)out[2], (float *)out[3], N,
                           &C->f);
    else
        hipLaunchKernelGGL(k_sweep_plain<double>, grid, block, 0, st, (const double *)in[0],
                           (const double *)in[1], (const double *)in[2], (const double *)in[3],
                           (double *)out[0], (double *)out[1], (double *)out[2], (double *)out[3], N,
                           &C->d);
}

}  // namespace lf
