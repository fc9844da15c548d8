// Lattice stencils of liblf: the Laplacian and the gradient energy it
// conserves, for the generic (one site per thread, global-memory) kernels.
//
//   ST = 7:  the 6-neighbour Laplacian of LATTICEEASY (Sainio,
//            arXiv:0911.5692, Sec. II.C); gradient energy = forward
//            differences |d+ f|^2.
//   ST = 27: the 27-point Laplacian the paper itself uses (Sec. II.C):
//            second-order accurate, fourth-order isotropic, weights
//            (centre, face, edge, corner) = (-128, 14, 3, 1) / 30.  The
//            gradient energy is its Dirichlet form, sum over the 13 bonds b
//            whose first nonzero of (dz, dy, dx) is +1 of
//            w_b (f(x+b) - f(x))^2, w = (14, 3, 1) / 30 by bond type, so that
//            sum_x grad2(x) = -sum_x f Lap f exactly.
//
// Both helpers return the RAW integer-weighted sums (no 1/dx^2 and, for
// ST = 27, no 1/30): every caller multiplies by the stencil weight gw
// (1 or 1/30, DevParams::gw) together with 1/dx^2.  A value functor
// v(dx, dy, dz) returns the neighbour at that offset (periodic wrap is the
// caller's); c is the centre value.
#pragma once

namespace lf {

template <int ST>
struct StencilW;
template <>
struct StencilW<7> {
    static constexpr double gw = 1.0;
};
template <>
struct StencilW<27> {
    static constexpr double gw = 1.0 / 30.0;
};

template <int ST, typename R, typename V>
__device__ inline R lap_raw(V v, R c)
{
    if constexpr (ST == 7) {
        return (((v(-1, 0, 0) + v(1, 0, 0)) + (v(0, -1, 0) + v(0, 1, 0))) + (v(0, 0, -1) + v(0, 0, 1))) - R(6) * c;
    } else {
        R face = (v(-1, 0, 0) + v(1, 0, 0)) + (v(0, -1, 0) + v(0, 1, 0)) + (v(0, 0, -1) + v(0, 0, 1));
        R edge = R(0), corner = R(0);
#pragma unroll
        for (int dz = -1; dz <= 1; dz += 2) {
            edge += (v(-1, 0, dz) + v(1, 0, dz)) + (v(0, -1, dz) + v(0, 1, dz));
            corner += (v(-1, -1, dz) + v(1, -1, dz)) + (v(-1, 1, dz) + v(1, 1, dz));
        }
        edge += (v(-1, -1, 0) + v(1, -1, 0)) + (v(-1, 1, 0) + v(1, 1, 0));
        return ((R(-128) * c + R(14) * face) + R(3) * edge) + corner;
    }
}

template <int ST, typename V>
__device__ inline double grad_raw(V v, double c)
{
    if constexpr (ST == 7) {
        const double t0 = v(1, 0, 0) - c, t1 = v(0, 1, 0) - c, t2 = v(0, 0, 1) - c;
        return t0 * t0 + t1 * t1 + t2 * t2;
    } else {
        auto sq = [&](int dx, int dy, int dz) {
            const double t = v(dx, dy, dz) - c;
            return t * t;
        };
        const double face = sq(1, 0, 0) + sq(0, 1, 0) + sq(0, 0, 1);
        const double edge = (sq(-1, 1, 0) + sq(1, 1, 0)) + (sq(0, -1, 1) + sq(0, 1, 1))
                          + (sq(-1, 0, 1) + sq(1, 0, 1));
        const double corner = (sq(-1, -1, 1) + sq(1, -1, 1)) + (sq(-1, 1, 1) + sq(1, 1, 1));
        return (14.0 * face + 3.0 * edge) + corner;
    }
}

// Index of (x+dx, y+dy, z+dz) mod N in an x-fastest N^3 array.
struct Wrap {
    int N, x, y, z;
    __device__ inline Wrap(int64_t i, int n) : N(n)
    {
        x = (int)(i % n);
        const int64_t t = i / n;
        y = (int)(t % n);
        z = (int)(t / n);
    }
    __device__ inline int64_t operator()(int dx, int dy, int dz) const
    {
        int xx = x + dx, yy = y + dy, zz = z + dz;
        xx += (xx < 0) ? N : ((xx >= N) ? -N : 0);
        yy += (yy < 0) ? N : ((yy >= N) ? -N : 0);
        zz += (zz < 0) ? N : ((zz >= N) ? -N : 0);
        return ((int64_t)zz * N + yy) * N + xx;
    }
};

}  // namespace lf
