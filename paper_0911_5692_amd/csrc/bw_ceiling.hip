// Streaming-bandwidth ceilings of MI355X (gfx950) for the byte mix of the
// FP32 leapfrog sweep: four N^3 FP32 arrays read and four written per step
// (32 B per site).  A standalone program (not part of liblf): it times, with
// HIP events, kernels that move exactly these bytes with no arithmetic, in
// three access orders:
//   flat   one element (4 or 16 B) per lane of a grid that covers the arrays
//          once, blocks in address order (no loop), and grid-stride loops;
//   march  the sweep's order: a block owns a TX x TY column tile and marches
//          a chunk of z-planes, loading plane z+1 while it stores plane z
//          (non-temporal stores), blocks in XCD-contiguous tile order;
//   chunk  the same march with z-chunks from 1 to N planes, from
//          short-lived blocks in address order to the sweep's long marches;
//   halo   a chunk of planes [z0, z1) copied with the sweep's read
//          footprint: d (arrays 0, 1) on planes z0-2 .. z1, rows y0-2 ..
//          y0+TY and columns x0-2 .. x0+TX+1, e (arrays 2, 3) on planes
//          z0-1 .. z1-1 with the row y0-1 and column x0-1 (what the 27-point
//          sweep reads, a superset of the 7-point one), from registers only:
//          what short chunks would cost a stencil sweep;
// plus read-only and write-only kernels.  Every configuration is timed over
// 20 launches after 5 warm-up launches; rates are the kernel's bytes (32 B
// per site for copies, 16 B for read or write only) over its average time.
//
// Usage: bw_ceiling [N]   (default 512; N in 256, 512, 768, 1024)
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#define CK(x)                                                                                      \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);       \
            exit(1);                                                                               \
        }                                                                                          \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- flat order

// One V per lane, grid covering n exactly (n a multiple of 256).
template <typename V>
__global__ void __launch_bounds__(256) k_flat(const V *__restrict__ a0, const V *__restrict__ a1,
                                              const V *__restrict__ a2, const V *__restrict__ a3, V *__restrict__ b0,
                                              V *__restrict__ b1, V *__restrict__ b2, V *__restrict__ b3, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const V x0 = a0[i], x1 = a1[i], x2 = a2[i], x3 = a3[i];
    __builtin_nontemporal_store(x0, b0 + i);
    __builtin_nontemporal_store(x1, b1 + i);
    __builtin_nontemporal_store(x2, b2 + i);
    __builtin_nontemporal_store(x3, b3 + i);
}

// Grid-stride loop, one V per lane per iteration.
template <typename V>
__global__ void __launch_bounds__(256) k_stride(const V *__restrict__ a0, const V *__restrict__ a1,
                                                const V *__restrict__ a2, const V *__restrict__ a3, V *__restrict__ b0,
                                                V *__restrict__ b1, V *__restrict__ b2, V *__restrict__ b3, long n)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const V x0 = a0[i], x1 = a1[i], x2 = a2[i], x3 = a3[i];
        __builtin_nontemporal_store(x0, b0 + i);
        __builtin_nontemporal_store(x1, b1 + i);
        __builtin_nontemporal_store(x2, b2 + i);
        __builtin_nontemporal_store(x3, b3 + i);
    }
}

// Read-only: one float per lane per array; the sum is stored only if it is
// exactly 1234.5 (never, for zero data), which keeps the loads.
__global__ void __launch_bounds__(256) k_read(const float *__restrict__ a0, const float *__restrict__ a1,
                                              const float *__restrict__ a2, const float *__restrict__ a3,
                                              float *__restrict__ out, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float s = (a0[i] + a1[i]) + (a2[i] + a3[i]);
    if (s == 1234.5f) out[0] = s;
}

__global__ void __launch_bounds__(256) k_write(float *__restrict__ b0, float *__restrict__ b1, float *__restrict__ b2,
                                               float *__restrict__ b3, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    __builtin_nontemporal_store(0.0f, b0 + i);
    __builtin_nontemporal_store(0.0f, b1 + i);
    __builtin_nontemporal_store(0.0f, b2 + i);
    __builtin_nontemporal_store(0.0f, b3 + i);
}

// ---------------------------------------------------------------- z-march order

__device__ inline int xcd_remap(int b, int nb)
{
    const int q = nb / 8;
    if (b >= q * 8) return b;
    return (b % 8) * q + b / 8;
}

// A TX x TY tile (TX divides N, 256 threads, TY a multiple of 256 / TX)
// marching planes [z0, z1): plane z+1 is loaded while plane z is stored.
template <int TX, int TY, bool REMAP>
__global__ void __launch_bounds__(256) k_march(const float *__restrict__ a0, const float *__restrict__ a1,
                                               const float *__restrict__ a2, const float *__restrict__ a3,
                                               float *__restrict__ b0, float *__restrict__ b1, float *__restrict__ b2,
                                               float *__restrict__ b3, int N, int zchunk, int ntx, int nty)
{
    constexpr int RPR = 256 / TX, KI = TY / RPR;
    static_assert(256 % TX == 0 && TY % RPR == 0, "tile shape");
    const int tile = REMAP ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tx = tile % ntx, r = tile / ntx, ty = r % nty, tz = r / nty;
    const int z0 = tz * zchunk, z1 = min(z0 + zchunk, N);
    const int t = threadIdx.x, cx = t % TX, cy = t / TX;
    const long NN = (long)N * N;
    int g[KI];
#pragma unroll
    for (int k = 0; k < KI; ++k) g[k] = (ty * TY + cy + RPR * k) * N + tx * TX + cx;
    float c[4][KI], nx[4][KI];
    auto load = [&](float (&v)[4][KI], int z) {
        const long o = (long)min(z, z1 - 1) * NN;  // past the chunk: an in-range plane, not used
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            v[0][k] = a0[o + g[k]];
            v[1][k] = a1[o + g[k]];
            v[2][k] = a2[o + g[k]];
            v[3][k] = a3[o + g[k]];
        }
    };
    load(c, z0);
    for (int z = z0; z < z1; ++z) {
        load(nx, z + 1);
        const long o = (long)z * NN;
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            __builtin_nontemporal_store(c[0][k], b0 + o + g[k]);
            __builtin_nontemporal_store(c[1][k], b1 + o + g[k]);
            __builtin_nontemporal_store(c[2][k], b2 + o + g[k]);
            __builtin_nontemporal_store(c[3][k], b3 + o + g[k]);
        }
#pragma unroll
        for (int k = 0; k < KI; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j][k] = nx[j][k];
    }
}

// ---------------------------------------------------------------- halo footprint

// Planes [z0, z1) of a TX x TY tile copied (arrays 0..3 at the tile's own
// sites) while the reads of the sweep's halo are made too: each loaded halo
// value feeds a sum that is stored only if it is exactly 1234.5 (never, for
// zero data).  Periodic wrap in x, y and z keeps every read in range.
template <int TX, int TY>
__global__ void __launch_bounds__(256) k_halo(const float *__restrict__ d1, const float *__restrict__ d2,
                                              const float *__restrict__ e1, const float *__restrict__ e2,
                                              float *__restrict__ b0, float *__restrict__ b1, float *__restrict__ b2,
                                              float *__restrict__ b3, float *__restrict__ out, int N, int zchunk,
                                              int ntx, int nty)
{
    constexpr int RPR = 256 / TX, KI = TY / RPR;
    // d halo: rows y0-2, y0-1, y0+TY (TX+4 wide from x0-2) and columns
    // x0-2, x0-1, x0+TX, x0+TX+1 of rows y0 .. y0+TY-1; e halo: row y0-1
    // (from x0-1 to x0+TX-1) and column x0-1 of rows y0 .. y0+TY-1
    constexpr int NHD = 3 * (TX + 4) + 4 * TY, NHM = (NHD + 255) / 256;
    constexpr int NHE = TX + 1 + TY, NEM = (NHE + 255) / 256;
    static_assert(256 % TX == 0 && TY % RPR == 0, "tile shape");
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, r = tile / ntx, ty = r % nty, tz = r / nty;
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = tz * zchunk, z1 = min(z0 + zchunk, N);
    const int t = threadIdx.x, cx = t % TX, cy = t / TX;
    const long NN = (long)N * N;
    auto wrap = [N](int v) { return ((v % N) + N) % N; };
    int g[KI], hd[NHM], he[NEM];
#pragma unroll
    for (int k = 0; k < KI; ++k) g[k] = (y0 + cy + RPR * k) * N + x0 + cx;
#pragma unroll
    for (int m = 0; m < NHM; ++m) {
        int c = t + 256 * m, x, y;
        if (c >= NHD) c = 0;  // a repeated cell: still in range
        if (c < 3 * (TX + 4)) {
            const int row = c / (TX + 4);
            x = c % (TX + 4) - 2;
            y = row == 0 ? -2 : (row == 1 ? -1 : TY);
        } else {
            const int cc = c - 3 * (TX + 4), col = cc / TY;
            y = cc % TY;
            x = col == 0 ? -2 : (col == 1 ? -1 : (col == 2 ? TX : TX + 1));
        }
        hd[m] = wrap(y0 + y) * N + wrap(x0 + x);
    }
#pragma unroll
    for (int m = 0; m < NEM; ++m) {
        const int c = t + 256 * m < NHE ? t + 256 * m : 0;
        const int x = c < TX + 1 ? c - 1 : -1, y = c < TX + 1 ? -1 : c - (TX + 1);
        he[m] = wrap(y0 + y) * N + wrap(x0 + x);
    }
    float acc = 0.f;
    for (int z = z0 - 2; z <= z1; ++z) {
        const long o = (long)wrap(z) * NN;
        float v1[KI], v2[KI], w1[KI], w2[KI];
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            v1[k] = d1[o + g[k]];
            v2[k] = d2[o + g[k]];
        }
#pragma unroll
        for (int m = 0; m < NHM; ++m) acc += d1[o + hd[m]] + d2[o + hd[m]];
        if (z >= z0 - 1 && z < z1) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                w1[k] = e1[o + g[k]];
                w2[k] = e2[o + g[k]];
            }
#pragma unroll
            for (int m = 0; m < NEM; ++m) acc += e1[o + he[m]] + e2[o + he[m]];
        }
        if (z >= z0 && z < z1) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                __builtin_nontemporal_store(v1[k], b0 + o + g[k]);
                __builtin_nontemporal_store(v2[k], b1 + o + g[k]);
                __builtin_nontemporal_store(w1[k], b2 + o + g[k]);
                __builtin_nontemporal_store(w2[k], b3 + o + g[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < KI; ++k) acc += v1[k] + v2[k];
        }
    }
    if (acc == 1234.5f) out[0] = acc;
}

// ---------------------------------------------------------------- driver

struct Arrays {
    float *a[4], *b[4];
    float *out;
    int N;
    long n;  // N^3
};

template <typename F>
static double time_ms(F launch)
{
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    for (int i = 0; i < 5; ++i) launch();
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0, 0));
    for (int i = 0; i < 20; ++i) launch();
    CK(hipEventRecord(e1, 0));
    CK(hipEventSynchronize(e1));
    CK(hipGetLastError());
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    return ms / 20.0;
}

static void report(const char *order, const char *what, double bytes, double ms)
{
    printf("| %s | %s | %.4f | %.0f | %.3f |\n", order, what, ms, bytes / ms / 1e6, bytes / ms / 1e6 / 8000.0);
    fflush(stdout);
}

template <typename V>
static void flat(const Arrays &A, const char *what)
{
    const long n = A.n * 4 / (long)sizeof(V);
    const double ms = time_ms([&] {
        hipLaunchKernelGGL(k_flat<V>, dim3((unsigned)(n / 256)), dim3(256), 0, 0, (const V *)A.a[0], (const V *)A.a[1],
                           (const V *)A.a[2], (const V *)A.a[3], (V *)A.b[0], (V *)A.b[1], (V *)A.b[2], (V *)A.b[3], n);
    });
    report("flat", what, 32.0 * A.n, ms);
}

template <typename V>
static void stride(const Arrays &A, int grid, const char *what)
{
    const long n = A.n * 4 / (long)sizeof(V);
    const double ms = time_ms([&] {
        hipLaunchKernelGGL(k_stride<V>, dim3(grid), dim3(256), 0, 0, (const V *)A.a[0], (const V *)A.a[1],
                           (const V *)A.a[2], (const V *)A.a[3], (V *)A.b[0], (V *)A.b[1], (V *)A.b[2], (V *)A.b[3], n);
    });
    char buf[96];
    snprintf(buf, sizeof buf, "%s, grid-stride loop, %d blocks", what, grid);
    report("flat", buf, 32.0 * A.n, ms);
}

template <int TX, int TY, bool REMAP>
static void march(const Arrays &A, int zchunk, const char *order)
{
    const int N = A.N, ntx = N / TX, nty = N / TY, nzc = (N + zchunk - 1) / zchunk;
    const double ms = time_ms([&] {
        hipLaunchKernelGGL((k_march<TX, TY, REMAP>), dim3(ntx * nty * nzc), dim3(256), 0, 0, A.a[0], A.a[1], A.a[2],
                           A.a[3], A.b[0], A.b[1], A.b[2], A.b[3], N, zchunk, ntx, nty);
    });
    char buf[128];
    snprintf(buf, sizeof buf, "%dx%d tiles, %d-plane chunks, %d blocks%s", TX, TY, zchunk, ntx * nty * nzc,
             REMAP ? ", XCD-contiguous" : "");
    report(order, buf, 32.0 * A.n, ms);
}

template <int TX, int TY>
static void halo(const Arrays &A, int zchunk)
{
    const int N = A.N, ntx = N / TX, nty = N / TY, nzc = (N + zchunk - 1) / zchunk;
    const double ms = time_ms([&] {
        hipLaunchKernelGGL((k_halo<TX, TY>), dim3(ntx * nty * nzc), dim3(256), 0, 0, A.a[0], A.a[1], A.a[2], A.a[3],
                           A.b[0], A.b[1], A.b[2], A.b[3], A.out, N, zchunk, ntx, nty);
    });
    char buf[128];
    snprintf(buf, sizeof buf, "%dx%d tiles, %d-plane chunks, %d blocks, XCD-contiguous", TX, TY, zchunk,
             ntx * nty * nzc);
    report("halo", buf, 32.0 * A.n, ms);
}

int main(int argc, char **argv)
{
    Arrays A;
    A.N = argc > 1 ? atoi(argv[1]) : 512;
    if (A.N < 256 || A.N > 1024 || A.N % 256) {
        fprintf(stderr, "N must be 256, 512, 768 or 1024\n");
        return 2;
    }
    A.n = (long)A.N * A.N * A.N;
    const size_t bytes = (size_t)A.n * 4;
    for (int j = 0; j < 4; ++j) {
        CK(hipMalloc(&A.a[j], bytes));
        CK(hipMalloc(&A.b[j], bytes));
        CK(hipMemset(A.a[j], 0, bytes));
        CK(hipMemset(A.b[j], 0, bytes));
    }
    CK(hipMalloc(&A.out, 256));
    CK(hipDeviceSynchronize());
    printf("Streaming rates for four %d^3 FP32 arrays read and four written (%.3f GB per pass)\n\n", A.N,
           32.0 * A.n / 1e9);
    printf("| order | kernel | ms | GB/s | of 8 TB/s |\n|---|---|---|---|---|\n");
    for (int i = 0; i < 3; ++i) flat<float>(A, "warm-up: 4 B per lane");  // brings the clocks up
    flat<float>(A, "4 B per lane");
    flat<f4>(A, "16 B per lane");
    for (int g : {1024, 4096, 32768}) stride<float>(A, g, "4 B per lane");
    for (int g : {1024, 4096, 32768}) stride<f4>(A, g, "16 B per lane");
    {
        const double ms = time_ms([&] {
            hipLaunchKernelGGL(k_read, dim3((unsigned)(A.n / 256)), dim3(256), 0, 0, A.a[0], A.a[1], A.a[2], A.a[3],
                               A.out, A.n);
        });
        report("flat", "read only, 4 B per lane", 16.0 * A.n, ms);
        const double ms2 = time_ms([&] {
            hipLaunchKernelGGL(k_write, dim3((unsigned)(A.n / 256)), dim3(256), 0, 0, A.b[0], A.b[1], A.b[2], A.b[3],
                               A.n);
        });
        report("flat", "write only, 4 B per lane", 16.0 * A.n, ms2);
    }
    const int N = A.N;
    march<128, 8, true>(A, N / 2, "march");
    march<128, 8, true>(A, N, "march");
    march<128, 8, false>(A, N / 2, "march");
    march<64, 8, true>(A, N / 2, "march");
    march<128, 4, true>(A, N / 2, "march");
    march<256, 4, true>(A, N / 2, "march");
    march<256, 1, false>(A, N, "march");
    for (int zc = 1; zc <= N; zc *= 2) march<256, 1, false>(A, zc, "chunk");
    for (int zc = 1; zc <= N; zc *= 4) march<128, 8, false>(A, zc, "chunk");
    for (int zc : {1, 2, 4, 8, 16, 64, N / 2}) halo<128, 8>(A, zc);
    for (int zc : {1, 4, 16, N / 2}) halo<256, 4>(A, zc);
    for (int zc : {1, 4, 16}) halo<256, 8>(A, zc);
    return 0;
}
