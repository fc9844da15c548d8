/*
 * FP64 CPU oracle for the staggered-leapfrog evolution of two interacting
 * scalar fields in an expanding FRW background, as described in
 * J. Sainio, "CUDAEASY - a GPU Accelerated Cosmological Lattice Program"
 * (arXiv:0911.5692), Sec. II.B.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's compute path may link,
 * load or call this file; it is used by the tests, by the package's smoke
 * check and by the benchmark's CPU-baseline leg.  It shares no code, header
 * or constant with the GPU library.
 *
 * It is deliberately plain: one loop per step of the method, in the order the
 * paper gives them, with no blocking or fusion, in double precision (and,
 * for the complex-step pin of the adjoint, in double _Complex).  OpenMP only
 * parallelises the site loops.  Built with -ffp-contract=off.
 *
 * Layout: each field is an N^3 array with x fastest: index (z*N + y)*N + x,
 * periodic in all three directions.
 *
 * Readings of the paper that this code fixes (where the paper is silent or
 * its printed formula is garbled):
 *   - the Laplacian is the 7-point (6-neighbour) one (Sec. II.C names it as
 *     LATTICEEASY's discretisation) unless the 27-point stencil the paper
 *     itself uses is selected; the gradient energy is the Dirichlet form of
 *     whichever stencil is in use;
 *   - the coefficient of the (a'/a)^2 f term in eq. (scalar-evo) is
 *     r(s - r + 2); the printed r(s - r - 2) does not follow from eq. (fe)
 *     under the rescaling of Sec. II.B (it would leave an (a'/a)^2 term in the
 *     conformal case r = 1, s = -1, where none exists);
 *   - a' is advanced with the time-centred (implicit midpoint) form of
 *     eq. (scale), so that the step is exactly time-reversible;
 *   - the kick of step k uses averages of the same fields f(k+1/2) it kicks
 *     (no lag between the field sweep and the scale-factor update);
 *   - both fields are kicked with the same-time values of both fields.
 *
 * Parity status: every function here is pinned by a CPU test against a
 * closed form, an identity or brute force (see the test files named
 * test_oracle_*.py); none is "parity unpinned".
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t N;       /* lattice sites per side */
    double L;        /* comoving box side, program units */
    double dt;       /* program time step */
    int32_t beta;    /* exponent of the dominant term c1 f^beta / beta */
    int32_t stencil; /* Laplacian: 7 (6 neighbours) or 27 (Sec. II.C) */
    double c1;       /* program-unit coupling of the dominant term */
    double G_re;     /* program-unit g^2 of the g^2 f1^2 f2^2 / 2 term */
    double r, s;     /* rescaling exponents, s - 2r + 3 = 0 */
    double kappa2;   /* 8 pi G / A^2 */
} orc_params;

#define IDX(x, y, z, N) ((((int64_t)(z)) * (N) + (y)) * (N) + (x))

/* powers of a for the degree-beta and degree-4 monomials of V_pr */
static double p1_of(const orc_params *p) { return -2.0 * p->s + (2.0 - p->beta) * p->r; }
static double p2_of(const orc_params *p) { return -2.0 * p->s - 2.0 * p->r; }

/* ---- real instantiation ------------------------------------------------ */
#define T double
#define T_SQRT(x) sqrt(x)
#define T_POW(x, y) pow((x), (y))
#define FN(name) orc_##name
#define PAR_FOR _Pragma("omp parallel for schedule(static)")
#define REDUCE_FOR _Pragma("omp parallel for schedule(static) reduction(+:sg,sv)")
#define REDUCE_FOR5 _Pragma("omp parallel for schedule(static) reduction(+:k1,k2,g1,g2,pv)")
#include "lf_oracle_core.inc"
#undef T
#undef T_SQRT
#undef T_POW
#undef FN
#undef PAR_FOR
#undef REDUCE_FOR
#undef REDUCE_FOR5

/* ---- complex instantiation (complex-step differentiation) -------------- */
#define T double _Complex
#define T_SQRT(x) csqrt(x)
#define T_POW(x, y) cpow((x), (y))
#define FN(name) orcz_##name
#define PAR_FOR
#define REDUCE_FOR
#define REDUCE_FOR5
#include "lf_oracle_core.inc"
#undef T
#undef T_SQRT
#undef T_POW
#undef FN
#undef PAR_FOR
#undef REDUCE_FOR
#undef REDUCE_FOR5

/* ======================================================================== */
/* Exported real entry points                                               */
/* ======================================================================== */

int orc_abi(void) { return 1; }

/* Parameter check: the rescaling constraint s - 2r + 3 = 0 of Sec. II.B. */
int orc_check_params(const orc_params *p)
{
    if (p->N < 1 || p->L <= 0.0 || p->dt <= 0.0 || p->beta < 2) return 1;
    if (p->stencil != 7 && p->stencil != 27) return 3;
    if (fabs(p->s - 2.0 * p->r + 3.0) > 1e-12) return 2;
    return 0;
}

void orc_laplacian(const orc_params *p, const double *f, double *out)
{
    const int64_t N = p->N;
    const double dx = p->L / (double)N, inv_dx2 = 1.0 / (dx * dx);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z)
        for (int64_t y = 0; y < N; ++y)
            for (int64_t x = 0; x < N; ++x)
                out[IDX(x, y, z, N)] = orc_lap_site(p, f, N, x, y, z, inv_dx2);
}

void orc_grad2(const orc_params *p, const double *f, double *out)
{
    const int64_t N = p->N;
    const double dx = p->L / (double)N, inv_dx2 = 1.0 / (dx * dx);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z)
        for (int64_t y = 0; y < N; ++y)
            for (int64_t x = 0; x < N; ++x)
                out[IDX(x, y, z, N)] = orc_grad2_site(p, f, N, x, y, z, inv_dx2);
}

/* out[0] = Sg, out[1] = SV at scale factor a (see orc_reduce in the core). */
void orc_averages(const orc_params *p, const double *f1, const double *f2, double a, double *out)
{
    orc_reduce(p, p->G_re, f1, f2, a, out);
}

/* out: a'_{k+1}, a'_{k+1/2}, a''_{k+1/2}, a_{k+3/2} */
void orc_scale_step(const orc_params *p, double a, double w, double Sg, double SV, double *out)
{
    double adh, add, an;
    double u = orc_scale_update(p, a, w, Sg, SV, &adh, &add, &an);
    out[0] = u; out[1] = adh; out[2] = add; out[3] = an;
}

void orc_desync_state(const orc_params *p, double *f1, double *f2, const double *v1,
                      const double *v2, double a0, double ad0, double *a_half)
{
    orc_desync(p, f1, f2, v1, v2, a0, ad0, a_half);
}

/* Advance n steps from the desynchronised state.  tape: NULL or 5*n doubles. */
void orc_evolve(const orc_params *p, double *f1, double *f2, double *v1, double *v2,
                double *a_half, double *ad, int64_t nsteps, double *tape)
{
    for (int64_t k = 0; k < nsteps; ++k)
        orc_step(p, p->G_re, f1, f2, v1, v2, a_half, ad, tape ? tape + 5 * k : NULL);
}

/* out[9]: a, a', K1, K2, G1, G2, P, rho, R at the synchronised time. */
void orc_energy(const orc_params *p, const double *f1, const double *f2, const double *v1,
                const double *v2, double a_half, double ad, double *out)
{
    const int64_t N3 = p->N * p->N * p->N;
    double *fs = (double *)malloc(2 * N3 * sizeof(double));
    orc_energies(p, p->G_re, f1, f2, v1, v2, a_half, ad, fs, fs + N3, out);
    free(fs);
}

/* Program-unit initial state (Sec. II.B, conversion to program units):
 * on entry v1, v2 hold the physical time derivatives already rescaled,
 * u_i = (A/B) a^(r-s) dphi_i/dt; f1, f2 hold f(0).  The Friedmann constraint
 *   a'^2 = (kappa^2/3) a^(2-2r) rho_pr,
 *   rho_pr = sum_i <u_i^2/2 + a^(-2s-2)|grad+ f_i|^2/2> + <V_pr>,
 * gives a'_0 (taken positive: an expanding universe); then
 *   v_i = u_i + r (a'_0/a_0) f_i.
 * Returns a'_0 and overwrites v1, v2. */
double orc_init_physical(const orc_params *p, const double *f1, const double *f2,
                         double *v1, double *v2, double a0)
{
    const int64_t N = p->N, N3 = N * N * N;
    const double dx = p->L / (double)N, inv_dx2 = 1.0 / (dx * dx);
    const double r = p->r, s = p->s;
    double ap1 = pow(a0, p1_of(p)), ap2 = pow(a0, p2_of(p));
    double kin = 0.0, grad = 0.0, pot = 0.0;
#pragma omp parallel for schedule(static) reduction(+:kin,grad,pot)
    for (int64_t z = 0; z < N; ++z)
        for (int64_t y = 0; y < N; ++y)
            for (int64_t x = 0; x < N; ++x) {
                int64_t i = IDX(x, y, z, N);
                kin += 0.5 * (v1[i] * v1[i] + v2[i] * v2[i]);
                grad += orc_grad2_site(p, f1, N, x, y, z, inv_dx2) + orc_grad2_site(p, f2, N, x, y, z, inv_dx2);
                pot += orc_vpr(p, p->G_re, f1[i], f2[i], ap1, ap2);
            }
    double rho = (kin + 0.5 * pow(a0, -2.0 * s - 2.0) * grad + pot) / (double)N3;
    double ad0 = sqrt((p->kappa2 / 3.0) * pow(a0, 2.0 - 2.0 * r) * rho);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N3; ++i) {
        v1[i] += r * (ad0 / a0) * f1[i];
        v2[i] += r * (ad0 / a0) * f2[i];
    }
    return ad0;
}

/* Energy density and pressure per site at the synchronised time (eq. rho-pres
 * in program units; the same rescaling takes rho and p to rho_pr, p_pr):
 *   rho(x) = sum_i [K_i(x) + G_i(x)] + V_pr,   p(x) = sum_i [K_i(x) - G_i(x)/3] - V_pr
 *   K_i = (v_i - r (a'/a) f_i)^2 / 2,   G_i = a^(-2s-2) |grad+ f_i|^2 / 2
 * with f = f(k+1/2) - dt/2 v(k), a_k = a_{k+1/2} - dt/2 a'_k.  rho, p may be
 * NULL.  out: <rho>, <p>, w = <p>/<rho>. */
void orc_rho_p(const orc_params *p, const double *f1, const double *f2, const double *v1,
               const double *v2, double a_half, double ad, double *rho, double *pr, double *out)
{
    const int64_t N = p->N, N3 = N * N * N;
    const double dx = p->L / (double)N, inv_dx2 = 1.0 / (dx * dx), h = 0.5 * p->dt;
    const double r = p->r, s = p->s;
    double *fs = (double *)malloc(2 * N3 * sizeof(double));
    double *fs1 = fs, *fs2 = fs + N3;
    const double a = a_half - h * ad, hub = ad / a;
    for (int64_t i = 0; i < N3; ++i) {
        fs1[i] = f1[i] - h * v1[i];
        fs2[i] = f2[i] - h * v2[i];
    }
    const double gfac = 0.5 * pow(a, -2.0 * s - 2.0);
    const double ap1 = pow(a, p1_of(p)), ap2 = pow(a, p2_of(p));
    double srho = 0.0, sp = 0.0;
#pragma omp parallel for schedule(static) reduction(+:srho,sp)
    for (int64_t z = 0; z < N; ++z)
        for (int64_t y = 0; y < N; ++y)
            for (int64_t x = 0; x < N; ++x) {
                int64_t i = IDX(x, y, z, N);
                double q1 = v1[i] - r * hub * fs1[i], q2 = v2[i] - r * hub * fs2[i];
                double K = 0.5 * (q1 * q1 + q2 * q2);
                double G = gfac * (orc_grad2_site(p, fs1, N, x, y, z, inv_dx2) + orc_grad2_site(p, fs2, N, x, y, z, inv_dx2));
                double V = orc_vpr(p, p->G_re, fs1[i], fs2[i], ap1, ap2);
                double rr = K + G + V, pp = K - G / 3.0 - V;
                if (rho) rho[i] = rr;
                if (pr) pr[i] = pp;
                srho += rr;
                sp += pp;
            }
    out[0] = srho / (double)N3;
    out[1] = sp / (double)N3;
    out[2] = out[1] / out[0];
    free(fs);
}

/* ---- complex-step entry points ----------------------------------------- */
/* Same map as orc_desync_state / orc_evolve / orc_energy over complex state
 * and a complex G; arrays are interleaved (re, im) pairs. */
void orcz_desync_state(const orc_params *p, double _Complex *f1, double _Complex *f2,
                       const double _Complex *v1, const double _Complex *v2,
                       const double *a0, const double *ad0, double *a_half)
{
    double _Complex ah;
    orcz_desync(p, f1, f2, v1, v2, a0[0] + I * a0[1], ad0[0] + I * ad0[1], &ah);
    a_half[0] = creal(ah); a_half[1] = cimag(ah);
}

void orcz_evolve(const orc_params *p, const double *G, double _Complex *f1, double _Complex *f2,
                 double _Complex *v1, double _Complex *v2, double *a_half, double *ad,
                 int64_t nsteps)
{
    double _Complex g = G[0] + I * G[1];
    double _Complex ah = a_half[0] + I * a_half[1], w = ad[0] + I * ad[1];
    for (int64_t k = 0; k < nsteps; ++k) orcz_step(p, g, f1, f2, v1, v2, &ah, &w, NULL);
    a_half[0] = creal(ah); a_half[1] = cimag(ah);
    ad[0] = creal(w); ad[1] = cimag(w);
}

void orcz_energy(const orc_params *p, const double *G, const double _Complex *f1,
                 const double _Complex *f2, const double _Complex *v1, const double _Complex *v2,
                 const double *a_half, const double *ad, double *out /* 9 complex */)
{
    const int64_t N3 = p->N * p->N * p->N;
    double _Complex *fs = (double _Complex *)malloc(2 * N3 * sizeof(double _Complex));
    double _Complex res[9];
    orcz_energies(p, G[0] + I * G[1], f1, f2, v1, v2, a_half[0] + I * a_half[1],
                  ad[0] + I * ad[1], fs, fs + N3, res);
    for (int i = 0; i < 9; ++i) { out[2 * i] = creal(res[i]); out[2 * i + 1] = cimag(res[i]); }
    free(fs);
}

#include "lf_oracle_adjoint.inc"
