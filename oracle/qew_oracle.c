/*
 * qew_oracle.c -- plain FP64 CPU oracle for the quenched Edwards-Wilkinson
 * (QEW) relaxation of Ferrero, Bustingorry and Kolton, "Non-steady relaxation
 * and critical exponents at the depinning transition" (arXiv:1211.7275).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU product path never
 * links, imports or calls it, and it shares no source with the GPU library.
 *
 * What it computes, step by step, in the order the paper states it:
 *   - Eq. (1) with eta = 1: du/dt = c d2u/dx2 + F_p(u, x) + f.
 *   - Sec. III B: x discretised into L sites (dx = 1), u continuous, explicit
 *     Euler integration, periodic boundary in x.
 *   - Sec. III B: the pinning force comes from uncorrelated random numbers at
 *     the integer values of u and x, generated on demand, and a cubic spline
 *     between them.  Random field (RF): the numbers are forces.  Random bond
 *     (RB): the numbers are potential values and F_p = -dU/du (Sec. II).
 *   - Sec. II, Eqs. (3)-(5): v = spatial mean of the total force (equal to the
 *     mean of du/dt), the centre of mass, and the quadratic width w^2.
 *   - Sec. II: flat start u(x, 0) = 0.
 *
 * Readings where the paper is silent (the random-number generator, its
 * keying, the float conversion, the Gaussian method and the spline type live
 * in the paper's supplemental material, which is not available):
 *   - generator: Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3" (SC'11);
 *   - keying: counter = (j, (uint32)n, disorder id, 0), key = (seed low word,
 *     seed high word), j = site, n = integer u (signed, two's complement);
 *   - RF value: m = x0 >> 8, R = (2m + 1 - 2^24) / 2^24, uniform in (-1, 1);
 *   - RB value: a = x0 >> 9, b = x1 >> 9, U1 = (2a+1)/2^24, U2 = (2b+1)/2^24,
 *     R = sqrt(-2 ln U1) cos(2 pi U2) (Box-Muller, cosine branch), N(0, 1);
 *   - spline: uniform Catmull-Rom (cardinal, tension 1/2) over the nodes
 *     n-1 .. n+2, which is local, C^1 and exact at the nodes;
 *   - node values are multiplied by `strength`;
 *   - the Euler update is synchronous (every site reads step-m values);
 *   - Sec. IV C, Case 3 (RB, Gaussian potential, linear spline): between
 *     integers the potential is linear, so F_p = -(V(n+1) - V(n)) on
 *     [n, n+1), discontinuous at the integers;
 *   - Sec. IV C, Case 4 (RF, Gaussian forces, no interpolation): F_p = R(n)
 *     on [n, n+1) (the value of the integer below u);
 *   - optional transverse period M (Sec. III B: the u direction can be made
 *     periodic): node n is node n mod M (M = 0: no period).
 *
 * Precision and order: everything is IEEE binary64, round to nearest, and the
 * file must be built with -ffp-contract=off so that no multiply-add is fused.
 * Expression orders are fixed and written out below.  Sums use Neumaier
 * compensation in index order.
 *
 * Parity status: every function here is pinned by the CPU tests (known-answer
 * vectors, spline identities, closed forms at zero disorder, the mean-force
 * identity, no-passing, node statistics, and a 60-digit re-evaluation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QO_RF 0      /* random field, uniform force values, Catmull-Rom  */
#define QO_RB 1      /* random bond, Gaussian potential, Catmull-Rom     */
#define QO_RB_LIN 2  /* random bond, Gaussian potential, linear spline   */
#define QO_RF_PC 3   /* random field, Gaussian forces, no interpolation  */

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the Philox S-box */
/* on a 4-word counter with a 2-word key bumped by Weyl constants.     */
/* ------------------------------------------------------------------ */
void qo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t prod0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Batch form used by the tests: ctr is [n][4], out is [n][4]. */
void qo_philox_many(const uint32_t *ctr, uint64_t seed, uint32_t *out, int64_t n)
{
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    for (int64_t i = 0; i < n; ++i)
        qo_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* ------------------------------------------------------------------ */
/* Disorder node value R(j, n) at integer u = n of column j (unscaled). */
/* ------------------------------------------------------------------ */
double qo_node(int kind, uint64_t seed, uint32_t disorder_id, int64_t j, int64_t n, int64_t period)
{
    uint32_t ctr[4], key[2], x[4];
    if (period > 0) n = ((n % period) + period) % period;
    ctr[0] = (uint32_t)j;
    ctr[1] = (uint32_t)(int32_t)n;          /* two's complement of the signed cell */
    ctr[2] = disorder_id;
    ctr[3] = 0u;                            /* stream tag 0: disorder nodes */
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
    qo_philox4x32_10(ctr, key, x);
    if (kind == QO_RF) {
        int64_t m = (int64_t)(x[0] >> 8);                  /* 24 random bits */
        int64_t odd = 2 * m + 1 - ((int64_t)1 << 24);      /* odd integer in (-2^24, 2^24) */
        return (double)odd / 16777216.0;                   /* exact */
    } else {
        double a = (double)(x[0] >> 9), b = (double)(x[1] >> 9);   /* 23 bits each */
        double U1 = (2.0 * a + 1.0) / 16777216.0;          /* in (0, 1), exact */
        double U2 = (2.0 * b + 1.0) / 16777216.0;
        double radius = sqrt(-2.0 * log(U1));
        double angle = 2.0 * M_PI * U2;
        return radius * cos(angle);
    }
}

/* ------------------------------------------------------------------ */
/* Uniform Catmull-Rom spline through p[0..3] at nodes -1, 0, 1, 2,     */
/* evaluated at s in [0, 1) (between p[1] and p[2]).                    */
/*   value(s) = 1/2 [ 2 p1 + (p2 - p0) s + (2p0 - 5p1 + 4p2 - p3) s^2   */
/*                    + (-p0 + 3p1 - 3p2 + p3) s^3 ]                    */
/* ------------------------------------------------------------------ */
double qo_cr_value(const double p[4], double s)
{
    double c0 = 2.0 * p[1];
    double c1 = p[2] - p[0];
    double c2 = 2.0 * p[0] - 5.0 * p[1] + 4.0 * p[2] - p[3];
    double c3 = -p[0] + 3.0 * p[1] - 3.0 * p[2] + p[3];
    return 0.5 * (c0 + s * (c1 + s * (c2 + s * c3)));
}

/* d value / ds */
double qo_cr_slope(const double p[4], double s)
{
    double c1 = p[2] - p[0];
    double c2 = 2.0 * p[0] - 5.0 * p[1] + 4.0 * p[2] - p[3];
    double c3 = -p[0] + 3.0 * p[1] - 3.0 * p[2] + p[3];
    return 0.5 * (c1 + s * (2.0 * c2 + s * (3.0 * c3)));
}

/* ------------------------------------------------------------------ */
/* Pinning force F_p(u, j) (Sec. III B; RB: F_p = -dU/du, Sec. II).     */
/* ------------------------------------------------------------------ */
double qo_pinning(int kind, double strength, uint64_t seed, uint32_t disorder_id,
                  int64_t j, double u, int64_t period)
{
    if (strength == 0.0) return 0.0;
    double nf = floor(u);
    int64_t n = (int64_t)nf;
    double s = u - nf;                       /* exact for |u| < 2^52 */
    if (kind == QO_RB_LIN) {                 /* F_p = -(V(n+1) - V(n)) */
        double v0 = strength * qo_node(kind, seed, disorder_id, j, n, period);
        double v1 = strength * qo_node(kind, seed, disorder_id, j, n + 1, period);
        return -(v1 - v0);
    }
    if (kind == QO_RF_PC)                    /* F_p = R(n) */
        return strength * qo_node(kind, seed, disorder_id, j, n, period);
    double p[4];
    for (int i = 0; i < 4; ++i)
        p[i] = strength * qo_node(kind, seed, disorder_id, j, n - 1 + i, period);
    if (kind == QO_RF)
        return qo_cr_value(p, s);
    return -qo_cr_slope(p, s);
}

/* Interpolated potential U(u, j) of the random-bond kinds (tests only):
 * Catmull-Rom (QO_RB) or linear (QO_RB_LIN) in u. */
double qo_potential(int kind, double strength, uint64_t seed, uint32_t disorder_id, int64_t j,
                    double u, int64_t period)
{
    double nf = floor(u);
    int64_t n = (int64_t)nf;
    if (kind == QO_RB_LIN) {
        double v0 = strength * qo_node(kind, seed, disorder_id, j, n, period);
        double v1 = strength * qo_node(kind, seed, disorder_id, j, n + 1, period);
        return v0 + (v1 - v0) * (u - nf);
    }
    double p[4];
    for (int i = 0; i < 4; ++i)
        p[i] = strength * qo_node(QO_RB, seed, disorder_id, j, n - 1 + i, period);
    return qo_cr_value(p, u - nf);
}

/* ------------------------------------------------------------------ */
/* Total force on every site at one time (Eq. (1), periodic in x):      */
/*   F_j = ((c * ((u_{j+1} + u_{j-1}) - 2 u_j)) + f) + F_p(u_j, j)      */
/* ------------------------------------------------------------------ */
void qo_forces(int kind, double strength, uint64_t seed, uint32_t disorder_id, int64_t period,
               int64_t L, double c, double f, const double *u, double *F)
{
    int64_t j;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (j = 0; j < L; ++j) {
        int64_t jm = (j == 0) ? L - 1 : j - 1;
        int64_t jp = (j == L - 1) ? 0 : j + 1;
        double lap = (u[jp] + u[jm]) - 2.0 * u[j];
        double fp = qo_pinning(kind, strength, seed, disorder_id, j, u[j], period);
        F[j] = ((c * lap) + f) + fp;
    }
}

/* Neumaier-compensated sum in index order. */
static double qo_sum(const double *x, int64_t n)
{
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) comp += (s - t) + x[i];
        else comp += (x[i] - t) + s;
        s = t;
    }
    return s + comp;
}

/* Sec. II, Eqs. (3)-(5) for one sample: v = mean force, ubar = mean u,
 * w2 = mean (u - ubar)^2 (two passes). */
void qo_measure(int64_t L, const double *u, const double *F,
                double *v, double *ubar, double *w2)
{
    double *d = (double *)malloc((size_t)L * sizeof(double));
    double mean_u = qo_sum(u, L) / (double)L;
    for (int64_t j = 0; j < L; ++j) {
        double e = u[j] - mean_u;
        d[j] = e * e;
    }
    *v = qo_sum(F, L) / (double)L;
    *ubar = mean_u;
    *w2 = qo_sum(d, L) / (double)L;
    free(d);
}

/* One synchronous Euler step: u_new = u + dt * F (Sec. III B). */
void qo_euler(int64_t L, double dt, const double *u, const double *F, double *u_new)
{
    for (int64_t j = 0; j < L; ++j) u_new[j] = u[j] + dt * F[j];
}

/*
 * Evolve one sample from the state `u` (taken to be the state at step
 * `step0`) up to step `n_steps`.  At every step m in meas_steps with
 * step0 <= m <= n_steps the observables of the state at step m are written
 * to v/ubar/w2[index of m]; entries for m < step0 are left untouched.  On
 * return `u` holds the state at step n_steps.  Returns 0, or -1 on bad input.
 */
int qo_run(int kind, double strength, uint64_t seed, uint32_t disorder_id, int64_t period,
           int64_t L, double c, double dt, double f,
           int64_t step0, int64_t n_steps, const int64_t *meas_steps, int32_t n_meas,
           double *u, double *v, double *ubar, double *w2)
{
    if (L < 1 || step0 < 0 || n_steps < step0) return -1;
    double *F = (double *)malloc((size_t)L * sizeof(double));
    double *un = (double *)malloc((size_t)L * sizeof(double));
    if (!F || !un) { free(F); free(un); return -1; }
    int32_t mi = 0;
    while (mi < n_meas && meas_steps[mi] < step0) ++mi;
    for (int64_t m = step0; m <= n_steps; ++m) {
        int measure = (mi < n_meas && meas_steps[mi] == m);
        if (!measure && m == n_steps) break;
        qo_forces(kind, strength, seed, disorder_id, period, L, c, f, u, F);
        if (measure) {
            qo_measure(L, u, F, &v[mi], &ubar[mi], &w2[mi]);
            ++mi;
        }
        if (m == n_steps) break;
        qo_euler(L, dt, u, F, un);
        memcpy(u, un, (size_t)L * sizeof(double));
    }
    free(F);
    free(un);
    return 0;
}

/*
 * Light-cone window of a long chain.  One Euler step of the discretised
 * Eq. (1) couples a site only to its two neighbours, so site j after m steps
 * depends on the state and the disorder within distance m of j and on
 * nothing else.  This evolves W consecutive sites whose column indices (the
 * Philox counter word j) are (j0 + i) mod L_global, i = 0..W-1, closing the
 * window on itself at its ends.  The closure is wrong only within distance m
 * of the two ends after m steps; sites i in [m, W - m) are those of the full
 * periodic chain of length L_global.  `u` holds the window's state on entry
 * and on return.  Returns 0, or -1 on bad input.
 */
int qo_run_window(int kind, double strength, uint64_t seed, uint32_t disorder_id, int64_t period,
                  int64_t L_global, int64_t j0, int64_t W, double c, double dt, double f,
                  int64_t n_steps, double *u)
{
    if (W < 3 || L_global < 1 || n_steps < 0) return -1;
    double *F = (double *)malloc((size_t)W * sizeof(double));
    double *un = (double *)malloc((size_t)W * sizeof(double));
    if (!F || !un) { free(F); free(un); return -1; }
    for (int64_t m = 0; m < n_steps; ++m) {
        int64_t i;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (i = 0; i < W; ++i) {
            int64_t im = (i == 0) ? W - 1 : i - 1;
            int64_t ip = (i == W - 1) ? 0 : i + 1;
            int64_t j = ((j0 + i) % L_global + L_global) % L_global;
            double lap = (u[ip] + u[im]) - 2.0 * u[i];
            double fp = qo_pinning(kind, strength, seed, disorder_id, j, u[i], period);
            F[i] = ((c * lap) + f) + fp;
        }
        qo_euler(W, dt, u, F, un);
        memcpy(u, un, (size_t)W * sizeof(double));
    }
    free(F);
    free(un);
    return 0;
}

/* Mean over j in [0, L) of the unscaled node value R(j, n) (Neumaier sum). */
double qo_mean_node(int kind, uint64_t seed, uint32_t disorder_id, int64_t L, int64_t n)
{
    double s = 0.0, comp = 0.0;
    for (int64_t j = 0; j < L; ++j) {
        double x = qo_node(kind, seed, disorder_id, j, n, 0);
        double t = s + x;
        if (fabs(s) >= fabs(x)) comp += (s - t) + x;
        else comp += (x - t) + s;
        s = t;
    }
    return (s + comp) / (double)L;
}

/* Thread control for the OpenMP site loop (1 = serial). */
void qo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int qo_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Critical configuration of a sample periodic in u (period M > 0), Sec. III A
 * (its definition: the pinned solution of c d2u/dx2 + F_p(u, x) + f = 0 with
 * the largest f).  One relaxation: Euler steps of Eq. (1) at drive f from u
 * (in place) until
 *   - every |F_j| <= tol: a pinned configuration (returns 0);
 *   - min_j (u_j - u_ref_j) >= M: the line has advanced by a full period of
 *     the medium, which it cannot do if a pinned configuration exists at this
 *     f (started below one, a forward-moving line never passes it, and its
 *     translates by M are pinned too), so f is above the critical force
 *     (returns 1);
 *   - max_steps steps were taken (returns 2: undecided).
 * *steps receives the number of steps taken.  Returns -1 on bad input.
 */
int qo_relax(int kind, double strength, uint64_t seed, uint32_t disorder_id, int64_t period,
             int64_t L, double c, double dt, double f, double *u, const double *u_ref,
             int64_t max_steps, double tol, int64_t *steps)
{
    if (L < 1 || period < 1 || max_steps < 0 || !(tol > 0)) return -1;
    double *F = (double *)malloc((size_t)L * sizeof(double));
    double *un = (double *)malloc((size_t)L * sizeof(double));
    if (!F || !un) { free(F); free(un); return -1; }
    int rc = 2;
    int64_t m = 0;
    for (;; ++m) {
        qo_forces(kind, strength, seed, disorder_id, period, L, c, f, u, F);
        double fmax = 0.0, adv = INFINITY;
        for (int64_t j = 0; j < L; ++j) {
            if (fabs(F[j]) > fmax) fmax = fabs(F[j]);
            if (u[j] - u_ref[j] < adv) adv = u[j] - u_ref[j];
        }
        if (fmax <= tol) { rc = 0; break; }
        if (adv >= (double)period) { rc = 1; break; }
        if (m == max_steps) break;
        qo_euler(L, dt, u, F, un);
        memcpy(u, un, (size_t)L * sizeof(double));
    }
    *steps = m;
    free(F);
    free(un);
    return rc;
}
