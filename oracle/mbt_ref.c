/*
 * mbt_ref.c -- plain FP64 CPU reference tracker (the oracle).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU library.  Written to be
 * read against the paper (arXiv:1809.00391) one step at a time: no blocking,
 * no fusion, no reordering of the turn beyond what the text and the written
 * readings state.  Sequential over bunches in bucket order; the per-particle
 * update of one bunch may run on several OpenMP threads, but every particle is
 * independent there and every sum is taken afterwards in particle order, so
 * results do not depend on the thread count.
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 */
#include "mbt_ref.h"

#include <complex.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586
#define PI 3.141592653589793
#define MAX_RES 16

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox-4x32-10 + Box-Muller.                              */
/* ------------------------------------------------------------------------ */

/* Philox-4x32 as published by Salmon, Moraes, Dror and Shaw (SC'11, "Parallel
 * random numbers: as easy as 1, 2, 3"): each round multiplies words 0 and 2
 * by the two round multipliers, keeps the 64-bit products split into high and
 * low halves, and permutes/xors them with words 1 and 3 and the round key; the
 * key is advanced by the two Weyl constants between rounds.  10 rounds. */
void mbt_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0, 1] from 64 random bits: the top 53 bits scaled by 2^-53,
 * plus half a step (2^-54); never 0, so the logarithm below is finite. */
static double uniform_open(uint32_t lo, uint32_t hi)
{
    uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(x >> 11) * 0x1.0p-53 + 0x1.0p-54;
}

/* Box and Muller (1958): r = sqrt(-2 ln u1), theta = 2 pi u2;
 * (r cos theta, r sin theta) are two independent unit normals. */
void mbt_ref_normal_pair(uint64_t seed, const uint32_t c[4], double z[2])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    mbt_ref_philox4x32_10(c, key, w);
    double u1 = uniform_open(w[0], w[1]);
    double u2 = uniform_open(w[2], w[3]);
    double r = sqrt(-2.0 * log(u1));
    double theta = TWO_PI * u2;
    z[0] = r * cos(theta);
    z[1] = r * sin(theta);
}

/* ------------------------------------------------------------------------ */
/* Wakes (Sec. 2.3): resonator wake function, binned table, wake potential.  */
/* ------------------------------------------------------------------------ */

/* Longitudinal wake of a resonator (R_s, Q, omega_r): with alpha = omega_r/2Q
 * and wbar = sqrt(omega_r^2 - alpha^2),
 *   W(t) = 2 alpha R_s exp(-alpha t) [cos(wbar t) - (alpha/wbar) sin(wbar t)]
 * for t > 0; zero before the source passes (causality). */
double mbt_ref_resonator_wake(const mbt_ref_resonator *r, double t)
{
    if (t < 0.0)
        return 0.0;
    double wr = TWO_PI * r->fr_Hz;
    double alpha = wr / (2.0 * r->q);
    double wbar = sqrt(wr * wr - alpha * alpha);
    return 2.0 * alpha * r->rs_ohm * exp(-alpha * t) *
           (cos(wbar * t) - (alpha / wbar) * sin(wbar * t));
}

/* x^2 exp(-a x^2) / (x^6 + 8) integrated over [0, inf): for a >= 1 after
 * x = s / sqrt(a) over s in [0, 7] (the rest is below 1e-20 of the total);
 * for a < 1 as [0, 1] in x plus [0, 1] in y = 1/x.  Composite Simpson with
 * 2n and n intervals combined by one Richardson step (Boole's rule). */
static double rw_f_large(double s, double a)
{
    return s * s * exp(-s * s) / (8.0 + s * s * s * s * s * s / (a * a * a));
}
static double rw_f_x(double x, double a) { return x * x * exp(-a * x * x) / (x * x * x * x * x * x + 8.0); }
static double rw_f_y(double y, double a)
{
    if (y == 0.0)
        return 0.0;
    return y * y * exp(-a / (y * y)) / (1.0 + 8.0 * y * y * y * y * y * y);
}
static double simpson(double (*f)(double, double), double a, double lo, double hi, int n)
{
    double h = (hi - lo) / n, sum = f(lo, a) + f(hi, a);
    for (int i = 1; i < n; ++i)
        sum += (i & 1 ? 4.0 : 2.0) * f(lo + i * h, a);
    return sum * h / 3.0;
}
static double boole(double (*f)(double, double), double a, double lo, double hi)
{
    const int n = 20000;
    double s2 = simpson(f, a, lo, hi, 2 * n), s1 = simpson(f, a, lo, hi, n);
    return s2 + (s2 - s1) / 15.0;
}
static double rw_integral(double a)
{
    if (a >= 1.0)
        return boole(rw_f_large, a, 0.0, 7.0) / (a * sqrt(a));
    return boole(rw_f_x, a, 0.0, 1.0) + boole(rw_f_y, a, 0.0, 1.0);
}

double mbt_ref_rw_wake(const mbt_ref_rw *rw, double t)
{
    if (t < 0.0)
        return 0.0;
    const double c = 299792458.0, z0 = 376.730313668;
    const double b = rw->radius_m;
    const double s0 = cbrt(2.0 * b * b / (z0 * rw->conductivity_S_m));
    const double u = c * t / s0;
    const double amp = 4.0 * z0 * c * rw->length_m / (PI * b * b);
    return amp * (exp(-u) * cos(sqrt(3.0) * u) / 3.0 - (sqrt(2.0) / PI) * rw_integral(u));
}

static int rw_ok(const mbt_ref_rw *rw)
{
    return rw && isfinite(rw->radius_m) && rw->radius_m > 0.0 && isfinite(rw->conductivity_S_m) &&
           rw->conductivity_S_m > 0.0 && isfinite(rw->length_m) && rw->length_m > 0.0;
}

static int grid_ok(const mbt_ref_grid *g)
{
    return g && g->nbins >= 1 && g->nbins <= 4096 && isfinite(g->tau_min_s) &&
           isfinite(g->tau_max_s) && g->tau_min_s < g->tau_max_s;
}

static int res_ok(const mbt_ref_resonator *r)
{
    return isfinite(r->rs_ohm) && r->rs_ohm >= 0.0 && isfinite(r->q) && r->q > 0.5 &&
           isfinite(r->fr_Hz) && r->fr_Hz > 0.0;
}

/* Table of the total wake (sum over resonators, Sec. 2.3) sampled at the
 * centre-to-centre distance k*Delta of two bins.  At k = 0 a particle sees
 * half the wake its own bin leaves behind (fundamental theorem of beam
 * loading), i.e. W(0+)/2 = alpha R_s. */
int mbt_ref_wake_table(int32_t nres, const mbt_ref_resonator *res, const mbt_ref_grid *g,
                       double *W)
{
    if (!grid_ok(g) || nres < 0 || (nres > 0 && !res) || !W)
        return MBT_REF_EINVAL;
    double delta_t = (g->tau_max_s - g->tau_min_s) / (double)g->nbins;
    for (int32_t k = 0; k < g->nbins; ++k)
        W[k] = 0.0;
    for (int32_t i = 0; i < nres; ++i) {
        if (!res_ok(&res[i]))
            return MBT_REF_EINVAL;
        W[0] += 0.5 * mbt_ref_resonator_wake(&res[i], 0.0);
        for (int32_t k = 1; k < g->nbins; ++k)
            W[k] += mbt_ref_resonator_wake(&res[i], (double)k * delta_t);
    }
    return MBT_REF_OK;
}

int mbt_ref_wake_table_rw(int32_t nres, const mbt_ref_resonator *res, const mbt_ref_rw *rw,
                          const mbt_ref_grid *g, double *W)
{
    int rc = mbt_ref_wake_table(nres, res, g, W);
    if (rc || !rw)
        return rc;
    if (!rw_ok(rw))
        return MBT_REF_EINVAL;
    double delta_t = (g->tau_max_s - g->tau_min_s) / (double)g->nbins;
    W[0] += 0.5 * mbt_ref_rw_wake(rw, 0.0);
    for (int32_t k = 1; k < g->nbins; ++k)
        W[k] += mbt_ref_rw_wake(rw, (double)k * delta_t);
    return MBT_REF_OK;
}

/* Bin k covers [tau_min + k Delta, tau_min + (k+1) Delta); the index is
 * floor((tau - tau_min) * (nbins / (tau_max - tau_min))). */
int32_t mbt_ref_bin_index(const mbt_ref_grid *g, double tau)
{
    double inv_delta = (double)g->nbins / (g->tau_max_s - g->tau_min_s);
    double x = (tau - g->tau_min_s) * inv_delta;
    if (!(x >= 0.0) || !(x < (double)g->nbins))
        return -1;
    return (int32_t)floor(x);
}

/* Number of macro-particles per bin (Sec. 2.3, binning and counting). */
int mbt_ref_histogram(const mbt_ref_grid *g, int64_t n, const double *tau, uint32_t *counts,
                      int64_t *out_of_grid)
{
    if (!grid_ok(g) || n < 0 || (n > 0 && !tau) || !counts)
        return MBT_REF_EINVAL;
    int64_t oog = 0;
    for (int32_t k = 0; k < g->nbins; ++k)
        counts[k] = 0;
    for (int64_t j = 0; j < n; ++j) {
        int32_t k = mbt_ref_bin_index(g, tau[j]);
        if (k < 0)
            ++oog;
        else
            ++counts[k];
    }
    if (out_of_grid)
        *out_of_grid = oog;
    return MBT_REF_OK;
}

/* Wake voltage at bin k from the charge in bins m <= k (earlier or equal
 * arrival): V[k] = q * sum_{m=0..k} W[k-m] c[m], summed with m ascending. */
int mbt_ref_wake_potential(int32_t nbins, const double *W, const uint32_t *counts,
                           double q_per_particle, double *V)
{
    if (nbins < 1 || !W || !counts || !V)
        return MBT_REF_EINVAL;
    for (int32_t k = 0; k < nbins; ++k) {
        double acc = 0.0;
        for (int32_t m = 0; m <= k; ++m)
            acc += W[k - m] * (double)counts[m];
        V[k] = q_per_particle * acc;
    }
    return MBT_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Transverse wakes (Sec. 2.3, Eq. 6 second line; long-range resistive wall). */
/* ------------------------------------------------------------------------ */

/* Transverse wake of a resonator (R_s in Ohm/m, Q, omega_r): with
 * alpha = omega_r / 2Q and wbar = sqrt(omega_r^2 - alpha^2),
 *   W_T(t) = (R_s omega_r^2 / (Q wbar)) exp(-alpha t) sin(wbar t), t > 0;
 * it vanishes at t = 0 and before the source passes. */
double mbt_ref_transverse_resonator_wake(const mbt_ref_resonator *r, double t)
{
    if (!(t > 0.0))
        return 0.0;
    double wr = TWO_PI * r->fr_Hz;
    double alpha = wr / (2.0 * r->q);
    double wbar = sqrt(wr * wr - alpha * alpha);
    return r->rs_ohm * wr * wr / (r->q * wbar) * exp(-alpha * t) * sin(wbar * t);
}

/* Thick-wall transverse resistive-wall wake far behind the source: the
 * impedance Z_T = (2 c / (b^2 w)) Z_L with Z_L = (L / (2 pi b)) (1 + i)
 * sqrt(w mu0 / (2 sigma)) transforms to (L / (pi b^3)) sqrt(Z0 c / (pi sigma t)). */
double mbt_ref_transverse_rw_wake(const mbt_ref_rw *rw, double t)
{
    if (!(t > 0.0))
        return 0.0;
    const double c = 299792458.0, z0 = 376.730313668;
    const double b = rw->radius_m;
    return rw->length_m / (PI * b * b * b) * sqrt(z0 * c / (PI * rw->conductivity_S_m * t));
}

int mbt_ref_transverse_wake_table(int32_t nres, const mbt_ref_resonator *res,
                                  const mbt_ref_grid *g, double *T)
{
    if (!grid_ok(g) || nres < 0 || (nres > 0 && !res) || !T)
        return MBT_REF_EINVAL;
    double delta_t = (g->tau_max_s - g->tau_min_s) / (double)g->nbins;
    for (int32_t k = 0; k < g->nbins; ++k)
        T[k] = 0.0;
    for (int32_t i = 0; i < nres; ++i) {
        if (!res_ok(&res[i]))
            return MBT_REF_EINVAL;
        for (int32_t k = 1; k < g->nbins; ++k)
            T[k] += mbt_ref_transverse_resonator_wake(&res[i], (double)k * delta_t);
    }
    return MBT_REF_OK;
}

/* Sec. 2.3: count the particles of every bin and sum their x (the dipole
 * moment of the bin times its count). */
int mbt_ref_dipole_histogram(const mbt_ref_grid *g, int64_t n, const double *tau,
                             const double *x, uint32_t *counts, double *X)
{
    if (!grid_ok(g) || n < 0 || (n > 0 && (!tau || !x)) || !counts || !X)
        return MBT_REF_EINVAL;
    for (int32_t k = 0; k < g->nbins; ++k) {
        counts[k] = 0;
        X[k] = 0.0;
    }
    for (int64_t j = 0; j < n; ++j) {
        int32_t k = mbt_ref_bin_index(g, tau[j]);
        if (k >= 0) {
            ++counts[k];
            X[k] += x[j];
        }
    }
    return MBT_REF_OK;
}

/* Eq. 6, second line: the kick on bin k comes from the dipoles of the bins
 * that passed before it, U[k] = scale * sum_{m<k} T[k-m] X[m]. */
int mbt_ref_transverse_kicks(int32_t nbins, const double *T, const double *X, double scale,
                             double *U)
{
    if (nbins < 1 || !T || !X || !U)
        return MBT_REF_EINVAL;
    for (int32_t k = 0; k < nbins; ++k) {
        double acc = 0.0;
        for (int32_t m = 0; m < k; ++m)
            acc += T[k - m] * X[m];
        U[k] = scale * acc;
    }
    return MBT_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Harmonic cavity.                                                          */
/* ------------------------------------------------------------------------ */

/* Flat-potential harmonic cavity of order n: the total voltage
 * V(tau) = Vrf [sin(phi_s - w tau) + k sin(n phi_h - n w tau)] has V(0) = U0
 * and V'(0) = V''(0) = 0.  Those three conditions give
 *   sin phi_s = n^2/(n^2-1) U0/Vrf,
 *   k^2 = 1/n^2 - (U0/Vrf)^2/(n^2-1),
 *   cos(n phi_h) = -cos(phi_s)/(k n),  sin(n phi_h) = -sin(phi_s)/(k n^2).
 * The cavity returned keeps that phase and runs at frac * k. */
int mbt_ref_hc_flat_fraction(const mbt_ref_ring *ring, int32_t n, double frac, mbt_ref_hc *out)
{
    if (!ring || !out || n < 2 || !(frac > 0.0) || !(ring->v_rf_V > 0.0) ||
        !(ring->u0_eV >= 0.0) || ring->alpha_c == 0.0)
        return MBT_REF_EINVAL;
    double r = ring->u0_eV / ring->v_rf_V;
    double nn = (double)n * (double)n;
    double s_fp = nn / (nn - 1.0) * r;
    double k2 = 1.0 / nn - r * r / (nn - 1.0);
    if (!(s_fp <= 1.0) || !(k2 > 0.0))
        return MBT_REF_EINVAL;
    double k_fp = sqrt(k2);
    double c_fp = sqrt(1.0 - s_fp * s_fp);
    if (ring->alpha_c < 0.0)
        c_fp = -c_fp;
    double cos_nphi = -c_fp / (k_fp * (double)n);
    double sin_nphi = -s_fp / (k_fp * nn);
    out->n = n;
    out->v_ratio = frac * k_fp;
    out->phase_n_rad = atan2(sin_nphi, cos_nphi);
    return MBT_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Simulation object.                                                        */
/* ------------------------------------------------------------------------ */

struct mbt_ref_sim {
    mbt_ref_ring ring;
    /* derived ring constants */
    double T0, T_rf, w_rf, phi_s, D, noise, drift;
    /* harmonic cavity */
    int hc_on;
    mbt_ref_hc hc;
    /* fill */
    int32_t M;
    int32_t *bucket;
    double *current;
    int32_t *stream;
    /* short-range wake */
    int sr_on;
    mbt_ref_grid grid;
    int32_t n_sr;
    mbt_ref_resonator sr[MAX_RES];
    int rw_on;
    mbt_ref_rw rw;
    double *W; /* rebuilt by prepare() */
    /* long-range resonators */
    int32_t n_lr;
    mbt_ref_resonator lr[MAX_RES];
    double lr_alpha[MAX_RES], lr_wbar[MAX_RES];
    double complex lr_c[MAX_RES];
    double complex phasor[MAX_RES];
    double complex *gap; /* [n_lr][M] rotation into bunch b's bucket */
    /* transverse plane */
    int tr_on;
    mbt_ref_transverse tr;
    double tr_qfrac, tr_gamma, tr_noise_x, tr_noise_xp;
    int32_t n_tw;
    mbt_ref_resonator tw[MAX_RES];
    double *T; /* transverse wake table, rebuilt by prepare() */
    int lrrw_on;
    mbt_ref_lrrw lrrw;
    double *H; /* [turns][M] centroid history of the long-range wall */
    /* particles */
    int64_t N;
    double *tau, *delta;
    double *x, *xp; /* transverse coordinates (with the plane on) */
    uint64_t seed;
    int64_t turn;
    int prepared;
    char err[256];
};

static int fail(mbt_ref_sim *s, int code, const char *fmt, ...)
{
    if (s) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(s->err, sizeof s->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

const char *mbt_ref_last_error(const mbt_ref_sim *s) { return s ? s->err : "null simulation"; }

int mbt_ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int mbt_ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Synchronous phase: the RF (plus harmonic cavity) restores exactly U0 at
 * tau = 0, and the branch is chosen so that alpha_c * dV/dphase > 0 (the
 * stable one for either sign of the momentum compaction). */
static int solve_phi_s(mbt_ref_sim *s)
{
    double sin_phi = s->ring.u0_eV / s->ring.v_rf_V;
    if (s->hc_on)
        sin_phi -= s->hc.v_ratio * sin(s->hc.phase_n_rad);
    if (!(fabs(sin_phi) <= 1.0))
        return fail(s, MBT_REF_EINVAL, "no synchronous phase: |sin phi_s| = %g > 1", fabs(sin_phi));
    double phi = asin(sin_phi);
    s->phi_s = (s->ring.alpha_c > 0.0) ? phi : (PI - phi);
    return MBT_REF_OK;
}

int mbt_ref_create(const mbt_ref_ring *ring, mbt_ref_sim **out)
{
    if (!ring || !out)
        return MBT_REF_EINVAL;
    *out = NULL;
    const mbt_ref_ring *r = ring;
    if (!(r->energy_eV > 0.0) || !isfinite(r->energy_eV) || !(r->f_rf_Hz > 0.0) ||
        !isfinite(r->f_rf_Hz) || !(r->v_rf_V > 0.0) || !isfinite(r->v_rf_V) ||
        !isfinite(r->alpha_c) || r->alpha_c == 0.0 || !(r->u0_eV >= 0.0) ||
        !isfinite(r->u0_eV) || !(r->tau_long_s > 0.0) || !(r->sigma_delta >= 0.0) ||
        !isfinite(r->sigma_delta) || r->harmonic < 1 || !(r->u0_eV < r->v_rf_V))
        return MBT_REF_EINVAL;
    mbt_ref_sim *s = calloc(1, sizeof *s);
    if (!s)
        return MBT_REF_ENOMEM;
    s->ring = *r;
    /* Revolution period from the RF: h buckets of 1/f_rf each. */
    s->T0 = (double)r->harmonic / r->f_rf_Hz;
    s->T_rf = 1.0 / r->f_rf_Hz;
    s->w_rf = TWO_PI * r->f_rf_Hz;
    /* Eq. 5: one damping coefficient D per turn; with damping on delta alone
     * the amplitude decays as (1-D)^(n/2), so D = 2 T0 / tau_L. */
    s->D = 2.0 * s->T0 / r->tau_long_s;
    s->noise = r->sigma_delta * sqrt(2.0 * s->D);
    /* Eq. 2 drift coefficient. */
    s->drift = r->alpha_c * s->T0;
    int rc = solve_phi_s(s);
    if (rc) {
        free(s);
        return rc;
    }
    *out = s;
    return MBT_REF_OK;
}

void mbt_ref_destroy(mbt_ref_sim *s)
{
    if (!s)
        return;
    free(s->bucket);
    free(s->current);
    free(s->stream);
    free(s->W);
    free(s->gap);
    free(s->tau);
    free(s->delta);
    free(s->x);
    free(s->xp);
    free(s->T);
    free(s->H);
    free(s);
}

int mbt_ref_derived(const mbt_ref_sim *s, double out[5])
{
    if (!s || !out)
        return MBT_REF_EINVAL;
    out[0] = s->phi_s;
    out[1] = s->T0;
    out[2] = s->D;
    out[3] = s->noise;
    out[4] = s->drift;
    return MBT_REF_OK;
}

int mbt_ref_set_harmonic_cavity(mbt_ref_sim *s, const mbt_ref_hc *hc)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (hc && (hc->n < 2 || !isfinite(hc->v_ratio) || hc->v_ratio < 0.0 ||
               !isfinite(hc->phase_n_rad)))
        return fail(s, MBT_REF_EINVAL, "bad harmonic cavity");
    int old_on = s->hc_on;
    mbt_ref_hc old = s->hc;
    s->hc_on = hc != NULL;
    if (hc)
        s->hc = *hc;
    int rc = solve_phi_s(s);
    if (rc) {
        s->hc_on = old_on;
        s->hc = old;
        solve_phi_s(s);
    }
    return rc;
}

int mbt_ref_set_fill(mbt_ref_sim *s, int32_t M, const int32_t *bucket, const double *current_A,
                     const int32_t *stream)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (s->tau)
        return fail(s, MBT_REF_ESTATE, "fill must be set before particles");
    if (M < 1 || M > s->ring.harmonic || !bucket || !current_A)
        return fail(s, MBT_REF_EINVAL, "bad fill size");
    for (int32_t b = 0; b < M; ++b) {
        if (bucket[b] < 0 || bucket[b] >= s->ring.harmonic || (b > 0 && bucket[b] <= bucket[b - 1]))
            return fail(s, MBT_REF_EINVAL, "buckets must be strictly increasing in [0,h)");
        if (!(current_A[b] >= 0.0) || !isfinite(current_A[b]))
            return fail(s, MBT_REF_EINVAL, "bunch currents must be finite and >= 0");
        if (stream && stream[b] < 0)
            return fail(s, MBT_REF_EINVAL, "stream ordinals must be >= 0");
    }
    free(s->bucket);
    free(s->current);
    free(s->stream);
    s->bucket = malloc(sizeof(int32_t) * (size_t)M);
    s->current = malloc(sizeof(double) * (size_t)M);
    s->stream = malloc(sizeof(int32_t) * (size_t)M);
    if (!s->bucket || !s->current || !s->stream)
        return fail(s, MBT_REF_ENOMEM, "out of memory");
    for (int32_t b = 0; b < M; ++b) {
        s->bucket[b] = bucket[b];
        s->current[b] = current_A[b];
        s->stream[b] = stream ? stream[b] : b;
    }
    s->M = M;
    free(s->H);
    s->H = NULL;
    s->prepared = 0;
    return MBT_REF_OK;
}

int mbt_ref_set_short_range(mbt_ref_sim *s, int32_t nres, const mbt_ref_resonator *res,
                            const mbt_ref_grid *g)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (!g) {
        s->sr_on = 0;
        s->n_sr = 0;
        s->prepared = 0;
        return MBT_REF_OK;
    }
    if (!grid_ok(g) || nres < 0 || nres > MAX_RES || (nres > 0 && !res))
        return fail(s, MBT_REF_EINVAL, "bad short-range wake or grid");
    for (int32_t i = 0; i < nres; ++i)
        if (!res_ok(&res[i]))
            return fail(s, MBT_REF_EINVAL, "resonator %d: need Rs >= 0, Q > 0.5, fr > 0", i);
    s->sr_on = 1;
    s->grid = *g;
    s->n_sr = nres;
    for (int32_t i = 0; i < nres; ++i)
        s->sr[i] = res[i];
    s->prepared = 0;
    return MBT_REF_OK;
}

int mbt_ref_set_long_range(mbt_ref_sim *s, int32_t nres, const mbt_ref_resonator *res)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (nres < 0 || nres > MAX_RES || (nres > 0 && !res))
        return fail(s, MBT_REF_EINVAL, "bad long-range resonator list");
    for (int32_t i = 0; i < nres; ++i)
        if (!res_ok(&res[i]))
            return fail(s, MBT_REF_EINVAL, "resonator %d: need Rs >= 0, Q > 0.5, fr > 0", i);
    s->n_lr = nres;
    for (int32_t i = 0; i < nres; ++i) {
        s->lr[i] = res[i];
        double wr = TWO_PI * res[i].fr_Hz;
        double alpha = wr / (2.0 * res[i].q);
        double wbar = sqrt(wr * wr - alpha * alpha);
        s->lr_alpha[i] = alpha;
        s->lr_wbar[i] = wbar;
        /* W(t) = Re[c exp((-alpha + i wbar) t)] with c = 2 alpha Rs (1 + i alpha/wbar). */
        s->lr_c[i] = 2.0 * alpha * res[i].rs_ohm * (1.0 + I * (alpha / wbar));
        s->phasor[i] = 0.0;
    }
    s->prepared = 0;
    return MBT_REF_OK;
}

int mbt_ref_set_resistive_wall(mbt_ref_sim *s, const mbt_ref_rw *rw)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (rw && !rw_ok(rw))
        return fail(s, MBT_REF_EINVAL, "resistive wall: need radius, conductivity, length > 0");
    s->rw_on = rw != NULL;
    if (rw)
        s->rw = *rw;
    s->prepared = 0;
    return MBT_REF_OK;
}

/* Build the wake table (short-range resonators plus the long-range ones, whose
 * same-bunch same-turn part acts through the bins) and the gap rotations. */
static int prepare(mbt_ref_sim *s)
{
    if (s->prepared)
        return MBT_REF_OK;
    if (s->M < 1)
        return fail(s, MBT_REF_ESTATE, "fill not set");
    free(s->W);
    s->W = NULL;
    if (s->sr_on) {
        mbt_ref_resonator all[2 * MAX_RES];
        int32_t n = 0;
        for (int32_t i = 0; i < s->n_sr; ++i)
            all[n++] = s->sr[i];
        for (int32_t i = 0; i < s->n_lr; ++i)
            all[n++] = s->lr[i];
        s->W = malloc(sizeof(double) * (size_t)s->grid.nbins);
        if (!s->W)
            return fail(s, MBT_REF_ENOMEM, "out of memory");
        int rc = mbt_ref_wake_table_rw(n, all, s->rw_on ? &s->rw : NULL, &s->grid, s->W);
        if (rc)
            return fail(s, rc, "wake table");
    }
    free(s->T);
    s->T = NULL;
    if (s->sr_on && s->tr_on) {
        s->T = malloc(sizeof(double) * (size_t)s->grid.nbins);
        if (!s->T)
            return fail(s, MBT_REF_ENOMEM, "out of memory");
        int rc = mbt_ref_transverse_wake_table(s->n_tw, s->tw, &s->grid, s->T);
        if (rc)
            return fail(s, rc, "transverse wake table");
    }
    if (s->tr_on && s->lrrw_on && !s->H) {
        s->H = calloc((size_t)s->lrrw.turns * (size_t)s->M, sizeof(double));
        if (!s->H)
            return fail(s, MBT_REF_ENOMEM, "out of memory");
    }
    free(s->gap);
    s->gap = NULL;
    if (s->n_lr > 0) {
        s->gap = malloc(sizeof(double complex) * (size_t)s->n_lr * (size_t)s->M);
        if (!s->gap)
            return fail(s, MBT_REF_ENOMEM, "out of memory");
        for (int32_t r = 0; r < s->n_lr; ++r) {
            for (int32_t b = 0; b < s->M; ++b) {
                /* Buckets between the previous filled bucket and this one;
                 * the first bunch follows the last one of the previous turn. */
                int32_t g = (b == 0) ? (s->ring.harmonic - s->bucket[s->M - 1] + s->bucket[0])
                                     : (s->bucket[b] - s->bucket[b - 1]);
                double t = (double)g * s->T_rf;
                s->gap[(size_t)r * s->M + b] =
                    exp(-s->lr_alpha[r] * t) *
                    (cos(s->lr_wbar[r] * t) + I * sin(s->lr_wbar[r] * t));
            }
        }
    }
    s->prepared = 1;
    return MBT_REF_OK;
}

int mbt_ref_alloc_particles(mbt_ref_sim *s, int64_t N, uint64_t seed)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (s->M < 1)
        return fail(s, MBT_REF_ESTATE, "fill not set");
    if (N < 1 || N > ((int64_t)1 << 33))
        return fail(s, MBT_REF_EINVAL, "N must be in [1, 2^33]");
    size_t n = (size_t)s->M * (size_t)N;
    free(s->tau);
    free(s->delta);
    s->tau = calloc(n, sizeof(double));
    s->delta = calloc(n, sizeof(double));
    if (!s->tau || !s->delta) {
        free(s->tau);
        free(s->delta);
        s->tau = s->delta = NULL;
        return fail(s, MBT_REF_ENOMEM, "out of memory for %zu particles", n);
    }
    free(s->x);
    free(s->xp);
    s->x = s->xp = NULL;
    if (s->tr_on) {
        s->x = calloc(n, sizeof(double));
        s->xp = calloc(n, sizeof(double));
        if (!s->x || !s->xp)
            return fail(s, MBT_REF_ENOMEM, "out of memory for %zu transverse particles", n);
    }
    s->N = N;
    s->seed = seed;
    s->turn = 0;
    for (int32_t r = 0; r < MAX_RES; ++r)
        s->phasor[r] = 0.0;
    if (s->H)
        memset(s->H, 0, sizeof(double) * (size_t)s->lrrw.turns * (size_t)s->M);
    return MBT_REF_OK;
}

/* Initial distribution: independent Gaussians in tau and delta, one
 * Box-Muller pair per particle from the INIT stream (tag 1). */
int mbt_ref_init_gaussian(mbt_ref_sim *s, int64_t N, double sigma_tau_s, double sigma_delta,
                          uint64_t seed)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (!(sigma_tau_s >= 0.0) || !(sigma_delta >= 0.0) || !isfinite(sigma_tau_s) ||
        !isfinite(sigma_delta))
        return fail(s, MBT_REF_EINVAL, "sigmas must be finite and >= 0");
    int rc = mbt_ref_alloc_particles(s, N, seed);
    if (rc)
        return rc;
    for (int32_t b = 0; b < s->M; ++b) {
        double *tau = s->tau + (size_t)b * (size_t)N;
        double *del = s->delta + (size_t)b * (size_t)N;
        for (int64_t j = 0; j < N; ++j) {
            uint32_t c[4] = {(uint32_t)j, (uint32_t)s->stream[b], 0u, 1u};
            double z[2];
            mbt_ref_normal_pair(seed, c, z);
            tau[j] = sigma_tau_s * z[0];
            del[j] = sigma_delta * z[1];
        }
    }
    return MBT_REF_OK;
}

int mbt_ref_set_particles(mbt_ref_sim *s, int32_t bunch, const double *tau, const double *delta)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (!s->tau)
        return fail(s, MBT_REF_ESTATE, "particles not allocated");
    if (bunch < 0 || bunch >= s->M || !tau || !delta)
        return fail(s, MBT_REF_EINVAL, "bad bunch index or null array");
    memcpy(s->tau + (size_t)bunch * (size_t)s->N, tau, sizeof(double) * (size_t)s->N);
    memcpy(s->delta + (size_t)bunch * (size_t)s->N, delta, sizeof(double) * (size_t)s->N);
    return MBT_REF_OK;
}

int mbt_ref_get_particles(const mbt_ref_sim *s, int32_t bunch, double *tau, double *delta)
{
    if (!s || !s->tau || bunch < 0 || bunch >= s->M || !tau || !delta)
        return MBT_REF_EINVAL;
    memcpy(tau, s->tau + (size_t)bunch * (size_t)s->N, sizeof(double) * (size_t)s->N);
    memcpy(delta, s->delta + (size_t)bunch * (size_t)s->N, sizeof(double) * (size_t)s->N);
    return MBT_REF_OK;
}

int mbt_ref_set_transverse(mbt_ref_sim *s, const mbt_ref_transverse *tr)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (!tr) {
        s->tr_on = 0;
        free(s->x);
        free(s->xp);
        s->x = s->xp = NULL;
        s->prepared = 0;
        return MBT_REF_OK;
    }
    if (!isfinite(tr->tune) || !isfinite(tr->chromaticity) || !isfinite(tr->alpha) ||
        !(tr->beta_m > 0.0) || !isfinite(tr->beta_m) || !isfinite(tr->disp_m) ||
        !isfinite(tr->disp_prime) || !(tr->emittance_m >= 0.0) || !isfinite(tr->emittance_m) ||
        !(tr->tau_damp_s > 0.0))
        return fail(s, MBT_REF_EINVAL, "bad transverse plane");
    s->tr = *tr;
    /* the one-turn matrix depends on the phase modulo 2 pi: the integer part
     * of the tune is dropped, exactly (Sterbenz) */
    s->tr_qfrac = tr->tune - floor(tr->tune);
    s->tr_gamma = (1.0 + tr->alpha * tr->alpha) / tr->beta_m;
    /* Eq. 5: noise sigma sqrt(D_x) with D_x = 2 T0 / tau (as for delta) */
    double dx = 2.0 * s->T0 / tr->tau_damp_s;
    s->tr_noise_x = sqrt(tr->emittance_m * tr->beta_m) * sqrt(dx);
    s->tr_noise_xp = sqrt(tr->emittance_m * s->tr_gamma) * sqrt(dx);
    if (!s->tr_on && s->tau) {
        size_t n = (size_t)s->M * (size_t)s->N;
        s->x = calloc(n, sizeof(double));
        s->xp = calloc(n, sizeof(double));
        if (!s->x || !s->xp) {
            free(s->x);
            free(s->xp);
            s->x = s->xp = NULL;
            return fail(s, MBT_REF_ENOMEM, "out of memory");
        }
    }
    s->tr_on = 1;
    s->prepared = 0;
    return MBT_REF_OK;
}

int mbt_ref_set_transverse_wake(mbt_ref_sim *s, int32_t nres, const mbt_ref_resonator *res)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (nres < 0 || nres > MAX_RES || (nres > 0 && !res))
        return fail(s, MBT_REF_EINVAL, "bad transverse resonator list");
    for (int32_t i = 0; i < nres; ++i)
        if (!res_ok(&res[i]))
            return fail(s, MBT_REF_EINVAL, "resonator %d: need Rs >= 0, Q > 0.5, fr > 0", i);
    s->n_tw = nres;
    for (int32_t i = 0; i < nres; ++i)
        s->tw[i] = res[i];
    s->prepared = 0;
    return MBT_REF_OK;
}

int mbt_ref_set_transverse_rw(mbt_ref_sim *s, const mbt_ref_lrrw *rw)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (rw) {
        mbt_ref_rw w = {rw->radius_m, rw->conductivity_S_m, rw->length_m};
        if (!rw_ok(&w) || rw->turns < 1 || rw->turns > 1024)
            return fail(s, MBT_REF_EINVAL, "resistive wall: need radius, conductivity, length > 0 "
                                           "and 1 <= turns <= 1024");
        s->lrrw = *rw;
    }
    s->lrrw_on = rw != NULL;
    free(s->H);
    s->H = NULL;
    s->prepared = 0;
    return MBT_REF_OK;
}

/* Matched Gaussian betatron coordinates from the INIT stream, tag 4: one
 * Box-Muller pair per particle, z0 for x and z1 for x'. */
int mbt_ref_init_transverse(mbt_ref_sim *s, double emittance_m, double offset_m)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (!s->tr_on || !s->x)
        return fail(s, MBT_REF_ESTATE, "transverse plane or particles not set");
    if (!(emittance_m >= 0.0) || !isfinite(emittance_m) || !isfinite(offset_m))
        return fail(s, MBT_REF_EINVAL, "emittance must be finite and >= 0");
    const double sx = sqrt(emittance_m * s->tr.beta_m), sxp = sqrt(emittance_m / s->tr.beta_m);
    for (int32_t b = 0; b < s->M; ++b) {
        double *x = s->x + (size_t)b * (size_t)s->N;
        double *xp = s->xp + (size_t)b * (size_t)s->N;
        for (int64_t j = 0; j < s->N; ++j) {
            uint32_t c[4] = {(uint32_t)j, (uint32_t)s->stream[b], 0u, 4u};
            double z[2];
            mbt_ref_normal_pair(s->seed, c, z);
            x[j] = offset_m + sx * z[0];
            xp[j] = sxp * (z[1] - s->tr.alpha * z[0]);
        }
    }
    if (s->H)
        memset(s->H, 0, sizeof(double) * (size_t)s->lrrw.turns * (size_t)s->M);
    return MBT_REF_OK;
}

int mbt_ref_set_transverse_particles(mbt_ref_sim *s, int32_t bunch, const double *x,
                                     const double *xp)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (!s->x)
        return fail(s, MBT_REF_ESTATE, "transverse particles not allocated");
    if (bunch < 0 || bunch >= s->M || !x || !xp)
        return fail(s, MBT_REF_EINVAL, "bad bunch index or null array");
    memcpy(s->x + (size_t)bunch * (size_t)s->N, x, sizeof(double) * (size_t)s->N);
    memcpy(s->xp + (size_t)bunch * (size_t)s->N, xp, sizeof(double) * (size_t)s->N);
    return MBT_REF_OK;
}

int mbt_ref_get_transverse_particles(const mbt_ref_sim *s, int32_t bunch, double *x, double *xp)
{
    if (!s || !s->x || bunch < 0 || bunch >= s->M || !x || !xp)
        return MBT_REF_EINVAL;
    memcpy(x, s->x + (size_t)bunch * (size_t)s->N, sizeof(double) * (size_t)s->N);
    memcpy(xp, s->xp + (size_t)bunch * (size_t)s->N, sizeof(double) * (size_t)s->N);
    return MBT_REF_OK;
}

int mbt_ref_get_rw_history(const mbt_ref_sim *s, double *H)
{
    if (!s || !H || !s->lrrw_on || s->M < 1)
        return MBT_REF_EINVAL;
    size_t n = (size_t)s->lrrw.turns * (size_t)s->M;
    if (s->H)
        memcpy(H, s->H, sizeof(double) * n);
    else
        memset(H, 0, sizeof(double) * n);
    return MBT_REF_OK;
}

int mbt_ref_set_rw_history(mbt_ref_sim *s, const double *H)
{
    if (!s || !H)
        return MBT_REF_EINVAL;
    if (!s->lrrw_on || !s->tr_on || s->M < 1)
        return fail(s, MBT_REF_ESTATE, "no long-range resistive wall");
    int rc = prepare(s);
    if (rc)
        return rc;
    memcpy(s->H, H, sizeof(double) * (size_t)s->lrrw.turns * (size_t)s->M);
    return MBT_REF_OK;
}

int mbt_ref_get_state(const mbt_ref_sim *s, int64_t *turn, uint64_t *seed, double *phasors)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (turn)
        *turn = s->turn;
    if (seed)
        *seed = s->seed;
    if (phasors)
        for (int32_t r = 0; r < s->n_lr; ++r) {
            phasors[2 * r] = creal(s->phasor[r]);
            phasors[2 * r + 1] = cimag(s->phasor[r]);
        }
    return MBT_REF_OK;
}

int mbt_ref_set_state(mbt_ref_sim *s, int64_t turn, uint64_t seed, const double *phasors)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (turn < 0 || turn > (int64_t)UINT32_MAX)
        return fail(s, MBT_REF_EINVAL, "turn out of range");
    s->turn = turn;
    s->seed = seed;
    if (phasors)
        for (int32_t r = 0; r < s->n_lr; ++r)
            s->phasor[r] = phasors[2 * r] + I * phasors[2 * r + 1];
    return MBT_REF_OK;
}

/* Neumaier's compensated summation, used for the bunch statistics. */
typedef struct {
    double sum, comp;
} csum;

static void csum_add(csum *c, double x)
{
    double t = c->sum + x;
    if (fabs(c->sum) >= fabs(x))
        c->comp += (c->sum - t) + x;
    else
        c->comp += (x - t) + c->sum;
    c->sum = t;
}

static double csum_get(const csum *c) { return c->sum + c->comp; }

/* Sec. 2.4: mean and rms of tau and delta over all N particles (population
 * rms), two passes. */
static void bunch_moments(int64_t N, const double *tau, const double *del, double m[4])
{
    csum st = {0, 0}, sd = {0, 0};
    for (int64_t j = 0; j < N; ++j) {
        csum_add(&st, tau[j]);
        csum_add(&sd, del[j]);
    }
    double mt = csum_get(&st) / (double)N;
    double md = csum_get(&sd) / (double)N;
    csum vt = {0, 0}, vd = {0, 0};
    for (int64_t j = 0; j < N; ++j) {
        csum_add(&vt, (tau[j] - mt) * (tau[j] - mt));
        csum_add(&vd, (del[j] - md) * (del[j] - md));
    }
    m[0] = mt;
    m[1] = md;
    m[2] = sqrt(csum_get(&vt) / (double)N);
    m[3] = sqrt(csum_get(&vd) / (double)N);
}

/* One turn of one bunch: binning, wake potential, long-range voltage seen,
 * then the single-particle map for every particle, then the bunch's deposit
 * into the long-range phasors. */
static int track_bunch(mbt_ref_sim *s, int32_t b, uint32_t *counts, double *V, double *dep,
                       double *X, double *U)
{
    const int64_t N = s->N;
    double *tau = s->tau + (size_t)b * (size_t)N;
    double *del = s->delta + (size_t)b * (size_t)N;
    const int tr_on = s->tr_on;
    double *xs = tr_on ? s->x + (size_t)b * (size_t)N : NULL;
    double *xps = tr_on ? s->xp + (size_t)b * (size_t)N : NULL;
    /* Charge carried by one macro-particle: bunch charge I_b T0 over N. */
    const double q_pp = s->current[b] * s->T0 / (double)N;

    /* Sec. 2.3: assign particles to bins, count them (and sum their x: the
     * bins' dipole moments), build the wake potential of the bunch at every
     * bin and, with the transverse plane, every bin's transverse kick. */
    if (s->sr_on) {
        if (tr_on) {
            mbt_ref_dipole_histogram(&s->grid, N, tau, xs, counts, X);
            mbt_ref_transverse_kicks(s->grid.nbins, s->T, X, q_pp / s->ring.energy_eV, U);
        } else {
            mbt_ref_histogram(&s->grid, N, tau, counts, NULL);
        }
        mbt_ref_wake_potential(s->grid.nbins, s->W, counts, q_pp, V);
    }

    /* Long-range resonators: rotate each phasor across the gap from the
     * previous filled bucket; this is the voltage the bunch sees. */
    double complex seen[MAX_RES];
    for (int32_t r = 0; r < s->n_lr; ++r) {
        s->phasor[r] *= s->gap[(size_t)r * s->M + b];
        seen[r] = s->phasor[r];
    }

    /* Deposit terms exp((alpha - i wbar) tau_j), taken on tau before the drift. */
    const int32_t n_lr = s->n_lr;
#pragma omp parallel for schedule(static) if (N >= 4096)
    for (int64_t j = 0; j < N; ++j) {
        for (int32_t r = 0; r < n_lr; ++r) {
            double e = exp(s->lr_alpha[r] * tau[j]);
            dep[(size_t)(2 * r) * N + j] = e * cos(s->lr_wbar[r] * tau[j]);
            dep[(size_t)(2 * r + 1) * N + j] = -e * sin(s->lr_wbar[r] * tau[j]);
        }
    }

    const double E0 = s->ring.energy_eV, Vrf = s->ring.v_rf_V, U0 = s->ring.u0_eV;
    const double w = s->w_rf, phi_s = s->phi_s, D = s->D, noise = s->noise, drift = s->drift;
    const int hc_on = s->hc_on;
    const double k_hc = s->hc.v_ratio, nphi = s->hc.phase_n_rad, n_hc = (double)s->hc.n;
    const int sr_on = s->sr_on;
    const uint32_t stream = (uint32_t)s->stream[b], turn = (uint32_t)s->turn;
    const uint64_t seed = s->seed;

#pragma omp parallel for schedule(static) if (N >= 4096)
    for (int64_t j = 0; j < N; ++j) {
        double t = tau[j];
        const double d_in = del[j];
        /* Eq. 1: energy gain in the RF (main cavity plus harmonic cavity)
         * minus the energy radiated per turn. */
        double e_rf = Vrf * sin(phi_s - w * t);
        if (hc_on)
            e_rf += k_hc * Vrf * sin(nphi - n_hc * w * t);
        double dE = e_rf - U0;
        /* Eq. 6: every particle in bin k loses the bunch's wake voltage V[k];
         * particles outside the grid get no short-range kick. */
        int32_t k = -1;
        if (sr_on) {
            k = mbt_ref_bin_index(&s->grid, t);
            if (k >= 0)
                dE -= V[k];
        }
        if (tr_on) {
            /* Eq. 6, second line: the bin's transverse wake kick. */
            double xp = xps[j];
            if (k >= 0)
                xp += U[k];
            /* Eqs. 3-4: betatron rotation about the dispersive orbit
             * (D delta, D' delta) by the chromatic phase advance. */
            const double psi = TWO_PI * (s->tr_qfrac + s->tr.chromaticity * d_in);
            const double cs = cos(psi), sn = sin(psi);
            const double al = s->tr.alpha, be = s->tr.beta_m, ga = s->tr_gamma;
            const double xb = xs[j] - s->tr.disp_m * d_in;
            const double xpb = xp - s->tr.disp_prime * d_in;
            double x2 = s->tr.disp_m * d_in + (cs + al * sn) * xb + be * sn * xpb;
            double xp2 = s->tr.disp_prime * d_in - ga * sn * xb + (cs - al * sn) * xpb;
            /* Eq. 5: x' shrinks by the momentum ratio across the RF energy
             * gain (adiabatic damping), then both get their noise. */
            xp2 = xp2 * ((1.0 + d_in) / (1.0 + d_in + e_rf / E0));
            if (s->tr_noise_x > 0.0 || s->tr_noise_xp > 0.0) {
                uint32_t cx[4] = {(uint32_t)(j >> 1), stream, turn, 2u};
                uint32_t cxp[4] = {(uint32_t)(j >> 1), stream, turn, 3u};
                double zx[2], zxp[2];
                mbt_ref_normal_pair(seed, cx, zx);
                mbt_ref_normal_pair(seed, cxp, zxp);
                x2 += s->tr_noise_x * zx[j & 1];
                xp2 += s->tr_noise_xp * zxp[j & 1];
            }
            xs[j] = x2;
            xps[j] = xp2;
        }
        /* Long-range: voltage Re[V~ exp((-alpha + i wbar) tau)]. */
        for (int32_t r = 0; r < n_lr; ++r) {
            double e = exp(-s->lr_alpha[r] * t);
            double c = cos(s->lr_wbar[r] * t), sn = sin(s->lr_wbar[r] * t);
            dE -= e * (creal(seen[r]) * c - cimag(seen[r]) * sn);
        }
        double d = d_in + dE / E0;
        /* Eq. 5: radiation damping and quantum excitation. */
        d = d * (1.0 - D);
        if (noise > 0.0) {
            uint32_t c[4] = {(uint32_t)(j >> 1), stream, turn, 0u};
            double z[2];
            mbt_ref_normal_pair(seed, c, z);
            d += noise * z[j & 1];
        }
        del[j] = d;
        /* Eq. 2: drift with the updated energy deviation. */
        tau[j] = t + drift * d;
    }

    /* The bunch's passage adds q_pp * c * sum_j exp((alpha - i wbar) tau_j)
     * to each long-range phasor. */
    for (int32_t r = 0; r < n_lr; ++r) {
        csum re = {0, 0}, im = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            csum_add(&re, dep[(size_t)(2 * r) * N + j]);
            csum_add(&im, dep[(size_t)(2 * r + 1) * N + j]);
        }
        double complex A = csum_get(&re) + I * csum_get(&im);
        s->phasor[r] += q_pp * s->lr_c[r] * A;
    }
    return MBT_REF_OK;
}

/* Sec. 2.3, last paragraph: once every bunch has passed and its statistics
 * are updated, each bunch b gets the long-range resistive-wall kick of the
 * passages before its own in that turn: bunches b' < b of the same turn and
 * every bunch of the earlier turns kept in the history, each source a rigid
 * dipole of charge I_b' T0 at its centroid.  `target` is the turn whose
 * passages receive the kick; H holds the centroids of turns target-K+1 ..
 * target.  kick[b] is added to x' of every particle of bunch b. */
static void rw_kicks(const mbt_ref_sim *s, int64_t target, double *kick)
{
    const int32_t K = s->lrrw.turns, M = s->M;
    const mbt_ref_rw w = {s->lrrw.radius_m, s->lrrw.conductivity_S_m, s->lrrw.length_m};
    for (int32_t b = 0; b < M; ++b) {
        double acc = 0.0;
        for (int32_t age = K - 1; age >= 0; --age) { /* oldest source turn first */
            const int64_t m = target - age;
            if (m < 0)
                continue;
            const double *row = s->H + (size_t)(m % K) * (size_t)M;
            for (int32_t bs = 0; bs < M; ++bs) {
                if (age == 0 && bs >= b)
                    break;
                const double dt = (double)age * s->T0 +
                                  (double)(s->bucket[b] - s->bucket[bs]) * s->T_rf;
                acc += s->current[bs] * s->T0 * row[bs] * mbt_ref_transverse_rw_wake(&w, dt);
            }
        }
        kick[b] = acc / s->ring.energy_eV;
    }
}

int mbt_ref_track(mbt_ref_sim *s, int64_t nturns, double *moments, uint32_t *counts,
                  int32_t stride)
{
    return mbt_ref_track2(s, nturns, moments, NULL, counts, stride);
}

int mbt_ref_track2(mbt_ref_sim *s, int64_t nturns, double *moments, double *tmoments,
                   uint32_t *counts, int32_t stride)
{
    if (!s)
        return MBT_REF_EINVAL;
    if (tmoments && !s->tr_on)
        return fail(s, MBT_REF_EINVAL, "transverse moments need the transverse plane");
    if (!s->tau)
        return fail(s, MBT_REF_ESTATE, "particles not initialised");
    if (nturns < 0 || s->turn + nturns > (int64_t)UINT32_MAX + 1)
        return fail(s, MBT_REF_EINVAL, "bad turn count");
    if (counts && (!s->sr_on || stride < 1))
        return fail(s, MBT_REF_EINVAL, "profiles need a grid and stride >= 1");
    int rc = prepare(s);
    if (rc)
        return rc;
    const int32_t nb = s->sr_on ? s->grid.nbins : 1;
    const int rw = s->tr_on && s->lrrw_on;
    uint32_t *cnt = malloc(sizeof(uint32_t) * (size_t)nb);
    double *V = malloc(sizeof(double) * (size_t)nb);
    double *X = malloc(sizeof(double) * (size_t)nb);
    double *U = malloc(sizeof(double) * (size_t)nb);
    double *kick = malloc(sizeof(double) * (size_t)s->M);
    double *dep = s->n_lr ? malloc(sizeof(double) * 2 * (size_t)s->n_lr * (size_t)s->N) : NULL;
    if (!cnt || !V || !X || !U || !kick || (s->n_lr && !dep)) {
        free(cnt);
        free(V);
        free(X);
        free(U);
        free(kick);
        free(dep);
        return fail(s, MBT_REF_ENOMEM, "out of memory");
    }
    rc = MBT_REF_OK;
    for (int64_t t = 0; t < nturns && !rc; ++t) {
        if (rw) {
            /* the wall's kick of the previous turn's passages, given after
             * all bunches of that turn (applied here, before this turn) */
            rw_kicks(s, s->turn - 1, kick);
            for (int32_t b = 0; b < s->M; ++b)
                for (int64_t j = 0; j < s->N; ++j)
                    s->xp[(size_t)b * s->N + j] += kick[b];
        }
        for (int32_t b = 0; b < s->M; ++b) {
            track_bunch(s, b, cnt, V, dep, X, U);
            double m[4];
            bunch_moments(s->N, s->tau + (size_t)b * s->N, s->delta + (size_t)b * s->N, m);
            if (!isfinite(m[0]) || !isfinite(m[1]) || !isfinite(m[2]) || !isfinite(m[3])) {
                rc = fail(s, MBT_REF_ENUMERIC, "non-finite moment at turn %lld bunch %d",
                          (long long)s->turn, b);
                break;
            }
            if (moments)
                memcpy(moments + ((size_t)t * s->M + b) * 4, m, sizeof m);
            if (s->tr_on) {
                double mx[4];
                bunch_moments(s->N, s->x + (size_t)b * s->N, s->xp + (size_t)b * s->N, mx);
                if (!isfinite(mx[0]) || !isfinite(mx[1]) || !isfinite(mx[2]) || !isfinite(mx[3])) {
                    rc = fail(s, MBT_REF_ENUMERIC, "non-finite transverse moment at turn %lld "
                              "bunch %d", (long long)s->turn, b);
                    break;
                }
                if (tmoments)
                    memcpy(tmoments + ((size_t)t * s->M + b) * 4, mx, sizeof mx);
                if (rw)
                    s->H[(size_t)(s->turn % s->lrrw.turns) * s->M + b] = mx[0];
            }
        }
        if (rc)
            break;
        if (counts && t % stride == 0) {
            size_t row = (size_t)(t / stride);
            for (int32_t b = 0; b < s->M; ++b)
                mbt_ref_histogram(&s->grid, s->N, s->tau + (size_t)b * s->N,
                                  counts + (row * s->M + b) * (size_t)nb, NULL);
        }
        s->turn += 1;
    }
    free(cnt);
    free(V);
    free(X);
    free(U);
    free(kick);
    free(dep);
    return rc;
}
