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
    /* particles */
    int64_t N;
    double *tau, *delta;
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
    s->N = N;
    s->seed = seed;
    s->turn = 0;
    for (int32_t r = 0; r < MAX_RES; ++r)
        s->phasor[r] = 0.0;
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
static int track_bunch(mbt_ref_sim *s, int32_t b, uint32_t *counts, double *V, double *dep)
{
    const int64_t N = s->N;
    double *tau = s->tau + (size_t)b * (size_t)N;
    double *del = s->delta + (size_t)b * (size_t)N;
    /* Charge carried by one macro-particle: bunch charge I_b T0 over N. */
    const double q_pp = s->current[b] * s->T0 / (double)N;

    /* Sec. 2.3: assign particles to bins, count them, build the wake
     * potential of the bunch at every bin. */
    if (s->sr_on) {
        mbt_ref_histogram(&s->grid, N, tau, counts, NULL);
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
        /* Eq. 1: energy gain in the RF (main cavity plus harmonic cavity)
         * minus the energy radiated per turn. */
        double dE = Vrf * sin(phi_s - w * t);
        if (hc_on)
            dE += k_hc * Vrf * sin(nphi - n_hc * w * t);
        dE -= U0;
        /* Eq. 6: every particle in bin k loses the bunch's wake voltage V[k];
         * particles outside the grid get no short-range kick. */
        if (sr_on) {
            int32_t k = mbt_ref_bin_index(&s->grid, t);
            if (k >= 0)
                dE -= V[k];
        }
        /* Long-range: voltage Re[V~ exp((-alpha + i wbar) tau)]. */
        for (int32_t r = 0; r < n_lr; ++r) {
            double e = exp(-s->lr_alpha[r] * t);
            double c = cos(s->lr_wbar[r] * t), sn = sin(s->lr_wbar[r] * t);
            dE -= e * (creal(seen[r]) * c - cimag(seen[r]) * sn);
        }
        double d = del[j] + dE / E0;
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

int mbt_ref_track(mbt_ref_sim *s, int64_t nturns, double *moments, uint32_t *counts,
                  int32_t stride)
{
    if (!s)
        return MBT_REF_EINVAL;
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
    uint32_t *cnt = malloc(sizeof(uint32_t) * (size_t)nb);
    double *V = malloc(sizeof(double) * (size_t)nb);
    double *dep = s->n_lr ? malloc(sizeof(double) * 2 * (size_t)s->n_lr * (size_t)s->N) : NULL;
    if (!cnt || !V || (s->n_lr && !dep)) {
        free(cnt);
        free(V);
        free(dep);
        return fail(s, MBT_REF_ENOMEM, "out of memory");
    }
    for (int64_t t = 0; t < nturns; ++t) {
        for (int32_t b = 0; b < s->M; ++b) {
            track_bunch(s, b, cnt, V, dep);
            double m[4];
            bunch_moments(s->N, s->tau + (size_t)b * s->N, s->delta + (size_t)b * s->N, m);
            if (!isfinite(m[0]) || !isfinite(m[1]) || !isfinite(m[2]) || !isfinite(m[3])) {
                free(cnt);
                free(V);
                free(dep);
                return fail(s, MBT_REF_ENUMERIC, "non-finite moment at turn %lld bunch %d",
                            (long long)s->turn, b);
            }
            if (moments)
                memcpy(moments + ((size_t)t * s->M + b) * 4, m, sizeof m);
        }
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
    free(dep);
    return MBT_REF_OK;
}
