/*
 * mbt_ref.h -- plain FP64 CPU reference tracker for longitudinal multi-bunch
 * macro-particle tracking (Xu, Locans, Adelmann, Stingelin, "Calculation of
 * Longitudinal Collective Instabilities with mbtrack-cuda", arXiv:1809.00391).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU tracker
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the GPU library; both are written from the
 * paper (Sec. 2.2 Eqs. 1, 2 and 5; Sec. 2.3 Eq. 6 and the binning steps;
 * Sec. 2.4 statistics) and from the same written readings of it.
 *
 * Conventions
 *   - tau is the arrival-time offset from the bucket centre in seconds
 *     (tau > 0 arrives later); delta = dE/E0 (Sec. 2.2).
 *   - All floating point is IEEE binary64; the library is built without
 *     fast-math and with floating-point contraction off.
 *   - Every call returns 0 on success or a negative MBT_REF_E* code; the
 *     message of the last failure is kept in the simulation object.
 *   - Particle arrays are bunch-major: element [b*N + j] is particle j of the
 *     b-th filled bunch (bunches ordered by increasing bucket index).
 */
#ifndef MBT_REF_H
#define MBT_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MBT_REF_OK = 0,
    MBT_REF_EINVAL = -1,   /* bad argument */
    MBT_REF_ESTATE = -2,   /* call made in the wrong order */
    MBT_REF_ENOMEM = -3,   /* host allocation failed */
    MBT_REF_ENUMERIC = -5  /* non-finite coordinate or moment */
};

typedef struct {
    double energy_eV;    /* E0, beam energy in eV                           */
    double f_rf_Hz;      /* main RF frequency                               */
    double v_rf_V;       /* main RF peak voltage                            */
    double alpha_c;      /* momentum compaction (sign kept)                 */
    double u0_eV;        /* energy radiated per turn; 0 switches SR loss off */
    double tau_long_s;   /* longitudinal amplitude damping time; +inf = off */
    double sigma_delta;  /* equilibrium relative energy spread; 0 = no noise*/
    int32_t harmonic;    /* h, buckets per turn                             */
} mbt_ref_ring;

typedef struct {
    int32_t n;           /* harmonic of the cavity (n >= 2)                 */
    double v_ratio;      /* k = V_hc / V_rf                                 */
    double phase_n_rad;  /* n * phi_h: cavity phase in its own radians      */
} mbt_ref_hc;

typedef struct {
    double rs_ohm;       /* shunt impedance                                 */
    double q;            /* quality factor, > 0.5                           */
    double fr_Hz;        /* resonant frequency                              */
} mbt_ref_resonator;

typedef struct {
    int32_t nbins;       /* number of bins, 1..4096                          */
    double tau_min_s;    /* grid covers [tau_min, tau_max)                  */
    double tau_max_s;
} mbt_ref_grid;

/* Round resistive pipe: radius b, DC conductivity, length (the paper's
 * validation used a copper chamber of 10 mm radius around the whole ring). */
typedef struct {
    double radius_m;
    double conductivity_S_m;
    double length_m;
} mbt_ref_rw;

typedef struct mbt_ref_sim mbt_ref_sim;

/* ---- free functions (also used as pins) ---------------------------------- */

/* Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void mbt_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* One Box-Muller pair from Philox(key = seed, counter = c).  z[0] uses the
 * cosine branch, z[1] the sine branch. */
void mbt_ref_normal_pair(uint64_t seed, const uint32_t c[4], double z[2]);

/* Resonator wake W(t) in V/C for t > 0 (0 for t < 0; W(0+) at t == 0). */
double mbt_ref_resonator_wake(const mbt_ref_resonator *r, double t);

/* Short-range resistive-wall wake of a round pipe in V/C (Bane and Sands,
 * 1995): with z = c t, s0 = (2 b^2 / (Z0 sigma))^(1/3),
 *   W = (4 Z0 c L / (pi b^2)) [ exp(-z/s0) cos(sqrt(3) z/s0) / 3
 *        - (sqrt(2)/pi) int_0^inf x^2 exp(-x^2 z/s0) / (x^6 + 8) dx ],
 * so W(0+) = Z0 c L / (pi b^2).  0 for t < 0.  Parity unpinned beyond the
 * tests' closed-form limits and impedance transform. */
double mbt_ref_rw_wake(const mbt_ref_rw *rw, double t);

/* Wake table on a grid: W[0] = sum W(0+)/2, W[k] = sum W(k*Delta), over the
 * resonators and the resistive wall (rw may be NULL). */
int mbt_ref_wake_table_rw(int32_t nres, const mbt_ref_resonator *res, const mbt_ref_rw *rw,
                          const mbt_ref_grid *g, double *W);

/* Wake table on a grid: W[0] = sum W(0+)/2, W[k] = sum W(k*Delta). */
int mbt_ref_wake_table(int32_t nres, const mbt_ref_resonator *res,
                       const mbt_ref_grid *g, double *W);

/* Bin index of tau on the grid, or -1 when outside [tau_min, tau_max). */
int32_t mbt_ref_bin_index(const mbt_ref_grid *g, double tau);

/* Line-density histogram of n particles (counts has g->nbins entries). */
int mbt_ref_histogram(const mbt_ref_grid *g, int64_t n, const double *tau,
                      uint32_t *counts, int64_t *out_of_grid);

/* Binned wake potential V[k] = q_per_particle * sum_{m<=k} W[k-m] c[m]. */
int mbt_ref_wake_potential(int32_t nbins, const double *W, const uint32_t *counts,
                           double q_per_particle, double *V);

/* Harmonic cavity at a fraction of the flat-potential voltage. */
int mbt_ref_hc_flat_fraction(const mbt_ref_ring *ring, int32_t n, double frac,
                             mbt_ref_hc *out);

/* ---- simulation object ---------------------------------------------------- */

int  mbt_ref_create(const mbt_ref_ring *ring, mbt_ref_sim **out);
void mbt_ref_destroy(mbt_ref_sim *s);
const char *mbt_ref_last_error(const mbt_ref_sim *s);

int mbt_ref_set_harmonic_cavity(mbt_ref_sim *s, const mbt_ref_hc *hc /* NULL = none */);
/* bucket[] strictly increasing in [0, h); current_A[] >= 0; stream[] (may be
 * NULL) gives each bunch's random-stream ordinal, default = its index b. */
int mbt_ref_set_fill(mbt_ref_sim *s, int32_t M, const int32_t *bucket,
                     const double *current_A, const int32_t *stream);
int mbt_ref_set_short_range(mbt_ref_sim *s, int32_t nres, const mbt_ref_resonator *res,
                            const mbt_ref_grid *g /* NULL = no short-range kick */);
int mbt_ref_set_long_range(mbt_ref_sim *s, int32_t nres, const mbt_ref_resonator *res);
/* Resistive wall added to the short-range table (acts only with a grid);
 * NULL removes it. */
int mbt_ref_set_resistive_wall(mbt_ref_sim *s, const mbt_ref_rw *rw);

int mbt_ref_init_gaussian(mbt_ref_sim *s, int64_t N, double sigma_tau_s,
                          double sigma_delta, uint64_t seed);
/* Allocates (or reuses) N particles per bunch; zero-filled until set. */
int mbt_ref_alloc_particles(mbt_ref_sim *s, int64_t N, uint64_t seed);
int mbt_ref_set_particles(mbt_ref_sim *s, int32_t bunch, const double *tau,
                          const double *delta);
int mbt_ref_get_particles(const mbt_ref_sim *s, int32_t bunch, double *tau,
                          double *delta);

/* Track nturns turns.  moments: [nturns][M][4] = mean tau, mean delta,
 * rms tau, rms delta of the state after each turn (may be NULL).  counts:
 * [ceil(nturns/stride)][M][nbins] histograms of the state after turns
 * 0, stride, 2*stride, ... of this call (may be NULL). */
int mbt_ref_track(mbt_ref_sim *s, int64_t nturns, double *moments,
                  uint32_t *counts, int32_t stride);

/* Checkpoint: turn counter, seed and long-range phasors ([nlr][2] re, im). */
int mbt_ref_get_state(const mbt_ref_sim *s, int64_t *turn, uint64_t *seed, double *phasors);
int mbt_ref_set_state(mbt_ref_sim *s, int64_t turn, uint64_t seed, const double *phasors);

/* Derived constants, for inspection: phi_s, T0, D (per-turn damping),
 * noise amplitude s, drift coefficient alpha_c*T0. */
int mbt_ref_derived(const mbt_ref_sim *s, double out[5]);

/* Number of OpenMP threads the per-particle loop uses (1 without OpenMP). */
int mbt_ref_threads(void);

/* Threads for the per-particle loop from now on (n >= 1; results do not
 * depend on it).  Returns the number in effect. */
int mbt_ref_set_threads(int n);

#ifdef __cplusplus
}
#endif

#endif /* MBT_REF_H */
