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

/* One transverse plane, (x, x') (Sec. 2.2 Eqs. 3-5; the horizontal plane
 * with its dispersion, or the vertical one with D = D' = 0). */
typedef struct {
    double tune;          /* betatron tune Q per turn; only frac(Q) enters the matrix  */
    double chromaticity;  /* Q' = dQ/ddelta: phase advance 2 pi (frac(Q) + Q' delta)    */
    double alpha;         /* Twiss alpha at the observation point                       */
    double beta_m;        /* Twiss beta [m], > 0; gamma = (1 + alpha^2) / beta           */
    double disp_m;        /* dispersion D [m]                                           */
    double disp_prime;    /* dispersion slope D'                                        */
    double emittance_m;   /* equilibrium emittance eps: the noise scales are
                             sigma_x = sqrt(eps beta), sigma_x' = sqrt(eps gamma)       */
    double tau_damp_s;    /* amplitude damping time of the plane, D_x = 2 T0 / tau;
                             +inf (or eps = 0) switches the plane's noise off          */
} mbt_ref_transverse;

/* Long-range transverse resistive wall (Sec. 2.3, last paragraph): a round
 * pipe of the given radius, DC conductivity and length, acting from every
 * earlier bunch passage of the last `turns` turns (the present one included). */
typedef struct {
    double radius_m;
    double conductivity_S_m;
    double length_m;
    int32_t turns;        /* 1 .. 1024 */
} mbt_ref_lrrw;

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
 * so W(0+) = Z0 c L / (pi b^2).  0 for t < 0.  Pinned by W(0+), the
 * thick-wall z^-3/2 tail and its Fourier transform, which must equal the
 * round-pipe impedance with DC conductivity at five frequencies spanning
 * 0.05 to 10 c/s0. */
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

/* Transverse wake of a resonator with R_s in Ohm/m: for t > 0
 *   W_T(t) = (R_s omega_r^2 / (Q wbar)) exp(-alpha t) sin(wbar t)  [V/(C m)],
 * 0 for t <= 0. */
double mbt_ref_transverse_resonator_wake(const mbt_ref_resonator *r, double t);

/* Long-range transverse wake of a thick resistive round pipe (the 1/sqrt(t)
 * law of the low-frequency impedance), for t > 0:
 *   W_T(t) = (L / (pi b^3)) sqrt(Z0 c / (pi sigma t))  [V/(C m)]; 0 for t <= 0. */
double mbt_ref_transverse_rw_wake(const mbt_ref_rw *rw, double t);

/* Transverse wake table: T[0] = 0, T[k] = sum over resonators of W_T(k Delta). */
int mbt_ref_transverse_wake_table(int32_t nres, const mbt_ref_resonator *res,
                                  const mbt_ref_grid *g, double *T);

/* Counts and dipole sums of n particles: X[k] = sum of x over the particles
 * in bin k, added in particle order (the bin's dipole moment times its
 * count). */
int mbt_ref_dipole_histogram(const mbt_ref_grid *g, int64_t n, const double *tau,
                             const double *x, uint32_t *counts, double *X);

/* Transverse kick of bin k from the dipole sums of the bins before it
 * (Eq. 6, second line): U[k] = scale * sum_{m<k} T[k-m] X[m], m ascending;
 * scale = q_per_particle / E0. */
int mbt_ref_transverse_kicks(int32_t nbins, const double *T, const double *X, double scale,
                             double *U);

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

/* Transverse plane (NULL switches it off).  Must precede the particles.
 * MBT_REF_EINVAL on beta <= 0, eps < 0, tau <= 0 or a non-finite value. */
int mbt_ref_set_transverse(mbt_ref_sim *s, const mbt_ref_transverse *tr);
/* Transverse short-range resonators (R_s in Ohm/m), on the short-range grid. */
int mbt_ref_set_transverse_wake(mbt_ref_sim *s, int32_t nres, const mbt_ref_resonator *res);
/* Long-range transverse resistive wall (NULL: off). */
int mbt_ref_set_transverse_rw(mbt_ref_sim *s, const mbt_ref_lrrw *rw);
/* Matched Gaussian (x, x') for every particle from the INIT stream (tag 4):
 * x = offset + sqrt(eps beta) z0, x' = sqrt(eps / beta) (z1 - alpha z0);
 * clears the resistive-wall history.  Needs the transverse plane and the
 * particles allocated. */
int mbt_ref_init_transverse(mbt_ref_sim *s, double emittance_m, double offset_m);
int mbt_ref_set_transverse_particles(mbt_ref_sim *s, int32_t bunch, const double *x,
                                     const double *xp);
int mbt_ref_get_transverse_particles(const mbt_ref_sim *s, int32_t bunch, double *x,
                                     double *xp);
/* As mbt_ref_track, plus tmoments [nturns][M][4] = mean x, mean x', rms x,
 * rms x' of the state after each turn (may be NULL; needs the plane). */
int mbt_ref_track2(mbt_ref_sim *s, int64_t nturns, double *moments, double *tmoments,
                   uint32_t *counts, int32_t stride);
/* Resistive-wall history: bunch centroids <x> of the last `turns` turns,
 * [turns][M], row r holding the turn t with t mod turns == r (zeros for
 * turns before 0).  Part of a checkpoint, beside mbt_ref_get_state. */
int mbt_ref_get_rw_history(const mbt_ref_sim *s, double *H);
int mbt_ref_set_rw_history(mbt_ref_sim *s, const double *H);

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
