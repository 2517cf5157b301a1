/*
 * mbt.h -- C ABI of the MI355X longitudinal multi-bunch macro-particle tracker.
 *
 * The library advances macro-particles of electron bunches in a storage ring
 * turn by turn in the longitudinal plane, with the method of Xu, Locans,
 * Adelmann and Stingelin, "Calculation of Longitudinal Collective
 * Instabilities with mbtrack-cuda" (arXiv:1809.00391):
 *   - single-particle map: RF energy gain minus radiated energy (Sec. 2.2,
 *     Eq. 1), radiation damping and quantum excitation (Eq. 5, delta line),
 *     drift with the momentum compaction (Eq. 2);
 *   - optional harmonic cavity (Sec. 2.2, last paragraph);
 *   - short-range wake: particles binned on a fixed grid, wake potential of
 *     the binned line density, kick per bin (Sec. 2.3, Eq. 6);
 *   - long-range resonators acting bunch to bunch (Sec. 4 study of a cavity
 *     higher-order mode) through one complex phasor per resonator;
 *   - per-bunch statistics every turn (Sec. 2.4).
 *
 * Units: tau in seconds (arrival-time offset from the bucket centre, tau > 0
 * arrives later), delta = dE/E0, energies in eV, voltages in V, currents in A.
 * All particle arithmetic is IEEE binary64 on the GPU.
 *
 * General conventions
 *   - Every call returns MBT_OK (0) or a negative MBT_E* code; nothing throws
 *     or aborts across the ABI: a failed host allocation inside a call
 *     returns MBT_ENOMEM, and a setter that fails leaves the previous
 *     setting in force.  mbt_last_error() returns the message of the last
 *     failing call on a context.
 *   - A context is used by one host thread at a time.
 *   - Host pointers are borrowed for the duration of the call only; output
 *     arrays are allocated by the caller with the sizes stated below.
 *   - Device memory (particle state and workspace) is allocated by the caller
 *     and handed over with mbt_bind(); the library never allocates device
 *     memory.  It allocates a small amount of pinned host memory at bind
 *     time for its asynchronous output copies.
 *   - Work is enqueued on the caller's HIP stream given to mbt_bind().
 *   - Call order: mbt_create -> [mbt_set_harmonic_cavity] -> mbt_set_fill ->
 *     [mbt_set_short_range] -> [mbt_set_long_range] -> mbt_query_bytes ->
 *     mbt_bind -> (mbt_init_gaussian | mbt_set_particles + mbt_set_state) ->
 *     mbt_track ...  Out-of-order calls return MBT_ESTATE.
 */
#ifndef MBT_H
#define MBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define MBT_OK 0
#define MBT_EINVAL (-1)   /* invalid argument                                 */
#define MBT_ESTATE (-2)   /* call made in the wrong order                     */
#define MBT_ENOSPC (-3)   /* caller buffer smaller than mbt_query_bytes says  */
#define MBT_EDEVICE (-4)  /* HIP runtime error; message kept                  */
#define MBT_ENUMERIC (-5) /* non-finite bunch moment detected                 */
#define MBT_ENOMEM (-6)   /* host allocation failed                           */

/* Where a particle array lives (mbt_set_particles / mbt_get_particles). */
#define MBT_HOST 0
#define MBT_DEVICE 1

/* Limits. */
#define MBT_MAX_BINS 4096       /* short-range grid bins                     */
#define MBT_MAX_SHORT_RANGE 16  /* resonators summed into the wake table     */
#define MBT_MAX_LONG_RANGE 4    /* long-range resonators (phasors)           */

/* Ring and main RF (the lattice parameters of the paper's Table 1 that act in
 * the longitudinal plane).  T0 = harmonic / f_rf_Hz. */
typedef struct {
    double energy_eV;   /* E0 > 0                                             */
    double f_rf_Hz;     /* main RF frequency > 0                              */
    double v_rf_V;      /* main RF peak voltage > u0_eV                       */
    double alpha_c;     /* momentum compaction, nonzero, sign kept            */
    double u0_eV;       /* energy radiated per turn >= 0 (Eq. 1 U_rad)        */
    double tau_long_s;  /* longitudinal amplitude damping time > 0; +inf: off */
    double sigma_delta; /* equilibrium relative energy spread >= 0 (Eq. 5)    */
    int32_t harmonic;   /* h >= 1                                             */
} mbt_ring;

/* Harmonic cavity at fixed voltage: adds k*V_rf*sin(n*phi_h - n*w_rf*tau). */
typedef struct {
    int32_t n;          /* harmonic of the cavity, >= 2                       */
    double v_ratio;     /* k = V_hc / V_rf >= 0                               */
    double phase_n_rad; /* n*phi_h                                            */
} mbt_hc;

/* Resonator impedance (Sec. 2.3: the total wake is a sum of resonators). */
typedef struct {
    double rs_ohm;      /* shunt impedance >= 0                               */
    double q;           /* quality factor > 0.5                               */
    double fr_Hz;       /* resonant frequency > 0                             */
} mbt_resonator;

/* Fixed binning grid relative to the bucket centre (Sec. 2.3): bin k covers
 * [tau_min + k*D, tau_min + (k+1)*D) with D = (tau_max - tau_min)/nbins; the
 * index is floor((tau - tau_min) * (nbins / (tau_max - tau_min))). */
typedef struct {
    int32_t nbins;      /* 1 .. MBT_MAX_BINS                                  */
    double tau_min_s;
    double tau_max_s;   /* > tau_min_s                                        */
} mbt_grid;

/* Round resistive pipe for the short-range resistive-wall wake (the wake
 * benchmark of Sec. 3: a copper chamber of 10 mm radius along the whole
 * ring). */
typedef struct {
    double radius_m;         /* b > 0                                         */
    double conductivity_S_m; /* DC conductivity > 0 (copper 5.8e7)            */
    double length_m;         /* pipe length > 0 (e.g. the circumference)      */
} mbt_resistive_wall;

/* Per-bunch statistics after a turn (Sec. 2.4): means and population rms
 * over all macro-particles of the bunch. */
typedef struct {
    double mean_tau;
    double mean_delta;
    double rms_tau;
    double rms_delta;
} mbt_moments;

typedef struct mbt_ctx mbt_ctx;

/* Message for a return code (static string). */
const char *mbt_strerror(int code);

/* Message of the last failing call on ctx (never NULL). */
const char *mbt_last_error(const mbt_ctx *ctx);

/* Create a context for one tracking job on the current HIP device.
 * Validates the ring (Sec. 2.2, Eqs. 1, 2, 5): MBT_EINVAL if E0 <= 0,
 * f_rf <= 0, V_rf <= u0, u0 < 0, alpha_c == 0, tau_long <= 0,
 * sigma_delta < 0, harmonic < 1 or any value is NaN.  The synchronous phase
 * solves V_rf sin(phi_s) = u0 on the branch with alpha_c cos(phi_s) > 0.
 * *out receives the context (NULL on failure); free it with mbt_destroy. */
int mbt_create(const mbt_ring *ring, mbt_ctx **out);

/* Free a context (NULL is allowed).  Does not free caller-owned device
 * memory; synchronises the bound stream first. */
void mbt_destroy(mbt_ctx *ctx);

/* Harmonic cavity of order n at frac times the flat-potential voltage, with
 * the flat-potential phase (total voltage and its first two derivatives match
 * U0, 0, 0 at tau = 0).  MBT_EINVAL if n < 2, frac <= 0 or no flat-potential
 * solution exists for this ring. */
int mbt_hc_flat_fraction(const mbt_ring *ring, int32_t n, double frac, mbt_hc *out);

/* Set (hc != NULL) or remove (hc == NULL) the harmonic cavity (Sec. 2.2) and
 * re-solve phi_s from V_rf sin(phi_s) + k V_rf sin(n phi_h) = u0.
 * MBT_EINVAL if no synchronous phase exists; the previous cavity is kept. */
int mbt_set_harmonic_cavity(mbt_ctx *ctx, const mbt_hc *hc);

/* Filling pattern (Sec. 4): M bunches in buckets bucket[0] < ... < bucket[M-1]
 * within [0, h), bunch currents current_A[b] >= 0 (bunch charge I_b * T0).
 * stream (may be NULL) gives each bunch's random-stream ordinal (default b):
 * the noise of bunch b is keyed by (seed, turn, stream[b], particle), so two
 * bunches with the same ordinal and seed see the same noise.
 * Must precede mbt_bind (MBT_ESTATE after it). */
int mbt_set_fill(mbt_ctx *ctx, int32_t M, const int32_t *bucket, const double *current_A,
                 const int32_t *stream);

/* Short-range wake (Sec. 2.3, Eq. 6): nres resonators summed into one wake
 * table sampled at bin distances (self term W(0+)/2), on grid *g.  Particles
 * outside the grid get no short-range kick.  g == NULL removes the
 * short-range kick.  MBT_EINVAL on Q <= 0.5, Rs < 0, fr <= 0, nbins outside
 * [1, MBT_MAX_BINS], tau_min >= tau_max or nres > MBT_MAX_SHORT_RANGE.
 * Must precede mbt_bind. */
int mbt_set_short_range(mbt_ctx *ctx, int32_t nres, const mbt_resonator *res,
                        const mbt_grid *g);

/* Short-range resistive-wall wake of a round pipe added to the wake table
 * (rw == NULL removes it): with z = c t and s0 = (2 b^2 / (Z0 sigma))^(1/3),
 * W = (4 Z0 c L / (pi b^2)) [exp(-z/s0) cos(sqrt(3) z/s0)/3 - (sqrt(2)/pi)
 * int_0^inf x^2 exp(-x^2 z/s0)/(x^6 + 8) dx] (Bane and Sands, 1995), sampled
 * at bin distances like the resonators (W(0+)/2 for the bin itself).  Acts
 * only with a grid.  MBT_EINVAL on a non-positive or non-finite value.
 * Must precede mbt_bind. */
int mbt_set_resistive_wall(mbt_ctx *ctx, const mbt_resistive_wall *rw);

/* ---- Transverse plane ------------------------------------------------------
 * One transverse plane (x in m, x' in rad) tracked beside (tau, delta): the
 * betatron map of Sec. 2.2 (Eqs. 3-5), the transverse wake kick of Sec. 2.3
 * (Eq. 6, second line) and the long-range resistive wall applied after all
 * bunches of a turn (Sec. 2.3, last paragraph).  The longitudinal map is
 * unchanged.  Per turn and particle, in this order, with delta and tau the
 * values before this turn's kick and k the bin of tau:
 *   x' += the bunch's long-range resistive-wall kick (from the passages of
 *         the previous turn and the turns before it, see below);
 *   x' += U[k]  (the bin's transverse wake kick; none outside the grid);
 *   xb = x - D delta, xb' = x' - D' delta, psi = 2 pi (frac(Q) + Q' delta),
 *   x  <- D delta  + (cos psi + alpha sin psi) xb + beta sin psi xb',
 *   x' <- D' delta - gamma sin psi xb + (cos psi - alpha sin psi) xb'
 *         (rotation about the dispersive orbit, gamma = (1 + alpha^2)/beta);
 *   x' *= (1 + delta) / (1 + delta + e_rf/E0)  (adiabatic damping across the
 *         energy gain e_rf of the main and harmonic cavities);
 *   x += sqrt(eps beta D_x) z, x' += sqrt(eps gamma D_x) z', D_x =
 *         2 T0 / tau_damp, z and z' from Philox counters (particle/2, stream
 *         ordinal, turn, 2) and (particle/2, stream ordinal, turn, 3), the
 *         pair's cosine branch for even particles, its sine branch for odd.
 * U[k] = (q_pp / E0) sum_{m<k} T[k-m] X[m]: T[j] the summed transverse wake
 * of the resonators at bin distance j (T[0] = 0), X[m] the sum of x over the
 * particles in bin m (the bin's dipole moment times its count).  X is summed
 * as an exact integer multiple of 2^-52 m after rounding each x to that grid
 * (at most 1.1e-16 m per particle), so it does not depend on the order of
 * the particles; |X| of a bin must stay below 2^11 m.
 * Jobs with the plane compute their longitudinal wake in FP64 (the
 * matrix-core modes return MBT_EINVAL) and cannot join a batch.
 *
 * The plane, its wake and its wall are set before mbt_bind; NULL switches
 * each off.  MBT_EINVAL on beta <= 0, eps < 0, tau_damp <= 0 or a non-finite
 * value. */
typedef struct {
    double tune;          /* betatron tune Q; only frac(Q) enters              */
    double chromaticity;  /* Q': phase advance 2 pi (frac(Q) + Q' delta)       */
    double alpha;         /* Twiss alpha at the observation point              */
    double beta_m;        /* Twiss beta > 0                                    */
    double disp_m;        /* dispersion D                                      */
    double disp_prime;    /* dispersion slope D'                               */
    double emittance_m;   /* equilibrium emittance eps >= 0 (noise scale)      */
    double tau_damp_s;    /* amplitude damping time > 0; +inf or eps 0: no noise */
} mbt_transverse;
int mbt_set_transverse(mbt_ctx *ctx, const mbt_transverse *tr);

/* Transverse short-range resonators (R_s in Ohm/m), on the short-range grid:
 * W_T(t) = (R_s w_r^2 / (Q wbar)) exp(-alpha t) sin(wbar t) for t > 0.
 * nres <= MBT_MAX_SHORT_RANGE; acts only with a grid. */
int mbt_set_transverse_wake(mbt_ctx *ctx, int32_t nres, const mbt_resonator *res);

/* Long-range transverse resistive wall of a round pipe (thick wall,
 * W_T(t) = (L / (pi b^3)) sqrt(Z0 c / (pi sigma t))): each bunch b gets, at
 * the start of turn n, the kick (1/E0) sum I_b' T0 <x>_b' W_T(t) over the
 * passages of bunches b' < b in turn n - 1 and of every bunch in turns
 * n - K .. n - 2 (turns >= 0), each a rigid dipole of charge I_b' T0 at its
 * centroid <x>_b' after that turn, t the time from that passage to bunch b's
 * passage in turn n - 1.  Cost K M^2 terms per turn. */
typedef struct {
    double radius_m;
    double conductivity_S_m;
    double length_m;
    int32_t turns;        /* K, 1 .. 1024 */
} mbt_transverse_rw;
int mbt_set_transverse_rw(mbt_ctx *ctx, const mbt_transverse_rw *rw);

/* Matched Gaussian betatron coordinates for every particle: x = offset +
 * sqrt(eps beta) z0, x' = sqrt(eps / beta) (z1 - alpha z0), (z0, z1) one
 * Box-Muller pair of Philox with key = the seed in force (mbt_init_gaussian
 * or mbt_set_state) and counter (particle, stream ordinal, 0, 4).  Clears
 * the wall's centroid history.  MBT_ESTATE without the plane or binding. */
int mbt_init_transverse(mbt_ctx *ctx, double emittance_m, double offset_m);

/* Copy N transverse coordinates of a bunch in or out (as mbt_set_particles /
 * mbt_get_particles; x' as stored, before any pending wall kick). */
int mbt_set_transverse_particles(mbt_ctx *ctx, int32_t bunch, const double *x, const double *xp,
                                 int32_t where);
int mbt_get_transverse_particles(mbt_ctx *ctx, int32_t bunch, double *x, double *xp,
                                 int32_t where);

/* Per-bunch transverse statistics after a turn (Sec. 2.4). */
typedef struct {
    double mean_x;
    double mean_xp;
    double rms_x;
    double rms_xp;
} mbt_tmoments;

/* As mbt_track, plus tout: host array [nturns][M] of transverse moments
 * after each turn (may be NULL; MBT_EINVAL if not NULL without the plane). */
int mbt_track2(mbt_ctx *ctx, int64_t nturns, mbt_moments *out, mbt_tmoments *tout,
               uint32_t *counts, int32_t stride);

/* Wall history for a checkpoint: bunch centroids <x> of the last K turns,
 * [K][M], row r holding turn t with t mod K == r (zeros for turns never
 * tracked).  MBT_ESTATE without a wall or binding. */
int mbt_get_rw_history(mbt_ctx *ctx, double *H);
int mbt_set_rw_history(mbt_ctx *ctx, const double *H);

/* Long-range resonators (Sec. 4 higher-order mode): each acts on later
 * bunch passages through a complex phasor rotated bucket to bucket; its
 * same-bunch same-turn part acts through the short-range table, to which it
 * is added when a grid is set.  nres <= MBT_MAX_LONG_RANGE.
 * Must precede mbt_bind. */
int mbt_set_long_range(mbt_ctx *ctx, int32_t nres, const mbt_resonator *res);

/* Device bytes the caller must provide for N macro-particles per bunch:
 * *state_bytes for the particle coordinates (tau and delta, FP64,
 * bunch-major with rows padded to a multiple of 64 particles) and
 * *work_bytes for tables, histograms, partial sums and output rings.
 * MBT_ESTATE if the fill is not set; MBT_EINVAL if N < 1 or N > 2^32. */
int mbt_query_bytes(const mbt_ctx *ctx, int64_t N, size_t *state_bytes, size_t *work_bytes);

/* Bind caller-owned device memory and a HIP stream (hipStream_t passed as
 * void*, NULL = default stream).  d_state and d_work must be 256-byte
 * aligned device pointers of at least the queried sizes (MBT_ENOSPC
 * otherwise).  Uploads the wake table and per-bunch constants, clears the
 * workspace.  The caller keeps ownership and must keep the memory alive until
 * mbt_destroy.  Binding again (e.g. a new N) replaces the previous binding. */
int mbt_bind(mbt_ctx *ctx, int64_t N, void *d_state, size_t state_bytes, void *d_work,
             size_t work_bytes, void *hip_stream);

/* Bind without allocating, for callers that cannot allocate device or
 * pinned host memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  As mbt_bind, except that the workspace is
 * the library's own static device array of MBT_STATIC_WORK_BYTES on the
 * current device (held by each device the library runs on until the process
 * ends), and no pinned host memory is taken: this call makes no hipMalloc,
 * hipHostMalloc, hipFree or event creation (its tables are built in ordinary
 * host memory), and mbt_track on the context copies moments and profiles
 * straight into the caller's host arrays.  The caller still provides d_state
 * (256-byte aligned, state_bytes from mbt_query_bytes).
 *   - One static workspace per device, shared by every such binding there: a
 *     later mbt_bind_static on the same device takes it over, and every call
 *     that uses the earlier context's workspace then returns MBT_ESTATE until
 *     that context is bound again.  Calls that overlap on one device (other
 *     host threads, other streams) race on it.
 *   - Binding clears the workspace, so nothing of a previous binding's
 *     contents carries over.
 *   - A context bound this way cannot join a batch (MBT_EINVAL).
 *   - MBT_ENOSPC if the job's workspace (work_bytes of mbt_query_bytes)
 *     exceeds MBT_STATIC_WORK_BYTES; MBT_EINVAL on a null or misaligned
 *     d_state, as mbt_bind. */
#define MBT_STATIC_WORK_BYTES (64u << 20)
int mbt_bind_static(mbt_ctx *ctx, int64_t N, void *d_state, size_t state_bytes, void *hip_stream);

/* Initial distribution: tau ~ N(0, sigma_tau_s), delta ~ N(0, sigma_delta)
 * per particle from one Box-Muller pair of Philox-4x32-10 with key = seed and
 * counter = (particle, stream ordinal, 0, 1).  Sets turn = 0, the seed, and
 * clears the long-range phasors; with the transverse plane also x = x' = 0
 * and the wall's history.  Asynchronous on the bound stream. */
int mbt_init_gaussian(mbt_ctx *ctx, double sigma_tau_s, double sigma_delta, uint64_t seed);

/* Copy N coordinates of bunch `bunch` in (where == MBT_HOST: host arrays,
 * synchronous; MBT_DEVICE: device arrays, asynchronous on the bound stream). */
int mbt_set_particles(mbt_ctx *ctx, int32_t bunch, const double *tau, const double *delta,
                      int32_t where);

/* Copy N coordinates of bunch `bunch` out; synchronises the bound stream. */
int mbt_get_particles(mbt_ctx *ctx, int32_t bunch, double *tau, double *delta, int32_t where);

/* Track nturns turns (nturns < 2^31) from the stored turn counter (so a
 * checkpoint resumes).
 *   out:    host array [nturns][M] of moments after each turn (may be NULL)
 *   counts: host array [ceil(nturns/stride)][M][nbins] of bin counts of the
 *           state after turns 0, stride, 2*stride, ... of this call (may be
 *           NULL; needs a grid and stride >= 1)
 * Each turn, for every bunch in bucket order: the kick (RF + harmonic cavity
 * - U0 - short-range wake of the bin - long-range voltage), damping and
 * quantum excitation with noise keyed by (seed, turn, stream ordinal,
 * particle/2), then the drift (Sec. 2.2-2.4).  Three kernel launches per
 * turn on the bound stream; the host does not wait on the device inside the
 * loop except to copy a full output ring out.  Blocks until done.
 * MBT_ENUMERIC if a bunch moment became non-finite. */
int mbt_track(mbt_ctx *ctx, int64_t nturns, mbt_moments *out, uint32_t *counts,
              int32_t stride);

/* Current line density: counts [M][nbins] of the present state on the grid
 * (Sec. 2.3 binning).  Synchronises the bound stream. */
int mbt_profile(mbt_ctx *ctx, uint32_t *counts);

/* Binned wake potential [M][nbins] in V that the next turn would apply
 * (Sec. 2.3): V[b][k] = (I_b T0 / N) sum_{m<=k} W[k-m] counts[b][m].
 * Synchronises the bound stream. */
int mbt_wake_potential(mbt_ctx *ctx, double *V);

/* Wake table W[nbins] in V/C (W[0] = sum of W(0+)/2, W[k] = sum of W(k D)). */
int mbt_wake_table(const mbt_ctx *ctx, double *W);

/* Checkpoint state: turn counter, seed and the long-range phasors
 * (phasors: [n_long_range][2] real, imaginary in V; may be NULL).  Together
 * with the particle coordinates this resumes a run bit for bit. */
int mbt_get_state(mbt_ctx *ctx, int64_t *turn, uint64_t *seed, double *phasors);
int mbt_set_state(mbt_ctx *ctx, int64_t turn, uint64_t seed, const double *phasors);

/* Kernel timing for measurement.  With every > 0, mbt_track records HIP
 * events on the bound stream around the push launch and around the
 * between-turn launches (phasor scan; prep or wake kernel) of every
 * `every`-th turn (at most 4096 turns per call) and adds their elapsed times
 * to running totals; every = 0 switches it off and clears the totals.  The
 * event records themselves take GPU time (several microseconds per bracketed
 * turn), so sparse brackets disturb a throughput measurement least.
 * mbt_get_timing returns the totals in milliseconds and the number of timed
 * launches (any pointer may be NULL). */
int mbt_set_timing(mbt_ctx *ctx, int32_t every);
int mbt_get_timing(const mbt_ctx *ctx, double *push_ms, int64_t *push_launches,
                   double *prep_ms, int64_t *prep_launches);

/* Launch shape of the push: nsub LDS sub-histograms per workgroup (0: a
 * default from nbins) and push_grid persistent workgroups (0: one workgroup
 * per push tile, 8192 particles for all but small jobs).  Neither changes
 * any result bit: histograms are integer sums and each tile's partial sums
 * keep their order.
 * MBT_EINVAL if the LDS image of the push would exceed 64 KiB. */
int mbt_set_launch(mbt_ctx *ctx, int32_t nsub, int32_t push_grid);

/* Arithmetic of the short-range wake potential V = qpp * T(W) * counts
 * (Sec. 2.3), the product of the lower-triangular Toeplitz matrix of the wake
 * table with the bunches' line densities:
 *   MBT_WAKE_FP64   FP64 convolution on the vector units (default; the
 *                   reference arithmetic, within 1e-13 of the FP64 oracle)
 *   MBT_WAKE_FP32   matrix cores: W/s in FP32 (s a power of two near max|W|),
 *                   counts exact in FP32 below 2^24, FP32 accumulation
 *   MBT_WAKE_BF16X2 matrix cores: W/s as the sum of two BF16 terms, each
 *                   count split exactly into 8-bit BF16 parts, FP32
 *                   accumulation per part, parts combined in FP64
 *   MBT_WAKE_BF16X3 as BF16X2 with three BF16 terms of W
 * Particle coordinates, sums and phasors stay FP64 in every mode.  May be
 * called at any time; the next call that tracks rebuilds the wake
 * potential.  A job's mode is fixed while it belongs to a batch. */
#define MBT_WAKE_FP64 0
#define MBT_WAKE_FP32 1
#define MBT_WAKE_BF16X2 2
#define MBT_WAKE_BF16X3 3
int mbt_set_wake_precision(mbt_ctx *ctx, int32_t mode);

/* ---- Batches -------------------------------------------------------------
 * A batch advances several bound jobs (contexts on one device) together:
 * each turn's launches cover every bunch of every job -- the phasor scan of
 * all jobs with long-range resonators, the push of all tiles (one launch per
 * distinct long-range resonator count), the between-turn work of all
 * bunches (the prep for FP64-wake jobs, one wake launch per matrix-core
 * arithmetic for the others).  Each job keeps its
 * own seed, turn counter, workspace and reduction layout, so its results are
 * bit for bit those of tracking it alone with mbt_track.  A job in a batch
 * must not be tracked on its own or rebound while the batch exists; destroy
 * the batch first.
 *
 * mbt_batch_query_bytes: device bytes of the batch's descriptor and item
 * tables (caller-owned, 256-byte aligned).  mbt_batch_create: builds the
 * tables in d_work on hip_stream (NULL: default stream) and creates a private
 * stream for graph capture.  MBT_EINVAL on duplicate jobs, jobs on different
 * devices, njobs outside [1, 65535]; MBT_ESTATE if a job is not bound. */
typedef struct mbt_batch mbt_batch;
int mbt_batch_query_bytes(mbt_ctx *const *jobs, int32_t njobs, size_t *work_bytes);
int mbt_batch_create(mbt_ctx *const *jobs, int32_t njobs, void *d_work, size_t work_bytes,
                     void *hip_stream, mbt_batch **out);
void mbt_batch_destroy(mbt_batch *batch);
const char *mbt_batch_last_error(const mbt_batch *batch);

/* graph_turns >= 2: turns are captured once as a HIP graph of that many
 * turns (rounded down to even, and at most what each job's moment ring and
 * profile ring allow) and replayed; the turn counter lives in device memory,
 * so a replay needs no parameter update.  0 or 1: launches are issued turn
 * by turn.  autotune = 1: on the
 * first call with enough turns, the push's sub-histogram count and
 * persistent grid are timed over real turns and the fastest kept, cached per
 * process by (resonator count, bins, item count); these choices change no
 * result bit. */
int mbt_batch_configure(mbt_batch *batch, int32_t graph_turns, int32_t autotune);

/* Push groups of the batch and their present launch shape: per group the
 * long-range resonator count, sub-histograms and workgroups (arrays of at
 * least MBT_MAX_LONG_RANGE + 1 entries; any may be NULL except ngroups). */
int mbt_batch_launch_info(const mbt_batch *batch, int32_t *ngroups, int32_t *nlr, int32_t *nsub,
                          int32_t *grid);

/* Kernel timing of a batch, for measurement: as mbt_set_timing /
 * mbt_get_timing, on the batch's stream.  The push total covers every push
 * group of a bracketed turn; the between-turn total covers the phasor scan
 * and the prep and wake kernels.  While every > 0 the batch issues its
 * turns eagerly (a captured graph holds no events).  every = 0 switches
 * timing off and clears the totals. */
int mbt_batch_set_timing(mbt_batch *batch, int32_t every);
int mbt_batch_get_timing(const mbt_batch *batch, double *push_ms, int64_t *push_launches,
                         double *between_ms, int64_t *between_launches);

/* Track nturns turns of every job.  out[j] (host [nturns][M_j], or NULL) and
 * counts[j] (host [ceil(nturns/stride[j])][M_j][nbins_j], or NULL) as in
 * mbt_track; out, counts and stride may themselves be NULL.  Blocks until
 * done.  MBT_ENUMERIC names the first job with a non-finite moment. */
int mbt_batch_track(mbt_batch *batch, int64_t nturns, mbt_moments *const *out,
                    uint32_t *const *counts, const int32_t *stride);

/* Raw Philox-4x32-10 blocks on the device (the generator behind the noise,
 * Salmon et al. SC'11): out[i][0..3] = philox(ctr[i][0..3], key), for
 * n counters.  ctr and out are device arrays; asynchronous on hip_stream. */
int mbt_philox4x32_10(int64_t n, const uint32_t *ctr, uint32_t key0, uint32_t key1,
                      uint32_t *out, void *hip_stream);

/* Device-to-device copy of `bytes` bytes from src to dst with the library's
 * own streaming kernel (16-byte accesses): the achievable-bandwidth yardstick
 * for the push's traffic (the measurement protocol compares the push with
 * both this copy and the published HBM peak).  src and dst are device
 * pointers, 16-byte aligned, not overlapping; bytes a multiple of 16 (0 is a
 * no-op).  Asynchronous on hip_stream.  MBT_EINVAL on a violated condition
 * (nothing is launched), MBT_EDEVICE if the launch fails. */
int mbt_stream_copy(const void *src, void *dst, int64_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MBT_H */
