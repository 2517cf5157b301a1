// mbt_internal.h -- device-side job descriptors and kernel launchers of the
// tracker (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbt {

constexpr int kMaxLR = 4;            // long-range resonators
#ifndef MBT_PUSH_THREADS
#define MBT_PUSH_THREADS 256
#endif
#ifndef MBT_PAIRS_PER_THREAD
#define MBT_PAIRS_PER_THREAD 16
#endif
constexpr int kPushThreads = MBT_PUSH_THREADS;         // wavefronts of 64
constexpr int kPairsPerThread = MBT_PAIRS_PER_THREAD;  // most particle pairs per thread per tile
constexpr int kPartTr = 4 + 2 * kMaxLR;      // first transverse slot of a tile partial
constexpr int kPartStride = kPartTr + 4;     // doubles per tile partial:
                                             // tau, tau^2, delta, delta^2, deposits,
                                             // x, x^2, x', x'^2
constexpr int kPrepThreads = 256;
constexpr int kConvOutMax = 64;      // wake-potential bins per prep workgroup, at most
constexpr int kConvOutMin = 16;      // ... and at least
constexpr int kRowAlign = 64;        // particle rows padded to 64 doubles (512 B)

// Per-turn constants of the single-particle map and the binning grid.
struct MapConst {
    double inv_E0;        // 1/E0 [1/eV]
    double w_rf;          // 2 pi f_rf [rad/s]
    double rf_a;          // V_rf sin(phi_s) / E0
    double rf_b;          // V_rf cos(phi_s) / E0
    double u0_e;          // U0 / E0
    double one_minus_D;   // 1 - D, D = 2 T0 / tau_L
    double noise;         // sigma_E sqrt(2 D)
    double drift;         // alpha_c T0 [s]
    double hc_a;          // k V_rf sin(n phi_h) / E0
    double hc_b;          // k V_rf cos(n phi_h) / E0
    int hc_n;             // harmonic of the cavity
    int hc_on;
    int sr_on;
    int noise_on;
    int nbins;
    double tau_min;       // grid start [s]
    double inv_delta;     // nbins / (tau_max - tau_min)
    double nbins_d;       // nbins as a double
    double lr_alpha[kMaxLR];  // omega_r / 2Q
    double lr_wbar[kMaxLR];   // sqrt(omega_r^2 - alpha^2)
};

// Constants of the transverse plane (Sec. 2.2 Eqs. 3-5, Sec. 2.3).
struct TransConst {
    double qfrac;         // frac(Q)
    double chrom;         // Q'
    double alpha, beta, gamma;
    double disp, disp_p;  // D, D'
    double noise_x;       // sqrt(eps beta D_x)
    double noise_xp;      // sqrt(eps gamma D_x)
    int noise_on;
    int rw_turns;         // K of the long-range wall (0: off)
    double rw_amp;        // L / (pi b^3) [1/m^2]
    double rw_arg;        // Z0 c / (pi sigma) [s]: W_T(t) = rw_amp sqrt(rw_arg / t)
    double T0, T_rf;
};

// Fixed-point scale of the dipole sums: x is summed as round(x 2^52) in int64.
constexpr double kDipoleScale = 4503599627370496.0;  // 2^52
constexpr double kDipoleUnit = 1.0 / kDipoleScale;

// Everything a kernel needs about one job, resident in device memory.  The
// turn counter lives on the device in two slots, so a captured run of turns
// replays without parameter updates: the launches of one turn carry a phase
// p (alternating 0, 1, 0, ... from the start of a call); during the push of
// turn n and the prep after it clock[p] reads n (modulo 2^32), and one prep
// workgroup per job writes n + 1 into clock[1 - p], which no launch of this
// turn reads.
struct JobDesc {
    MapConst c;
    double *tau;              // [M][ld]
    double *delta;            // [M][ld]
    int64_t ld;               // row stride in doubles
    int64_t N;                // particles per bunch
    int M;
    int ntiles;               // push tiles per bunch
    int ppt;                  // particle pairs per thread in a push tile (pairs_per_thread)
    int nsub;                 // LDS sub-histograms in the push
    int nlr;                  // long-range resonators
    int mom_slots;            // moment ring rows (power of two)
    int prof_stride;          // profile every prof_stride-th turn (0: off)
    int prof_slots;           // profile ring rows (power of two)
    uint32_t base;            // first turn of the present call: ring rows count from it
    uint32_t key0, key1;      // Philox key = seed
    int wake_mode;            // 0: FP64 convolution in the prep; else k_wake (WakeMode)
    int count_parts;          // 8-bit parts of a bin count (< 2^(8 count_parts))
    double wake_scale;        // power of two: the MFMA tables hold W / wake_scale
    const uint16_t *Wbf;      // [3][nbins] BF16 parts of W / wake_scale (hi, lo, lo2)
    const float *Wf32;        // [nbins] W / wake_scale rounded to FP32
    const double *W;          // [nbins] wake table
    const double *qpp;        // [M] charge per macro-particle
    const double *gap;        // [nlr][M][2] rotation into bunch b's bucket
    const double *qc;         // [nlr][M][2] qpp_b * c_r
    const uint32_t *stream;   // [M] random-stream ordinals
    double *V;                // [M][nbins] wake potential
    double *partials;         // [M][ntiles][kPartStride] tile sums
    double *S;                // [nlr][M][2] deposit sums
    double *seen;             // [nlr][M][2] voltage seen by each bunch
    double *phasor;           // [nlr][2]
    double *mom_ring;         // [mom_slots][M][4]
    uint32_t *counts;         // [2][M][max(nbins,1)] histograms by turn parity
    uint32_t *prof_ring;      // [prof_slots][M][nbins]
    uint32_t *status;         // bit 0: non-finite moment
    uint32_t *clock;          // [2] turn counter by launch phase (see below)
    int conv_out;             // wake-potential bins per prep workgroup (16, 32 or 64)
    // transverse plane (tr_on = 0: none of the fields below is used)
    int tr_on;
    TransConst t;
    double *x;                // [M][ld]
    double *xp;               // [M][ld]
    const double *Tt;         // [nbins] transverse wake table
    double *U;                // [M][nbins] transverse kick per bin [rad]
    unsigned long long *Xq;   // [2][M][nbins] dipole sums (int64, units 2^-52 m) by turn parity
    double *tmom_ring;        // [mom_slots][M][4]
    double *H;                // [rw_turns][M] bunch centroids <x> by turn mod K
    double *rwk;              // [M] wall kick for the next turn [rad]
    const int32_t *bucket;    // [M] bucket of each bunch
    const double *qb;         // [M] bunch charge I_b T0 [C]
};

// One unit of work: a tile (push) or a wake-potential chunk (prep) of a bunch.
struct Item {
    uint16_t job;
    uint16_t bunch;
    uint32_t part;
};

// Arithmetic of the short-range wake potential.
enum WakeMode {
    kWakeFP64 = 0,    // FP64 convolution on the vector units (the reference arithmetic)
    kWakeFP32 = 1,    // FP32 W x exact FP32 counts on MFMA, FP32 accumulation
    kWakeBF16x2 = 2,  // W split in two BF16 terms x counts split in exact 8-bit BF16 parts
    kWakeBF16x3 = 3,  // as above with three BF16 terms of W
};

// Terms of the single-particle map fixed at compile time in a push kernel.
enum MapKind {
    kMapGeneric = 0,       // every switch read from the map constants
    kMapWakeNoise = 1,     // short-range wake and noise on, no harmonic cavity
    kMapWakeNoiseHC3 = 2,  // as above with a third-harmonic cavity
};

// Launch descriptors.
struct PushLaunch {
    int phase;                // slot of the turn counter this launch reads
    const JobDesc *jobs;
    const Item *items;
    int nitems;
    int nlr;                  // template group: every job of the items has this many
    int nbins_max;
    int nsub_max;
    int grid;                 // workgroups: nitems (one per item) or fewer (persistent)
    int map;                  // MapKind shared by every job of the items
    int stream;               // particle rows read and written with the non-temporal hint
    // persistent launches: [0..1] next item by phase, [2..3] finished
    // workgroups by phase; both 0 between launches (k_push rewinds them)
    uint32_t *ctr;
};
struct PrepLaunch {
    int phase;
    const JobDesc *jobs;
    const Item *items;        // (job, bunch, chunk)
    int nitems;
    int nlr_max;
    int nbins_max;
    // One job only: items are (0, i / inner, i % inner) and the turn counter
    // is clk[phase], so a workgroup need not read the item table before the
    // descriptor, nor the descriptor before the counter.  inner = 0: tables.
    int inner;
    const uint32_t *clk;
    int tr;                   // the job has the transverse plane (one job per launch)
};
struct WakeLaunch {
    int phase;
    const JobDesc *jobs;
    const Item *items;        // (job, 16-bunch tile, 16-bin output tile)
    int nitems;
    int mode;                 // WakeMode other than kWakeFP64; every job of the items has it
    int nbins_max;
    int inner;                // as in PrepLaunch
    const uint32_t *clk;
};
struct RwLaunch {
    int phase;
    const JobDesc *job;       // one job
    int M;
    const uint32_t *clk;      // its turn counter
};
struct ScanLaunch {
    const JobDesc *jobs;
    int njobs;
    int nlr_max;
};

hipError_t launch_push(const PushLaunch &l, bool push, hipStream_t s);
hipError_t launch_push_tr(const PushLaunch &l, bool push, hipStream_t s);
hipError_t launch_rw(const RwLaunch &l, hipStream_t s);
hipError_t launch_init_transverse(double *x, double *xp, int64_t ld, int64_t N, int M,
                                  const uint32_t *stream, double sx, double sxp, double alpha,
                                  double offset, uint32_t key0, uint32_t key1, hipStream_t s);
size_t push_tr_lds_bytes(int nbins, int nsub);
hipError_t launch_prep(const PrepLaunch &l, hipStream_t s);
hipError_t launch_scan(const ScanLaunch &l, hipStream_t s);
hipError_t launch_wake(const WakeLaunch &l, hipStream_t s);
hipError_t launch_init_gauss(double *tau, double *delta, int64_t ld, int64_t N, int M,
                             const uint32_t *stream, double sig_tau, double sig_delta,
                             uint32_t key0, uint32_t key1, hipStream_t s);
hipError_t launch_philox(int64_t n, const uint32_t *ctr, uint32_t key0, uint32_t key1,
                         uint32_t *out, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);
size_t wake_lds_bytes(int mode, int nbins_max);
size_t push_lds_bytes(int nbins, int nsub);
int conv_chunks(int nbins, int conv_out);
int conv_width(int M, int nbins);
int pairs_per_thread(int M, int64_t N);
constexpr int kWakeBins = 16;     // output bins per k_wake workgroup (one 16 x 16 MFMA tile)
constexpr int kWakeBunches = 16;  // bunches per k_wake workgroup

}  // namespace mbt
