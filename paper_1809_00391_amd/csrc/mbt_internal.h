// mbt_internal.h -- parameter blocks shared by the host runtime and the HIP
// kernels of the tracker (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbt {

constexpr int kMaxLR = 4;            // long-range resonators
#ifndef MBT_PUSH_THREADS
#define MBT_PUSH_THREADS 256
#endif
#ifndef MBT_PAIRS_PER_THREAD
#define MBT_PAIRS_PER_THREAD 8
#endif
constexpr int kPushThreads = MBT_PUSH_THREADS;         // wavefronts of 64
constexpr int kPairsPerThread = MBT_PAIRS_PER_THREAD;  // particle pairs per thread per tile
constexpr int kTile = kPushThreads * 2 * kPairsPerThread;  // particles per tile
constexpr int kPartStride = 4 + 2 * kMaxLR;  // doubles per tile partial
constexpr int kPrepThreads = 256;
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
    double lr_alpha[kMaxLR];  // omega_r / 2Q
    double lr_wbar[kMaxLR];   // sqrt(omega_r^2 - alpha^2)
};

// Push (and bin-only prologue) kernel arguments.
struct PushArgs {
    MapConst c;
    double *tau;              // [M][ld]
    double *delta;            // [M][ld]
    int64_t ld;               // row stride in doubles
    int64_t N;                // particles per bunch
    int M;
    int ntiles;               // tiles per bunch
    int nsub;                 // LDS sub-histograms
    const double *V;          // [M][nbins] wake potential (push only)
    const double *seen;       // [nlr][M][2] long-range voltage seen by each bunch
    const uint32_t *stream;   // [M] random-stream ordinals
    uint32_t *counts_out;     // [M][nbins] histogram of the new tau (atomics)
    double *partials;         // [M][ntiles][kPartStride]
    uint32_t key0, key1;      // Philox key = seed
    uint32_t turn;            // Philox counter word 2
};

// Between-turn kernel arguments: moments, wake potential, long-range scan.
struct PrepArgs {
    int M;
    int ntiles;
    int64_t N;
    int nbins;
    int nlr;
    int do_conv;              // compute V from counts_in
    int do_scan;              // advance the long-range phasors
    const double *partials;   // [M][ntiles][kPartStride] from the last push/prologue
    double *mom_out;          // [M][4] moments slot or nullptr
    const uint32_t *counts_in;   // [M][nbins]
    uint32_t *counts_clear;      // [M][nbins] zeroed for the next push
    const double *W;          // [nbins] wake table
    const double *qpp;        // [M] charge per macro-particle I_b T0 / N
    double *V;                // [M][nbins]
    const double *gap;        // [nlr][M][2] rotation into bunch b's bucket
    const double *qc;         // [nlr][M][2] qpp_b * c_r
    double *S;                // [nlr][M][2] deposit sums of each bunch
    double *phasor;           // [nlr][2] state
    double *seen;             // [nlr][M][2]
    uint32_t *status;         // bit 0: non-finite moment
};

// Kernel launchers (mbt_kernels.hip).
hipError_t launch_push(const PushArgs &a, int nlr, bool push, hipStream_t s);
hipError_t launch_prep(const PrepArgs &a, hipStream_t s);
hipError_t launch_init_gauss(double *tau, double *delta, int64_t ld, int64_t N, int M,
                             const uint32_t *stream, double sig_tau, double sig_delta,
                             uint32_t key0, uint32_t key1, hipStream_t s);
hipError_t launch_philox(int64_t n, const uint32_t *ctr, uint32_t key0, uint32_t key1,
                         uint32_t *out, hipStream_t s);
size_t push_lds_bytes(int nbins, int nsub);
int push_nsub(int nbins);

}  // namespace mbt
