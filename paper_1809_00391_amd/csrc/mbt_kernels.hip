// mbt_kernels.hip -- HIP kernels of the longitudinal multi-bunch tracker for
// CDNA4 (gfx950).
//
// One turn is two launches on the caller's stream (three with long-range
// resonators; a batch mixing FP64 and matrix-core jobs adds the wake kernel
// beside the prep), each covering every bunch of every job it is given (jobs
// are described by device-resident descriptors, work by item lists, and each
// job's turn counter lives on the device, so a turn can be captured once and
// replayed), in this order:
//   k_scan  (one workgroup per job, only with long-range resonators): the
//           long-range phasors through the bunches in bucket order (a scan
//           of affine maps);
//   k_push  (tiles of 8192 particles): the single-particle map of every particle
//           (Sec. 2.2: Eq. 1 kick with RF, harmonic cavity and U0; Eq. 6
//           short-range kick of the particle's bin; long-range kick; Eq. 5
//           damping and quantum excitation; Eq. 2 drift), then -- on the new
//           tau, which is exactly the tau the next turn bins -- the LDS
//           histogram, the long-range deposit sums and the moment sums;
//   k_prep  (FP64 wake; per bunch, one workgroup per chunk of 16-64 bins):
//           finishes the push's per-bunch sums (moments, Sec. 2.4, and
//           long-range deposits), builds each bunch's binned wake potential
//           from its line density (Sec. 2.3), and writes the job's next turn
//           counter;
//   k_wake  (matrix-core wake modes, in place of k_prep; one workgroup per
//           16 bunches x 16 bins): the same between-turn work, with the wake
//           potential as a Toeplitz-by-histograms product on the MFMA units.
// Particle coordinates are FP64 structure-of-arrays rows, one row per bunch;
// each thread moves pairs of neighbouring particles with 16-byte loads and
// stores, and one Philox block gives both particles of a pair their noise.
// No floating-point atomics: all floating sums are fixed-order tile partials,
// so a run is bit-reproducible; histograms use integer atomics.
#include <algorithm>

#include "mbt_internal.h"
#include "mbt_fastmath.h"

namespace mbt {

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox_round(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                             uint32_t &x3, uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
}

// a ^ b ^ k in one instruction: v_bitop3_b32 evaluates any three-input
// bitwise function given by its truth table, and 0x96 is the one that is 1
// where an odd number of the inputs are 1.  k is wavefront-uniform (a round
// key) and is read from a scalar register.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    __asm__("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// A round after the first, where every word of the state varies across the
// wavefront: the same function as philox_round, with each three-way XOR in
// one instruction instead of two.
__device__ __forceinline__ void philox_round_v(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                               uint32_t &x3, uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = xor3((uint32_t)(p1 >> 32), x1, k0);
    const uint32_t y2 = xor3((uint32_t)(p0 >> 32), x3, k1);
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
}

__device__ __forceinline__ void philox10(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                         uint32_t k0, uint32_t k1)
{
    // The key is uniform across the wavefront; marking it as redefined here
    // keeps the compiler from hoisting all ten round keys out of the particle
    // loop (twenty scalar registers), so each round adds its Weyl step with
    // one scalar instruction instead.
    __asm__ volatile("" : "+s"(k0), "+s"(k1));
    // The first round in plain code: three of the four counter words are
    // uniform, and the compiler folds their part into scalar instructions.
    philox_round(x0, x1, x2, x3, k0, k1);
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        philox_round_v(x0, x1, x2, x3, k0, k1);
    }
}

// 53 random bits to a double in (0, 1]: never 0, so the logarithm is finite.
// The value is u = (x >> 11) 2^-53 + 2^-54 with x = hi 2^32 + lo, rounded
// once.  Spelled as hi 2^-32 + ((lo >> 11) 2^-53 + 2^-54): the inner scaling
// and sum are exact ((2 (lo >> 11) + 1) 2^-54 needs 22 bits) and the FMA
// rounds the exact total once, so the result is the same double, without
// the 64-bit shift and the second conversion's scaling.
__device__ __forceinline__ double u01_open0(uint32_t lo, uint32_t hi)
{
    const double low = ldexp((double)(lo >> 11), -53) + 0x1.0p-54;
    return fma((double)hi, 0x1.0p-32, low);
}

// Box-Muller pair from one Philox block: z0 = r cos(theta), z1 = r sin(theta).
// u1 rounds to 1 with probability 2^-53 (the largest 53-bit value plus the
// half step is a tie that rounds up); -2 ln u1 is then -0, where the
// reciprocal-square-root form of the square root gives NaN, so the argument
// is raised to the smallest normal double first (r = 2^-511 instead of 0).
__device__ __forceinline__ void normal_pair(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1, double &z0, double &z1)
{
    philox10(c0, c1, c2, c3, k0, k1);
    const double u1 = u01_open0(c0, c1);
    const double u2 = u01_open0(c2, c3);
    const double r = sqrt_pos(fmax(-2.0 * log_unit(u1), 0x1.0p-1022));
    double s, c;
    sincos_2pi(u2, s, c);
    z0 = r * c;
    z1 = r * s;
}

// ---------------------------------------------------------------------------
// Map pieces.
// ---------------------------------------------------------------------------

// Whether p holds on every active lane of the wavefront: the lane mask of
// the comparison that produced p against the execution mask, with no vector
// instruction beyond that comparison (__all materialises p first).
__device__ __forceinline__ bool wave_all(bool p)
{
    return __builtin_amdgcn_ballot_w64(p) == __builtin_amdgcn_read_exec();
}

// Slot of tau in a per-bin LDS table with a guard slot on each side: the bin
// index on the grid, -1 below it, nbins at or above it (the maxNum clamp
// sends NaN to -1; the conversion saturates), so that either guard stands
// for "outside the grid".  Within the grid it is the index bin_of gives.
__device__ __forceinline__ int bin_slot(const MapConst &c, double t)
{
    const double x = floor((t - c.tau_min) * c.inv_delta);
    return min((int)fmax(x, -1.0), c.nbins);
}

// Bin of tau on the fixed grid; -1 outside [tau_min, tau_max) (and for NaN).
__device__ __forceinline__ int bin_of(const MapConst &c, double t)
{
    const double x = (t - c.tau_min) * c.inv_delta;
    // both comparisons evaluated (no short-circuit), so this is a select,
    // not a branch; NaN fails both
    const bool in = (x >= 0.0) & (x < c.nbins_d);
    return (int)(in ? x : -1.0);
}

// sin and cos of x: when every lane of the wavefront has |x| <= pi/4 the
// minimax polynomials apply directly (the pi/2 reduction would be the
// identity, so the result is bit for bit the same); otherwise reduce first.
__device__ __forceinline__ void sincos_wave(double x, double &s, double &c)
{
    constexpr double kPio4 = 0.7853981633974483;
    if (wave_all(fabs(x) <= kPio4))
        sincos_poly(x, s, c);
    else
        sincos_cw(x, s, c);
}

// exp(y) for the long-range decay across a bunch: the degree-3 Taylor form
// without a per-lane branch when every lane has |y| < 1e-4 (the branch
// exp_small takes lane by lane there, so the result is the same).
__device__ __forceinline__ double exp_wave(double y)
{
    if (wave_all(fabs(y) < 1e-4))
        return exp_taylor3(y);
    return exp_small(y);
}

// sin and cos of the RF phase x = w_rf tau of a pair of particles.  Near the
// synchronous particle (every lane of the wavefront within |x| <= pi/4) the
// minimax polynomials apply directly; otherwise reduce by pi/2 first.
__device__ __forceinline__ void rf_phase(double x0, double x1, double &s0, double &c0, double &s1,
                                         double &c1)
{
    constexpr double kPio4 = 0.7853981633974483;
    if (wave_all(fmax(fabs(x0), fabs(x1)) <= kPio4)) {
        sincos_poly(x0, s0, c0);
        sincos_poly(x1, s1, c1);
    } else {
        sincos_cw(x0, s0, c0);
        sincos_cw(x1, s1, c1);
    }
}

// Which terms of the map are on: read from the map constants in the generic
// kernel (MAP = kMapGeneric), fixed at compile time in the specialisations
// for the usual configurations, which frees the registers and branches the
// flags cost.  A specialised kernel computes exactly what the generic one
// does for the same constants.
template <int MAP>
__device__ __forceinline__ bool hc_on(const MapConst &c)
{
    return MAP == kMapGeneric ? c.hc_on != 0 : MAP == kMapWakeNoiseHC3;
}
template <int MAP>
__device__ __forceinline__ bool sr_on(const MapConst &c)
{
    return MAP == kMapGeneric ? c.sr_on != 0 : true;
}
template <int MAP>
__device__ __forceinline__ bool noise_on(const MapConst &c)
{
    return MAP == kMapGeneric ? c.noise_on != 0 : true;
}

// Kick, damping + quantum excitation, drift of one particle (Sec. 2.2 Eqs. 1,
// 5, 2 with the Eq. 6 short-range kick and the long-range kick), all energy
// terms in units of E0:
//   RF:  V_rf sin(phi_s - w tau)/E0 = a cos(w tau) - b sin(w tau)
//   HC:  k V_rf sin(n phi_h - n w tau)/E0 = a_h cos(n w tau) - b_h sin(n w tau)
//   wake: vb = the bin's V/E0 (staged in LDS already divided by E0; read
//         before the noise so that the LDS latency hides behind it)
//   long range: Re[(V~/E0) exp((-alpha + i wbar) tau)]
// Energy gain in the main and harmonic cavities over E0, from sin and cos of
// w_rf tau.
template <int MAP>
__device__ __forceinline__ double rf_energy(const MapConst &c, double sx, double cx)
{
    double k = fma(c.rf_a, cx, -c.rf_b * sx);
    if (hc_on<MAP>(c)) {
        double sn, cn;
        multiple_angle(MAP == kMapWakeNoiseHC3 ? 3 : c.hc_n, sx, cx, sn, cn);
        k += fma(c.hc_a, cn, -c.hc_b * sn);
    }
    return k;
}

// The rest of the kick after the cavities' gain erf, then damping, noise
// and drift.
template <int NLR>
__device__ __forceinline__ void kick_rest(const MapConst &c, double k, const double vb,
                                          const double (&seen)[NLR > 0 ? NLR : 1][2], double z,
                                          double &t, double &d)
{
    k -= c.u0_e;
    k -= vb;  // the bin's wake voltage: 0 outside the grid or without a wake
#pragma unroll
    for (int r = 0; r < NLR; ++r) {
        const double e = exp_wave(-c.lr_alpha[r] * t);
        double s, co;
        sincos_wave(c.lr_wbar[r] * t, s, co);
        k -= e * fma(seen[r][0], co, -seen[r][1] * s);
    }
    const double dn = fma(c.noise, z, (d + k) * c.one_minus_D);
    d = dn;
    t = fma(c.drift, dn, t);
}

template <int NLR, int MAP>
__device__ __forceinline__ void kick_drift(const MapConst &c, const double vb,
                                           const double (&seen)[NLR > 0 ? NLR : 1][2], double sx,
                                           double cx, double z, double &t, double &d)
{
    double k = rf_energy<MAP>(c, sx, cx);
    k -= c.u0_e;
    k -= vb;  // the bin's wake voltage: 0 outside the grid or without a wake
#pragma unroll
    for (int r = 0; r < NLR; ++r) {
        const double e = exp_wave(-c.lr_alpha[r] * t);
        double s, co;
        sincos_wave(c.lr_wbar[r] * t, s, co);
        k -= e * fma(seen[r][0], co, -seen[r][1] * s);
    }
    // z = 0 without noise, and then the FMA returns dn unchanged
    const double dn = fma(c.noise, z, (d + k) * c.one_minus_D);
    d = dn;
    t = fma(c.drift, dn, t);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Per-particle epilogue on the new coordinates: histogram, sums of x and x^2
// for the moments, long-range deposit sums.  The moment sums are plain (no
// shift): bunch centroids stay within a few rms of the bucket centre, so the
// variance keeps full precision, and the result depends only on the present
// state, which makes a checkpointed run resume bit for bit.
// The deposit phase is evaluated from the post-drift tau itself (not
// rotated from the kick's phase), so the bin-only prologue of a resumed run
// computes exactly the same sums as the push it replaces.
template <int NLR, int MAP>
__device__ __forceinline__ void epilogue(const MapConst &c, uint32_t *hist_w, double t, double d,
                                         double *acc)
{
    if (sr_on<MAP>(c)) {
        // particles outside the grid go to a guard slot (-1 or nb), never merged
        atomicAdd(&hist_w[bin_slot(c, t)], 1u);
    }
    acc[0] += t;
    acc[1] = fma(t, t, acc[1]);
    acc[2] += d;
    acc[3] = fma(d, d, acc[3]);
#pragma unroll
    for (int r = 0; r < NLR; ++r) {
        const double e = exp_wave(c.lr_alpha[r] * t);
        double s, co;
        sincos_wave(c.lr_wbar[r] * t, s, co);
        acc[4 + 2 * r] = fma(e, co, acc[4 + 2 * r]);
        acc[5 + 2 * r] = fma(-e, s, acc[5 + 2 * r]);
    }
}

// LDS of the push: V/E0 of every bin with a zero guard on each side for
// "outside the grid", the sub-histograms (every bin with a guard slot on each
// side), and the wavefront partial sums.
size_t push_lds_bytes(int nbins, int nsub)
{
    size_t v = (size_t)(nbins + 2) * sizeof(double);
    size_t h = (size_t)nsub * (size_t)(nbins + 2) * sizeof(uint32_t);
    h = (h + 7) & ~(size_t)7;
    return v + h + (size_t)(kPushThreads / 64) * kPartStride * sizeof(double);
}

int conv_chunks(int nbins, int conv_out)
{
    return nbins > 0 ? (nbins + conv_out - 1) / conv_out : 1;
}

// Particle pairs per thread in a job's push tiles: the most (16: tiles of
// 8192 particles) unless the job then has fewer than 512 tiles, when the
// largest of 8, 4, 2, 1 that gives at least 512 tiles (or 1) is taken: a
// small job's turn is bound by the serial work of one tile, not by
// bandwidth.  A function of the job's shape alone, so a job's tile partition
// (and the order of its sums) is the same alone and in any batch.
int pairs_per_thread(int M, int64_t N)
{
    int p = kPairsPerThread;
    while (p > 1) {
        const int64_t tile = 2LL * kPushThreads * p;
        if ((int64_t)M * ((N + tile - 1) / tile) >= 512)
            break;
        p /= 2;
    }
    return p;
}

// Prep chunk width of a job: the widest of 64, 32, 16 bins that still gives
// at least 256 prep workgroups (one per compute unit), so that few large
// bunches get more threads per output bin and many bunches keep few
// workgroups.
int conv_width(int M, int nbins)
{
    int w = kConvOutMax;
    while (w > kConvOutMin && (int64_t)M * conv_chunks(nbins, w) < 256)
        w /= 2;
    return w;
}

// Map and epilogue of the pair (t0, d0), (t1, d1) = particles 2p, 2p + 1
// (the second only if `two`); the pushed coordinates are returned in place.
template <int NLR, bool PUSH, int MAP>
__device__ __forceinline__ void pair_compute(const MapConst &c, uint32_t key0, uint32_t key1,
                                             uint32_t turn, const double *Vs,
                                             const double (&seen)[NLR > 0 ? NLR : 1][2],
                                             uint32_t *hist_w, uint32_t p, uint32_t stream,
                                             bool two, double &t0, double &t1, double &d0,
                                             double &d1, double *acc)
{
    if (PUSH) {
        double vb0 = 0.0, vb1 = 0.0;
        if (sr_on<MAP>(c)) {
            vb0 = Vs[bin_slot(c, t0)];
            vb1 = Vs[bin_slot(c, t1)];
        }
        double z0 = 0.0, z1 = 0.0;
        if (noise_on<MAP>(c))
            normal_pair(p, stream, turn, 0u, key0, key1, z0, z1);
        double s0, c0, s1, c1;
        rf_phase(c.w_rf * t0, c.w_rf * t1, s0, c0, s1, c1);
        kick_drift<NLR, MAP>(c, vb0, seen, s0, c0, z0, t0, d0);
        kick_drift<NLR, MAP>(c, vb1, seen, s1, c1, z1, t1, d1);
    }
    epilogue<NLR, MAP>(c, hist_w, t0, d0, acc);
    if (two)
        epilogue<NLR, MAP>(c, hist_w, t1, d1, acc);
}

// Pointers known to address global memory: loads and stores through them
// compile to global (not flat) instructions, which the compiler cannot infer
// for pointers read from a descriptor.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
typedef double dvec2 __attribute__((ext_vector_type(2)));  // one 16-byte access

// Particle-row accesses of the push.  The push reads every coordinate once
// and writes it once per turn.  When the particle state of the launch is
// larger than the 256 MB Infinity Cache it cannot stay there between turns,
// and the loads and stores carry the non-temporal hint (NT = true): on the
// full fill (774 MB) this made the push 2.5-3.5% faster, with the hint on
// the loads alone or on the stores alone changing nothing.  A state that
// fits (the 128 MB current scan) is read back from the cache every turn,
// and there the hint made the push 14% slower, so it keeps the default.
template <bool NT, class T>
__device__ __forceinline__ T ld_row(const gptr<T> p)
{
    if (NT)
        return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st_row(gptr<T> p, T v)
{
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// ---------------------------------------------------------------------------
// k_push: an item is one tile of 512 ppt particles (8192 for all but small
// jobs) of one bunch of one job.  With one workgroup (256 threads) per item
// (ctr = null, grid = nitems) the hardware hands out the items; a persistent
// launch (grid < nitems) takes them from the launch's counter ctr[phase]
// instead, each workgroup fetching its next item while it works on the
// present one, so that every compute unit of every XCD stays busy until the
// list is done (a fixed blockIdx -> XCD assignment would leave the faster
// XCDs idle at the end).  The last workgroup to finish rewinds the counter
// (ctr[2 + phase] counts finished workgroups), so the next launch in this
// phase starts from item 0.  Which workgroup takes which tile changes no
// result bit: every tile has its own partial-sum slot.
// PUSH = false is the bin-only prologue that produces the histogram,
// deposits and moment sums of the present state without moving it.  Both
// write the histogram into counts[(clock + 1) & 1]: during the push of turn
// n the clock reads n, during the prologue at the start of turn n it reads
// n - 1.  Full tiles run a loop without bounds checks that loads the next
// pair before computing the current one.
// ---------------------------------------------------------------------------
// Occupancy: without long-range resonators the push fits in about 100
// registers; with one resonator it is held to 128 (a few spills outside the
// particle loop), so both run four workgroups (four waves per SIMD) per
// compute unit; with more resonators, the compiler's choice (two), since
// capping them spills inside the loop.
template <int NLR>
constexpr int push_min_blocks() { return NLR <= 1 ? 4 : 1; }

template <int NLR, bool PUSH, int MAP, bool NT>
__global__ __launch_bounds__(kPushThreads, push_min_blocks<NLR>()) void k_push(
    const JobDesc *__restrict__ jobs, const Item *__restrict__ items, const int nitems,
    const int grid, const int phase, uint32_t *__restrict__ ctr)
{
    extern __shared__ double smem[];
    __shared__ int s_next;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int NP = 4 + 2 * NLR;

    int it = blockIdx.x;
    if (ctr) {
        if (tid == 0)
            s_next = (int)atomicAdd(&ctr[phase], 1u);
        __syncthreads();
        it = s_next;
    }
    while (it < nitems) {
        uint32_t next = 0;
        if (ctr && tid == 0)
            next = atomicAdd(&ctr[phase], 1u);  // in flight while this tile is pushed
        // descriptors are read-only here, so these loads are scalar
        const Item item = items[it];
        const JobDesc &J = jobs[item.job];
        const MapConst &c = J.c;
        const int nb = c.nbins, nbx = nb > 0 ? nb : 1;
        const int b = item.bunch;
        const uint32_t tile = item.part;
        const uint32_t clock = __builtin_amdgcn_readfirstlane(J.clock[phase]);
        const uint32_t turn = clock;  // push of turn n runs with the clock at n

        double *Vs = smem + 1;  // [-1 .. nb]
        uint32_t *hist = reinterpret_cast<uint32_t *>(smem + nb + 2);
        const int nbh = nb + 2;  // sub-histogram stride: the bins and a guard slot on each side
        double *red = smem + nb + 2 + ((J.nsub * nbh + 1) >> 1);

        for (int k = tid; k < J.nsub * nbh; k += kPushThreads)
            hist[k] = 0u;
        if (PUSH && sr_on<MAP>(c))
            for (int k = tid - 1; k <= nb; k += kPushThreads)
                Vs[k] = k >= 0 && k < nb ? J.V[(size_t)b * nb + k] * c.inv_E0 : 0.0;
        __syncthreads();
        uint32_t *hist_w = hist + 1 + (J.nsub > 0 ? (wave % J.nsub) * nbh : 0);

        double seen[NLR > 0 ? NLR : 1][2];
#pragma unroll
        for (int r = 0; r < NLR; ++r) {
            seen[r][0] = J.seen[((size_t)r * J.M + b) * 2 + 0] * c.inv_E0;
            seen[r][1] = J.seen[((size_t)r * J.M + b) * 2 + 1] * c.inv_E0;
        }
        const uint32_t stream = J.stream[b];
        const gptr<double> tau = (gptr<double>)(J.tau + (size_t)b * J.ld);
        const gptr<double> del = (gptr<double>)(J.delta + (size_t)b * J.ld);
        double acc[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i)
            acc[i] = 0.0;

        // Indices within the bunch fit 32 bits (N <= 2^32, a pair index < 2^31).
        const int ppt = J.ppt;  // pairs per thread in this job's tiles
        const uint32_t pair0 = tile * (uint32_t)(kPushThreads * ppt);
        if ((int64_t)(pair0 + kPushThreads * ppt) * 2 <= J.N) {
            uint32_t p = pair0 + (uint32_t)tid;
            dvec2 tv = ld_row<NT>(reinterpret_cast<gptr<dvec2>>(tau + 2u * p));
            dvec2 dv = ld_row<NT>(reinterpret_cast<gptr<dvec2>>(del + 2u * p));
#ifndef MBT_PUSH_UNROLL
#define MBT_PUSH_UNROLL 1
#endif
#pragma unroll MBT_PUSH_UNROLL
            for (int s = 0; s < ppt; ++s) {
                dvec2 tn = tv, dn = dv;
                if (s + 1 < ppt) {
                    tn = ld_row<NT>(reinterpret_cast<gptr<dvec2>>(tau + 2u * (p + kPushThreads)));
                    dn = ld_row<NT>(reinterpret_cast<gptr<dvec2>>(del + 2u * (p + kPushThreads)));
                }
                double t0 = tv.x, t1 = tv.y, d0 = dv.x, d1 = dv.y;
                pair_compute<NLR, PUSH, MAP>(c, J.key0, J.key1, turn, Vs, seen, hist_w, p, stream, true,
                                        t0, t1, d0, d1, acc);
                if (PUSH) {
                    st_row<NT>(reinterpret_cast<gptr<dvec2>>(tau + 2u * p), dvec2{t0, t1});
                    st_row<NT>(reinterpret_cast<gptr<dvec2>>(del + 2u * p), dvec2{d0, d1});
                }
                tv = tn;
                dv = dn;
                p += kPushThreads;
            }
        } else {
            const uint32_t n_last = (uint32_t)(J.N - 1);  // last particle index
#pragma unroll 1
            for (int s = 0; s < ppt; ++s) {
                const uint32_t p = pair0 + (uint32_t)(s * kPushThreads + tid);
                const uint32_t j0 = 2u * p;
                if (j0 > n_last)
                    break;
                const bool two = j0 < n_last;
                double t0, t1 = 0.0, d0, d1 = 0.0;
                if (two) {
                    const dvec2 tv = ld_row<NT>(reinterpret_cast<gptr<dvec2>>(tau + j0));
                    const dvec2 dv = ld_row<NT>(reinterpret_cast<gptr<dvec2>>(del + j0));
                    t0 = tv.x; t1 = tv.y; d0 = dv.x; d1 = dv.y;
                } else {
                    t0 = ld_row<NT>(tau + j0);
                    d0 = ld_row<NT>(del + j0);
                }
                pair_compute<NLR, PUSH, MAP>(c, J.key0, J.key1, turn, Vs, seen, hist_w, p, stream, two,
                                        t0, t1, d0, d1, acc);
                if (PUSH) {
                    if (two) {
                        st_row<NT>(reinterpret_cast<gptr<dvec2>>(tau + j0), dvec2{t0, t1});
                        st_row<NT>(reinterpret_cast<gptr<dvec2>>(del + j0), dvec2{d0, d1});
                    } else {
                        st_row<NT>(tau + j0, t0);
                        st_row<NT>(del + j0, d0);
                    }
                }
            }
        }

        // Fixed-order tile reduction: wave butterflies, then waves in order.
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const double v = wave_sum(acc[i]);
            if (lane == 0)
                red[wave * kPartStride + i] = v;
        }
        __syncthreads();
        if (tid < NP) {
            double sum = red[tid];
            for (int w = 1; w < kPushThreads / 64; ++w)
                sum += red[w * kPartStride + tid];
            J.partials[((size_t)b * J.ntiles + tile) * kPartStride + tid] = sum;
        }
        // Merge the LDS sub-histograms into the bunch's histogram.
        if (sr_on<MAP>(c)) {
            uint32_t *out = J.counts + ((size_t)((clock + 1u) & 1u) * J.M + b) * nbx;
            for (int k = tid; k < nb; k += kPushThreads) {
                uint32_t sum = 0;
                for (int q = 0; q < J.nsub; ++q)
                    sum += hist[q * nbh + 1 + k];
                if (sum)
                    atomicAdd(&out[k], sum);
            }
        }
        if (ctr && tid == 0)
            s_next = (int)next;
        __syncthreads();  // LDS is reused by the next item
        it = ctr ? s_next : it + grid;
    }
    if (ctr && tid == 0) {
        // every fetch of this workgroup has returned; the last workgroup to
        // get here rewinds the counters for the next launch in this phase
        if (atomicAdd(&ctr[2 + phase], 1u) == (uint32_t)grid - 1u) {
            atomicExch(&ctr[phase], 0u);
            atomicExch(&ctr[2 + phase], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// k_prep: one workgroup per (job, bunch, chunk of 16-64 bins).  After the
// push of turn n (the counter reads n) it finishes the tile sums of the state after
// turn n (moments into the ring row of that turn, deposit sums S), records
// that state's histogram on profile turns, builds 64 bins of the wake
// potential from it, and clears the histogram buffer the push of turn n + 1
// fills; one workgroup per job then writes n + 1 into the other counter slot.
// The bin-only prologue is followed by the same prep with the counter at
// n - 1.
// ---------------------------------------------------------------------------

// Moments of bunch b from the tile sums of the last push (Sec. 2.4), and
// the bunch's long-range deposit sums S[r][b] = sum_j exp((alpha - i wbar) tau_j).
template <int NLR>
__device__ void finish_sums(const JobDesc &J, int b, uint32_t clock)
{
    constexpr int NP = 4 + 2 * NLR;
    __shared__ double sred[kPrepThreads / 64][NP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int np = 4 + 2 * J.nlr;
    double s[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i)
        s[i] = 0.0;
    for (int t = tid; t < J.ntiles; t += kPrepThreads) {
        const double *p = J.partials + ((size_t)b * J.ntiles + t) * kPartStride;
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (i < np)
                s[i] += p[i];
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double v = wave_sum(s[i]);
        if (lane == 0)
            sred[wave][i] = v;
    }
    __syncthreads();
    if (tid < NP) {
        double tot = sred[0][tid];
        for (int w = 1; w < kPrepThreads / 64; ++w)
            tot += sred[w][tid];
        sred[0][tid] = tot;
    }
    __syncthreads();
    // turns since the start of the call; the state before its first turn
    // (rel = -1) is neither stored nor recorded
    const int32_t rel = (int32_t)(clock - J.base);
    if (tid == 0) {
        const double invN = 1.0 / (double)J.N;
        const double mt = sred[0][0] * invN, md = sred[0][2] * invN;
        const double vt = sred[0][1] * invN - mt * mt, vd = sred[0][3] * invN - md * md;
        if (rel >= 0) {
            double *m = J.mom_ring + ((size_t)(rel & (J.mom_slots - 1)) * J.M + b) * 4;
            m[0] = mt;
            m[1] = md;
            m[2] = sqrt(vt > 0.0 ? vt : 0.0);
            m[3] = sqrt(vd > 0.0 ? vd : 0.0);
        }
        if (!isfinite(mt) || !isfinite(md) || !isfinite(vt) || !isfinite(vd))
            atomicOr(J.status, 1u);
    }
    if (tid < 2 * J.nlr)
        J.S[((size_t)(tid >> 1) * J.M + b) * 2 + (tid & 1)] = sred[0][4 + tid];
    // histogram of this state on every prof_stride-th turn of the call
    if (J.prof_stride > 0 && rel >= 0 && rel % J.prof_stride == 0) {
        const int nb = J.c.nbins;
        const uint32_t *src = J.counts + ((size_t)((clock + 1u) & 1u) * J.M + b) * nb;
        const int row = (rel / J.prof_stride) & (J.prof_slots - 1);
        uint32_t *dst = J.prof_ring + ((size_t)row * J.M + b) * nb;
        for (int k = tid; k < nb; k += kPrepThreads)
            dst[k] = src[k];
    }
}

// Bins [k0, k1) of bunch b's wake potential (Sec. 2.3):
// V[k] = qpp * sum_{m<=k} W[k-m] c[m].  A workgroup takes w = conv_out
// bins with K = 256 / w threads per output bin, each summing every K-th
// source bin with two accumulators; the K partial sums are added by a
// butterfly across the K lanes (a fixed order).
__device__ void conv_chunk(const JobDesc &J, int b, int chunk, uint32_t clock, double *psm)
{
    __shared__ int s_lo;
    const int w = J.conv_out, K = kPrepThreads / w;
    const int tid = threadIdx.x;
    const int nb = J.c.nbins;
    const int k0 = chunk * w, k1 = min(k0 + w, nb);
    const uint32_t *cin = J.counts + ((size_t)((clock + 1u) & 1u) * J.M + b) * nb;
    uint32_t *cclr = J.counts + ((size_t)(clock & 1u) * J.M + b) * nb;
    double *sW = psm;        // W[0 .. k1)
    double *sc = psm + nb;   // c[0 .. k1)
    if (tid == 0)
        s_lo = k1;
    __syncthreads();
    int lo = k1;             // first occupied bin: nothing below it contributes
    // every load of a pass is issued before its first store, so a pass costs
    // one memory latency
    for (int ks = 0; ks < k1; ks += 4 * kPrepThreads) {
        double wv[4];
        uint32_t cv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = ks + tid + u * kPrepThreads;
            wv[u] = k < k1 ? J.W[k] : 0.0;
            cv[u] = k < k1 ? cin[k] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = ks + tid + u * kPrepThreads;
            if (k < k1) {
                sW[k] = wv[u];
                sc[k] = (double)cv[u];
                if (cv[u] && k < lo)
                    lo = k;
            }
        }
    }
    if (lo < k1)
        atomicMin(&s_lo, lo);
    __syncthreads();
    lo = s_lo;
    // the K ways of an output are consecutive lanes of one wavefront (K is
    // 4, 8 or 16)
    const int o = tid / K, q = tid % K;  // output, way
    const int k = k0 + o;
    double acc0 = 0.0, acc1 = 0.0;
    if (k < k1) {
        int m = lo + q;
        for (; m + K <= k; m += 2 * K) {
            acc0 = fma(sW[k - m], sc[m], acc0);
            acc1 = fma(sW[k - m - K], sc[m + K], acc1);
        }
        if (m <= k)
            acc0 = fma(sW[k - m], sc[m], acc0);
    }
    // fixed-order butterfly over the K ways, every lane taking part
    double v = acc0 + acc1;
    for (int off = K >> 1; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    if (q == 0 && k < k1)
        J.V[(size_t)b * nb + k] = J.qpp[b] * v;
    for (int kk = k0 + tid; kk < k1; kk += kPrepThreads)
        cclr[kk] = 0u;
}

template <int NLR>
__device__ __forceinline__ void prep_body(const PrepLaunch &L, const Item &item, const JobDesc &J,
                                          const uint32_t clock, double *psm)
{
    if (item.part == 0)
        finish_sums<NLR>(J, item.bunch, clock);
    // jobs whose wake potential comes from the matrix cores have no prep
    // items: k_wake does their between-turn work
    if (J.c.sr_on)
        conv_chunk(J, item.bunch, (int)item.part, clock, psm);
}

template <int NLR>
__global__ __launch_bounds__(kPrepThreads) void k_prep(const PrepLaunch L)
{
    extern __shared__ double psm[];
    const int bx = blockIdx.x;
    const Item item = L.inner > 0 ? Item{0, (uint16_t)(bx / L.inner), (uint32_t)(bx % L.inner)}
                                  : L.items[bx];
    const JobDesc &J = L.jobs[item.job];
    const uint32_t clock = L.clk ? L.clk[L.phase] : J.clock[L.phase];
    prep_body<NLR>(L, item, J, clock, psm);
    // the next turn's counter, in the slot no launch of this turn reads
    if (item.bunch == 0 && item.part == 0 && threadIdx.x == 0)
        J.clock[L.phase ^ 1] = clock + 1u;
}// ---------------------------------------------------------------------------
// k_wake: the short-range wake potential of all bunches as one product of
// the lower-triangular Toeplitz matrix T[k][m] = W[k - m] (Sec. 2.3) with
// the matrix of line densities C[m][b] (bin m, bunch b), on the matrix
// cores: V[b][k] = qpp_b sum_m T[k][m] C[m][b].
//   FP32:   W / s rounded to FP32, counts exact in FP32 (below 2^24),
//           v_mfma_f32_16x16x4_f32, FP32 accumulation.
//   BF16xn: W / s = W_0 + W_1 (+ W_2), each term BF16 (8 significant bits,
//           so the residual after n terms is about 2^-9n of W); every count
//           c = sum_p c_p 2^(8p) with 8-bit parts c_p, each exact in BF16;
//           v_mfma_f32_16x16x16_bf16 accumulates sum_q T_q C_p in FP32 per
//           part p; the parts are combined in FP64.
// s is a power of two near max |W|, so the tables are O(1).  A workgroup
// covers one 16 x 16 output tile (16 bins x 16 bunches); its four
// wavefronts take interleaved 16-bin steps of the reduction over m, which
// stops at the diagonal, and their four partial tiles are added in
// wavefront order in FP64.  MFMA 16x16 operand layout (lane l,
// element r): A[l % 16][4 (l / 16) + r], B[4 (l / 16) + r][l % 16], and the
// result C[4 (l / 16) + r][l % 16]; for the f32 form with K = 4,
// A[l % 16][l / 16] and B[l / 16][l % 16].
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// An integer in [0, 256] as BF16: its float has at most 8 significant bits,
// so the upper half of the float is the exact BF16.
__device__ __forceinline__ short small_int_bf16(uint32_t v)
{
    return (short)(__float_as_uint((float)v) >> 16);
}

// Moments and deposit sums of bunch b by one wavefront (the calling lanes
// are its 64 lanes): the additions of finish_sums's workgroup, in the same
// order (its four 64-thread slices one after another, each slice's lanes
// summing every 256th tile, then a butterfly), so the results are the same
// doubles.  Used where a wavefront, not a workgroup, is free for the bunch.
// A slice with no tile adds +0.0, which changes no total (a sum of tile
// partials that start from +0.0 is never -0.0), so the slices past the
// last tile are skipped.
__device__ __forceinline__ void finish_sums_wave(const JobDesc &J, int b, uint32_t clock, int lane)
{
    const int np = 4 + 2 * J.nlr;
    double tot[kPartStride];
#pragma unroll
    for (int i = 0; i < kPartStride; ++i)
        tot[i] = 0.0;
#pragma unroll 1
    for (int w = 0; w < kPrepThreads / 64 && 64 * w < J.ntiles; ++w) {
        double s[kPartStride];
#pragma unroll
        for (int i = 0; i < kPartStride; ++i)
            s[i] = 0.0;
        for (int t = 64 * w + lane; t < J.ntiles; t += kPrepThreads) {
            const double *p = J.partials + ((size_t)b * J.ntiles + t) * kPartStride;
#pragma unroll
            for (int i = 0; i < kPartStride; ++i)
                if (i < np)
                    s[i] += p[i];
        }
#pragma unroll
        for (int i = 0; i < kPartStride; ++i)
            if (i < np) {
                const double v = wave_sum(s[i]);
                tot[i] = w == 0 ? v : tot[i] + v;
            }
    }
    const int32_t rel = (int32_t)(clock - J.base);
    if (lane == 0) {
        const double invN = 1.0 / (double)J.N;
        const double mt = tot[0] * invN, md = tot[2] * invN;
        const double vt = tot[1] * invN - mt * mt, vd = tot[3] * invN - md * md;
        if (rel >= 0) {
            double *m = J.mom_ring + ((size_t)(rel & (J.mom_slots - 1)) * J.M + b) * 4;
            m[0] = mt;
            m[1] = md;
            m[2] = sqrt(vt > 0.0 ? vt : 0.0);
            m[3] = sqrt(vd > 0.0 ? vd : 0.0);
        }
        if (!isfinite(mt) || !isfinite(md) || !isfinite(vt) || !isfinite(vd))
            atomicOr(J.status, 1u);
    }
#pragma unroll
    for (int i = 0; i < 2 * kMaxLR; ++i)
        if (lane == i && i < 2 * J.nlr)
            J.S[((size_t)(i >> 1) * J.M + b) * 2 + (i & 1)] = tot[4 + i];
}

// Bins of the count block staged in LDS at a time, and the row stride of the
// staged block (in words): rows start 16 bytes apart modulo the 32 banks, so
// the 16 rows a wavefront reads at once fall into different banks.
constexpr int kWakeStage = 256;
__host__ __device__ constexpr int wake_stage_stride(int width) { return ((width + 3) & ~3) + 4; }
// Partial output tiles of the four wavefronts: [wave][part][element][lane].
constexpr int kWakeRed = 4 * 4 * 4 * 64;

size_t wake_lds_bytes(int mode, int nbins_max)
{
    const int kmax = std::min(nbins_max, 4096);
    const size_t w = mode == kWakeFP32 ? (size_t)kmax * 4
                                       : (size_t)(mode == kWakeBF16x2 ? 2 : 3) * kmax * 2;
    const size_t c = (size_t)kWakeBunches * wake_stage_stride(std::min(kmax, kWakeStage)) * 4;
    return ((w + 15) & ~(size_t)15) + c + (size_t)kWakeRed * sizeof(float);
}

// The whole between-turn work of a job whose wake potential is computed on
// the matrix cores (it has no prep items).  A workgroup takes 16 bunches x
// 16 output bins: it finishes the tile sums of its share of those bunches,
// one wavefront per bunch; multiplies the wake table by the bunches'
// histograms staged in LDS; records the histogram tile on profile turns;
// clears the tile of the histogram buffer the next push fills; one
// workgroup per job writes the next turn into the other counter slot.
template <int MODE>
__global__ __launch_bounds__(256) void k_wake(const WakeLaunch L)
{
    extern __shared__ double wsm[];
    const int bx = blockIdx.x;
    const Item item = L.inner > 0 ? Item{0, (uint16_t)(bx / L.inner), (uint32_t)(bx % L.inner)}
                                  : L.items[bx];
    const JobDesc &J = L.jobs[item.job];
    const int nb = J.c.nbins, M = J.M;
    const int b0 = (int)item.bunch * kWakeBunches;
    const int nbt = min(kWakeBunches, M - b0);  // bunches of this tile
    const int kb = (int)item.part * kWakeBins;   // output bins kb .. kb + 15
    const int nparts = (nb + kWakeBins - 1) / kWakeBins;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t clock = L.clk ? L.clk[L.phase] : J.clock[L.phase];
    const uint32_t *cnt = J.counts + (size_t)((clock + 1u) & 1u) * M * nb;
    constexpr int NW = MODE == kWakeFP32 ? 1 : (MODE == kWakeBF16x2 ? 2 : 3);

    // W (or its parts) at distances [0, kmax) and the histograms of the
    // tile's bunches, a block of bins at a time, are staged in LDS.  Every
    // load of a pass is issued before its first store, and the first pass
    // of both before the sums, so their memory latencies overlap.
    const int kmax = min(nb, kb + kWakeBins);  // source bins [0, kmax) reach the tile
    float *wf = reinterpret_cast<float *>(wsm);
    uint16_t *wb = reinterpret_cast<uint16_t *>(wsm);
    const int wbytes = MODE == kWakeFP32 ? kmax * 4 : NW * kmax * 2;
    uint32_t *sc = reinterpret_cast<uint32_t *>(reinterpret_cast<unsigned char *>(wsm) +
                                                ((wbytes + 15) & ~15));
    const int cst = wake_stage_stride(min(kmax, kWakeStage));
    float *red = reinterpret_cast<float *>(sc + kWakeBunches * cst);
    float wv32[4];
    uint16_t wv16[NW][4];
    auto load_w = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + tid + 256 * u;
            if (MODE == kWakeFP32) {
                wv32[u] = k < kmax ? J.Wf32[k] : 0.f;
            } else {
#pragma unroll
                for (int q = 0; q < NW; ++q)
                    wv16[q][u] = k < kmax ? J.Wbf[(size_t)q * nb + k] : (uint16_t)0;
            }
        }
    };
    auto store_w = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + tid + 256 * u;
            if (k < kmax) {
                if (MODE == kWakeFP32) {
                    wf[k] = wv32[u];
                } else {
#pragma unroll
                    for (int q = 0; q < NW; ++q)
                        wb[q * kmax + k] = wv16[q][u];
                }
            }
        }
    };
    uint32_t cv[kWakeBunches];
    auto load_counts = [&](int mb, int width) {
#pragma unroll
        for (int r = 0; r < kWakeBunches; ++r)
            cv[r] = (r < nbt && tid < width) ? cnt[(size_t)(b0 + r) * nb + mb + tid] : 0u;
    };
    auto store_counts = [&](int width) {
#pragma unroll
        for (int r = 0; r < kWakeBunches; ++r)
            if (r < nbt && tid < width)
                sc[r * cst + tid] = cv[r];
    };
    load_w(0);
    load_counts(0, min(kWakeStage, kmax));

    // Sums of the tile's bunches b0 + j with j = part, part + nparts, ...
    // (every bunch of the tile exactly once over its workgroups), the i-th
    // of them by wavefront i mod 4.
    for (int j = (int)item.part, i = 0; j < nbt; j += nparts, ++i)
        if ((i & 3) == wave)
            finish_sums_wave(J, b0 + j, clock, lane);

    store_w(0);
    for (int k0 = 1024; k0 < kmax; k0 += 1024) {
        load_w(k0);
        store_w(k0);
    }

    const int i = lane & 15, g = lane >> 4;
    const bool bok = i < nbt;      // this lane's column is a bunch of the job
    const bool rok = kb + i < nb;  // row of this lane's A operand inside the grid
    floatx4 acc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
        acc[p] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int np = J.count_parts;
    for (int mb = 0; mb < kmax; mb += kWakeStage) {
        // histogram bins [mb, mb + width) of the tile's bunches
        const int width = min(kWakeStage, kmax - mb);
        if (mb > 0)
            load_counts(mb, width);
        __syncthreads();  // W staged; the previous block's readers are done
        store_counts(width);
        __syncthreads();
        const uint32_t *crow = sc + (bok ? i : 0) * cst;  // bin m at crow[m - mb]
        const int m1 = mb + width;
        // this wavefront's steps: m0 = mb + 16 (wave + 4 t)
        for (int m0 = mb + 16 * wave; m0 < m1; m0 += 64) {
            if (MODE == kWakeFP32) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int m = m0 + 4 * s + g;
                    const int d = kb + i - m;
                    const float a = (rok && d >= 0) ? wf[d] : 0.f;
                    const float c = (bok && m < m1) ? (float)crow[m - mb] : 0.f;
                    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, c, acc[0], 0, 0, 0);
                }
            } else {
                const int mg = m0 + 4 * g;
                uint32_t c[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    c[r] = (bok && mg + r < m1) ? crow[mg + r - mb] : 0u;
                bf16x4 a[NW];
                const int d0 = kb + i - mg;
#pragma unroll
                for (int q = 0; q < NW; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        a[q][r] = (rok && d0 - r >= 0) ? (short)wb[q * kmax + d0 - r] : (short)0;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    if (p >= np)
                        break;
                    bf16x4 bp;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        bp[r] = small_int_bf16((c[r] >> (8 * p)) & 255u);
#pragma unroll
                    for (int q = 0; q < NW; ++q)
                        acc[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[q], bp, acc[p], 0, 0, 0);
                }
            }
        }
    }
    // the four partial tiles, then each thread one element of the tile:
    // column i = lane % 16, row 4 (lane / 16) + r with r = tid / 64
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[((wave * 4 + p) * 4 + r) * 64 + lane] = acc[p][r];
    __syncthreads();
    {
        const int r = wave;  // element handled by this thread
        const int k = kb + 4 * g + r;
        if (bok && k < nb) {
            const int nparts_sum = MODE == kWakeFP32 ? 1 : np;
            double v = 0.0, w = 1.0;
            for (int p = 0; p < nparts_sum; ++p, w *= 256.0) {
                double sp = (double)red[((0 * 4 + p) * 4 + r) * 64 + lane];
#pragma unroll
                for (int ww = 1; ww < 4; ++ww)
                    sp += (double)red[((ww * 4 + p) * 4 + r) * 64 + lane];
                v = fma(w, sp, v);
            }
            J.V[(size_t)(b0 + i) * nb + k] = J.qpp[b0 + i] * J.wake_scale * v;
        }
    }

    // the histogram tile on every prof_stride-th turn of the call
    const int32_t rel = (int32_t)(clock - J.base);
    const int tw = kmax - kb;  // bins of this tile
    if (J.prof_stride > 0 && rel >= 0 && rel % J.prof_stride == 0) {
        const int row = (rel / J.prof_stride) & (J.prof_slots - 1);
        for (int e = tid; e < nbt * tw; e += 256) {
            const int r = e / tw, k = kb + e % tw;
            J.prof_ring[((size_t)row * M + b0 + r) * nb + k] = cnt[(size_t)(b0 + r) * nb + k];
        }
    }
    // clear the tile of the buffer the next push fills
    uint32_t *cclr = J.counts + (size_t)(clock & 1u) * M * nb;
    for (int e = tid; e < nbt * tw; e += 256)
        cclr[(size_t)(b0 + e / tw) * nb + kb + e % tw] = 0u;
    // the next turn's counter, in the slot no launch of this turn reads
    if (item.bunch == 0 && item.part == 0 && tid == 0)
        J.clock[L.phase ^ 1] = clock + 1u;
}

// ---------------------------------------------------------------------------
// k_scan: one workgroup per job with long-range resonators, before the push.
// Carries the job's long-range phasors through the bunches in bucket order.  Passing bunch b maps the phasor x to G_b x + D_b (rotation
// across the gap from the previous filled bucket, then the bunch's deposit
// D_b = qpp_b c_r S_b); the bunch sees G_b x.  The chain of M affine maps is
// evaluated as a scan: each thread composes a contiguous run of bunches, a
// Hillis-Steele scan over the 256 composed maps (fixed order, so
// deterministic) gives each run its incoming phasor, and each thread then
// replays its run to record what every bunch sees.
// ---------------------------------------------------------------------------
struct cplx {
    double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b)
{
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx cmuladd(cplx a, cplx b, cplx c)
{
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}

__global__ __launch_bounds__(kPrepThreads) void k_scan(const ScanLaunch L)
{
    __shared__ cplx mA[kPrepThreads], mB[kPrepThreads];  // composed maps
    const JobDesc &J = L.jobs[blockIdx.x];
    const int tid = threadIdx.x;
    const int M = J.M;
    const int run = (M + kPrepThreads - 1) / kPrepThreads;
    const int b_lo = min(tid * run, M), b_hi = min(b_lo + run, M);
#pragma unroll 1
    for (int r = 0; r < J.nlr; ++r) {
        cplx *seen = reinterpret_cast<cplx *>(J.seen) + (size_t)r * M;
        const cplx *gap = reinterpret_cast<const cplx *>(J.gap) + (size_t)r * M;
        const cplx *qc = reinterpret_cast<const cplx *>(J.qc) + (size_t)r * M;
        const cplx *S = reinterpret_cast<const cplx *>(J.S) + (size_t)r * M;
        // 1. this thread's run: compose x -> G_b x + qc_b S_b over its bunches
        cplx A = {1.0, 0.0}, B = {0.0, 0.0};
        for (int b = b_lo; b < b_hi; ++b) {
            const cplx G = gap[b];
            A = cmul(G, A);
            B = cmuladd(G, B, cmul(qc[b], S[b]));
        }
        mA[tid] = A;
        mB[tid] = B;
        __syncthreads();
        // 2. inclusive scan of the maps: map[t] <- map[t] o map[t - d]
        for (int d = 1; d < kPrepThreads; d <<= 1) {
            cplx nA = mA[tid], nB = mB[tid];
            if (tid >= d) {
                const cplx pA = mA[tid - d], pB = mB[tid - d];
                nB = cmuladd(nA, pB, nB);
                nA = cmul(nA, pA);
            }
            __syncthreads();
            mA[tid] = nA;
            mB[tid] = nB;
            __syncthreads();
        }
        // 3. incoming phasor of this run, then replay the run
        const cplx x0 = {J.phasor[2 * r], J.phasor[2 * r + 1]};
        cplx x = x0;
        if (tid > 0)
            x = cmuladd(mA[tid - 1], x0, mB[tid - 1]);
        for (int b = b_lo; b < b_hi; ++b) {
            x = cmul(gap[b], x);
            seen[b] = x;
            const cplx D = cmul(qc[b], S[b]);
            x = {x.re + D.re, x.im + D.im};
        }
        __syncthreads();
        if (tid == kPrepThreads - 1) {
            const cplx xe = cmuladd(mA[tid], x0, mB[tid]);
            J.phasor[2 * r] = xe.re;
            J.phasor[2 * r + 1] = xe.im;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Transverse plane (Sec. 2.2 Eqs. 3-5; Sec. 2.3, Eq. 6 second line and the
// long-range resistive wall of its last paragraph).  k_push_tr is k_push with
// one transverse plane (x, x') moved beside (tau, delta): the same
// longitudinal arithmetic, plus per particle the wall kick of its bunch and
// the transverse wake kick of its bin on x', the betatron rotation about the
// dispersive orbit, adiabatic damping and the plane's noise; its epilogue
// adds the bins' dipole sums (exact integer sums in LDS, merged into the
// bunch's buffer with 64-bit integer atomics) and the sums of x, x^2, x',
// x'^2.  Every switch is read from the descriptor (no compile-time map).
// ---------------------------------------------------------------------------

// x rounded to the nearest multiple of 2^-52 m, as that integer (|x| < 2^11 m):
// the scaling is exact, rint rounds once, and the integral double is split
// into 32-bit halves exactly.
__device__ __forceinline__ unsigned long long dipole_q(double x)
{
    const double r = rint(x * kDipoleScale);
    const double hi = floor(r * 0x1.0p-32);
    const double lo = fma(hi, -4294967296.0, r);  // r - hi 2^32, in [0, 2^32), exact
    return ((unsigned long long)(long long)(int)hi << 32) + (unsigned long long)(uint32_t)lo;
}

// Transverse part of one particle's turn (the longitudinal state d is the
// value before the kick; erf the cavities' energy gain over E0).
__device__ __forceinline__ void betatron(const TransConst &tc, double din, double erf, double ub,
                                         double rwk, bool rw, double zx, double zxp, double &x,
                                         double &xp)
{
    double p = xp;
    if (rw)
        p = p + rwk;  // the wall's kick of the previous turn's passages
    p = p + ub;       // the bin's transverse wake kick (0 outside the grid)
    const double psi = 6.283185307179586 * (tc.qfrac + tc.chrom * din);
    double sn, cs;
    sincos_cw(psi, sn, cs);
    const double xb = x - tc.disp * din;
    const double xpb = p - tc.disp_p * din;
    double x2 = (tc.disp * din + (cs + tc.alpha * sn) * xb) + (tc.beta * sn) * xpb;
    double xp2 = (tc.disp_p * din - (tc.gamma * sn) * xb) + (cs - tc.alpha * sn) * xpb;
    xp2 = xp2 * ((1.0 + din) / ((1.0 + din) + erf));
    if (tc.noise_on) {
        x2 = x2 + tc.noise_x * zx;
        xp2 = xp2 + tc.noise_xp * zxp;
    }
    x = x2;
    xp = xp2;
}

// The four coordinates of a particle pair of the transverse push.
struct TrRows {
    dvec2 t, d, x, xp;
};
template <bool NT>
__device__ __forceinline__ TrRows load_tr_rows(const gptr<double> rt, const gptr<double> rd,
                                               const gptr<double> rx, const gptr<double> rxp,
                                               uint32_t j0)
{
    return TrRows{ld_row<NT>(reinterpret_cast<gptr<dvec2>>(rt + j0)),
                  ld_row<NT>(reinterpret_cast<gptr<dvec2>>(rd + j0)),
                  ld_row<NT>(reinterpret_cast<gptr<dvec2>>(rx + j0)),
                  ld_row<NT>(reinterpret_cast<gptr<dvec2>>(rxp + j0))};
}

template <int NLR, bool PUSH, bool NT>
__global__ __launch_bounds__(kPushThreads, 2) void k_push_tr(
    const JobDesc *__restrict__ jobs, const Item *__restrict__ items, const int nitems,
    const int grid, const int phase)
{
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int NP = 4 + 2 * NLR;
    constexpr int NA = NP + 4;  // + x, x^2, x', x'^2

    for (int it = blockIdx.x; it < nitems; it += grid) {
        const Item item = items[it];
        const JobDesc &J = jobs[item.job];
        const MapConst &c = J.c;
        const TransConst &tc = J.t;
        const int nb = c.nbins, nbx = nb > 0 ? nb : 1;
        const int b = item.bunch;
        const uint32_t tile = item.part;
        const uint32_t clock = __builtin_amdgcn_readfirstlane(J.clock[phase]);
        const uint32_t turn = clock;

        // LDS: V/E0 and U of every bin plus a zero slot, the dipole sums
        // (bins plus an outside slot), the sub-histograms, the wave sums
        double *Vs = smem;                        // [nb + 1]
        double *Us = Vs + nb + 1;                 // [nb + 1]
        unsigned long long *xh =
            reinterpret_cast<unsigned long long *>(Us + nb + 1);  // [nb + 1]
        uint32_t *hist = reinterpret_cast<uint32_t *>(xh + nb + 1);
        const int nbh = nb + 1;
        double *red = reinterpret_cast<double *>(xh + nb + 1) + ((J.nsub * nbh + 1) >> 1);

        for (int k = tid; k < J.nsub * nbh; k += kPushThreads)
            hist[k] = 0u;
        for (int k = tid; k <= nb; k += kPushThreads) {
            xh[k] = 0ull;
            if (PUSH && c.sr_on) {
                Vs[k] = k < nb ? J.V[(size_t)b * nb + k] * c.inv_E0 : 0.0;
                Us[k] = k < nb ? J.U[(size_t)b * nb + k] : 0.0;
            }
        }
        __syncthreads();
        uint32_t *hist_w = hist + (J.nsub > 0 ? (wave % J.nsub) * nbh : 0);

        double seen[NLR > 0 ? NLR : 1][2];
#pragma unroll
        for (int r = 0; r < NLR; ++r) {
            seen[r][0] = J.seen[((size_t)r * J.M + b) * 2 + 0] * c.inv_E0;
            seen[r][1] = J.seen[((size_t)r * J.M + b) * 2 + 1] * c.inv_E0;
        }
        const bool rw = tc.rw_turns > 0;
        const double rwk = rw ? J.rwk[b] : 0.0;
        const uint32_t stream = J.stream[b];
        const size_t row = (size_t)b * J.ld;
        double acc[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i)
            acc[i] = 0.0;

        const int ppt = J.ppt;
        const uint32_t pair0 = tile * (uint32_t)(kPushThreads * ppt);
        const uint32_t n_last = (uint32_t)(J.N - 1);
        const gptr<double> rt = (gptr<double>)(J.tau + row), rd = (gptr<double>)(J.delta + row);
        const gptr<double> rx = (gptr<double>)(J.x + row), rxp = (gptr<double>)(J.xp + row);
        // The map and epilogue of the pair (particles j0, j0 + 1; the second
        // only if `two`), coordinates in place.
        auto pair = [&](uint32_t p, bool two, double (&t)[2], double (&d)[2], double (&x)[2],
                        double (&xp)[2]) {
            if (PUSH) {
                double vb[2] = {0.0, 0.0}, ub[2] = {0.0, 0.0};
                if (c.sr_on) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const int k = bin_of(c, t[i]);
                        vb[i] = Vs[k >= 0 ? k : nb];
                        ub[i] = Us[k >= 0 ? k : nb];
                    }
                }
                double z[2] = {0.0, 0.0}, zx[2] = {0.0, 0.0}, zxp[2] = {0.0, 0.0};
                if (c.noise_on)
                    normal_pair(p, stream, turn, 0u, J.key0, J.key1, z[0], z[1]);
                if (tc.noise_on) {
                    normal_pair(p, stream, turn, 2u, J.key0, J.key1, zx[0], zx[1]);
                    normal_pair(p, stream, turn, 3u, J.key0, J.key1, zxp[0], zxp[1]);
                }
                double sx[2], cx[2];
                rf_phase(c.w_rf * t[0], c.w_rf * t[1], sx[0], cx[0], sx[1], cx[1]);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const double erf = rf_energy<kMapGeneric>(c, sx[i], cx[i]);
                    betatron(tc, d[i], erf, ub[i], rwk, rw, zx[i], zxp[i], x[i], xp[i]);
                    kick_rest<NLR>(c, erf, vb[i], seen, z[i], t[i], d[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if (i == 1 && !two)
                    break;
                if (c.sr_on) {
                    const int k = bin_of(c, t[i]);
                    atomicAdd(&hist_w[k >= 0 ? k : nb], 1u);
                    atomicAdd(&xh[k >= 0 ? k : nb], dipole_q(x[i]));
                }
                acc[0] += t[i];
                acc[1] = fma(t[i], t[i], acc[1]);
                acc[2] += d[i];
                acc[3] = fma(d[i], d[i], acc[3]);
#pragma unroll
                for (int r = 0; r < NLR; ++r) {
                    const double e = exp_wave(c.lr_alpha[r] * t[i]);
                    double sn, co;
                    sincos_wave(c.lr_wbar[r] * t[i], sn, co);
                    acc[4 + 2 * r] = fma(e, co, acc[4 + 2 * r]);
                    acc[5 + 2 * r] = fma(-e, sn, acc[5 + 2 * r]);
                }
                acc[NP + 0] += x[i];
                acc[NP + 1] = fma(x[i], x[i], acc[NP + 1]);
                acc[NP + 2] += xp[i];
                acc[NP + 3] = fma(xp[i], xp[i], acc[NP + 3]);
            }
        };
        if ((int64_t)(pair0 + kPushThreads * ppt) * 2 <= J.N) {
            // full tile: 16-byte pair accesses, the next pair loaded before
            // the present one is pushed
            uint32_t p = pair0 + (uint32_t)tid;
            TrRows cur = load_tr_rows<NT>(rt, rd, rx, rxp, 2u * p);
#pragma unroll 1
            for (int s = 0; s < ppt; ++s) {
                TrRows nxt = cur;
                if (s + 1 < ppt)
                    nxt = load_tr_rows<NT>(rt, rd, rx, rxp, 2u * (p + kPushThreads));
                double t[2] = {cur.t.x, cur.t.y}, d[2] = {cur.d.x, cur.d.y};
                double x[2] = {cur.x.x, cur.x.y}, xp[2] = {cur.xp.x, cur.xp.y};
                pair(p, true, t, d, x, xp);
                if (PUSH) {
                    const uint32_t j0 = 2u * p;
                    st_row<NT>(reinterpret_cast<gptr<dvec2>>(rt + j0), dvec2{t[0], t[1]});
                    st_row<NT>(reinterpret_cast<gptr<dvec2>>(rd + j0), dvec2{d[0], d[1]});
                    st_row<NT>(reinterpret_cast<gptr<dvec2>>(rx + j0), dvec2{x[0], x[1]});
                    st_row<NT>(reinterpret_cast<gptr<dvec2>>(rxp + j0), dvec2{xp[0], xp[1]});
                }
                cur = nxt;
                p += kPushThreads;
            }
        } else {
#pragma unroll 1
            for (int s = 0; s < ppt; ++s) {
                const uint32_t p = pair0 + (uint32_t)(s * kPushThreads + tid);
                const uint32_t j0 = 2u * p;
                if (j0 > n_last)
                    break;
                const bool two = j0 < n_last;
                double t[2], d[2], x[2], xp[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const uint32_t j = i == 0 || two ? j0 + i : j0;
                    t[i] = ld_row<NT>(rt + j);
                    d[i] = ld_row<NT>(rd + j);
                    x[i] = ld_row<NT>(rx + j);
                    xp[i] = ld_row<NT>(rxp + j);
                }
                pair(p, two, t, d, x, xp);
                if (PUSH) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        if (i == 1 && !two)
                            break;
                        st_row<NT>(rt + j0 + i, t[i]);
                        st_row<NT>(rd + j0 + i, d[i]);
                        st_row<NT>(rx + j0 + i, x[i]);
                        st_row<NT>(rxp + j0 + i, xp[i]);
                    }
                }
            }
        }

        // Fixed-order tile reduction, as in k_push; the transverse sums go to
        // the partial's transverse slots.
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const double v = wave_sum(acc[i]);
            if (lane == 0)
                red[wave * kPartStride + i] = v;
        }
        __syncthreads();
        if (tid < NA) {
            double sum = red[tid];
            for (int w = 1; w < kPushThreads / 64; ++w)
                sum += red[w * kPartStride + tid];
            const int slot = tid < NP ? tid : kPartTr + (tid - NP);
            J.partials[((size_t)b * J.ntiles + tile) * kPartStride + slot] = sum;
        }
        if (c.sr_on) {
            const size_t off = ((size_t)((clock + 1u) & 1u) * J.M + b) * nbx;
            uint32_t *out = J.counts + off;
            unsigned long long *xout = J.Xq + off;
            for (int k = tid; k < nb; k += kPushThreads) {
                uint32_t sum = 0;
                for (int q = 0; q < J.nsub; ++q)
                    sum += hist[q * nbh + k];
                if (sum) {
                    atomicAdd(&out[k], sum);
                    atomicAdd(&xout[k], xh[k]);
                }
            }
        }
        __syncthreads();
    }
}

size_t push_tr_lds_bytes(int nbins, int nsub)
{
    size_t v = (size_t)3 * (nbins + 1) * sizeof(double);  // V, U, dipole sums
    size_t h = (size_t)nsub * (size_t)(nbins + 1) * sizeof(uint32_t);
    h = (h + 7) & ~(size_t)7;
    return v + h + (size_t)(kPushThreads / 64) * kPartStride * sizeof(double);
}

// Transverse moments of bunch b (Sec. 2.4) into the ring, and its centroid
// into the wall's history, from the transverse slots of the tile partials;
// the same fixed order as finish_sums.
__device__ void finish_sums_tr(const JobDesc &J, int b, uint32_t clock)
{
    __shared__ double tred[kPrepThreads / 64][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = tid; t < J.ntiles; t += kPrepThreads) {
        const double *p = J.partials + ((size_t)b * J.ntiles + t) * kPartStride + kPartTr;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            s[i] += p[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double v = wave_sum(s[i]);
        if (lane == 0)
            tred[wave][i] = v;
    }
    __syncthreads();
    const int32_t rel = (int32_t)(clock - J.base);
    if (tid == 0) {
        double tot[4];
        for (int i = 0; i < 4; ++i) {
            tot[i] = tred[0][i];
            for (int w = 1; w < kPrepThreads / 64; ++w)
                tot[i] += tred[w][i];
        }
        const double invN = 1.0 / (double)J.N;
        const double mx = tot[0] * invN, mp = tot[2] * invN;
        const double vx = tot[1] * invN - mx * mx, vp = tot[3] * invN - mp * mp;
        if (rel >= 0) {
            double *m = J.tmom_ring + ((size_t)(rel & (J.mom_slots - 1)) * J.M + b) * 4;
            m[0] = mx;
            m[1] = mp;
            m[2] = sqrt(vx > 0.0 ? vx : 0.0);
            m[3] = sqrt(vp > 0.0 ? vp : 0.0);
            if (J.t.rw_turns > 0)
                J.H[(size_t)(clock % (uint32_t)J.t.rw_turns) * J.M + b] = mx;
        }
        if (!isfinite(mx) || !isfinite(mp) || !isfinite(vx) || !isfinite(vp))
            atomicOr(J.status, 1u);
    }
    __syncthreads();
}

// Bins [k0, k1) of bunch b's transverse kick (Sec. 2.3, Eq. 6 second line):
// U[k] = (qpp / E0) sum_{m<k} T[k-m] X[m], X from the exact dipole sums.  The
// same chunking and fixed-order combination as conv_chunk (T[0] = 0, so the
// sum may run to m = k); clears the dipole buffer the next push fills.
__device__ void conv_chunk_tr(const JobDesc &J, int b, int chunk, uint32_t clock, double *psm)
{
    __shared__ int t_lo;
    const int w = J.conv_out, K = kPrepThreads / w;
    const int tid = threadIdx.x;
    const int nb = J.c.nbins;
    const int k0 = chunk * w, k1 = min(k0 + w, nb);
    const unsigned long long *xin = J.Xq + ((size_t)((clock + 1u) & 1u) * J.M + b) * nb;
    unsigned long long *xclr = J.Xq + ((size_t)(clock & 1u) * J.M + b) * nb;
    double *sT = psm;
    double *sX = psm + nb;
    __syncthreads();  // the LDS may still be read by the longitudinal chunk
    if (tid == 0)
        t_lo = k1;
    __syncthreads();
    int lo = k1;
    for (int k = tid; k < k1; k += kPrepThreads) {
        const long long q = (long long)xin[k];
        sT[k] = J.Tt[k];
        sX[k] = (double)q * kDipoleUnit;
        if (q != 0 && k < lo)
            lo = k;
    }
    if (lo < k1)
        atomicMin(&t_lo, lo);
    __syncthreads();
    lo = t_lo;
    const int o = tid / K, q = tid % K;
    const int k = k0 + o;
    double acc0 = 0.0, acc1 = 0.0;
    if (k < k1) {
        int m = lo + q;
        for (; m + K <= k; m += 2 * K) {
            acc0 = fma(sT[k - m], sX[m], acc0);
            acc1 = fma(sT[k - m - K], sX[m + K], acc1);
        }
        if (m <= k)
            acc0 = fma(sT[k - m], sX[m], acc0);
    }
    double v = acc0 + acc1;
    for (int off = K >> 1; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    if (q == 0 && k < k1)
        J.U[(size_t)b * nb + k] = (J.qpp[b] * J.c.inv_E0) * v;
    for (int kk = k0 + tid; kk < k1; kk += kPrepThreads)
        xclr[kk] = 0ull;
}

// The between-turn work of a job with the transverse plane: the prep's
// longitudinal work, then its transverse counterpart.
template <int NLR>
__global__ __launch_bounds__(kPrepThreads) void k_prep_tr(const PrepLaunch L)
{
    extern __shared__ double psm[];
    const int bx = blockIdx.x;
    const Item item = L.inner > 0 ? Item{0, (uint16_t)(bx / L.inner), (uint32_t)(bx % L.inner)}
                                  : L.items[bx];
    const JobDesc &J = L.jobs[item.job];
    const uint32_t clock = L.clk ? L.clk[L.phase] : J.clock[L.phase];
    prep_body<NLR>(L, item, J, clock, psm);
    if (item.part == 0)
        finish_sums_tr(J, item.bunch, clock);
    if (J.c.sr_on)
        conv_chunk_tr(J, item.bunch, (int)item.part, clock, psm);
    if (item.bunch == 0 && item.part == 0 && threadIdx.x == 0)
        J.clock[L.phase ^ 1] = clock + 1u;
}

// The long-range resistive wall (Sec. 2.3, last paragraph), after the prep
// has recorded the centroids of turn n (the counter reads n): the kick that
// bunch b's particles get at the start of turn n + 1, from the passages of
// bunches b' < b in turn n and of every bunch in turns n - K + 1 .. n - 1,
// each source a rigid dipole of charge I_b' T0 at its centroid.  One
// workgroup per bunch; the K M terms are split over the threads and combined
// in a fixed order.
__global__ __launch_bounds__(256) void k_rw(const RwLaunch L)
{
    __shared__ double wred[4];
    const JobDesc &J = *L.job;
    const TransConst &tc = J.t;
    const int b = blockIdx.x, tid = threadIdx.x;
    const uint32_t clock = L.clk[L.phase];
    // the turn whose passages receive the kick (-1 before the first turn)
    const int64_t target = (int64_t)J.base + (int64_t)(int32_t)(clock - J.base);
    const int K = tc.rw_turns, M = J.M;
    const int64_t nterms = (int64_t)(K - 1) * M + b;
    double acc = 0.0;
    for (int64_t i = tid; i < nterms; i += 256) {
        const int age = K - 1 - (int)(i / M);
        const int bs = (int)(i % M);
        const int64_t m = target - age;
        if (m < 0)
            continue;
        const double dt = (double)age * tc.T0 + (double)(J.bucket[b] - J.bucket[bs]) * tc.T_rf;
        const double wt = tc.rw_amp * sqrt(tc.rw_arg / dt);
        acc += J.qb[bs] * J.H[(size_t)(m % K) * M + bs] * wt;
    }
    const double v = wave_sum(acc);
    if ((tid & 63) == 0)
        wred[tid >> 6] = v;
    __syncthreads();
    if (tid == 0)
        J.rwk[b] = (((wred[0] + wred[1]) + wred[2]) + wred[3]) * J.c.inv_E0;
}

// Matched Gaussian (x, x'): one Box-Muller pair of the INIT stream, tag 4,
// per particle.
__global__ __launch_bounds__(256) void k_init_tr(double *x, double *xp, int64_t ld, int64_t N,
                                                 const uint32_t *stream, double sx, double sxp,
                                                 double alpha, double offset, uint32_t k0,
                                                 uint32_t k1)
{
    const int b = blockIdx.y;
    const uint32_t sb = stream[b];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        double z0, z1;
        normal_pair((uint32_t)j, sb, 0u, 4u, k0, k1, z0, z1);
        x[(size_t)b * ld + j] = offset + sx * z0;
        xp[(size_t)b * ld + j] = sxp * (z1 - alpha * z0);
    }
}

// ---------------------------------------------------------------------------
// Initial distribution and raw Philox.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_gauss(double *tau, double *delta, int64_t ld,
                                                    int64_t N, const uint32_t *stream,
                                                    double sig_t, double sig_d, uint32_t k0,
                                                    uint32_t k1)
{
    const int b = blockIdx.y;
    const uint32_t sb = stream[b];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        double z0, z1;
        normal_pair((uint32_t)j, sb, 0u, 1u, k0, k1, z0, z1);
        tau[(size_t)b * ld + j] = sig_t * z0;
        delta[(size_t)b * ld + j] = sig_d * z1;
    }
}

__global__ __launch_bounds__(256) void k_philox(int64_t n, const uint32_t *ctr, uint32_t k0,
                                                uint32_t k1, uint32_t *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t x0 = ctr[4 * i], x1 = ctr[4 * i + 1], x2 = ctr[4 * i + 2], x3 = ctr[4 * i + 3];
        philox10(x0, x1, x2, x3, k0, k1);
        out[4 * i] = x0;
        out[4 * i + 1] = x1;
        out[4 * i + 2] = x2;
        out[4 * i + 3] = x3;
    }
}

// Device-to-device copy in 16-byte elements, one per thread, in workgroups
// of 256 (4 KiB each): of the shapes measured on the MI355X (grid-stride
// loops with 4 or 8 loads in flight per thread, non-temporal accesses,
// 4-16 KiB per workgroup) the many small workgroups reach the highest
// bandwidth, above the runtime's own device copy.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4 *__restrict__ src,
                                                     u32x4 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        ((gptr<u32x4>)dst)[i] = ((gptr<const u32x4>)src)[i];
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <int NLR, int MAP>
static void push_launch(const PushLaunch &l, bool push, size_t lds, hipStream_t s)
{
    constexpr int map = NLR == 1 ? MAP : kMapGeneric;
    uint32_t *ctr = l.grid < l.nitems ? l.ctr : nullptr;
    if (push && l.stream)
        hipLaunchKernelGGL((k_push<NLR, true, map, true>), dim3(l.grid), dim3(kPushThreads), lds, s,
                           l.jobs, l.items, l.nitems, l.grid, l.phase, ctr);
    else if (push)
        hipLaunchKernelGGL((k_push<NLR, true, map, false>), dim3(l.grid), dim3(kPushThreads), lds,
                           s, l.jobs, l.items, l.nitems, l.grid, l.phase, ctr);
    else
        hipLaunchKernelGGL((k_push<NLR, false, kMapGeneric, false>), dim3(l.grid),
                           dim3(kPushThreads), lds, s, l.jobs, l.items, l.nitems, l.grid, l.phase,
                           ctr);
}

template <int NLR>
static hipError_t push_n(const PushLaunch &l, bool push, hipStream_t s)
{
    const size_t lds = push_lds_bytes(l.nbins_max, l.nsub_max);
    // measured: without long-range resonators the specialisations spill at
    // four waves per SIMD and run slower than the generic kernel; with one
    // resonator they are faster; more resonators keep the generic kernel
    switch (push && NLR == 1 ? l.map : kMapGeneric) {
    case kMapWakeNoise: push_launch<NLR, kMapWakeNoise>(l, push, lds, s); break;
    case kMapWakeNoiseHC3: push_launch<NLR, kMapWakeNoiseHC3>(l, push, lds, s); break;
    default: push_launch<NLR, kMapGeneric>(l, push, lds, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_push(const PushLaunch &l, bool push, hipStream_t s)
{
    if (l.nitems < 1 || l.grid < 1 || (l.grid < l.nitems && !l.ctr))
        return hipErrorInvalidValue;
    switch (l.nlr) {
    case 0: return push_n<0>(l, push, s);
    case 1: return push_n<1>(l, push, s);
    case 2: return push_n<2>(l, push, s);
    case 3: return push_n<3>(l, push, s);
    case 4: return push_n<4>(l, push, s);
    default: return hipErrorInvalidValue;
    }
}

template <int NLR>
static hipError_t push_tr_n(const PushLaunch &l, bool push, hipStream_t s)
{
    const size_t lds = push_tr_lds_bytes(l.nbins_max, l.nsub_max);
    if (push && l.stream)
        hipLaunchKernelGGL((k_push_tr<NLR, true, true>), dim3(l.grid), dim3(kPushThreads), lds, s,
                           l.jobs, l.items, l.nitems, l.grid, l.phase);
    else if (push)
        hipLaunchKernelGGL((k_push_tr<NLR, true, false>), dim3(l.grid), dim3(kPushThreads), lds, s,
                           l.jobs, l.items, l.nitems, l.grid, l.phase);
    else
        hipLaunchKernelGGL((k_push_tr<NLR, false, false>), dim3(l.grid), dim3(kPushThreads), lds,
                           s, l.jobs, l.items, l.nitems, l.grid, l.phase);
    return hipGetLastError();
}

hipError_t launch_push_tr(const PushLaunch &l, bool push, hipStream_t s)
{
    if (l.nitems < 1 || l.grid < 1)
        return hipErrorInvalidValue;
    switch (l.nlr) {
    case 0: return push_tr_n<0>(l, push, s);
    case 1: return push_tr_n<1>(l, push, s);
    case 2: return push_tr_n<2>(l, push, s);
    case 3: return push_tr_n<3>(l, push, s);
    case 4: return push_tr_n<4>(l, push, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rw(const RwLaunch &l, hipStream_t s)
{
    if (l.M < 1 || !l.job || !l.clk)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rw, dim3(l.M), dim3(256), 0, s, l);
    return hipGetLastError();
}

hipError_t launch_init_transverse(double *x, double *xp, int64_t ld, int64_t N, int M,
                                  const uint32_t *stream, double sx, double sxp, double alpha,
                                  double offset, uint32_t key0, uint32_t key1, hipStream_t s)
{
    int64_t bx = (N + 255) / 256;
    if (bx > 4096)
        bx = 4096;
    hipLaunchKernelGGL(k_init_tr, dim3((unsigned)bx, M), dim3(256), 0, s, x, xp, ld, N, stream,
                       sx, sxp, alpha, offset, key0, key1);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepLaunch &l, hipStream_t s)
{
    if (l.nitems < 1)
        return hipErrorInvalidValue;
    size_t lds = (size_t)2 * l.nbins_max * sizeof(double);
    if (lds == 0)
        lds = 16;
    if (l.tr) {
        switch (l.nlr_max) {
        case 0: hipLaunchKernelGGL((k_prep_tr<0>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
        case 1: hipLaunchKernelGGL((k_prep_tr<1>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
        case 2: hipLaunchKernelGGL((k_prep_tr<2>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
        case 3: hipLaunchKernelGGL((k_prep_tr<3>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
        case 4: hipLaunchKernelGGL((k_prep_tr<4>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (l.nlr_max) {
    case 0: hipLaunchKernelGGL((k_prep<0>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
    case 1: hipLaunchKernelGGL((k_prep<1>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
    case 2: hipLaunchKernelGGL((k_prep<2>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
    case 3: hipLaunchKernelGGL((k_prep<3>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
    case 4: hipLaunchKernelGGL((k_prep<4>), dim3(l.nitems), dim3(kPrepThreads), lds, s, l); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scan(const ScanLaunch &l, hipStream_t s)
{
    if (l.njobs < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan, dim3(l.njobs), dim3(kPrepThreads), 0, s, l);
    return hipGetLastError();
}

hipError_t launch_wake(const WakeLaunch &l, hipStream_t s)
{
    if (l.nitems < 1 || l.nbins_max < 1)
        return hipErrorInvalidValue;
    const size_t lds = wake_lds_bytes(l.mode, l.nbins_max);
    switch (l.mode) {
    case kWakeFP32:
        hipLaunchKernelGGL((k_wake<kWakeFP32>), dim3(l.nitems), dim3(256), lds, s, l);
        break;
    case kWakeBF16x2:
        hipLaunchKernelGGL((k_wake<kWakeBF16x2>), dim3(l.nitems), dim3(256), lds, s, l);
        break;
    case kWakeBF16x3:
        hipLaunchKernelGGL((k_wake<kWakeBF16x3>), dim3(l.nitems), dim3(256), lds, s, l);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init_gauss(double *tau, double *delta, int64_t ld, int64_t N, int M,
                             const uint32_t *stream, double sig_tau, double sig_delta,
                             uint32_t key0, uint32_t key1, hipStream_t s)
{
    int64_t bx = (N + 255) / 256;
    if (bx > 4096)
        bx = 4096;
    hipLaunchKernelGGL(k_init_gauss, dim3((unsigned)bx, M), dim3(256), 0, s, tau, delta, ld, N,
                       stream, sig_tau, sig_delta, key0, key1);
    return hipGetLastError();
}

hipError_t launch_philox(int64_t n, const uint32_t *ctr, uint32_t key0, uint32_t key1,
                         uint32_t *out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t bx = (n + 255) / 256;
    if (bx > 8192)
        bx = 8192;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)bx), dim3(256), 0, s, n, ctr, key0, key1, out);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s)
{
    const int64_t n = bytes / 16;
    if (n <= 0)
        return hipSuccess;
    const int64_t bx = (n + 255) / 256;
    if (bx > (int64_t)UINT32_MAX)
        return hipErrorInvalidValue;  // beyond 2^44 bytes
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)bx), dim3(256), 0, s,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n);
    return hipGetLastError();
}

}  // namespace mbt
