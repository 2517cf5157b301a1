// mbt_host.cpp -- host runtime behind the C ABI in include/mbt.h.
//
// Validates parameters, derives the turn-map constants, lays out the caller's
// workspace, and drives the per-turn launches on the caller's stream.  The
// turn loop never synchronises with the host: moments and profiles go to
// device rings that are copied to pinned host memory chunk by chunk.
#include "mbt.h"
#include "mbt_internal.h"
#include "mbt_rw.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <vector>

using namespace mbt;

// ---- Static workspace of mbt_bind_static -----------------------------------
// For callers that cannot allocate device memory: one array per device,
// resident until the process ends.  Host code never takes its name as an
// address (in host code it is only a stand-in for the device symbol): the
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and is kept in StaticWorkspace::ptr.
static __device__ __align__(256) unsigned char scratch[MBT_STATIC_WORK_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct StaticWorkspace {
    std::mutex mu;
    void *ptr[kMaxDevices] = {};           // device address of scratch, per device
    const mbt_ctx *owner[kMaxDevices] = {};  // context bound to it last
};

StaticWorkspace &static_ws()
{
    static StaticWorkspace w;
    return w;
}

}  // namespace

namespace {

constexpr double kTwoPi = 6.283185307179586;
constexpr double kPi = 3.141592653589793;

struct Resonator {
    double rs, q, fr;
    double alpha() const { return kTwoPi * fr / (2.0 * q); }
    double wbar() const
    {
        const double wr = kTwoPi * fr, a = alpha();
        return std::sqrt(wr * wr - a * a);
    }
    // Resonator wake for t >= 0 (W(0+) at t = 0), in V/C.
    double wake(double t) const
    {
        const double a = alpha(), wb = wbar();
        return 2.0 * a * rs * std::exp(-a * t) * (std::cos(wb * t) - (a / wb) * std::sin(wb * t));
    }
};

bool res_valid(const mbt_resonator &r)
{
    return std::isfinite(r.rs_ohm) && r.rs_ohm >= 0.0 && std::isfinite(r.q) && r.q > 0.5 &&
           std::isfinite(r.fr_Hz) && r.fr_Hz > 0.0;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// BF16 (the upper 16 bits of an IEEE single) nearest to x, ties to even,
// through the FP32 rounding of x; and its value.
uint16_t bf16_nearest(double x)
{
    const float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

int floor_pow2(size_t x)
{
    int p = 1;
    while ((size_t)p * 2 <= x && p < (1 << 30))
        p *= 2;
    return p;
}

constexpr size_t kLdsLimit = 64 * 1024;  // dynamic LDS of one push workgroup

// Offsets of every workspace region for a given job shape.
struct Layout {
    size_t desc, items_push, items_prep, items_wake, clock, status, pctr, Wbf, Wf32;
    size_t W, V, counts, partials, S, seen, gap, qc, phasor, qpp, stream, mom, prof;
    // transverse plane (empty regions without it)
    size_t Tt, U, Xq, tmom, H, rwk, bucket, qb;
    size_t total;
    int mom_slots, prof_slots, ntiles, ppt, nchunks, nwake, conv_out;
    int64_t ld;
    size_t state_bytes;
};

// tr: the job tracks a transverse plane; rw_turns: K of its wall (0: none).
Layout make_layout(int M, int64_t N, int nb, int nlr, bool tr = false, int rw_turns = 0)
{
    Layout L{};
    const int nbx = std::max(nb, 1);
    L.ld = (N + kRowAlign - 1) / kRowAlign * kRowAlign;
    L.ppt = pairs_per_thread(M, N);
    const int64_t tile = 2LL * kPushThreads * L.ppt;
    L.ntiles = (int)((N + tile - 1) / tile);
    L.conv_out = conv_width(M, nb);
    L.nchunks = conv_chunks(nb, L.conv_out);
    L.nwake = nb > 0 ? ((M + kWakeBunches - 1) / kWakeBunches) * ((nb + kWakeBins - 1) / kWakeBins) : 0;
    // output rings: powers of two, about 16 MB each at most
    const size_t moment_row = (size_t)M * 4 * sizeof(double);
    L.mom_slots = floor_pow2(std::max<size_t>(16, std::min<size_t>(1024, (16u << 20) / moment_row)));
    const size_t prof_row = (size_t)M * nbx * sizeof(uint32_t);
    L.prof_slots = floor_pow2(std::max<size_t>(1, std::min<size_t>(64, (16u << 20) / prof_row)));
    const int nl = std::max(nlr, 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.desc = take(sizeof(JobDesc));
    L.items_push = take((size_t)M * L.ntiles * sizeof(Item));
    L.items_prep = take((size_t)M * L.nchunks * sizeof(Item));
    L.items_wake = take((size_t)std::max(L.nwake, 1) * sizeof(Item));
    L.clock = take(2 * sizeof(uint32_t));
    L.status = take(sizeof(uint32_t));
    L.pctr = take(4 * sizeof(uint32_t));  // the persistent push's item counters
    L.W = take((size_t)nbx * sizeof(double));
    L.Wbf = take((size_t)3 * nbx * sizeof(uint16_t));
    L.Wf32 = take((size_t)nbx * sizeof(float));
    L.V = take((size_t)M * nbx * sizeof(double));
    L.counts = take((size_t)2 * M * nbx * sizeof(uint32_t));
    L.partials = take((size_t)M * L.ntiles * kPartStride * sizeof(double));
    L.S = take((size_t)nl * M * 2 * sizeof(double));
    L.seen = take((size_t)nl * M * 2 * sizeof(double));
    L.gap = take((size_t)nl * M * 2 * sizeof(double));
    L.qc = take((size_t)nl * M * 2 * sizeof(double));
    L.phasor = take((size_t)nl * 2 * sizeof(double));
    L.qpp = take((size_t)M * sizeof(double));
    L.stream = take((size_t)M * sizeof(uint32_t));
    L.mom = take((size_t)L.mom_slots * moment_row);
    L.prof = take((size_t)L.prof_slots * prof_row);
    const size_t ntr = tr ? 1 : 0;
    L.Tt = take(ntr * nbx * sizeof(double));
    L.U = take(ntr * M * nbx * sizeof(double));
    L.Xq = take(ntr * 2 * M * nbx * sizeof(unsigned long long));
    L.tmom = take(ntr * L.mom_slots * moment_row);
    L.H = take(ntr * (size_t)rw_turns * M * sizeof(double));
    L.rwk = take(ntr * M * sizeof(double));
    L.bucket = take(ntr * M * sizeof(int32_t));
    L.qb = take(ntr * M * sizeof(double));
    L.total = o;
    L.state_bytes = (size_t)(tr ? 4 : 2) * M * (size_t)L.ld * sizeof(double);
    return L;
}

// Default sub-histograms per push workgroup: several copies spread the LDS
// atomics of a wavefront over more banks when they fit.
int default_nsub(int nbins)
{
    if (nbins <= 0)
        return 0;
    int n = nbins <= 1024 ? 4 : (nbins <= 2048 ? 2 : 1);
    while (n > 1 && push_lds_bytes(nbins, n) > kLdsLimit)
        n /= 2;
    return n;
}

// A device ring of `slots` rows (power of two) that a kernel fills row by
// row, copied out to a host array through a pinned buffer of the ring's size.
// Rows are numbered from the start of the call; row r sits in slot
// r & (slots - 1).  Before work that writes rows [written, written + n) is
// enqueued, rows that would be overwritten are copied out first.
struct RingOut {
    const unsigned char *dev = nullptr;
    size_t row_bytes = 0;
    int slots = 0;
    unsigned char *dst = nullptr;  // host row 0 of this call (NULL: not wanted)
    int64_t flushed = 0, written = 0;
    // staging: the pinned copy of the ring and the event its last copy recorded
    unsigned char *pin = nullptr;
    hipEvent_t ev = nullptr;
    struct Piece { size_t pin_off; int64_t row; int64_t rows; };
    std::vector<Piece> pending;
};

}  // namespace

// Event pairs around launches, for measurement only.
struct Timer {
    static constexpr int kMax = 4096;
    int every = 0;
    std::vector<hipEvent_t> ev[2];  // [0]: push, [1]: between-turn (scan + prep)
    int n[2] = {0, 0};              // pairs recorded since the last collect
    double ms[2] = {0.0, 0.0};
    int64_t launches[2] = {0, 0};
};

// Pinned host image of what the host writes into a job's workspace.
struct Mirror {
    JobDesc desc;
    uint32_t clock[2];
};

struct mbt_ctx {
    // parameters
    mbt_ring ring{};
    double T0 = 0, T_rf = 0, w_rf = 0, phi_s = 0, D = 0, noise = 0, drift = 0;
    bool hc_on = false;
    mbt_hc hc{};
    int M = 0;
    std::vector<int32_t> bucket, stream;
    std::vector<double> current;
    bool sr_on = false;
    mbt_grid grid{};
    std::vector<Resonator> sr, lr;
    bool rw_on = false;
    ResistiveWall rw{};
    // transverse plane, its short-range resonators (R_s in Ohm/m) and wall
    bool tr_on = false;
    mbt_transverse tr{};
    std::vector<Resonator> tw;
    bool trw_on = false;
    mbt_transverse_rw trw{};
    // binding
    bool bound = false;
    int64_t N = 0;
    Layout L{};
    double *tau = nullptr, *delta = nullptr, *x = nullptr, *xp = nullptr;
    unsigned char *work = nullptr;
    hipStream_t stream_h = nullptr;
    int device = 0;
    Mirror *mirror = nullptr;  // pinned (or plain_mirror for a static binding)
    RingOut mom, prof, tmom;   // pinned staging of the output rings
    // mbt_bind_static: the workspace is the library's static array on `device`,
    // the mirror is plain host memory and the rings copy straight out
    bool static_ws = false;
    Mirror plain_mirror{};
    // launch shape (neither changes a result bit)
    int nsub = 0, push_grid = 0;
    // arithmetic of the wake potential (WakeMode) and its tables
    int wake_mode = kWakeFP64;
    int count_parts = 1;
    double wake_scale = 1.0;
    Timer timer;
    // run state
    bool have_particles = false;
    bool dirty = true;  // tile sums, histogram and wake potential do not describe the present state
    int64_t turn = 0;   // turns completed
    uint64_t seed = 0;
    char err[512] = "";

    template <class T> T *w(size_t off) const { return reinterpret_cast<T *>(work + off); }
    int nbins() const { return sr_on ? grid.nbins : 0; }
    int nlr() const { return (int)lr.size(); }
    int rw_turns() const { return tr_on && trw_on ? trw.turns : 0; }
    Layout layout(int64_t n) const
    {
        return make_layout(M, n, nbins(), nlr(), tr_on, rw_turns());
    }
};

struct mbt_batch;

namespace {

// Record a message on a context or batch (anything with an `err` buffer).
template <class C>
int fail(C *c, int code, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

// Body of an entry point: no C++ exception crosses the C ABI.  A failed host
// allocation (std::bad_alloc from a container) becomes MBT_ENOMEM, anything
// else MBT_EDEVICE, with the message kept on the context or batch.
template <class C, class F>
int guarded(C *c, F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(c, MBT_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(c, MBT_EDEVICE, "internal error: %s", e.what());
    } catch (...) {
        return fail(c, MBT_EDEVICE, "internal error");
    }
}

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), MBT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int solve_phi_s(mbt_ctx *c, bool hc_on, const mbt_hc &hc, double *phi)
{
    double s = c->ring.u0_eV / c->ring.v_rf_V;
    if (hc_on)
        s -= hc.v_ratio * std::sin(hc.phase_n_rad);
    if (!(std::fabs(s) <= 1.0))
        return fail(c, MBT_EINVAL, "no synchronous phase: |sin phi_s| = %g > 1", std::fabs(s));
    const double a = std::asin(s);
    // stable branch: alpha_c * cos(phi_s) > 0
    *phi = (c->ring.alpha_c > 0.0) ? a : (kPi - a);
    return MBT_OK;
}

MapConst map_const(const mbt_ctx *c)
{
    MapConst m{};
    const double E0 = c->ring.energy_eV;
    m.inv_E0 = 1.0 / E0;
    m.w_rf = c->w_rf;
    m.rf_a = c->ring.v_rf_V * std::sin(c->phi_s) / E0;
    m.rf_b = c->ring.v_rf_V * std::cos(c->phi_s) / E0;
    m.u0_e = c->ring.u0_eV / E0;
    m.one_minus_D = 1.0 - c->D;
    m.noise = c->noise;
    m.drift = c->drift;
    m.hc_on = c->hc_on ? 1 : 0;
    if (c->hc_on) {
        const double kv = c->hc.v_ratio * c->ring.v_rf_V;
        m.hc_a = kv * std::sin(c->hc.phase_n_rad) / E0;
        m.hc_b = kv * std::cos(c->hc.phase_n_rad) / E0;
        m.hc_n = c->hc.n;
    }
    m.sr_on = c->sr_on ? 1 : 0;
    m.noise_on = c->noise > 0.0 ? 1 : 0;
    m.nbins = c->nbins();
    m.nbins_d = (double)c->nbins();
    if (c->sr_on) {
        m.tau_min = c->grid.tau_min_s;
        m.inv_delta = (double)c->grid.nbins / (c->grid.tau_max_s - c->grid.tau_min_s);
    }
    for (size_t r = 0; r < c->lr.size(); ++r) {
        m.lr_alpha[r] = c->lr[r].alpha();
        m.lr_wbar[r] = c->lr[r].wbar();
    }
    return m;
}

// Descriptor of a bound job for a call that starts at turn `base` and records
// a profile every `prof_stride`-th turn (0: none).
JobDesc job_desc(const mbt_ctx *c, uint32_t base, int prof_stride)
{
    JobDesc d{};
    d.c = map_const(c);
    d.tau = c->tau;
    d.delta = c->delta;
    d.ld = c->L.ld;
    d.N = c->N;
    d.M = c->M;
    d.ntiles = c->L.ntiles;
    d.ppt = c->L.ppt;
    d.nsub = c->nsub;
    d.nlr = c->nlr();
    d.mom_slots = c->L.mom_slots;
    d.prof_stride = prof_stride;
    d.prof_slots = c->L.prof_slots;
    d.base = base;
    d.key0 = (uint32_t)c->seed;
    d.key1 = (uint32_t)(c->seed >> 32);
    d.wake_mode = c->sr_on ? c->wake_mode : kWakeFP64;
    d.count_parts = c->count_parts;
    d.wake_scale = c->wake_scale;
    d.Wbf = c->w<uint16_t>(c->L.Wbf);
    d.Wf32 = c->w<float>(c->L.Wf32);
    d.W = c->w<double>(c->L.W);
    d.qpp = c->w<double>(c->L.qpp);
    d.gap = c->w<double>(c->L.gap);
    d.qc = c->w<double>(c->L.qc);
    d.stream = c->w<uint32_t>(c->L.stream);
    d.V = c->w<double>(c->L.V);
    d.partials = c->w<double>(c->L.partials);
    d.S = c->w<double>(c->L.S);
    d.seen = c->w<double>(c->L.seen);
    d.phasor = c->w<double>(c->L.phasor);
    d.mom_ring = c->w<double>(c->L.mom);
    d.counts = c->w<uint32_t>(c->L.counts);
    d.prof_ring = c->w<uint32_t>(c->L.prof);
    d.status = c->w<uint32_t>(c->L.status);
    d.clock = c->w<uint32_t>(c->L.clock);
    d.conv_out = c->L.conv_out;
    d.tr_on = c->tr_on ? 1 : 0;
    if (c->tr_on) {
        const mbt_transverse &t = c->tr;
        TransConst &tc = d.t;
        tc.qfrac = t.tune - std::floor(t.tune);  // exact
        tc.chrom = t.chromaticity;
        tc.alpha = t.alpha;
        tc.beta = t.beta_m;
        tc.gamma = (1.0 + t.alpha * t.alpha) / t.beta_m;
        tc.disp = t.disp_m;
        tc.disp_p = t.disp_prime;
        // Eq. 5: noise sigma sqrt(D_x) with D_x = 2 T0 / tau_damp
        const double dx = 2.0 * c->T0 / t.tau_damp_s;
        tc.noise_x = std::sqrt(t.emittance_m * t.beta_m) * std::sqrt(dx);
        tc.noise_xp = std::sqrt(t.emittance_m * tc.gamma) * std::sqrt(dx);
        tc.noise_on = (tc.noise_x > 0.0 || tc.noise_xp > 0.0) ? 1 : 0;
        tc.rw_turns = c->rw_turns();
        if (tc.rw_turns > 0) {
            const double z0 = 376.730313668, cl = 299792458.0, rb = c->trw.radius_m;
            tc.rw_amp = c->trw.length_m / (kPi * rb * rb * rb);
            tc.rw_arg = z0 * cl / (kPi * c->trw.conductivity_S_m);
        }
        tc.T0 = c->T0;
        tc.T_rf = c->T_rf;
        d.x = c->x;
        d.xp = c->xp;
        d.Tt = c->w<double>(c->L.Tt);
        d.U = c->w<double>(c->L.U);
        d.Xq = c->w<unsigned long long>(c->L.Xq);
        d.tmom_ring = c->w<double>(c->L.tmom);
        d.H = c->w<double>(c->L.H);
        d.rwk = c->w<double>(c->L.rwk);
        d.bucket = c->w<int32_t>(c->L.bucket);
        d.qb = c->w<double>(c->L.qb);
    }
    return d;
}

// Which specialised push kernel fits the job (MapKind).
int map_kind(const mbt_ctx *c)
{
    if (!c->sr_on || !(c->noise > 0.0))
        return kMapGeneric;
    if (!c->hc_on)
        return kMapWakeNoise;
    return c->hc.n == 3 ? kMapWakeNoiseHC3 : kMapGeneric;
}

// Push items of a job: (job, bunch, tile), tile-major, so that the short
// last tile of every bunch is dispatched at the end of the launch (measured:
// 1.4% shorter push at the full fill than bunch-major).  The order of the
// items changes no result: each tile has its own partial-sum slot.
void push_items(const mbt_ctx *c, int job, std::vector<Item> &out)
{
    for (int t = 0; t < c->L.ntiles; ++t)
        for (int b = 0; b < c->M; ++b)
            out.push_back(Item{(uint16_t)job, (uint16_t)b, (uint32_t)t});
}

// Prep items of a job: (job, bunch, chunk of conv_out bins).
void prep_items(const mbt_ctx *c, int job, std::vector<Item> &out)
{
    for (int b = 0; b < c->M; ++b)
        for (int k = 0; k < c->L.nchunks; ++k)
            out.push_back(Item{(uint16_t)job, (uint16_t)b, (uint32_t)k});
}

// Wake items of a job: (job, 16-bunch tile, 16-bin output tile).
void wake_items(const mbt_ctx *c, int job, std::vector<Item> &out)
{
    const int nb = c->nbins();
    if (nb == 0)
        return;
    for (int bt = 0; bt < (c->M + kWakeBunches - 1) / kWakeBunches; ++bt)
        for (int kt = 0; kt < (nb + kWakeBins - 1) / kWakeBins; ++kt)
            out.push_back(Item{(uint16_t)job, (uint16_t)bt, (uint32_t)kt});
}

// A job whose wake potential k_wake computes on the matrix cores.
bool mfma_wake(const mbt_ctx *c) { return c->sr_on && c->wake_mode != kWakeFP64; }

// Launch tables of a set of jobs whose descriptors and item lists are in
// device memory.  Push items are grouped by the number of long-range
// resonators (a template parameter of the push).
struct Group {
    int item0 = 0, nitems = 0, nlr = 0, nbins_max = 0, nsub_max = 0, grid = 0;
    uint32_t *ctr = nullptr;  // item counters of a persistent launch (4 words)
    int map = kMapGeneric;  // compile-time map terms every job of the group shares
    bool stream = false;    // non-temporal particle-row accesses (see stream_rows)
};

// Particle state above which the push streams its rows with the
// non-temporal hint: the 256 MB Infinity Cache of the MI355X, which holds a
// smaller state from one turn to the next.
constexpr size_t kStreamBytes = (size_t)256 << 20;
bool stream_rows(size_t state_bytes) { return state_bytes > kStreamBytes; }
struct WakeGroup {
    int item0 = 0, nitems = 0, mode = 0, nbins_max = 0;
};
struct Engine {
    const JobDesc *jobs = nullptr;
    const Item *push_items = nullptr;
    const Item *prep_items = nullptr;
    const Item *wake_items = nullptr;
    int njobs = 0, nprep = 0, nlr_max = 0, nbins_max = 0;
    // a single job: prep chunks per bunch and wake tiles per 16-bunch tile,
    // and its turn counter, so that the between-turn kernels derive their
    // items and read the counter without the tables (the push keeps the
    // tables: two more arguments cost its one-resonator form registers)
    int one_chunks = 0, one_wparts = 0;
    const uint32_t *one_clock = nullptr;
    std::vector<Group> groups;
    std::vector<WakeGroup> wakes;  // jobs whose wake potential comes from k_wake
    // a single job with the transverse plane (batches hold none): its M and
    // whether its long-range wall needs the kick kernel after the prep
    bool tr = false, rw = false;
    int tr_M = 0;
};

PushLaunch push_launch(const Engine &e, const Group &g, int phase)
{
    PushLaunch l{};
    l.phase = phase;
    l.jobs = e.jobs;
    l.items = e.push_items + g.item0;
    l.nitems = g.nitems;
    l.nlr = g.nlr;
    l.nbins_max = g.nbins_max;
    l.nsub_max = g.nsub_max;
    l.grid = g.grid > 0 ? std::min(g.grid, g.nitems) : g.nitems;
    l.map = g.map;
    l.ctr = g.ctr;
    l.stream = g.stream ? 1 : 0;
    return l;
}

// Fill the single-job fields of an engine over job c (its items are the
// bunch-major tables prep_items / wake_items build).
void set_one_job(Engine &e, const mbt_ctx *c)
{
    e.one_chunks = c->L.nchunks;
    e.one_wparts = c->nbins() > 0 ? (c->nbins() + kWakeBins - 1) / kWakeBins : 0;
    e.one_clock = c->w<uint32_t>(c->L.clock);
}

hipError_t enqueue_push(const Engine &e, bool push, int phase, hipStream_t s)
{
    for (const Group &g : e.groups) {
        const PushLaunch l = push_launch(e, g, phase);
        hipError_t r = e.tr ? launch_push_tr(l, push, s) : launch_push(l, push, s);
        if (r != hipSuccess)
            return r;
    }
    return hipSuccess;
}

// The between-turn work after a push: sums, histograms, wake potential.
hipError_t enqueue_prep(const Engine &e, int phase, hipStream_t s)
{
    PrepLaunch l{};
    l.phase = phase;
    l.jobs = e.jobs;
    l.items = e.prep_items;
    l.nitems = e.nprep;
    l.nlr_max = e.nlr_max;
    l.nbins_max = e.nbins_max;
    l.inner = e.one_chunks;
    l.clk = e.one_clock;
    l.tr = e.tr ? 1 : 0;
    hipError_t r = e.nprep > 0 ? launch_prep(l, s) : hipSuccess;
    if (r == hipSuccess && e.rw) {
        RwLaunch w{};
        w.phase = phase;
        w.job = e.jobs;
        w.M = e.tr_M;
        w.clk = e.one_clock;
        r = launch_rw(w, s);
    }
    for (const WakeGroup &g : e.wakes) {
        if (r != hipSuccess)
            break;
        WakeLaunch w{};
        w.phase = phase;
        w.jobs = e.jobs;
        w.items = e.wake_items + g.item0;
        w.nitems = g.nitems;
        w.mode = g.mode;
        w.nbins_max = g.nbins_max;
        w.inner = e.one_wparts;
        w.clk = e.one_clock;
        r = launch_wake(w, s);
    }
    return r;
}

hipError_t enqueue_scan(const Engine &e, hipStream_t s)
{
    if (e.nlr_max == 0)
        return hipSuccess;  // nothing to scan; the prep advances the counters
    ScanLaunch l{};
    l.jobs = e.jobs;
    l.njobs = e.njobs;
    l.nlr_max = e.nlr_max;
    return launch_scan(l, s);
}

// One turn of every job in launch phase `phase`: phasor scan (with long-range
// resonators), push, prep (+ wake).  With a timer, four events bracket the
// three parts.
hipError_t enqueue_turn(const Engine &e, int phase, hipStream_t s, Timer *tm)
{
    hipEvent_t *ev = nullptr;
    if (tm && tm->n[0] < Timer::kMax)
        ev = &tm->ev[0][4 * tm->n[0]++];
    hipError_t r;
    if (ev && (r = hipEventRecord(ev[0], s)) != hipSuccess)
        return r;
    if ((r = enqueue_scan(e, s)) != hipSuccess)
        return r;
    if (ev && (r = hipEventRecord(ev[1], s)) != hipSuccess)
        return r;
    if ((r = enqueue_push(e, true, phase, s)) != hipSuccess)
        return r;
    if (ev && (r = hipEventRecord(ev[2], s)) != hipSuccess)
        return r;
    if ((r = enqueue_prep(e, phase, s)) != hipSuccess)
        return r;
    if (ev && (r = hipEventRecord(ev[3], s)) != hipSuccess)
        return r;
    return hipSuccess;
}

// Engine of one job, from the tables in its own workspace.
Engine single_engine(const mbt_ctx *c)
{
    Engine e;
    e.jobs = c->w<JobDesc>(c->L.desc);
    e.push_items = c->w<Item>(c->L.items_push);
    e.prep_items = c->w<Item>(c->L.items_prep);
    e.njobs = 1;
    e.nprep = mfma_wake(c) ? 0 : c->M * c->L.nchunks;  // k_wake does a matrix-core job's prep
    e.nlr_max = c->nlr();
    e.nbins_max = c->nbins();
    Group g;
    g.nitems = c->M * c->L.ntiles;
    g.nlr = c->nlr();
    g.nbins_max = c->nbins();
    g.nsub_max = c->nsub;
    g.grid = c->push_grid;
    g.map = map_kind(c);
    g.ctr = c->w<uint32_t>(c->L.pctr);
    g.stream = stream_rows(c->L.state_bytes);
    e.groups.push_back(g);
    e.wake_items = c->w<Item>(c->L.items_wake);
    if (c->sr_on && c->wake_mode != kWakeFP64) {
        WakeGroup w;
        w.nitems = c->L.nwake;
        w.mode = c->wake_mode;
        w.nbins_max = c->nbins();
        e.wakes.push_back(w);
    }
    set_one_job(e, c);
    e.tr = c->tr_on;
    e.rw = c->rw_turns() > 0;
    e.tr_M = c->M;
    return e;
}

// Start of a call on job c, enqueued on stream s: upload its descriptor
// (rings count from the present turn) and put the present turn into counter
// slot 0, where the call's first turn (phase 0) reads it.  If the tile sums,
// histogram and wake potential are stale, they are rebuilt first by a
// bin-only pass and a prep in phase 1 with the counter at turn - 1; that
// prep writes the turn into slot 0 itself.
int begin_call(mbt_ctx *c, int prof_stride, hipStream_t s)
{
    c->mirror->desc = job_desc(c, (uint32_t)c->turn, prof_stride);
    HIPCHK(c, hipMemcpyAsync(c->w<JobDesc>(c->L.desc), &c->mirror->desc, sizeof(JobDesc),
                             hipMemcpyHostToDevice, s));
    uint32_t *clock = c->w<uint32_t>(c->L.clock);
    if (!c->dirty) {
        c->mirror->clock[0] = (uint32_t)c->turn;
        HIPCHK(c, hipMemcpyAsync(clock, &c->mirror->clock[0], sizeof(uint32_t),
                                 hipMemcpyHostToDevice, s));
        return MBT_OK;
    }
    c->mirror->clock[1] = (uint32_t)(c->turn - 1);
    HIPCHK(c, hipMemcpyAsync(clock + 1, &c->mirror->clock[1], sizeof(uint32_t),
                             hipMemcpyHostToDevice, s));
    const int nbx = std::max(c->nbins(), 1);
    uint32_t *cnt = c->w<uint32_t>(c->L.counts) + (size_t)(c->turn & 1) * c->M * nbx;
    HIPCHK(c, hipMemsetAsync(cnt, 0, (size_t)c->M * nbx * sizeof(uint32_t), s));
    if (c->tr_on)
        HIPCHK(c, hipMemsetAsync(c->w<unsigned long long>(c->L.Xq) + (size_t)(c->turn & 1) * c->M * nbx,
                                 0, (size_t)c->M * nbx * sizeof(unsigned long long), s));
    const Engine e = single_engine(c);
    HIPCHK(c, enqueue_push(e, false, 1, s));
    HIPCHK(c, enqueue_prep(e, 1, s));
    c->dirty = false;
    return MBT_OK;
}

// --- output rings --------------------------------------------------------

int ring_alloc(mbt_ctx *c, RingOut &r, const void *dev, size_t row_bytes, int slots, bool pinned)
{
    r.dev = reinterpret_cast<const unsigned char *>(dev);
    r.row_bytes = row_bytes;
    r.slots = slots;
    if (!pinned)
        return MBT_OK;  // no staging: rows go straight into the caller's array
    HIPCHK(c, hipHostMalloc((void **)&r.pin, (size_t)slots * row_bytes, hipHostMallocDefault));
    HIPCHK(c, hipEventCreateWithFlags(&r.ev, hipEventDisableTiming));
    // a flush adds at most two pieces after landing the previous ones, so
    // the turn loop never allocates here
    r.pending.reserve(2);
    return MBT_OK;
}

void ring_free(RingOut &r)
{
    if (r.pin)
        (void)hipHostFree(r.pin);
    if (r.ev)
        (void)hipEventDestroy(r.ev);
    r = RingOut{};
}

void ring_start(RingOut &r, void *dst)
{
    r.dst = reinterpret_cast<unsigned char *>(dst);
    r.flushed = r.written = 0;
    r.pending.clear();
}

// Wait for the last copy out of the ring and move it to the host array.
hipError_t ring_land(RingOut &r)
{
    if (r.pending.empty())
        return hipSuccess;
    hipError_t e = hipEventSynchronize(r.ev);
    if (e != hipSuccess)
        return e;
    for (const RingOut::Piece &p : r.pending)
        std::memcpy(r.dst + (size_t)p.row * r.row_bytes, r.pin + p.pin_off,
                    (size_t)p.rows * r.row_bytes);
    r.pending.clear();
    return hipSuccess;
}

// Enqueue the copy of rows [flushed, written) (at most two contiguous runs
// of slots) into the pinned buffer.
hipError_t ring_flush(RingOut &r, hipStream_t s)
{
    if (!r.dst || r.written == r.flushed)
        return hipSuccess;
    if (!r.pin) {
        // no staging (static binding): copy the rows into the caller's host
        // array directly, in stream order
        for (int64_t row = r.flushed; row < r.written;) {
            const int64_t slot = row & (r.slots - 1);
            const int64_t n = std::min<int64_t>(r.written - row, r.slots - slot);
            hipError_t e = hipMemcpyAsync(r.dst + (size_t)row * r.row_bytes,
                                          r.dev + (size_t)slot * r.row_bytes,
                                          (size_t)n * r.row_bytes, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess)
                return e;
            row += n;
        }
        r.flushed = r.written;
        return hipSuccess;
    }
    hipError_t e = ring_land(r);
    if (e != hipSuccess)
        return e;
    int64_t row = r.flushed;
    while (row < r.written) {
        const int64_t slot = row & (r.slots - 1);
        const int64_t n = std::min<int64_t>(r.written - row, r.slots - slot);
        const size_t off = (size_t)slot * r.row_bytes;
        e = hipMemcpyAsync(r.pin + off, r.dev + off, (size_t)n * r.row_bytes,
                           hipMemcpyDeviceToHost, s);
        if (e != hipSuccess)
            return e;
        r.pending.push_back({off, row, n});
        row += n;
    }
    r.flushed = r.written;
    return hipEventRecord(r.ev, s);
}

// Make room for n more rows (n <= slots), then count them as written.
hipError_t ring_advance(RingOut &r, int64_t n, hipStream_t s)
{
    if (!r.dst || n == 0)
        return hipSuccess;
    if (r.written + n - r.flushed > r.slots) {
        hipError_t e = ring_flush(r, s);
        if (e != hipSuccess)
            return e;
    }
    r.written += n;
    return hipSuccess;
}

// Profile rows among the turns [t0, t0 + n) of a call with this stride.
int64_t profile_rows(int64_t t0, int64_t n, int stride)
{
    if (stride < 1)
        return 0;
    auto ceil_div = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
    return ceil_div(t0 + n, stride) - ceil_div(t0, stride);
}

// --- timing --------------------------------------------------------------

void timer_free(Timer &t)
{
    for (hipEvent_t e : t.ev[0])
        (void)hipEventDestroy(e);
    t.ev[0].clear();
}

hipError_t timer_set(Timer &t, int every)
{
    t.every = every;
    t.ms[0] = t.ms[1] = 0.0;
    t.launches[0] = t.launches[1] = 0;
    t.n[0] = 0;
    if (every > 0 && t.ev[0].empty()) {
        t.ev[0].resize(4 * Timer::kMax);
        for (hipEvent_t &e : t.ev[0]) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess)
                return r;
        }
    }
    return hipSuccess;
}

// After the stream has drained: add the recorded turns to the totals.
hipError_t timer_collect(Timer &t)
{
    for (int i = 0; i < t.n[0]; ++i) {
        const hipEvent_t *ev = &t.ev[0][4 * i];
        float a = 0.f, b = 0.f, p = 0.f;
        hipError_t r;
        if ((r = hipEventElapsedTime(&a, ev[0], ev[1])) != hipSuccess ||
            (r = hipEventElapsedTime(&p, ev[1], ev[2])) != hipSuccess ||
            (r = hipEventElapsedTime(&b, ev[2], ev[3])) != hipSuccess)
            return r;
        t.ms[0] += p;
        t.ms[1] += a + b;
    }
    t.launches[0] += t.n[0];
    t.launches[1] += t.n[0];
    t.n[0] = 0;
    return hipSuccess;
}

// Whether c is the context last bound to its device's static workspace.
bool owns_static(const mbt_ctx *c)
{
    StaticWorkspace &w = static_ws();
    std::lock_guard<std::mutex> g(w.mu);
    return c->device >= 0 && c->device < kMaxDevices && w.owner[c->device] == c;
}

void release_binding(mbt_ctx *c)
{
    if (c->bound)
        (void)hipStreamSynchronize(c->stream_h);
    ring_free(c->mom);
    ring_free(c->prof);
    ring_free(c->tmom);
    if (c->mirror && c->mirror != &c->plain_mirror)
        (void)hipHostFree(c->mirror);
    c->mirror = nullptr;
    if (c->static_ws) {
        StaticWorkspace &w = static_ws();
        std::lock_guard<std::mutex> g(w.mu);
        if (c->device >= 0 && c->device < kMaxDevices && w.owner[c->device] == c)
            w.owner[c->device] = nullptr;
        c->static_ws = false;
    }
    c->bound = false;
}

int need_bound(mbt_ctx *c)
{
    if (!c)
        return MBT_EINVAL;
    if (!c->bound)
        return fail(c, MBT_ESTATE, "context not bound: call mbt_bind first");
    if (c->static_ws && !owns_static(c))
        return fail(c, MBT_ESTATE, "a later mbt_bind_static on device %d took the static workspace: "
                    "bind this context again", c->device);
    return MBT_OK;
}

// Device address of the static workspace on the current device, looked up
// once per device (with that device current) and kept.
int static_workspace(mbt_ctx *c, int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(c, MBT_EINVAL, "device %d beyond the static workspace table", device);
    StaticWorkspace &w = static_ws();
    std::lock_guard<std::mutex> g(w.mu);
    if (!w.ptr[device]) {
        void *p = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255))
            return fail(c, MBT_EDEVICE, "static workspace address %p unusable", p);
        w.ptr[device] = p;
    }
    *out = reinterpret_cast<unsigned char *>(w.ptr[device]);
    return MBT_OK;
}

}  // namespace

extern "C" {

const char *mbt_strerror(int code)
{
    switch (code) {
    case MBT_OK: return "ok";
    case MBT_EINVAL: return "invalid argument";
    case MBT_ESTATE: return "call made in the wrong order";
    case MBT_ENOSPC: return "buffer smaller than required";
    case MBT_EDEVICE: return "HIP runtime error";
    case MBT_ENUMERIC: return "non-finite bunch moment";
    case MBT_ENOMEM: return "host allocation failed";
    default: return "unknown error";
    }
}

const char *mbt_last_error(const mbt_ctx *ctx) { return ctx ? ctx->err : "null context"; }

int mbt_create(const mbt_ring *r, mbt_ctx **out)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!out)
            return MBT_EINVAL;
        *out = nullptr;
        if (!r)
            return MBT_EINVAL;
        if (!(r->energy_eV > 0.0) || !std::isfinite(r->energy_eV) || !(r->f_rf_Hz > 0.0) ||
            !std::isfinite(r->f_rf_Hz) || !(r->v_rf_V > 0.0) || !std::isfinite(r->v_rf_V) ||
            !std::isfinite(r->alpha_c) || r->alpha_c == 0.0 || !(r->u0_eV >= 0.0) ||
            !std::isfinite(r->u0_eV) || !(r->tau_long_s > 0.0) || !(r->sigma_delta >= 0.0) ||
            !std::isfinite(r->sigma_delta) || r->harmonic < 1 || !(r->u0_eV < r->v_rf_V))
            return MBT_EINVAL;
        mbt_ctx *c = new (std::nothrow) mbt_ctx();
        if (!c)
            return MBT_ENOMEM;
        c->ring = *r;
        c->T0 = (double)r->harmonic / r->f_rf_Hz;
        c->T_rf = 1.0 / r->f_rf_Hz;
        c->w_rf = kTwoPi * r->f_rf_Hz;
        c->D = 2.0 * c->T0 / r->tau_long_s;  // per-turn damping of delta (Eq. 5)
        c->noise = r->sigma_delta * std::sqrt(2.0 * c->D);
        c->drift = r->alpha_c * c->T0;       // Eq. 2
        if (solve_phi_s(c, false, c->hc, &c->phi_s) != MBT_OK) {
            delete c;
            return MBT_EINVAL;
        }
        if (hipGetDevice(&c->device) != hipSuccess)
            c->device = 0;
        *out = c;
        return MBT_OK;
    });
}

void mbt_destroy(mbt_ctx *ctx)
{
    try {
        if (!ctx)
            return;
        release_binding(ctx);
        timer_free(ctx->timer);
        delete ctx;
    } catch (...) {
        // teardown does not allocate; nothing may leave the ABI
    }
}

int mbt_hc_flat_fraction(const mbt_ring *ring, int32_t n, double frac, mbt_hc *out)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!ring || !out || n < 2 || !(frac > 0.0) || !std::isfinite(frac) || !(ring->v_rf_V > 0.0) ||
            !(ring->u0_eV >= 0.0) || ring->alpha_c == 0.0)
            return MBT_EINVAL;
        // Flat potential: V(0) = U0, V'(0) = V''(0) = 0 for
        // V(tau) = V_rf [sin(phi_s - w tau) + k sin(n phi_h - n w tau)].
        const double u = ring->u0_eV / ring->v_rf_V;
        const double n2 = (double)n * (double)n;
        const double sin_s = n2 / (n2 - 1.0) * u;
        const double k2 = 1.0 / n2 - u * u / (n2 - 1.0);
        if (!(sin_s <= 1.0) || !(k2 > 0.0))
            return MBT_EINVAL;
        const double k = std::sqrt(k2);
        double cos_s = std::sqrt(1.0 - sin_s * sin_s);
        if (ring->alpha_c < 0.0)
            cos_s = -cos_s;
        out->n = n;
        out->v_ratio = frac * k;
        out->phase_n_rad = std::atan2(-sin_s / (k * n2), -cos_s / (k * (double)n));
        return MBT_OK;
    });
}

int mbt_set_harmonic_cavity(mbt_ctx *c, const mbt_hc *hc)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        mbt_hc h{};
        if (hc) {
            if (hc->n < 2 || !std::isfinite(hc->v_ratio) || hc->v_ratio < 0.0 ||
                !std::isfinite(hc->phase_n_rad))
                return fail(c, MBT_EINVAL, "bad harmonic cavity");
            h = *hc;
        }
        double phi = 0.0;
        int rc = solve_phi_s(c, hc != nullptr, h, &phi);
        if (rc)
            return rc;
        c->hc_on = hc != nullptr;
        c->hc = h;
        c->phi_s = phi;
        return MBT_OK;
    });
}

int mbt_set_fill(mbt_ctx *c, int32_t M, const int32_t *bucket, const double *current_A,
                 const int32_t *stream)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (c->bound)
            return fail(c, MBT_ESTATE, "fill must be set before mbt_bind");
        if (M < 1 || M > c->ring.harmonic || M > 65535 || !bucket || !current_A)
            return fail(c, MBT_EINVAL, "need 1 <= M <= min(h, 65535) and non-null arrays");
        for (int b = 0; b < M; ++b) {
            if (bucket[b] < 0 || bucket[b] >= c->ring.harmonic || (b > 0 && bucket[b] <= bucket[b - 1]))
                return fail(c, MBT_EINVAL, "buckets must be strictly increasing in [0, h)");
            if (!(current_A[b] >= 0.0) || !std::isfinite(current_A[b]))
                return fail(c, MBT_EINVAL, "bunch currents must be finite and >= 0");
            if (stream && stream[b] < 0)
                return fail(c, MBT_EINVAL, "stream ordinals must be >= 0");
        }
        // built aside and swapped in, so a failed allocation leaves the
        // previous fill in place
        std::vector<int32_t> bk(bucket, bucket + M), st(M);
        std::vector<double> cur(current_A, current_A + M);
        for (int b = 0; b < M; ++b)
            st[b] = stream ? stream[b] : b;
        c->bucket.swap(bk);
        c->current.swap(cur);
        c->stream.swap(st);
        c->M = M;
        return MBT_OK;
    });
}

int mbt_set_short_range(mbt_ctx *c, int32_t nres, const mbt_resonator *res, const mbt_grid *g)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (c->bound)
            return fail(c, MBT_ESTATE, "wakes must be set before mbt_bind");
        if (!g) {
            c->sr_on = false;
            c->sr.clear();
            return MBT_OK;
        }
        if (g->nbins < 1 || g->nbins > MBT_MAX_BINS || !std::isfinite(g->tau_min_s) ||
            !std::isfinite(g->tau_max_s) || !(g->tau_min_s < g->tau_max_s))
            return fail(c, MBT_EINVAL, "grid: need 1 <= nbins <= %d and tau_min < tau_max", MBT_MAX_BINS);
        if (nres < 0 || nres > MBT_MAX_SHORT_RANGE || (nres > 0 && !res))
            return fail(c, MBT_EINVAL, "need 0 <= nres <= %d", MBT_MAX_SHORT_RANGE);
        for (int i = 0; i < nres; ++i)
            if (!res_valid(res[i]))
                return fail(c, MBT_EINVAL, "resonator %d: need Rs >= 0, Q > 0.5, fr > 0", i);
        std::vector<Resonator> sr;
        for (int i = 0; i < nres; ++i)
            sr.push_back({res[i].rs_ohm, res[i].q, res[i].fr_Hz});
        c->sr.swap(sr);
        c->sr_on = true;
        c->grid = *g;
        return MBT_OK;
    });
}

int mbt_set_long_range(mbt_ctx *c, int32_t nres, const mbt_resonator *res)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (c->bound)
            return fail(c, MBT_ESTATE, "wakes must be set before mbt_bind");
        if (nres < 0 || nres > MBT_MAX_LONG_RANGE || (nres > 0 && !res))
            return fail(c, MBT_EINVAL, "need 0 <= nres <= %d", MBT_MAX_LONG_RANGE);
        for (int i = 0; i < nres; ++i)
            if (!res_valid(res[i]))
                return fail(c, MBT_EINVAL, "resonator %d: need Rs >= 0, Q > 0.5, fr > 0", i);
        std::vector<Resonator> lr;
        for (int i = 0; i < nres; ++i)
            lr.push_back({res[i].rs_ohm, res[i].q, res[i].fr_Hz});
        c->lr.swap(lr);
        return MBT_OK;
    });
}

int mbt_set_resistive_wall(mbt_ctx *c, const mbt_resistive_wall *rw)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (c->bound)
            return fail(c, MBT_ESTATE, "wakes must be set before mbt_bind");
        if (rw && !(std::isfinite(rw->radius_m) && rw->radius_m > 0.0 &&
                    std::isfinite(rw->conductivity_S_m) && rw->conductivity_S_m > 0.0 &&
                    std::isfinite(rw->length_m) && rw->length_m > 0.0))
            return fail(c, MBT_EINVAL, "resistive wall: need radius, conductivity and length > 0");
        c->rw_on = rw != nullptr;
        if (rw)
            c->rw = ResistiveWall{rw->radius_m, rw->conductivity_S_m, rw->length_m};
        return MBT_OK;
    });
}

int mbt_set_transverse(mbt_ctx *c, const mbt_transverse *tr)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (c->bound)
            return fail(c, MBT_ESTATE, "the transverse plane must be set before mbt_bind");
        if (!tr) {
            c->tr_on = false;
            return MBT_OK;
        }
        if (!std::isfinite(tr->tune) || !std::isfinite(tr->chromaticity) || !std::isfinite(tr->alpha) ||
            !(tr->beta_m > 0.0) || !std::isfinite(tr->beta_m) || !std::isfinite(tr->disp_m) ||
            !std::isfinite(tr->disp_prime) || !(tr->emittance_m >= 0.0) ||
            !std::isfinite(tr->emittance_m) || !(tr->tau_damp_s > 0.0))
            return fail(c, MBT_EINVAL, "transverse plane: need finite values, beta > 0, eps >= 0, "
                        "tau_damp > 0");
        if (c->wake_mode != kWakeFP64)
            return fail(c, MBT_EINVAL, "the transverse plane needs the FP64 wake");
        c->tr = *tr;
        c->tr_on = true;
        return MBT_OK;
    });
}

int mbt_set_transverse_wake(mbt_ctx *c, int32_t nres, const mbt_resonator *res)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (c->bound)
            return fail(c, MBT_ESTATE, "wakes must be set before mbt_bind");
        if (nres < 0 || nres > MBT_MAX_SHORT_RANGE || (nres > 0 && !res))
            return fail(c, MBT_EINVAL, "need 0 <= nres <= %d", MBT_MAX_SHORT_RANGE);
        for (int i = 0; i < nres; ++i)
            if (!res_valid(res[i]))
                return fail(c, MBT_EINVAL, "resonator %d: need Rs >= 0, Q > 0.5, fr > 0", i);
        std::vector<Resonator> tw;
        for (int i = 0; i < nres; ++i)
            tw.push_back({res[i].rs_ohm, res[i].q, res[i].fr_Hz});
        c->tw.swap(tw);
        return MBT_OK;
    });
}

int mbt_set_transverse_rw(mbt_ctx *c, const mbt_transverse_rw *rw)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (c->bound)
            return fail(c, MBT_ESTATE, "wakes must be set before mbt_bind");
        if (rw && !(std::isfinite(rw->radius_m) && rw->radius_m > 0.0 &&
                    std::isfinite(rw->conductivity_S_m) && rw->conductivity_S_m > 0.0 &&
                    std::isfinite(rw->length_m) && rw->length_m > 0.0 && rw->turns >= 1 &&
                    rw->turns <= 1024))
            return fail(c, MBT_EINVAL, "resistive wall: need radius, conductivity, length > 0 and "
                        "1 <= turns <= 1024");
        c->trw_on = rw != nullptr;
        if (rw)
            c->trw = *rw;
        return MBT_OK;
    });
}

int mbt_query_bytes(const mbt_ctx *c, int64_t N, size_t *state_bytes, size_t *work_bytes)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!c || !state_bytes || !work_bytes)
            return MBT_EINVAL;
        if (c->M < 1)
            return MBT_ESTATE;
        if (N < 1 || N > ((int64_t)1 << 32))
            return MBT_EINVAL;
        Layout L = c->layout(N);
        *state_bytes = L.state_bytes;
        *work_bytes = L.total;
        return MBT_OK;
    });
}

}  // extern "C"

namespace {

// mbt_bind and mbt_bind_static.  With `st` the workspace is the current
// device's static array (d_work and work_bytes are ignored), the host mirror
// is plain memory and the output rings have no pinned staging.
int bind_job(mbt_ctx *c, int64_t N, void *d_state, size_t state_bytes, void *d_work,
             size_t work_bytes, void *hip_stream, bool st)
{
    {
        if (!c)
            return MBT_EINVAL;
        if (c->M < 1)
            return fail(c, MBT_ESTATE, "fill not set");
        if (N < 1 || N > ((int64_t)1 << 32))
            return fail(c, MBT_EINVAL, "N must be in [1, 2^32]");
        if (!d_state || ((uintptr_t)d_state & 255) || (!st && (!d_work || ((uintptr_t)d_work & 255))))
            return fail(c, MBT_EINVAL, "device buffers must be non-null and 256-byte aligned");
        Layout L = c->layout(N);
        if (st && L.total > (size_t)MBT_STATIC_WORK_BYTES)
            return fail(c, MBT_ENOSPC, "the job needs %zu workspace bytes; the static workspace "
                        "holds %zu", L.total, (size_t)MBT_STATIC_WORK_BYTES);
        if (state_bytes < L.state_bytes || (!st && work_bytes < L.total))
            return fail(c, MBT_ENOSPC, "need %zu state and %zu workspace bytes", L.state_bytes, L.total);
        int device = 0;
        HIPCHK(c, hipGetDevice(&device));
        unsigned char *work = reinterpret_cast<unsigned char *>(d_work);
        if (st) {
            int rc = static_workspace(c, device, &work);
            if (rc)
                return rc;
        }
        release_binding(c);
        c->L = L;
        c->N = N;
        c->tau = reinterpret_cast<double *>(d_state);
        c->delta = c->tau + (size_t)c->M * L.ld;
        c->x = c->tr_on ? c->delta + (size_t)c->M * L.ld : nullptr;
        c->xp = c->tr_on ? c->x + (size_t)c->M * L.ld : nullptr;
        c->work = work;
        c->stream_h = reinterpret_cast<hipStream_t>(hip_stream);
        c->device = device;
        if (st) {
            // from here on this context owns the device's static workspace;
            // an earlier owner gets MBT_ESTATE until it is bound again
            StaticWorkspace &w = static_ws();
            std::lock_guard<std::mutex> g(w.mu);
            w.owner[device] = c;
            c->static_ws = true;
        }

        const int M = c->M, nb = c->nbins(), nbx = std::max(nb, 1), nlr = c->nlr();
        // Host-side tables.
        std::vector<double> W((size_t)nbx, 0.0);
        if (c->sr_on) {
            // Sum of all resonators sampled at bin distances (Sec. 2.3); the
            // long-range ones contribute their same-bunch, same-turn part here.
            const double dt = (c->grid.tau_max_s - c->grid.tau_min_s) / (double)nb;
            std::vector<Resonator> all = c->sr;
            all.insert(all.end(), c->lr.begin(), c->lr.end());
            for (const Resonator &r : all) {
                W[0] += 0.5 * r.wake(0.0);
                for (int k = 1; k < nb; ++k)
                    W[k] += r.wake((double)k * dt);
            }
            if (c->rw_on) {
                std::vector<double> gx, gw;
                gauss_legendre(24, gx, gw);
                W[0] += 0.5 * rw_wake(c->rw, 0.0, gx, gw);
                for (int k = 1; k < nb; ++k)
                    W[k] += rw_wake(c->rw, (double)k * dt, gx, gw);
            }
        }
        std::vector<double> qpp(M), gap((size_t)std::max(nlr, 1) * M * 2, 0.0),
            qc((size_t)std::max(nlr, 1) * M * 2, 0.0);
        std::vector<uint32_t> strm(M);
        for (int b = 0; b < M; ++b) {
            qpp[b] = c->current[b] * c->T0 / (double)N;
            strm[b] = (uint32_t)c->stream[b];
        }
        for (int r = 0; r < nlr; ++r) {
            const double a = c->lr[r].alpha(), wb = c->lr[r].wbar();
            // W(t) = Re[c_r exp((-alpha + i wbar) t)], c_r = 2 alpha Rs (1 + i alpha/wbar)
            const double cr = 2.0 * a * c->lr[r].rs, ci = 2.0 * a * c->lr[r].rs * (a / wb);
            for (int b = 0; b < M; ++b) {
                const int g = (b == 0) ? (c->ring.harmonic - c->bucket[M - 1] + c->bucket[0])
                                       : (c->bucket[b] - c->bucket[b - 1]);
                const double t = (double)g * c->T_rf;
                const double e = std::exp(-a * t);
                const size_t ix = ((size_t)r * M + b) * 2;
                gap[ix] = e * std::cos(wb * t);
                gap[ix + 1] = e * std::sin(wb * t);
                qc[ix] = qpp[b] * cr;
                qc[ix + 1] = qpp[b] * ci;
            }
        }
        std::vector<Item> pitems, citems, witems;
        pitems.reserve((size_t)M * L.ntiles);
        citems.reserve((size_t)M * L.nchunks);
        push_items(c, 0, pitems);
        prep_items(c, 0, citems);
        wake_items(c, 0, witems);
        // Matrix-core tables of the wake: W / s with s a power of two near max |W|,
        // as FP32 and as three BF16 terms (each the BF16 nearest to what the
        // previous ones leave).  Bin counts stay below 2^(8 count_parts).
        std::vector<uint16_t> wbf((size_t)3 * nbx, 0);
        std::vector<float> wf((size_t)nbx, 0.f);
        {
            double wmax = 0.0;
            for (double v : W)
                wmax = std::max(wmax, std::fabs(v));
            int e = 0;
            if (wmax > 0.0)
                std::frexp(wmax, &e);  // wmax = f 2^e, f in [1/2, 1)
            c->wake_scale = wmax > 0.0 ? std::ldexp(1.0, e) : 1.0;
            for (int k = 0; k < nbx; ++k) {
                double rest = W[k] / c->wake_scale;
                wf[k] = (float)rest;
                for (int q = 0; q < 3; ++q) {
                    const uint16_t h = bf16_nearest(rest);
                    wbf[(size_t)q * nbx + k] = h;
                    rest -= bf16_value(h);
                }
            }
            c->count_parts = 1;
            while (c->count_parts < 4 && (double)N >= std::ldexp(1.0, 8 * c->count_parts))
                ++c->count_parts;
        }
        HIPCHK(c, hipMemsetAsync(c->work, 0, L.total, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<double>(L.W), W.data(), W.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<double>(L.qpp), qpp.data(), qpp.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<double>(L.gap), gap.data(), gap.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<double>(L.qc), qc.data(), qc.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<uint32_t>(L.stream), strm.data(), strm.size() * sizeof(uint32_t),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<Item>(L.items_push), pitems.data(), pitems.size() * sizeof(Item),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<Item>(L.items_prep), citems.data(), citems.size() * sizeof(Item),
                                 hipMemcpyHostToDevice, c->stream_h));
        if (!witems.empty())
            HIPCHK(c, hipMemcpyAsync(c->w<Item>(L.items_wake), witems.data(), witems.size() * sizeof(Item),
                                     hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<uint16_t>(L.Wbf), wbf.data(), wbf.size() * sizeof(uint16_t),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->w<float>(L.Wf32), wf.data(), wf.size() * sizeof(float),
                                 hipMemcpyHostToDevice, c->stream_h));
        if (c->tr_on) {
            // transverse wake table on the grid (T[0] = 0), bunch buckets and
            // charges for the wall
            std::vector<double> T((size_t)nbx, 0.0), qb((size_t)M);
            if (c->sr_on) {
                const double dt = (c->grid.tau_max_s - c->grid.tau_min_s) / (double)nb;
                for (const Resonator &r : c->tw) {
                    const double wr = kTwoPi * r.fr, a = r.alpha(), wb = r.wbar();
                    const double amp = r.rs * wr * wr / (r.q * wb);
                    for (int k = 1; k < nb; ++k) {
                        const double t = (double)k * dt;
                        T[k] += amp * std::exp(-a * t) * std::sin(wb * t);
                    }
                }
            }
            for (int b = 0; b < M; ++b)
                qb[b] = c->current[b] * c->T0;
            HIPCHK(c, hipMemcpyAsync(c->w<double>(L.Tt), T.data(), T.size() * sizeof(double),
                                     hipMemcpyHostToDevice, c->stream_h));
            HIPCHK(c, hipMemcpyAsync(c->w<int32_t>(L.bucket), c->bucket.data(), (size_t)M * sizeof(int32_t),
                                     hipMemcpyHostToDevice, c->stream_h));
            HIPCHK(c, hipMemcpyAsync(c->w<double>(L.qb), qb.data(), qb.size() * sizeof(double),
                                     hipMemcpyHostToDevice, c->stream_h));
            HIPCHK(c, hipStreamSynchronize(c->stream_h));
        }
        HIPCHK(c, hipMemsetAsync(d_state, 0, L.state_bytes, c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        if (st)
            c->mirror = &c->plain_mirror;
        else
            HIPCHK(c, hipHostMalloc((void **)&c->mirror, sizeof(Mirror), hipHostMallocDefault));
        int rc = ring_alloc(c, c->mom, c->w<double>(L.mom), (size_t)M * sizeof(mbt_moments),
                            L.mom_slots, !st);
        if (!rc)
            rc = ring_alloc(c, c->prof, c->w<uint32_t>(L.prof), (size_t)M * nbx * sizeof(uint32_t),
                            L.prof_slots, !st);
        if (!rc && c->tr_on)
            rc = ring_alloc(c, c->tmom, c->w<double>(L.tmom), (size_t)M * sizeof(mbt_tmoments),
                            L.mom_slots, !st);
        if (rc) {
            release_binding(c);
            return rc;
        }
        if (c->nsub == 0 || push_lds_bytes(nb, c->nsub) > kLdsLimit)
            c->nsub = default_nsub(nb);
        if (nb == 0)
            c->nsub = 0;
        c->bound = true;
        c->have_particles = false;
        c->dirty = true;
        c->turn = 0;
        return MBT_OK;
    }
}

}  // namespace

extern "C" {

int mbt_bind(mbt_ctx *c, int64_t N, void *d_state, size_t state_bytes, void *d_work,
             size_t work_bytes, void *hip_stream)
{
    return guarded(c, [&]() -> int {
        return bind_job(c, N, d_state, state_bytes, d_work, work_bytes, hip_stream, false);
    });
}

int mbt_bind_static(mbt_ctx *c, int64_t N, void *d_state, size_t state_bytes, void *hip_stream)
{
    return guarded(c, [&]() -> int {
        return bind_job(c, N, d_state, state_bytes, nullptr, 0, hip_stream, true);
    });
}

int mbt_init_gaussian(mbt_ctx *c, double sigma_tau_s, double sigma_delta, uint64_t seed)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (!(sigma_tau_s >= 0.0) || !(sigma_delta >= 0.0) || !std::isfinite(sigma_tau_s) ||
            !std::isfinite(sigma_delta))
            return fail(c, MBT_EINVAL, "sigmas must be finite and >= 0");
        HIPCHK(c, launch_init_gauss(c->tau, c->delta, c->L.ld, c->N, c->M,
                                    c->w<uint32_t>(c->L.stream), sigma_tau_s, sigma_delta,
                                    (uint32_t)seed, (uint32_t)(seed >> 32), c->stream_h));
        HIPCHK(c, hipMemsetAsync(c->w<double>(c->L.phasor), 0,
                                 (size_t)std::max(c->nlr(), 1) * 2 * sizeof(double), c->stream_h));
        if (c->tr_on) {
            // a fresh start: the plane at rest until mbt_init_transverse, no wall history
            HIPCHK(c, hipMemsetAsync(c->x, 0, (size_t)2 * c->M * c->L.ld * sizeof(double), c->stream_h));
            if (c->rw_turns() > 0)
                HIPCHK(c, hipMemsetAsync(c->w<double>(c->L.H), 0,
                                         (size_t)c->rw_turns() * c->M * sizeof(double), c->stream_h));
        }
        c->seed = seed;
        c->turn = 0;
        c->have_particles = true;
        c->dirty = true;
        return MBT_OK;
    });
}

int mbt_set_particles(mbt_ctx *c, int32_t bunch, const double *tau, const double *delta,
                      int32_t where)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (bunch < 0 || bunch >= c->M || !tau || !delta || (where != MBT_HOST && where != MBT_DEVICE))
            return fail(c, MBT_EINVAL, "bad bunch index, null array or location");
        const size_t bytes = (size_t)c->N * sizeof(double);
        const hipMemcpyKind kind = where == MBT_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        double *dt = c->tau + (size_t)bunch * c->L.ld, *dd = c->delta + (size_t)bunch * c->L.ld;
        HIPCHK(c, hipMemcpyAsync(dt, tau, bytes, kind, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(dd, delta, bytes, kind, c->stream_h));
        if (where == MBT_HOST)
            HIPCHK(c, hipStreamSynchronize(c->stream_h));
        c->have_particles = true;
        c->dirty = true;
        return MBT_OK;
    });
}

int mbt_get_particles(mbt_ctx *c, int32_t bunch, double *tau, double *delta, int32_t where)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (bunch < 0 || bunch >= c->M || !tau || !delta || (where != MBT_HOST && where != MBT_DEVICE))
            return fail(c, MBT_EINVAL, "bad bunch index, null array or location");
        const size_t bytes = (size_t)c->N * sizeof(double);
        const hipMemcpyKind kind = where == MBT_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        HIPCHK(c, hipMemcpyAsync(tau, c->tau + (size_t)bunch * c->L.ld, bytes, kind, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(delta, c->delta + (size_t)bunch * c->L.ld, bytes, kind, c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        return MBT_OK;
    });
}

}  // extern "C"

namespace {

int track_job(mbt_ctx *c, int64_t nturns, mbt_moments *out, mbt_tmoments *tout, uint32_t *counts,
              int32_t stride)
{
    {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (!c->have_particles)
            return fail(c, MBT_ESTATE, "particles not initialised");
        if (nturns < 0 || nturns > INT32_MAX || c->turn + nturns > ((int64_t)1 << 32))
            return fail(c, MBT_EINVAL, "need nturns < 2^31 and the turn counter below 2^32");
        if (counts && (!c->sr_on || stride < 1))
            return fail(c, MBT_EINVAL, "profiles need a grid and stride >= 1");
        if (tout && !c->tr_on)
            return fail(c, MBT_EINVAL, "transverse moments need the transverse plane");
        if (nturns == 0)
            return MBT_OK;
        hipStream_t s = c->stream_h;
        rc = begin_call(c, counts ? stride : 0, s);
        if (rc)
            return rc;
        ring_start(c->mom, out);
        ring_start(c->prof, counts);
        ring_start(c->tmom, tout);
        const Engine e = single_engine(c);
        for (int64_t t = 0; t < nturns; ++t) {
            const bool timed = c->timer.every > 0 && (t % c->timer.every) == 0;
            HIPCHK(c, ring_advance(c->mom, 1, s));
            HIPCHK(c, ring_advance(c->prof, profile_rows(t, 1, stride), s));
            HIPCHK(c, ring_advance(c->tmom, 1, s));
            HIPCHK(c, enqueue_turn(e, (int)(t & 1), s, timed ? &c->timer : nullptr));
        }
        c->turn += nturns;
        HIPCHK(c, ring_flush(c->mom, s));
        HIPCHK(c, ring_flush(c->prof, s));
        HIPCHK(c, ring_flush(c->tmom, s));
        HIPCHK(c, hipStreamSynchronize(s));
        HIPCHK(c, ring_land(c->mom));
        HIPCHK(c, ring_land(c->prof));
        HIPCHK(c, ring_land(c->tmom));
        HIPCHK(c, timer_collect(c->timer));
        uint32_t status = 0;
        HIPCHK(c, hipMemcpy(&status, c->w<uint32_t>(c->L.status), sizeof status, hipMemcpyDeviceToHost));
        if (status) {
            HIPCHK(c, hipMemset(c->w<uint32_t>(c->L.status), 0, sizeof status));
            return fail(c, MBT_ENUMERIC, "non-finite bunch moment during turns %lld..%lld",
                        (long long)(c->turn - nturns), (long long)(c->turn - 1));
        }
        return MBT_OK;
    }
}

}  // namespace

extern "C" {

int mbt_track(mbt_ctx *c, int64_t nturns, mbt_moments *out, uint32_t *counts, int32_t stride)
{
    return guarded(c, [&]() -> int { return track_job(c, nturns, out, nullptr, counts, stride); });
}

int mbt_track2(mbt_ctx *c, int64_t nturns, mbt_moments *out, mbt_tmoments *tout, uint32_t *counts,
               int32_t stride)
{
    return guarded(c, [&]() -> int { return track_job(c, nturns, out, tout, counts, stride); });
}

int mbt_init_transverse(mbt_ctx *c, double emittance_m, double offset_m)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (!c->tr_on)
            return fail(c, MBT_ESTATE, "no transverse plane");
        if (!(emittance_m >= 0.0) || !std::isfinite(emittance_m) || !std::isfinite(offset_m))
            return fail(c, MBT_EINVAL, "emittance must be finite and >= 0, offset finite");
        const double sx = std::sqrt(emittance_m * c->tr.beta_m);
        const double sxp = std::sqrt(emittance_m / c->tr.beta_m);
        HIPCHK(c, launch_init_transverse(c->x, c->xp, c->L.ld, c->N, c->M, c->w<uint32_t>(c->L.stream),
                                         sx, sxp, c->tr.alpha, offset_m, (uint32_t)c->seed,
                                         (uint32_t)(c->seed >> 32), c->stream_h));
        if (c->rw_turns() > 0)
            HIPCHK(c, hipMemsetAsync(c->w<double>(c->L.H), 0,
                                     (size_t)c->rw_turns() * c->M * sizeof(double), c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        c->dirty = true;
        return MBT_OK;
    });
}

int mbt_set_transverse_particles(mbt_ctx *c, int32_t bunch, const double *x, const double *xp,
                                 int32_t where)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (!c->tr_on)
            return fail(c, MBT_ESTATE, "no transverse plane");
        if (bunch < 0 || bunch >= c->M || !x || !xp || (where != MBT_HOST && where != MBT_DEVICE))
            return fail(c, MBT_EINVAL, "bad bunch index, null array or location");
        const size_t bytes = (size_t)c->N * sizeof(double);
        const hipMemcpyKind kind = where == MBT_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        HIPCHK(c, hipMemcpyAsync(c->x + (size_t)bunch * c->L.ld, x, bytes, kind, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(c->xp + (size_t)bunch * c->L.ld, xp, bytes, kind, c->stream_h));
        if (where == MBT_HOST)
            HIPCHK(c, hipStreamSynchronize(c->stream_h));
        c->dirty = true;
        return MBT_OK;
    });
}

int mbt_get_transverse_particles(mbt_ctx *c, int32_t bunch, double *x, double *xp, int32_t where)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (!c->tr_on)
            return fail(c, MBT_ESTATE, "no transverse plane");
        if (bunch < 0 || bunch >= c->M || !x || !xp || (where != MBT_HOST && where != MBT_DEVICE))
            return fail(c, MBT_EINVAL, "bad bunch index, null array or location");
        const size_t bytes = (size_t)c->N * sizeof(double);
        const hipMemcpyKind kind = where == MBT_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        HIPCHK(c, hipMemcpyAsync(x, c->x + (size_t)bunch * c->L.ld, bytes, kind, c->stream_h));
        HIPCHK(c, hipMemcpyAsync(xp, c->xp + (size_t)bunch * c->L.ld, bytes, kind, c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        return MBT_OK;
    });
}

int mbt_get_rw_history(mbt_ctx *c, double *H)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (c->rw_turns() == 0)
            return fail(c, MBT_ESTATE, "no long-range resistive wall");
        if (!H)
            return fail(c, MBT_EINVAL, "null array");
        HIPCHK(c, hipMemcpyAsync(H, c->w<double>(c->L.H), (size_t)c->rw_turns() * c->M * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        return MBT_OK;
    });
}

int mbt_set_rw_history(mbt_ctx *c, const double *H)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (c->rw_turns() == 0)
            return fail(c, MBT_ESTATE, "no long-range resistive wall");
        if (!H)
            return fail(c, MBT_EINVAL, "null array");
        HIPCHK(c, hipMemcpyAsync(c->w<double>(c->L.H), H, (size_t)c->rw_turns() * c->M * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        c->dirty = true;  // the wall kick of the next turn comes from the new history
        return MBT_OK;
    });
}

int mbt_profile(mbt_ctx *c, uint32_t *counts)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (!counts || !c->sr_on)
            return fail(c, MBT_EINVAL, "need a grid and an output array");
        if (!c->have_particles)
            return fail(c, MBT_ESTATE, "particles not initialised");
        rc = begin_call(c, 0, c->stream_h);
        if (rc)
            return rc;
        // the prep leaves the present state's histogram in counts[turn & 1]
        const size_t bytes = (size_t)c->M * c->nbins() * sizeof(uint32_t);
        HIPCHK(c, hipMemcpyAsync(counts, c->w<uint32_t>(c->L.counts) + (size_t)(c->turn & 1) * c->M * c->nbins(),
                                 bytes, hipMemcpyDeviceToHost, c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        return MBT_OK;
    });
}

int mbt_wake_potential(mbt_ctx *c, double *V)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (!V || !c->sr_on)
            return fail(c, MBT_EINVAL, "need a grid and an output array");
        if (!c->have_particles)
            return fail(c, MBT_ESTATE, "particles not initialised");
        rc = begin_call(c, 0, c->stream_h);
        if (rc)
            return rc;
        HIPCHK(c, hipMemcpyAsync(V, c->w<double>(c->L.V), (size_t)c->M * c->nbins() * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream_h));
        HIPCHK(c, hipStreamSynchronize(c->stream_h));
        return MBT_OK;
    });
}

int mbt_wake_table(const mbt_ctx *c, double *W)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!c || !W)
            return MBT_EINVAL;
        if (!c->bound || !c->sr_on || (c->static_ws && !owns_static(c)))
            return MBT_ESTATE;
        if (hipMemcpy(W, c->w<double>(c->L.W), (size_t)c->nbins() * sizeof(double),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return MBT_EDEVICE;
        return MBT_OK;
    });
}

int mbt_get_state(mbt_ctx *c, int64_t *turn, uint64_t *seed, double *phasors)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (turn)
            *turn = c->turn;
        if (seed)
            *seed = c->seed;
        if (phasors && c->nlr() > 0) {
            HIPCHK(c, hipMemcpyAsync(phasors, c->w<double>(c->L.phasor), (size_t)c->nlr() * 2 * sizeof(double),
                                     hipMemcpyDeviceToHost, c->stream_h));
            HIPCHK(c, hipStreamSynchronize(c->stream_h));
        }
        return MBT_OK;
    });
}

int mbt_set_state(mbt_ctx *c, int64_t turn, uint64_t seed, const double *phasors)
{
    return guarded(c, [&]() -> int {
        int rc = need_bound(c);
        if (rc)
            return rc;
        if (turn < 0 || turn > ((int64_t)1 << 32))
            return fail(c, MBT_EINVAL, "turn out of range");
        if (c->nlr() > 0) {
            const size_t bytes = (size_t)c->nlr() * 2 * sizeof(double);
            if (phasors) {
                HIPCHK(c, hipMemcpyAsync(c->w<double>(c->L.phasor), phasors, bytes, hipMemcpyHostToDevice,
                                         c->stream_h));
                HIPCHK(c, hipStreamSynchronize(c->stream_h));
            } else {
                HIPCHK(c, hipMemsetAsync(c->w<double>(c->L.phasor), 0, bytes, c->stream_h));
            }
        }
        c->turn = turn;
        c->seed = seed;
        c->dirty = true;
        return MBT_OK;
    });
}

int mbt_set_timing(mbt_ctx *c, int32_t every)
{
    return guarded(c, [&]() -> int {
        if (!c || every < 0)
            return MBT_EINVAL;
        HIPCHK(c, timer_set(c->timer, every));
        return MBT_OK;
    });
}

int mbt_get_timing(const mbt_ctx *c, double *push_ms, int64_t *push_launches, double *prep_ms,
                   int64_t *prep_launches)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (push_ms)
            *push_ms = c->timer.ms[0];
        if (push_launches)
            *push_launches = c->timer.launches[0];
        if (prep_ms)
            *prep_ms = c->timer.ms[1];
        if (prep_launches)
            *prep_launches = c->timer.launches[1];
        return MBT_OK;
    });
}

int mbt_set_wake_precision(mbt_ctx *c, int32_t mode)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        if (mode < MBT_WAKE_FP64 || mode > MBT_WAKE_BF16X3)
            return fail(c, MBT_EINVAL, "unknown wake precision %d", mode);
        if (c->tr_on && mode != MBT_WAKE_FP64)
            return fail(c, MBT_EINVAL, "a job with the transverse plane keeps the FP64 wake");
        if (mode != c->wake_mode)
            c->dirty = true;  // the stored wake potential used the other arithmetic
        c->wake_mode = mode;
        return MBT_OK;
    });
}

int mbt_set_launch(mbt_ctx *c, int32_t nsub, int32_t push_grid)
{
    return guarded(c, [&]() -> int {
        if (!c)
            return MBT_EINVAL;
        const int nb = c->nbins();
        if (push_grid < 0 || nsub < 0 || (nb > 0 && nsub > 0 && push_lds_bytes(nb, nsub) > kLdsLimit))
            return fail(c, MBT_EINVAL, "need push_grid >= 0 and 0 <= nsub with the LDS image <= %zu bytes",
                        kLdsLimit);
        c->nsub = nb == 0 ? 0 : (nsub == 0 ? default_nsub(nb) : nsub);
        c->push_grid = push_grid;
        return MBT_OK;
    });
}

int mbt_philox4x32_10(int64_t n, const uint32_t *ctr, uint32_t key0, uint32_t key1, uint32_t *out,
                      void *hip_stream)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (n < 0 || (n > 0 && (!ctr || !out)))
            return MBT_EINVAL;
        if (launch_philox(n, ctr, key0, key1, out, reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
            return MBT_EDEVICE;
        return MBT_OK;
    });
}

int mbt_stream_copy(const void *src, void *dst, int64_t bytes, void *hip_stream)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (bytes < 0 || (bytes % 16) != 0)
            return MBT_EINVAL;
        if (bytes == 0)
            return MBT_OK;
        if (!src || !dst || (reinterpret_cast<uintptr_t>(src) & 15u) ||
            (reinterpret_cast<uintptr_t>(dst) & 15u))
            return MBT_EINVAL;
        const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
        if (a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes)
            return MBT_EINVAL;  // overlapping ranges
        if (launch_stream_copy(src, dst, bytes, reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
            return MBT_EDEVICE;
        return MBT_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: several bound jobs advanced together, every kernel launch
// covering all bunches of all jobs.  Optionally a run of turns is captured
// once as a HIP graph and replayed; optionally the launch shape of the push
// is tuned online on the first turns.
// ---------------------------------------------------------------------------

struct mbt_batch {
    std::vector<mbt_ctx *> jobs;
    unsigned char *work = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;   // private stream that graphs are captured on
    JobDesc *pin_desc = nullptr; // pinned [njobs]
    size_t off_push = 0, off_prep = 0, off_wake = 0, off_ctr = 0, total = 0;
    Engine eng;
    std::vector<int> wake_modes;  // each job's wake arithmetic when the batch was made
    int graph_turns = 0;
    bool autotune = false, tuned = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int exec_turns = 0, exec_phase = 0;  // captured turns and the phase of the first
    Timer timer;  // measurement only: bracketed turns run eagerly, never from a graph
    char err[512] = "";
};

namespace {

size_t batch_layout(mbt_ctx *const *jobs, int n, size_t *off_push, size_t *off_prep,
                    size_t *off_wake, size_t *off_ctr = nullptr)
{
    size_t np = 0, nc = 0, nw = 0;
    for (int j = 0; j < n; ++j) {
        np += (size_t)jobs[j]->M * jobs[j]->L.ntiles;
        nc += (size_t)jobs[j]->M * jobs[j]->L.nchunks;
        nw += (size_t)jobs[j]->L.nwake;
    }
    size_t o = align256((size_t)n * sizeof(JobDesc));
    *off_push = o;
    o = align256(o + np * sizeof(Item));
    *off_prep = o;
    o = align256(o + nc * sizeof(Item));
    *off_wake = o;
    o = align256(o + std::max<size_t>(nw, 1) * sizeof(Item));
    if (off_ctr)
        *off_ctr = o;
    // item counters of persistent push launches: four words per push group
    o = align256(o + (size_t)(kMaxLR + 1) * 4 * sizeof(uint32_t));
    return o;
}

void drop_graph(mbt_batch *B)
{
    if (B->exec)
        (void)hipGraphExecDestroy(B->exec);
    if (B->graph)
        (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->exec_turns = 0;
}

// Launch-shape choices found by the tuner, by (group nlr, largest nbins,
// log2 of the item count).
struct TuneKey {
    int nlr, nbins, log_items;
    bool operator<(const TuneKey &o) const
    {
        return nlr != o.nlr ? nlr < o.nlr : nbins != o.nbins ? nbins < o.nbins : log_items < o.log_items;
    }
};
struct TuneChoice {
    int nsub, grid;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune_cache;

TuneKey tune_key(const Group &g)
{
    int l = 0;
    while ((1 << (l + 1)) <= g.nitems && l < 30)
        ++l;
    return TuneKey{g.nlr, g.nbins_max, l};
}

// Set the sub-histogram count of every job of group gi (and the group's
// LDS bound) and its push grid.
void apply_choice(mbt_batch *B, int gi, TuneChoice ch)
{
    Group &g = B->eng.groups[gi];
    g.grid = ch.grid;
    g.nsub_max = 0;
    for (mbt_ctx *c : B->jobs)
        if (c->nlr() == g.nlr) {
            c->nsub = c->nbins() > 0 ? ch.nsub : 0;
            g.nsub_max = std::max(g.nsub_max, c->nsub);
        }
}

// Upload every job's descriptor (after begin_call has refreshed its mirror).
// The pinned image may still be read by an earlier copy: drain first.
int upload_descs(mbt_batch *B)
{
    HIPCHK(B, hipStreamSynchronize(B->stream));
    for (size_t j = 0; j < B->jobs.size(); ++j) {
        mbt_ctx *c = B->jobs[j];
        B->pin_desc[j] = c->mirror->desc;
        B->pin_desc[j].nsub = c->nsub;
    }
    HIPCHK(B, hipMemcpyAsync(B->work, B->pin_desc, B->jobs.size() * sizeof(JobDesc),
                             hipMemcpyHostToDevice, B->stream));
    return MBT_OK;
}

// Rings of every job for turns [t, t + n) of the call.
int batch_rings(mbt_batch *B, int64_t t, int64_t n, const int32_t *stride)
{
    for (size_t j = 0; j < B->jobs.size(); ++j) {
        mbt_ctx *c = B->jobs[j];
        HIPCHK(B, ring_advance(c->mom, n, B->stream));
        if (stride)
            HIPCHK(B, ring_advance(c->prof, profile_rows(t, n, stride[j]), B->stream));
    }
    return MBT_OK;
}

// Online tuning over real turns [t, t + budget): every candidate shape of
// every group runs for two turns with events around the push; the fastest
// (minimum over its turns) is kept and cached.  The shapes do not change any
// result bit, so the turns count as ordinary tracking.  Returns the turns used.
int64_t batch_tune(mbt_batch *B, int64_t t, int64_t budget, const int32_t *stride, int *rc)
{
    *rc = MBT_OK;
    std::vector<std::vector<TuneChoice>> cand(B->eng.groups.size());
    size_t ncand = 1;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (size_t gi = 0; gi < B->eng.groups.size(); ++gi) {
            const Group &g = B->eng.groups[gi];
            auto it = g_tune_cache.find(tune_key(g));
            if (it != g_tune_cache.end()) {
                cand[gi].push_back(it->second);
                continue;
            }
            std::vector<int> subs;
            if (g.nbins_max == 0)
                subs.push_back(0);
            else
                for (int n = 1; n <= 8; n *= 2)
                    if (push_lds_bytes(g.nbins_max, n) <= kLdsLimit)
                        subs.push_back(n);
            std::vector<int> grids = {0};
            for (int w : {512, 1024, 2048})
                if (w < g.nitems)
                    grids.push_back(w);
            for (int n : subs)
                for (int w : grids)
                    cand[gi].push_back({n, w});
            ncand = std::max(ncand, cand[gi].size());
        }
    }
    // every candidate runs `reps` turns, the candidates taken in turn within
    // each round, so that a drift of the clock over the tuning turns (it
    // rises over the first turns after idle) favours none of them
    const int reps = 3;
    if (ncand == 1) {  // all cached
        for (size_t gi = 0; gi < cand.size(); ++gi)
            apply_choice(B, (int)gi, cand[gi][0]);
        B->tuned = true;
        *rc = upload_descs(B);
        return 0;
    }
    if ((int64_t)ncand * reps > budget)
        return 0;  // too few turns in this call; tune on a later one
    std::vector<std::vector<float>> best(cand.size());
    for (size_t gi = 0; gi < cand.size(); ++gi)
        best[gi].assign(cand[gi].size(), 1e30f);
    std::vector<hipEvent_t> ev(2 * cand.size(), nullptr);
    for (hipEvent_t &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            for (hipEvent_t made : ev)
                if (made)
                    (void)hipEventDestroy(made);
            *rc = fail(B, MBT_EDEVICE, "hipEventCreate failed");
            return 0;
        }
    int64_t used = 0;
    for (int r = 0; r < reps && !*rc; ++r) {
        for (size_t k = 0; k < ncand && !*rc; ++k, ++used) {
            for (size_t gi = 0; gi < cand.size(); ++gi)
                apply_choice(B, (int)gi, cand[gi][std::min(k, cand[gi].size() - 1)]);
            if ((*rc = upload_descs(B)))
                break;
            if ((*rc = batch_rings(B, t + used, 1, stride)))
                break;
            const int phase = (int)((t + used) & 1);
            hipError_t e = enqueue_scan(B->eng, B->stream);
            for (size_t gi = 0; gi < cand.size() && e == hipSuccess; ++gi) {
                e = hipEventRecord(ev[2 * gi], B->stream);
                if (e == hipSuccess)
                    e = launch_push(push_launch(B->eng, B->eng.groups[gi], phase), true, B->stream);
                if (e == hipSuccess)
                    e = hipEventRecord(ev[2 * gi + 1], B->stream);
            }
            if (e == hipSuccess)
                e = enqueue_prep(B->eng, phase, B->stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(B->stream);
            for (size_t gi = 0; gi < cand.size() && e == hipSuccess; ++gi) {
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, ev[2 * gi], ev[2 * gi + 1]);
                const size_t kk = std::min(k, cand[gi].size() - 1);
                best[gi][kk] = std::min(best[gi][kk], ms);
            }
            if (e != hipSuccess)
                *rc = fail(B, MBT_EDEVICE, "tuning turn failed: %s", hipGetErrorString(e));
        }
    }
    for (hipEvent_t e : ev)
        (void)hipEventDestroy(e);
    if (*rc)
        return used;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (size_t gi = 0; gi < cand.size(); ++gi) {
            size_t k = std::min_element(best[gi].begin(), best[gi].end()) - best[gi].begin();
            // The default shape (default sub-histograms, one workgroup per
            // tile) stays unless a candidate beats it by more than 2%: three
            // turns per candidate do not resolve smaller differences.
            const Group &g = B->eng.groups[gi];
            const int dsub = g.nbins_max > 0 ? default_nsub(g.nbins_max) : 0;
            for (size_t d = 0; d < cand[gi].size(); ++d)
                if (cand[gi][d].nsub == dsub && cand[gi][d].grid == 0 &&
                    best[gi][k] > 0.98f * best[gi][d])
                    k = d;
            try {
                g_tune_cache[tune_key(B->eng.groups[gi])] = cand[gi][k];
            } catch (const std::bad_alloc &) {
                // the tuned turns are already tracked: keep the choice, uncached
            }
            apply_choice(B, (int)gi, cand[gi][k]);
        }
    }
    B->tuned = true;
    *rc = upload_descs(B);
    return used;
}

// Capture `turns` (even) turns of the batch as a graph (on the private
// stream), the first in launch phase `phase0`.
int batch_capture(mbt_batch *B, int turns, int phase0)
{
    drop_graph(B);
    HIPCHK(B, hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < turns && e == hipSuccess; ++k)
        e = enqueue_turn(B->eng, (phase0 + k) & 1, B->cap, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(B->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return fail(B, MBT_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    B->graph = g;
    HIPCHK(B, hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->exec_turns = turns;
    B->exec_phase = phase0;
    return MBT_OK;
}

}  // namespace

extern "C" {

int mbt_batch_query_bytes(mbt_ctx *const *jobs, int32_t njobs, size_t *work_bytes)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!jobs || njobs < 1 || njobs > 65535 || !work_bytes)
            return MBT_EINVAL;
        for (int j = 0; j < njobs; ++j) {
            if (!jobs[j] || !jobs[j]->bound)
                return MBT_ESTATE;
            if (jobs[j]->static_ws)
                return MBT_EINVAL;  // the static workspace is not a batch job's own
            if (jobs[j]->tr_on)
                return MBT_EINVAL;  // transverse jobs are tracked alone
        }
        size_t a, b, w;
        *work_bytes = batch_layout(jobs, njobs, &a, &b, &w);
        return MBT_OK;
    });
}

int mbt_batch_create(mbt_ctx *const *jobs, int32_t njobs, void *d_work, size_t work_bytes,
                     void *hip_stream, mbt_batch **out)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!out)
            return MBT_EINVAL;
        *out = nullptr;
        size_t need = 0;
        int rc = mbt_batch_query_bytes(jobs, njobs, &need);
        if (rc)
            return rc;
        if (!d_work || ((uintptr_t)d_work & 255))
            return MBT_EINVAL;
        if (work_bytes < need)
            return MBT_ENOSPC;
        for (int j = 0; j < njobs; ++j) {
            if (jobs[j]->device != jobs[0]->device)
                return MBT_EINVAL;
            for (int k = 0; k < j; ++k)
                if (jobs[k] == jobs[j])
                    return MBT_EINVAL;
        }
        mbt_batch *B = new (std::nothrow) mbt_batch();
        if (!B)
            return MBT_ENOMEM;
        B->jobs.assign(jobs, jobs + njobs);
        B->work = reinterpret_cast<unsigned char *>(d_work);
        B->stream = reinterpret_cast<hipStream_t>(hip_stream);
        B->total = batch_layout(jobs, njobs, &B->off_push, &B->off_prep, &B->off_wake, &B->off_ctr);
        // items grouped by long-range count, jobs in the order given
        std::vector<Item> pitems, citems;
        Engine &e = B->eng;
        // the batch's whole particle state is what a turn streams
        size_t state = 0;
        for (int j = 0; j < njobs; ++j)
            state += jobs[j]->L.state_bytes;
        for (int nlr = 0; nlr <= kMaxLR; ++nlr) {
            Group g;
            g.item0 = (int)pitems.size();
            g.nlr = nlr;
            g.map = -1;
            g.stream = stream_rows(state);
            for (int j = 0; j < njobs; ++j) {
                mbt_ctx *c = jobs[j];
                if (c->nlr() != nlr)
                    continue;
                push_items(c, j, pitems);
                g.nbins_max = std::max(g.nbins_max, c->nbins());
                g.nsub_max = std::max(g.nsub_max, c->nsub);
                const int k = map_kind(c);
                g.map = (g.map < 0 || g.map == k) ? k : kMapGeneric;
            }
            if (g.map < 0)
                g.map = kMapGeneric;
            g.nitems = (int)pitems.size() - g.item0;
            g.ctr = reinterpret_cast<uint32_t *>(B->work + B->off_ctr) + 4 * e.groups.size();
            if (g.nitems > 0)
                e.groups.push_back(g);
        }
        for (int j = 0; j < njobs; ++j) {
            if (!mfma_wake(jobs[j]))
                prep_items(jobs[j], j, citems);  // k_wake does a matrix-core job's prep
            e.nlr_max = std::max(e.nlr_max, jobs[j]->nlr());
            e.nbins_max = std::max(e.nbins_max, jobs[j]->nbins());
            B->wake_modes.push_back(jobs[j]->wake_mode);
        }
        // wake items grouped by arithmetic (a template parameter of k_wake)
        std::vector<Item> witems;
        for (int mode = kWakeFP32; mode <= kWakeBF16x3; ++mode) {
            WakeGroup g;
            g.item0 = (int)witems.size();
            g.mode = mode;
            for (int j = 0; j < njobs; ++j)
                if (jobs[j]->sr_on && jobs[j]->wake_mode == mode) {
                    wake_items(jobs[j], j, witems);
                    g.nbins_max = std::max(g.nbins_max, jobs[j]->nbins());
                }
            g.nitems = (int)witems.size() - g.item0;
            if (g.nitems > 0)
                e.wakes.push_back(g);
        }
        if (pitems.size() > (size_t)INT32_MAX || citems.size() > (size_t)INT32_MAX) {
            delete B;
            return MBT_EINVAL;
        }
        e.jobs = reinterpret_cast<const JobDesc *>(B->work);
        e.push_items = reinterpret_cast<const Item *>(B->work + B->off_push);
        e.prep_items = reinterpret_cast<const Item *>(B->work + B->off_prep);
        e.wake_items = reinterpret_cast<const Item *>(B->work + B->off_wake);
        e.njobs = njobs;
        e.nprep = (int)citems.size();
        if (njobs == 1)
            set_one_job(e, jobs[0]);
        auto bail = [&](hipError_t r) {
            std::snprintf(B->err, sizeof B->err, "batch setup failed: %s", hipGetErrorString(r));
            mbt_batch_destroy(B);
            return MBT_EDEVICE;
        };
        hipError_t r;
        if ((r = hipHostMalloc((void **)&B->pin_desc, (size_t)njobs * sizeof(JobDesc), hipHostMallocDefault)) != hipSuccess)
            return bail(r);
        if ((r = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking)) != hipSuccess)
            return bail(r);
        if ((r = hipMemcpyAsync(B->work + B->off_push, pitems.data(), pitems.size() * sizeof(Item),
                                hipMemcpyHostToDevice, B->stream)) != hipSuccess ||
            (r = hipMemcpyAsync(B->work + B->off_prep, citems.data(), citems.size() * sizeof(Item),
                                hipMemcpyHostToDevice, B->stream)) != hipSuccess ||
            (r = hipMemsetAsync(B->work + B->off_ctr, 0, (size_t)(kMaxLR + 1) * 4 * sizeof(uint32_t),
                                B->stream)) != hipSuccess ||
            (!witems.empty() &&
             (r = hipMemcpyAsync(B->work + B->off_wake, witems.data(), witems.size() * sizeof(Item),
                                 hipMemcpyHostToDevice, B->stream)) != hipSuccess) ||
            (r = hipStreamSynchronize(B->stream)) != hipSuccess)
            return bail(r);
        *out = B;
        return MBT_OK;
    });
}

void mbt_batch_destroy(mbt_batch *B)
{
    try {
        if (!B)
            return;
        (void)hipStreamSynchronize(B->stream);
        drop_graph(B);
        timer_free(B->timer);
        if (B->cap)
            (void)hipStreamDestroy(B->cap);
        if (B->pin_desc)
            (void)hipHostFree(B->pin_desc);
        delete B;
    } catch (...) {
        // teardown does not allocate; nothing may leave the ABI
    }
}

const char *mbt_batch_last_error(const mbt_batch *B) { return B ? B->err : "null batch"; }

int mbt_batch_configure(mbt_batch *B, int32_t graph_turns, int32_t autotune)
{
    return guarded(B, [&]() -> int {
        if (!B || graph_turns < 0 || graph_turns > 1024 || (autotune != 0 && autotune != 1))
            return MBT_EINVAL;
        if (graph_turns != B->graph_turns)
            drop_graph(B);
        B->graph_turns = graph_turns;
        B->autotune = autotune == 1;
        return MBT_OK;
    });
}

int mbt_batch_set_timing(mbt_batch *B, int32_t every)
{
    return guarded(B, [&]() -> int {
        if (!B || every < 0)
            return MBT_EINVAL;
        HIPCHK(B, timer_set(B->timer, every));
        return MBT_OK;
    });
}

int mbt_batch_get_timing(const mbt_batch *B, double *push_ms, int64_t *push_launches,
                         double *between_ms, int64_t *between_launches)
{
    if (!B)
        return MBT_EINVAL;
    if (push_ms)
        *push_ms = B->timer.ms[0];
    if (push_launches)
        *push_launches = B->timer.launches[0];
    if (between_ms)
        *between_ms = B->timer.ms[1];
    if (between_launches)
        *between_launches = B->timer.launches[1];
    return MBT_OK;
}

int mbt_batch_launch_info(const mbt_batch *B, int32_t *ngroups, int32_t *nlr, int32_t *nsub,
                          int32_t *grid)
{
    return guarded(static_cast<mbt_ctx *>(nullptr), [&]() -> int {
        if (!B || !ngroups)
            return MBT_EINVAL;
        *ngroups = (int32_t)B->eng.groups.size();
        for (size_t g = 0; g < B->eng.groups.size(); ++g) {
            const Group &G = B->eng.groups[g];
            if (nlr)
                nlr[g] = G.nlr;
            if (nsub)
                nsub[g] = G.nsub_max;
            if (grid)
                grid[g] = G.grid > 0 ? std::min(G.grid, G.nitems) : G.nitems;
        }
        return MBT_OK;
    });
}

int mbt_batch_track(mbt_batch *B, int64_t nturns, mbt_moments *const *out,
                    uint32_t *const *counts, const int32_t *stride)
{
    return guarded(B, [&]() -> int {
        if (!B)
            return MBT_EINVAL;
        const int nj = (int)B->jobs.size();
        if (nturns < 0 || nturns > INT32_MAX)
            return fail(B, MBT_EINVAL, "need 0 <= nturns < 2^31");
        for (int j = 0; j < nj; ++j) {
            mbt_ctx *c = B->jobs[j];
            if (!c->bound || !c->have_particles)
                return fail(B, MBT_ESTATE, "job %d: not bound or particles not initialised", j);
            if (c->turn + nturns > ((int64_t)1 << 32))
                return fail(B, MBT_EINVAL, "job %d: turn counter would pass 2^32", j);
            if (counts && counts[j] && (!c->sr_on || !stride || stride[j] < 1))
                return fail(B, MBT_EINVAL, "job %d: profiles need a grid and stride >= 1", j);
            if (c->wake_mode != B->wake_modes[j])
                return fail(B, MBT_ESTATE, "job %d: wake precision changed after the batch was made", j);
        }
        if (nturns == 0)
            return MBT_OK;
        // per-job strides (0: no profiles)
        std::vector<int32_t> st(nj, 0);
        for (int j = 0; j < nj; ++j)
            st[j] = (counts && counts[j]) ? stride[j] : 0;
        // earlier work on the jobs' own streams first
        for (mbt_ctx *c : B->jobs)
            if (c->stream_h != B->stream)
                HIPCHK(B, hipStreamSynchronize(c->stream_h));
        for (int j = 0; j < nj; ++j) {
            mbt_ctx *c = B->jobs[j];
            int rc = begin_call(c, st[j], B->stream);
            if (rc)
                return fail(B, rc, "job %d: %s", j, c->err);
            ring_start(c->mom, out ? out[j] : nullptr);
            ring_start(c->prof, st[j] ? counts[j] : nullptr);
        }
        // LDS bound of each push group from the jobs' present sub-histogram counts
        for (Group &g : B->eng.groups) {
            int ns = 0;
            for (mbt_ctx *c : B->jobs)
                if (c->nlr() == g.nlr)
                    ns = std::max(ns, c->nsub);
            if (ns != g.nsub_max)
                drop_graph(B);
            g.nsub_max = ns;
        }
        int rc = upload_descs(B);
        if (rc)
            return rc;
        int64_t t = 0;
        if (B->autotune && !B->tuned) {
            t = batch_tune(B, 0, nturns, st.data(), &rc);
            if (rc)
                return rc;
            if (B->tuned)
                drop_graph(B);
        }
        // turns per graph: whole rings' worth of rows at most
        // turns bracketed by timing events are launched eagerly
        int G = B->timer.every > 0 ? 0 : B->graph_turns;
        for (int j = 0; j < nj && G > 0; ++j) {
            mbt_ctx *c = B->jobs[j];
            G = std::min(G, c->L.mom_slots);
            if (st[j])
                G = (int)std::min<int64_t>(G, (int64_t)c->L.prof_slots * st[j]);
        }
        G &= ~1;  // an even number of turns leaves the launch phase where it began
        // capture only when this call replays the graph at least twice (or it is
        // already captured): a capture costs about as much as a few eager turns
        const bool have = B->exec_turns == G && B->exec_phase == (int)(t & 1);
        if (G >= 2 && (have ? t + G <= nturns : t + 2 * G <= nturns)) {
            if (B->exec_turns != G || B->exec_phase != (int)(t & 1))
                if ((rc = batch_capture(B, G, (int)(t & 1))))
                    return rc;
            for (; t + G <= nturns; t += G) {
                if ((rc = batch_rings(B, t, G, st.data())))
                    return rc;
                HIPCHK(B, hipGraphLaunch(B->exec, B->stream));
            }
        }
        for (; t < nturns; ++t) {
            if ((rc = batch_rings(B, t, 1, st.data())))
                return rc;
            const bool timed = B->timer.every > 0 && (t % B->timer.every) == 0;
            HIPCHK(B, enqueue_turn(B->eng, (int)(t & 1), B->stream, timed ? &B->timer : nullptr));
        }
        for (mbt_ctx *c : B->jobs) {
            c->turn += nturns;
            HIPCHK(B, ring_flush(c->mom, B->stream));
            HIPCHK(B, ring_flush(c->prof, B->stream));
        }
        HIPCHK(B, hipStreamSynchronize(B->stream));
        HIPCHK(B, timer_collect(B->timer));
        int bad = -1;
        for (int j = 0; j < nj; ++j) {
            mbt_ctx *c = B->jobs[j];
            HIPCHK(B, ring_land(c->mom));
            HIPCHK(B, ring_land(c->prof));
            uint32_t status = 0;
            HIPCHK(B, hipMemcpy(&status, c->w<uint32_t>(c->L.status), sizeof status, hipMemcpyDeviceToHost));
            if (status) {
                HIPCHK(B, hipMemset(c->w<uint32_t>(c->L.status), 0, sizeof status));
                if (bad < 0)
                    bad = j;
            }
        }
        if (bad >= 0)
            return fail(B, MBT_ENUMERIC, "job %d: non-finite bunch moment", bad);
        return MBT_OK;
    });
}

}  // extern "C"
