// mbt_host.cpp -- host runtime behind the C ABI in include/mbt.h.
//
// Validates parameters, derives the turn-map constants, lays out the caller's
// workspace, and drives the per-turn launches on the caller's stream.  The
// turn loop never synchronises with the host: moments and profiles go to
// device rings that are copied to pinned host memory chunk by chunk.
#include "mbt.h"
#include "mbt_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace mbt;

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

// Offsets of every workspace region for a given job shape.
struct Layout {
    size_t W, V, counts, partials, S, seen, gap, qc, phasor, qpp, stream, status, mom, prof;
    size_t total;
    int ring_turns, prof_slots, ntiles;
    int64_t ld;
    size_t state_bytes;
};

Layout make_layout(int M, int64_t N, int nb, int nlr)
{
    Layout L{};
    const int nbx = std::max(nb, 1);
    L.ld = (N + kRowAlign - 1) / kRowAlign * kRowAlign;
    L.ntiles = (int)((N + kTile - 1) / kTile);
    const size_t moment_row = (size_t)M * 4 * sizeof(double);
    L.ring_turns = (int)std::max<size_t>(16, std::min<size_t>(1024, (16u << 20) / moment_row));
    const size_t prof_row = (size_t)M * nbx * sizeof(uint32_t);
    L.prof_slots = (int)std::max<size_t>(1, std::min<size_t>(64, (16u << 20) / prof_row));
    const int nl = std::max(nlr, 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.W = take((size_t)nbx * sizeof(double));
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
    L.status = take(sizeof(uint32_t));
    L.mom = take((size_t)L.ring_turns * moment_row);
    L.prof = take((size_t)L.prof_slots * prof_row);
    L.total = o;
    L.state_bytes = (size_t)2 * M * (size_t)L.ld * sizeof(double);
    return L;
}

// One pending device->pinned->caller copy.
struct Pending {
    hipEvent_t ev = nullptr;
    void *dst = nullptr;
    size_t bytes = 0;
    bool busy = false;
};

}  // namespace

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
    // binding
    bool bound = false;
    int64_t N = 0;
    Layout L{};
    double *tau = nullptr, *delta = nullptr;
    unsigned char *work = nullptr;
    hipStream_t stream_h = nullptr;
    int device = 0;
    // pinned staging (two buffers each for moments and profiles)
    void *pin_mom[2] = {nullptr, nullptr};
    void *pin_prof[2] = {nullptr, nullptr};
    Pending pend_mom[2], pend_prof[2];
    // kernel timing (measurement only)
    int timing_every = 0;
    std::vector<hipEvent_t> ev_push, ev_prep;  // start/end pairs
    int n_push_ev = 0, n_prep_ev = 0;          // pairs recorded in this call
    double push_ms = 0.0, prep_ms = 0.0;
    int64_t push_launches = 0, prep_launches = 0;
    // run state
    bool have_particles = false;
    bool dirty = true;  // partials/histogram do not describe the present state
    int64_t turn = 0;
    uint64_t seed = 0;
    char err[512] = "";

    template <class T> T *w(size_t off) const { return reinterpret_cast<T *>(work + off); }
    int nbins() const { return sr_on ? grid.nbins : 0; }
    int nlr() const { return (int)lr.size(); }
};

namespace {

int fail(mbt_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
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

PushArgs push_args(const mbt_ctx *c, bool for_push)
{
    PushArgs a{};
    a.c = map_const(c);
    a.tau = c->tau;
    a.delta = c->delta;
    a.ld = c->L.ld;
    a.N = c->N;
    a.M = c->M;
    a.ntiles = c->L.ntiles;
    a.nsub = push_nsub(c->nbins());
    a.V = c->w<double>(c->L.V);
    a.seen = c->w<double>(c->L.seen);
    a.stream = c->w<uint32_t>(c->L.stream);
    const int64_t cbuf = for_push ? ((c->turn + 1) & 1) : (c->turn & 1);
    a.counts_out = c->w<uint32_t>(c->L.counts) + (size_t)cbuf * c->M * std::max(c->nbins(), 1);
    a.partials = c->w<double>(c->L.partials);
    a.key0 = (uint32_t)c->seed;
    a.key1 = (uint32_t)(c->seed >> 32);
    a.turn = (uint32_t)c->turn;
    return a;
}

// prep(n) at the present turn n: moments of the state at the start of turn n
// (into mom_out if given), wake potential, phasor scan.
PrepArgs prep_args(const mbt_ctx *c, bool conv, bool scan, double *mom_out)
{
    PrepArgs p{};
    const int nbx = std::max(c->nbins(), 1);
    p.M = c->M;
    p.ntiles = c->L.ntiles;
    p.N = c->N;
    p.nbins = c->nbins();
    p.nlr = c->nlr();
    p.do_conv = (conv && c->sr_on) ? 1 : 0;
    p.do_scan = (scan && c->nlr() > 0) ? 1 : 0;
    p.partials = c->w<double>(c->L.partials);
    p.mom_out = mom_out;
    p.counts_in = c->w<uint32_t>(c->L.counts) + (size_t)(c->turn & 1) * c->M * nbx;
    p.counts_clear = c->w<uint32_t>(c->L.counts) + (size_t)((c->turn + 1) & 1) * c->M * nbx;
    p.W = c->w<double>(c->L.W);
    p.qpp = c->w<double>(c->L.qpp);
    p.V = c->w<double>(c->L.V);
    p.gap = c->w<double>(c->L.gap);
    p.qc = c->w<double>(c->L.qc);
    p.S = c->w<double>(c->L.S);
    p.phasor = c->w<double>(c->L.phasor);
    p.seen = c->w<double>(c->L.seen);
    p.status = c->w<uint32_t>(c->L.status);
    return p;
}

// Bin-only pass over the present state: histogram, deposits and moment sums
// that the next prep consumes.
int prologue(mbt_ctx *c)
{
    if (!c->dirty)
        return MBT_OK;
    const int nbx = std::max(c->nbins(), 1);
    uint32_t *cnt = c->w<uint32_t>(c->L.counts) + (size_t)(c->turn & 1) * c->M * nbx;
    HIPCHK(c, hipMemsetAsync(cnt, 0, (size_t)c->M * nbx * sizeof(uint32_t), c->stream_h));
    HIPCHK(c, launch_push(push_args(c, false), c->nlr(), false, c->stream_h));
    c->dirty = false;
    return MBT_OK;
}

int wait_pending(mbt_ctx *c, Pending &p, const void *src)
{
    if (!p.busy)
        return MBT_OK;
    HIPCHK(c, hipEventSynchronize(p.ev));
    std::memcpy(p.dst, src, p.bytes);
    p.busy = false;
    return MBT_OK;
}

// Copy `bytes` of a device ring to `dst` through pinned buffer `slot`.
int stage_out(mbt_ctx *c, int slot, bool prof, const void *dev, void *dst, size_t bytes)
{
    Pending &p = prof ? c->pend_prof[slot] : c->pend_mom[slot];
    void *pin = prof ? c->pin_prof[slot] : c->pin_mom[slot];
    int rc = wait_pending(c, p, pin);
    if (rc)
        return rc;
    HIPCHK(c, hipMemcpyAsync(pin, dev, bytes, hipMemcpyDeviceToHost, c->stream_h));
    HIPCHK(c, hipEventRecord(p.ev, c->stream_h));
    p.dst = dst;
    p.bytes = bytes;
    p.busy = true;
    return MBT_OK;
}

int drain(mbt_ctx *c)
{
    for (int i = 0; i < 2; ++i) {
        int rc = wait_pending(c, c->pend_mom[i], c->pin_mom[i]);
        if (rc)
            return rc;
        rc = wait_pending(c, c->pend_prof[i], c->pin_prof[i]);
        if (rc)
            return rc;
    }
    return MBT_OK;
}

constexpr int kMaxTimed = 4096;

void destroy_timing_events(mbt_ctx *c)
{
    for (hipEvent_t e : c->ev_push)
        (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_prep)
        (void)hipEventDestroy(e);
    c->ev_push.clear();
    c->ev_prep.clear();
}

// Launch helpers that bracket a launch with a timing event pair when asked.
int timed_push(mbt_ctx *c, bool timed)
{
    const bool t = timed && c->n_push_ev < kMaxTimed;
    if (t)
        HIPCHK(c, hipEventRecord(c->ev_push[2 * c->n_push_ev], c->stream_h));
    HIPCHK(c, launch_push(push_args(c, true), c->nlr(), true, c->stream_h));
    if (t)
        HIPCHK(c, hipEventRecord(c->ev_push[2 * c->n_push_ev++ + 1], c->stream_h));
    return MBT_OK;
}

int timed_prep(mbt_ctx *c, bool timed, double *slot)
{
    const bool t = timed && c->n_prep_ev < kMaxTimed;
    if (t)
        HIPCHK(c, hipEventRecord(c->ev_prep[2 * c->n_prep_ev], c->stream_h));
    HIPCHK(c, launch_prep(prep_args(c, true, true, slot), c->stream_h));
    if (t)
        HIPCHK(c, hipEventRecord(c->ev_prep[2 * c->n_prep_ev++ + 1], c->stream_h));
    return MBT_OK;
}

// After the stream has drained: add the recorded pairs to the totals.
int collect_timing(mbt_ctx *c)
{
    for (int i = 0; i < c->n_push_ev; ++i) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_push[2 * i], c->ev_push[2 * i + 1]));
        c->push_ms += ms;
    }
    for (int i = 0; i < c->n_prep_ev; ++i) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_prep[2 * i], c->ev_prep[2 * i + 1]));
        c->prep_ms += ms;
    }
    c->push_launches += c->n_push_ev;
    c->prep_launches += c->n_prep_ev;
    c->n_push_ev = c->n_prep_ev = 0;
    return MBT_OK;
}

void release_binding(mbt_ctx *c)
{
    if (c->bound)
        (void)hipStreamSynchronize(c->stream_h);
    for (int i = 0; i < 2; ++i) {
        if (c->pin_mom[i])
            (void)hipHostFree(c->pin_mom[i]);
        if (c->pin_prof[i])
            (void)hipHostFree(c->pin_prof[i]);
        c->pin_mom[i] = c->pin_prof[i] = nullptr;
        if (c->pend_mom[i].ev)
            (void)hipEventDestroy(c->pend_mom[i].ev);
        if (c->pend_prof[i].ev)
            (void)hipEventDestroy(c->pend_prof[i].ev);
        c->pend_mom[i] = Pending{};
        c->pend_prof[i] = Pending{};
    }
    c->bound = false;
}

int need_bound(mbt_ctx *c)
{
    if (!c)
        return MBT_EINVAL;
    if (!c->bound)
        return fail(c, MBT_ESTATE, "context not bound: call mbt_bind first");
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
}

void mbt_destroy(mbt_ctx *ctx)
{
    if (!ctx)
        return;
    release_binding(ctx);
    destroy_timing_events(ctx);
    delete ctx;
}

int mbt_hc_flat_fraction(const mbt_ring *ring, int32_t n, double frac, mbt_hc *out)
{
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
}

int mbt_set_harmonic_cavity(mbt_ctx *c, const mbt_hc *hc)
{
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
}

int mbt_set_fill(mbt_ctx *c, int32_t M, const int32_t *bucket, const double *current_A,
                 const int32_t *stream)
{
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
    c->M = M;
    c->bucket.assign(bucket, bucket + M);
    c->current.assign(current_A, current_A + M);
    c->stream.resize(M);
    for (int b = 0; b < M; ++b)
        c->stream[b] = stream ? stream[b] : b;
    return MBT_OK;
}

int mbt_set_short_range(mbt_ctx *c, int32_t nres, const mbt_resonator *res, const mbt_grid *g)
{
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
    c->sr_on = true;
    c->grid = *g;
    c->sr.clear();
    for (int i = 0; i < nres; ++i)
        c->sr.push_back({res[i].rs_ohm, res[i].q, res[i].fr_Hz});
    return MBT_OK;
}

int mbt_set_long_range(mbt_ctx *c, int32_t nres, const mbt_resonator *res)
{
    if (!c)
        return MBT_EINVAL;
    if (c->bound)
        return fail(c, MBT_ESTATE, "wakes must be set before mbt_bind");
    if (nres < 0 || nres > MBT_MAX_LONG_RANGE || (nres > 0 && !res))
        return fail(c, MBT_EINVAL, "need 0 <= nres <= %d", MBT_MAX_LONG_RANGE);
    for (int i = 0; i < nres; ++i)
        if (!res_valid(res[i]))
            return fail(c, MBT_EINVAL, "resonator %d: need Rs >= 0, Q > 0.5, fr > 0", i);
    c->lr.clear();
    for (int i = 0; i < nres; ++i)
        c->lr.push_back({res[i].rs_ohm, res[i].q, res[i].fr_Hz});
    return MBT_OK;
}

int mbt_query_bytes(const mbt_ctx *c, int64_t N, size_t *state_bytes, size_t *work_bytes)
{
    if (!c || !state_bytes || !work_bytes)
        return MBT_EINVAL;
    if (c->M < 1)
        return MBT_ESTATE;
    if (N < 1 || N > ((int64_t)1 << 32))
        return MBT_EINVAL;
    Layout L = make_layout(c->M, N, c->nbins(), c->nlr());
    *state_bytes = L.state_bytes;
    *work_bytes = L.total;
    return MBT_OK;
}

int mbt_bind(mbt_ctx *c, int64_t N, void *d_state, size_t state_bytes, void *d_work,
             size_t work_bytes, void *hip_stream)
{
    if (!c)
        return MBT_EINVAL;
    if (c->M < 1)
        return fail(c, MBT_ESTATE, "fill not set");
    if (N < 1 || N > ((int64_t)1 << 32))
        return fail(c, MBT_EINVAL, "N must be in [1, 2^32]");
    if (!d_state || !d_work || ((uintptr_t)d_state & 255) || ((uintptr_t)d_work & 255))
        return fail(c, MBT_EINVAL, "device buffers must be non-null and 256-byte aligned");
    Layout L = make_layout(c->M, N, c->nbins(), c->nlr());
    if (state_bytes < L.state_bytes || work_bytes < L.total)
        return fail(c, MBT_ENOSPC, "need %zu state and %zu workspace bytes", L.state_bytes, L.total);
    release_binding(c);
    c->L = L;
    c->N = N;
    c->tau = reinterpret_cast<double *>(d_state);
    c->delta = c->tau + (size_t)c->M * L.ld;
    c->work = reinterpret_cast<unsigned char *>(d_work);
    c->stream_h = reinterpret_cast<hipStream_t>(hip_stream);
    HIPCHK(c, hipGetDevice(&c->device));

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
    HIPCHK(c, hipMemsetAsync(d_state, 0, L.state_bytes, c->stream_h));
    HIPCHK(c, hipStreamSynchronize(c->stream_h));
    const size_t mom_bytes = (size_t)L.ring_turns * M * 4 * sizeof(double);
    const size_t prof_bytes = (size_t)L.prof_slots * M * nbx * sizeof(uint32_t);
    for (int i = 0; i < 2; ++i) {
        HIPCHK(c, hipHostMalloc(&c->pin_mom[i], mom_bytes, hipHostMallocDefault));
        HIPCHK(c, hipHostMalloc(&c->pin_prof[i], prof_bytes, hipHostMallocDefault));
        HIPCHK(c, hipEventCreateWithFlags(&c->pend_mom[i].ev, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->pend_prof[i].ev, hipEventDisableTiming));
    }
    c->bound = true;
    c->have_particles = false;
    c->dirty = true;
    c->turn = 0;
    return MBT_OK;
}

int mbt_init_gaussian(mbt_ctx *c, double sigma_tau_s, double sigma_delta, uint64_t seed)
{
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
    c->seed = seed;
    c->turn = 0;
    c->have_particles = true;
    c->dirty = true;
    return MBT_OK;
}

int mbt_set_particles(mbt_ctx *c, int32_t bunch, const double *tau, const double *delta,
                      int32_t where)
{
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
}

int mbt_get_particles(mbt_ctx *c, int32_t bunch, double *tau, double *delta, int32_t where)
{
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
}

int mbt_track(mbt_ctx *c, int64_t nturns, mbt_moments *out, uint32_t *counts, int32_t stride)
{
    int rc = need_bound(c);
    if (rc)
        return rc;
    if (!c->have_particles)
        return fail(c, MBT_ESTATE, "particles not initialised");
    if (nturns < 0 || c->turn + nturns > ((int64_t)1 << 32))
        return fail(c, MBT_EINVAL, "turn counter would pass 2^32");
    if (counts && (!c->sr_on || stride < 1))
        return fail(c, MBT_EINVAL, "profiles need a grid and stride >= 1");
    if (nturns == 0)
        return MBT_OK;
    rc = prologue(c);
    if (rc)
        return rc;
    const int M = c->M, nbx = std::max(c->nbins(), 1);
    const int K = c->L.ring_turns, P = c->L.prof_slots;
    const size_t mom_row = (size_t)M * 4 * sizeof(double);
    const size_t prof_row = (size_t)M * nbx * sizeof(uint32_t);
    double *ring = c->w<double>(c->L.mom);
    uint32_t *pring = c->w<uint32_t>(c->L.prof);
    int mom_chunk = 0, prof_chunk = 0;
    int64_t mom_from = 0;   // first turn of the moment chunk being filled
    int64_t prof_from = 0;  // first profile row of the chunk being filled
    int64_t prof_rows = 0;

    for (int64_t t = 0; t < nturns; ++t) {
        const bool timed = c->timing_every > 0 && (t % c->timing_every) == 0;
        // prep(n): moments of the state after turn t-1 of this call
        double *slot = (out && t > 0) ? ring + (size_t)((t - 1) % K) * M * 4 : nullptr;
        rc = timed_prep(c, timed, slot);
        if (rc)
            return rc;
        if (out && t > 0 && (t - 1) % K == K - 1) {
            rc = stage_out(c, mom_chunk & 1, false, ring, out + (size_t)mom_from * M,
                           (size_t)K * mom_row);
            if (rc)
                return rc;
            ++mom_chunk;
            mom_from = t;
        }
        rc = timed_push(c, timed);
        if (rc)
            return rc;
        c->turn += 1;
        if (counts && t % stride == 0) {
            const uint32_t *src = c->w<uint32_t>(c->L.counts) + (size_t)(c->turn & 1) * M * nbx;
            const int64_t row = t / stride;
            HIPCHK(c, hipMemcpyAsync(pring + (size_t)(row % P) * M * nbx, src, prof_row,
                                     hipMemcpyDeviceToDevice, c->stream_h));
            ++prof_rows;
            if (row % P == P - 1) {
                rc = stage_out(c, prof_chunk & 1, true, pring,
                               counts + (size_t)prof_from * M * nbx, (size_t)P * prof_row);
                if (rc)
                    return rc;
                ++prof_chunk;
                prof_from = row + 1;
            }
        }
    }
    // Moments of the final state.
    double *slot = out ? ring + (size_t)((nturns - 1) % K) * M * 4 : nullptr;
    HIPCHK(c, launch_prep(prep_args(c, false, false, slot), c->stream_h));
    if (out && nturns > mom_from)
        rc = stage_out(c, mom_chunk & 1, false, ring, out + (size_t)mom_from * M,
                       (size_t)(nturns - mom_from) * mom_row);
    if (rc)
        return rc;
    if (counts && prof_rows > prof_from)
        rc = stage_out(c, prof_chunk & 1, true, pring, counts + (size_t)prof_from * M * nbx,
                       (size_t)(prof_rows - prof_from) * prof_row);
    if (rc)
        return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream_h));
    rc = drain(c);
    if (rc)
        return rc;
    rc = collect_timing(c);
    if (rc)
        return rc;
    uint32_t status = 0;
    HIPCHK(c, hipMemcpy(&status, c->w<uint32_t>(c->L.status), sizeof status, hipMemcpyDeviceToHost));
    if (status) {
        HIPCHK(c, hipMemset(c->w<uint32_t>(c->L.status), 0, sizeof status));
        return fail(c, MBT_ENUMERIC, "non-finite bunch moment during turns %lld..%lld",
                    (long long)(c->turn - nturns), (long long)(c->turn - 1));
    }
    return MBT_OK;
}

int mbt_profile(mbt_ctx *c, uint32_t *counts)
{
    int rc = need_bound(c);
    if (rc)
        return rc;
    if (!counts || !c->sr_on)
        return fail(c, MBT_EINVAL, "need a grid and an output array");
    if (!c->have_particles)
        return fail(c, MBT_ESTATE, "particles not initialised");
    rc = prologue(c);
    if (rc)
        return rc;
    const size_t bytes = (size_t)c->M * c->nbins() * sizeof(uint32_t);
    HIPCHK(c, hipMemcpyAsync(counts, c->w<uint32_t>(c->L.counts) + (size_t)(c->turn & 1) * c->M * c->nbins(),
                             bytes, hipMemcpyDeviceToHost, c->stream_h));
    HIPCHK(c, hipStreamSynchronize(c->stream_h));
    return MBT_OK;
}

int mbt_wake_potential(mbt_ctx *c, double *V)
{
    int rc = need_bound(c);
    if (rc)
        return rc;
    if (!V || !c->sr_on)
        return fail(c, MBT_EINVAL, "need a grid and an output array");
    if (!c->have_particles)
        return fail(c, MBT_ESTATE, "particles not initialised");
    rc = prologue(c);
    if (rc)
        return rc;
    HIPCHK(c, launch_prep(prep_args(c, true, false, nullptr), c->stream_h));
    HIPCHK(c, hipMemcpyAsync(V, c->w<double>(c->L.V), (size_t)c->M * c->nbins() * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream_h));
    HIPCHK(c, hipStreamSynchronize(c->stream_h));
    return MBT_OK;
}

int mbt_wake_table(const mbt_ctx *c, double *W)
{
    if (!c || !W)
        return MBT_EINVAL;
    if (!c->bound || !c->sr_on)
        return MBT_ESTATE;
    if (hipMemcpy(W, c->w<double>(c->L.W), (size_t)c->nbins() * sizeof(double),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return MBT_EDEVICE;
    return MBT_OK;
}

int mbt_get_state(mbt_ctx *c, int64_t *turn, uint64_t *seed, double *phasors)
{
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
}

int mbt_set_state(mbt_ctx *c, int64_t turn, uint64_t seed, const double *phasors)
{
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
}

int mbt_set_timing(mbt_ctx *c, int32_t every)
{
    if (!c || every < 0)
        return MBT_EINVAL;
    c->timing_every = every;
    c->push_ms = c->prep_ms = 0.0;
    c->push_launches = c->prep_launches = 0;
    c->n_push_ev = c->n_prep_ev = 0;
    if (every > 0 && c->ev_push.empty()) {
        c->ev_push.resize(2 * kMaxTimed);
        c->ev_prep.resize(2 * kMaxTimed);
        for (hipEvent_t &e : c->ev_push)
            HIPCHK(c, hipEventCreate(&e));
        for (hipEvent_t &e : c->ev_prep)
            HIPCHK(c, hipEventCreate(&e));
    }
    return MBT_OK;
}

int mbt_get_timing(const mbt_ctx *c, double *push_ms, int64_t *push_launches, double *prep_ms,
                   int64_t *prep_launches)
{
    if (!c)
        return MBT_EINVAL;
    if (push_ms)
        *push_ms = c->push_ms;
    if (push_launches)
        *push_launches = c->push_launches;
    if (prep_ms)
        *prep_ms = c->prep_ms;
    if (prep_launches)
        *prep_launches = c->prep_launches;
    return MBT_OK;
}

int mbt_philox4x32_10(int64_t n, const uint32_t *ctr, uint32_t key0, uint32_t key1, uint32_t *out,
                      void *hip_stream)
{
    if (n < 0 || (n > 0 && (!ctr || !out)))
        return MBT_EINVAL;
    if (launch_philox(n, ctr, key0, key1, out, reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return MBT_EDEVICE;
    return MBT_OK;
}

}  // extern "C"
