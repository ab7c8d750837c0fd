// Host runtime of the droplet-population ensembles (include/dp.h): argument
// checks, the workspace layout, launches and read-back.  Every step of the
// computation runs in the kernels of dp_kernels.hip.
#include "dp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "dp_internal.h"

namespace {

using dp::kMaxMoments;
using dp::kSlots;

thread_local std::string g_err;
std::mutex g_live_mu;
std::set<const void*> g_live;

constexpr int kMaxHistBins = 4096;
constexpr int64_t kMaxSamples = int64_t(1) << 24;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t off_mem = 0, off_order = 0, off_state = 0, off_V = 0, off_slot = 0, off_series = 0, off_statm = 0,
           off_stat = 0, off_hist = 0, total = 0;
};

Layout layout(int32_t m, int64_t total_n, int64_t J)
{
    Layout L;
    size_t o = 0;
    L.off_mem = o;
    o = align_up(o + sizeof(dp::Member) * (size_t)m);
    L.off_order = o;
    o = align_up(o + sizeof(int32_t) * (size_t)m);
    L.off_state = o;
    o = align_up(o + sizeof(dp::State) * (size_t)m);
    L.off_V = o;
    o = align_up(o + sizeof(double) * (size_t)total_n);
    L.off_slot = o;
    o = align_up(o + sizeof(int32_t) * (size_t)total_n);
    L.off_series = o;
    o = align_up(o + sizeof(double) * kSlots * (size_t)m * (size_t)J);
    L.off_statm = o;
    o = align_up(o + sizeof(int32_t) * (size_t)m);
    L.off_stat = o;
    o = align_up(o + sizeof(double) * ((size_t)kMaxMoments * (size_t)J + 2));
    L.off_hist = o;
    o = align_up(o + sizeof(uint64_t) * (kMaxHistBins + 2));
    L.total = o;
    return L;
}

// Checks shared by dp_workspace_bytes and dp_create; J and the droplet total
// on success, a message on failure.
bool check_args(const int32_t* n, int32_t m, const dp_params* prm, int64_t& J, int64_t& total_n,
                std::string& why)
{
    char buf[256];
    if (!n || m < 1 || !prm) {
        why = "need n, m >= 1 and params";
        return false;
    }
    total_n = 0;
    for (int32_t i = 0; i < m; ++i) {
        if (n[i] < 1 || n[i] > dp::kMaxN) {
            snprintf(buf, sizeof buf, "member %d: need 1 <= n <= %d droplets, got %d", i, dp::kMaxN, n[i]);
            why = buf;
            return false;
        }
        total_n += n[i];
    }
    const dp_params& p = *prm;
    if (!(std::isfinite(p.t_end) && p.t_end >= 0.0) || !(std::isfinite(p.dt_sample) && p.dt_sample > 0.0) ||
        !(std::isfinite(p.rtol) && p.rtol > 0.0) || !(std::isfinite(p.atol) && p.atol > 0.0) ||
        !(std::isfinite(p.h0) && p.h0 > 0.0) || p.max_attempts < 1) {
        why = "need t_end >= 0, dt_sample > 0, rtol > 0, atol > 0, h0 > 0 (finite) and max_attempts >= 1";
        return false;
    }
    const double js = p.t_end / p.dt_sample;
    if (js > (double)(kMaxSamples - 1)) {
        snprintf(buf, sizeof buf, "t_end / dt_sample = %g exceeds %lld samples", js, (long long)kMaxSamples);
        why = buf;
        return false;
    }
    J = (int64_t)std::llround(js) + 1;
    return true;
}

}  // namespace

struct dp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    unsigned char* ws = nullptr;
    std::vector<int32_t> n;
    std::vector<int64_t> off;
    dp_params prm{};
    int64_t J = 0;
    int per = 1;
    bool started = false;
    Layout L;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::string err;

    dp::Member* d_mem() { return reinterpret_cast<dp::Member*>(ws + L.off_mem); }
    int32_t* d_order() { return reinterpret_cast<int32_t*>(ws + L.off_order); }
    dp::State* d_state() { return reinterpret_cast<dp::State*>(ws + L.off_state); }
    double* d_V() { return reinterpret_cast<double*>(ws + L.off_V); }
    int32_t* d_slot() { return reinterpret_cast<int32_t*>(ws + L.off_slot); }
    double* d_series() { return reinterpret_cast<double*>(ws + L.off_series); }
    int32_t* d_statm() { return reinterpret_cast<int32_t*>(ws + L.off_statm); }
    double* d_stat() { return reinterpret_cast<double*>(ws + L.off_stat); }
    unsigned long long* d_hist() { return reinterpret_cast<unsigned long long*>(ws + L.off_hist); }

    dp::Args args()
    {
        dp::Args a{};
        a.mem = d_mem();
        a.order = d_order();
        a.st = d_state();
        a.V = d_V();
        a.slot = d_slot();
        a.series = d_series();
        a.J = J;
        a.dts = prm.dt_sample;
        a.rtol = prm.rtol;
        a.atol = prm.atol;
        a.h0 = prm.h0;
        a.max_total = prm.max_attempts;
        return a;
    }
    int32_t m() const { return (int32_t)n.size(); }
};

namespace {

ch_status fail(dp_ctx* ctx, ch_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_err = buf;
    return st;
}

#define DPCHK(ctx, expr)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, CH_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

bool is_live(const dp_ctx* ctx)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(ctx) != 0;
}

ch_status check_ctx(dp_ctx* ctx)
{
    if (!ctx) return fail(nullptr, CH_EINVAL, "ctx is NULL");
    if (!is_live(ctx)) return fail(nullptr, CH_ESTATE, "unknown or destroyed context");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CH_EDEVICE, "hipSetDevice failed");
    return CH_OK;
}

ch_status read_states(dp_ctx* ctx, std::vector<dp::State>& st)
{
    st.resize(ctx->m());
    DPCHK(ctx, hipMemcpyAsync(st.data(), ctx->d_state(), sizeof(dp::State) * st.size(), hipMemcpyDeviceToHost,
                              ctx->stream));
    DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

// Members for a statistics call (uploaded to the workspace) and the samples
// every one of them has recorded.
ch_status stat_setup(dp_ctx* ctx, const int32_t* members, int32_t nm, std::vector<int32_t>& list, int64_t& count)
{
    if (!ctx->started) return fail(ctx, CH_ESTATE, "radii not set");
    if (members) {
        // the device list holds m entries (indices may repeat)
        if (nm < 1 || nm > ctx->m()) return fail(ctx, CH_EINVAL, "need 1 <= nm <= %d, got %d", ctx->m(), nm);
        list.assign(members, members + nm);
        for (int32_t v : list)
            if (v < 0 || v >= ctx->m()) return fail(ctx, CH_EINVAL, "member %d out of range", v);
    } else {
        list.resize(ctx->m());
        std::iota(list.begin(), list.end(), 0);
    }
    std::vector<dp::State> st;
    ch_status s = read_states(ctx, st);
    if (s != CH_OK) return s;
    count = ctx->J;
    for (int32_t v : list) {
        if (st[v].status >= dp::kUnderflow)
            return fail(ctx, st[v].status == dp::kNonFinite ? CH_ENONFINITE : CH_ESTATE,
                        "member %d stopped with state %d", v, st[v].status);
        count = std::min<int64_t>(count, st[v].jn);
    }
    DPCHK(ctx, hipMemcpyAsync(ctx->d_statm(), list.data(), sizeof(int32_t) * list.size(), hipMemcpyHostToDevice,
                              ctx->stream));
    return CH_OK;
}

bool window_range(double dts, int64_t count, double t1, double t2, int64_t& j0, int64_t& j1)
{
    j0 = -1;
    j1 = -1;
    for (int64_t j = 0; j < count; ++j) {
        const double t = (double)j * dts;
        if (t >= t1 && t <= t2) {
            if (j0 < 0) j0 = j;
            j1 = j;
        }
    }
    return j0 >= 0;
}

}  // namespace

extern "C" {

const char* dp_last_error(const dp_ctx* ctx)
{
    if (ctx && is_live(ctx)) return ctx->err.c_str();
    return g_err.c_str();
}

size_t dp_workspace_bytes(const int32_t* n, int32_t m, const dp_params* prm)
{
    int64_t J, total_n;
    std::string why;
    if (!check_args(n, m, prm, J, total_n, why)) return 0;
    return layout(m, total_n, J).total;
}

ch_status dp_create(const int32_t* n, int32_t m, const dp_params* prm, void* d_workspace, size_t ws_bytes,
                    void* hip_stream, dp_ctx** out)
{
    if (!out) return fail(nullptr, CH_EINVAL, "out is NULL");
    *out = nullptr;
    int64_t J, total_n;
    std::string why;
    if (!check_args(n, m, prm, J, total_n, why)) return fail(nullptr, CH_EINVAL, "%s", why.c_str());
    const Layout L = layout(m, total_n, J);
    if (!d_workspace || ((uintptr_t)d_workspace & 255u) != 0)
        return fail(nullptr, CH_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(nullptr, CH_EINVAL, "workspace of %zu bytes, need %zu", ws_bytes, L.total);
    auto* ctx = new dp_ctx;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return fail(nullptr, CH_EDEVICE, "hipGetDevice failed");
    }
    ctx->stream = (hipStream_t)hip_stream;
    ctx->ws = (unsigned char*)d_workspace;
    ctx->n.assign(n, n + m);
    ctx->prm = *prm;
    ctx->J = J;
    ctx->L = L;
    ctx->off.resize(m);
    std::vector<dp::Member> mem(m);
    int64_t o = 0;
    int32_t nmax = 0;
    for (int32_t i = 0; i < m; ++i) {
        ctx->off[i] = o;
        mem[i].off = o;
        mem[i].n = n[i];
        o += n[i];
        nmax = std::max(nmax, n[i]);
    }
    ctx->per = dp::per_thread(nmax);
    // the longest members start first
    std::vector<int32_t> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
    hipError_t e = hipMemcpyAsync(ctx->d_mem(), mem.data(), sizeof(dp::Member) * m, hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->d_order(), order.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev0);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev1);
    if (e != hipSuccess) {
        if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
        delete ctx;
        return fail(nullptr, CH_EDEVICE, "setting up the context failed: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(ctx);
    }
    *out = ctx;
    return CH_OK;
}

ch_status dp_set_radii(dp_ctx* ctx, const double* host_radii)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (!host_radii) return fail(ctx, CH_EINVAL, "radii are NULL");
    const size_t total = (size_t)(ctx->off.back() + ctx->n.back());
    for (size_t i = 0; i < total; ++i)
        if (!std::isfinite(host_radii[i])) return fail(ctx, CH_EINVAL, "radius %zu is not finite", i);
    // the init kernel cubes the radii in place and records sample 0
    DPCHK(ctx, hipMemcpyAsync(ctx->d_V(), host_radii, sizeof(double) * total, hipMemcpyHostToDevice, ctx->stream));
    DPCHK(ctx, dp::launch_init(ctx->args(), ctx->m(), ctx->per, ctx->stream));
    DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->started = true;
    return CH_OK;
}

ch_status dp_advance(dp_ctx* ctx, int64_t attempts)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (!ctx->started) return fail(ctx, CH_ESTATE, "radii not set");
    if (attempts < 1) return fail(ctx, CH_EINVAL, "need attempts >= 1");
    DPCHK(ctx, dp::launch_steps(ctx->args(), ctx->m(), ctx->per, attempts, ctx->stream));
    return CH_OK;
}

ch_status dp_run(dp_ctx* ctx, int64_t attempts, int64_t* launches, double* kernel_ms)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (!ctx->started) return fail(ctx, CH_ESTATE, "radii not set");
    if (attempts < 1) return fail(ctx, CH_EINVAL, "need attempts >= 1");
    int64_t nl = 0;
    double ms = 0.0;
    std::vector<dp::State> s;
    // every launch makes at least one attempt for every running member, and
    // a member stops at max_attempts, so the loop ends
    for (;;) {
        if ((st = read_states(ctx, s)) != CH_OK) return st;
        int32_t bad = -1, running = 0;
        for (int32_t i = 0; i < ctx->m(); ++i) {
            if (s[i].status == dp::kRunning) ++running;
            if (s[i].status >= dp::kUnderflow && bad < 0) bad = i;
        }
        if (launches) *launches = nl;
        if (kernel_ms) *kernel_ms = ms;
        if (bad >= 0) {
            const int32_t code = s[bad].status;
            return fail(ctx, code == dp::kNonFinite ? CH_ENONFINITE : CH_ESTATE,
                        "member %d stopped at t = %.17g: %s", bad, s[bad].t,
                        code == dp::kNonFinite  ? "non-finite error estimate"
                        : code == dp::kUnderflow ? "step size underflow"
                                                 : "attempt limit reached");
        }
        if (running == 0) return CH_OK;
        DPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
        DPCHK(ctx, dp::launch_steps(ctx->args(), ctx->m(), ctx->per, attempts, ctx->stream));
        DPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
        DPCHK(ctx, hipEventSynchronize(ctx->ev1));
        float e = 0.0f;
        DPCHK(ctx, hipEventElapsedTime(&e, ctx->ev0, ctx->ev1));
        ms += e;
        ++nl;
    }
}

ch_status dp_member_info(dp_ctx* ctx, int32_t member, double* t, int64_t* accepted, int64_t* rejected,
                         int32_t* state, int64_t* samples, double* evals)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (member < 0 || member >= ctx->m()) return fail(ctx, CH_EINVAL, "member %d out of range", member);
    if (!ctx->started) return fail(ctx, CH_ESTATE, "radii not set");
    dp::State s;
    DPCHK(ctx, hipMemcpyAsync(&s, ctx->d_state() + member, sizeof s, hipMemcpyDeviceToHost, ctx->stream));
    DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (t) *t = s.t;
    if (accepted) *accepted = s.acc;
    if (rejected) *rejected = s.rej;
    if (state) *state = s.status;
    if (samples) *samples = s.jn;
    if (evals) *evals = s.evals;
    return CH_OK;
}

ch_status dp_get_volumes(dp_ctx* ctx, int32_t member, double* host_dst)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (member < 0 || member >= ctx->m() || !host_dst) return fail(ctx, CH_EINVAL, "bad member or NULL dst");
    if (!ctx->started) return fail(ctx, CH_ESTATE, "radii not set");
    DPCHK(ctx, hipMemcpyAsync(host_dst, ctx->d_V() + ctx->off[member], sizeof(double) * ctx->n[member],
                              hipMemcpyDeviceToHost, ctx->stream));
    DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

ch_status dp_series(dp_ctx* ctx, int32_t member, double* out, int64_t cap, int64_t* count)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (member < 0 || member >= ctx->m() || !out || !count || cap < 0)
        return fail(ctx, CH_EINVAL, "bad member, NULL out/count or cap < 0");
    if (!ctx->started) return fail(ctx, CH_ESTATE, "radii not set");
    dp::State s;
    DPCHK(ctx, hipMemcpyAsync(&s, ctx->d_state() + member, sizeof s, hipMemcpyDeviceToHost, ctx->stream));
    DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t c = std::min<int64_t>(cap, s.jn);
    *count = c;
    if (c > 0) {
        DPCHK(ctx, hipMemcpyAsync(out, ctx->d_series() + (size_t)member * ctx->J * kSlots,
                                  sizeof(double) * kSlots * (size_t)c, hipMemcpyDeviceToHost, ctx->stream));
        DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return CH_OK;
}

ch_status dp_ensemble_moments(dp_ctx* ctx, const int32_t* members, int32_t nm, int32_t pmax, double* t,
                              double* mu, int64_t cap, int64_t* count)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (pmax < 1 || pmax > kMaxMoments || cap < 0 || !mu || !count)
        return fail(ctx, CH_EINVAL, "need 1 <= pmax <= %d, cap >= 0, mu and count", kMaxMoments);
    std::vector<int32_t> list;
    int64_t J;
    if ((st = stat_setup(ctx, members, nm, list, J)) != CH_OK) return st;
    J = std::min<int64_t>(J, cap);
    *count = J;
    if (J > 0) {
        DPCHK(ctx, dp::launch_moments(ctx->d_series(), ctx->J, ctx->d_statm(), (int32_t)list.size(), J, pmax,
                                      ctx->d_stat(), ctx->stream));
        std::vector<double> buf(kMaxMoments * (size_t)J);
        DPCHK(ctx, hipMemcpyAsync(buf.data(), ctx->d_stat(), sizeof(double) * buf.size(), hipMemcpyDeviceToHost,
                                  ctx->stream));
        DPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int64_t j = 0; j < J; ++j) {
            if (t) t[j] = (double)j * ctx->prm.dt_sample;
            for (int p = 0; p < pmax; ++p) mu[j * pmax + p] = buf[j * kMaxMoments + p];
        }
    } else {
        DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return CH_OK;
}

ch_status dp_ensemble_window(dp_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2,
                             double* beta0, double* k)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (!(t1 <= t2)) return fail(ctx, CH_EINVAL, "need t1 <= t2");
    std::vector<int32_t> list;
    int64_t J;
    if ((st = stat_setup(ctx, members, nm, list, J)) != CH_OK) return st;
    int64_t j0, j1;
    double out[2] = {std::nan(""), std::nan("")};
    if (window_range(ctx->prm.dt_sample, J, t1, t2, j0, j1)) {
        double* d_out = ctx->d_stat() + kMaxMoments * (size_t)ctx->J;
        DPCHK(ctx, dp::launch_moments(ctx->d_series(), ctx->J, ctx->d_statm(), (int32_t)list.size(), j1 + 1, 2,
                                      ctx->d_stat(), ctx->stream));
        DPCHK(ctx, dp::launch_window(ctx->d_stat(), j0, j1, ctx->prm.dt_sample, d_out, ctx->stream));
        DPCHK(ctx, hipMemcpyAsync(out, d_out, sizeof out, hipMemcpyDeviceToHost, ctx->stream));
    }
    DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (beta0) *beta0 = out[0];
    if (k) *k = out[1];
    return CH_OK;
}

ch_status dp_beta_histogram(dp_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2, double lo,
                            double hi, int32_t nbins, uint64_t* counts)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (!(t1 <= t2) || !(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi) || nbins < 1 ||
        nbins > kMaxHistBins || !counts)
        return fail(ctx, CH_EINVAL, "need t1 <= t2, finite lo < hi, 1 <= nbins <= %d and counts", kMaxHistBins);
    std::vector<int32_t> list;
    int64_t J;
    if ((st = stat_setup(ctx, members, nm, list, J)) != CH_OK) return st;
    DPCHK(ctx, dp::launch_zero(ctx->d_hist(), nbins + 2, ctx->stream));
    int64_t j0, j1;
    if (window_range(ctx->prm.dt_sample, J, t1, t2, j0, j1))
        DPCHK(ctx, dp::launch_hist(ctx->d_series(), ctx->J, ctx->d_statm(), (int32_t)list.size(), j0, j1, lo, hi,
                                   nbins, ctx->d_hist(), ctx->stream));
    static_assert(sizeof(unsigned long long) == sizeof(uint64_t), "64-bit counters");
    DPCHK(ctx, hipMemcpyAsync(counts, ctx->d_hist(), sizeof(uint64_t) * (nbins + 2), hipMemcpyDeviceToHost,
                              ctx->stream));
    DPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

ch_status dp_destroy(dp_ctx* ctx)
{
    if (!ctx) return fail(nullptr, CH_EINVAL, "ctx is NULL");
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!g_live.erase(ctx)) return fail(nullptr, CH_ESTATE, "unknown or destroyed context");
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipEventDestroy(ctx->ev0);
    (void)hipEventDestroy(ctx->ev1);
    delete ctx;
    return CH_OK;
}

}  // extern "C"
