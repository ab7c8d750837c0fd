// Host runtime of libch.so: argument validation, size classes and tile plans,
// workspace layout, line-solve coefficients, launch sequencing, HIP graphs and
// the autotuner.  All device work is done by the kernels in ch_kernels.hip.
#include "../../include/ch.h"
#include "ch_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

using namespace chk;

namespace {

thread_local std::string g_err;
std::mutex g_live_mu;
std::set<const void*> g_live;  // contexts created and not yet destroyed

bool is_live(const void* p)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(p) != 0;
}

constexpr size_t kAlign = 256;
constexpr size_t kLdsLimit = 160 * 1024 - 1024;  // gfx950: 160 KiB per workgroup, minus statics
// The size classes of a step run on up to kMaxStreams streams; the class
// with the most sites among those of at least 2 * kMinSplit members is split
// in two while there are fewer classes than streams.
constexpr int kMaxStreams = 4;
constexpr int kMaxHistBins = 4096;
constexpr int kMinSplit = 4;
constexpr int64_t kMaxBlocks = (int64_t)1 << 31;  // kernels index blocks in 32 bits

size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

struct ColPlan {
    int cy = 0, b = 0, P = 0;
    int64_t cols = 0, stride = 0, run = 0, outer = 0, nblocks = 0;
};

struct ClassPlan {
    int dim = 2, nx = 0, ny = 0, nz = 1;
    std::vector<int> members;
    int nfixed = 0;  // member count of a plan built without a member list (ch_step_static)
    bool cn = false; // Crank-Nicolson variant of the scheme (theta = 1/2; 2D)
    // pass A
    int cx = 0, rl = 1, waves = 4, units = 1, P = 0, rpw = 0, R = 0, bands = 0, pitch = 0;
    int wl = 0;          // wavefronts per x-line (0: a line within one wavefront, P <= 64)
    bool split = false;  // RHS tile pass, then the x-solve in place (wide FP64 lines; units = 0)
    int64_t bpmA = 0;  // pass-A blocks per member
    int64_t bpmP = 0;  // diagnostics partials per member (pass-A blocks, or RHS tiles of the split form)
    int64_t nblocksA = 0;
    size_t ldsA = 0;
    ColPlan col[3];  // [1] = y, [2] = z
    // workspace
    size_t off_mids = 0, off_partials = 0;
    int64_t partial_cap = 0;  // blocks
};

struct Layout {
    size_t off_mem = 0, off_C = 0, off_W = 0, off_steps = 0, off_nstamp = 0, off_flags = 0;
    size_t off_series = 0, off_energy = 0, off_beta = 0, total = 0;
    size_t off_statm = 0, off_stat = 0, off_hist = 0;  // ensemble statistics
    int64_t total_elems = 0;
    std::vector<int64_t> moff;  // element offset per member
};

int elem_size(int prec) { return prec == 0 ? 8 : 4; }

int64_t class_size(const ClassPlan& c) { return c.nfixed > 0 ? c.nfixed : (int64_t)c.members.size(); }

int lds_pos(int xx, int cx, int pad) { return xx + (xx / cx) * pad; }

int64_t split_tiles(int nx, int ny) { return (int64_t)(nx / kTileX) * ((ny + kTileY - 1) / kTileY); }

// x-lines of more than 64 chunks: a line spans P / 64 wavefronts of a
// 4-wavefront block (2D, one line per lane, one unit per block).  units = 0
// asks for the split form.
bool planA_wide(ClassPlan& c, int prec, int cx, int rl, int waves, int units)
{
    const int P = c.nx / cx;
    const bool split = units == 0;
    if (c.dim != 2 || c.cn || rl != 1 || waves != kPassAThreads / 64 || (units != 1 && !split)) return false;
    if (P % 64 || !passA_wide_has(prec, cx, P / 64, split)) return false;
    if (split && c.nx % kTileX) return false;
    const int wl = P / 64;
    const int R = waves / wl;
    const int pad = passA_pad(prec), halo = passA_halo(prec);
    if (cx % halo) return false;
    const int pitch = lds_pos(c.nx + 2 * halo - 1, cx, pad) + 1;
    // staged rows: the R lines and their stencil rows, or (split) the lines only
    const size_t lds = (size_t)(split ? R : R + 3) * pitch * elem_size(prec);
    if (lds > kLdsLimit) return false;
    c.cx = cx;
    c.rl = 1;
    c.waves = waves;
    c.units = units;
    c.P = P;
    c.rpw = 0;
    c.R = R;
    c.wl = wl;
    c.split = split;
    c.bands = (c.ny + R - 1) / R;
    c.pitch = pitch;
    c.ldsA = lds;
    c.bpmA = c.bands;
    c.bpmP = split ? split_tiles(c.nx, c.ny) : c.bpmA;
    c.nblocksA = class_size(c) * c.bpmA;
    return c.nblocksA < kMaxBlocks && class_size(c) * c.bpmP < kMaxBlocks;
}

bool planA(ClassPlan& c, int prec, int cx, int rl, int waves, int units)
{
    if (cx < 1 || c.nx % cx) return false;
    const int P = c.nx / cx;
    if (P > 64) return planA_wide(c, prec, cx, rl, waves, units);
    if (!passA_has(c.dim, cx, rl, units, c.cn)) return false;
    if (P < 1) return false;
    if (waves < 1 || waves > kPassAThreads / 64) return false;
    const int rpw = (64 / P) * rl;
    const int R = waves * rpw;
    const int pad = passA_pad(prec), halo = passA_halo(prec);
    if (cx % halo) return false;
    const int pitch = lds_pos(c.nx + 2 * halo - 1, cx, pad) + 1;
    const int planes = c.dim == 3 ? 4 : 1;
    const size_t lds = (size_t)planes * (R + (c.cn ? 4 : 3)) * pitch * elem_size(prec);
    if (lds > kLdsLimit) return false;
    if (units > 1) {
        // a wavefront's share of the plane a unit adds must fit the prefetch
        // registers (rows round-robin over wavefronts, 64-vector segments per
        // row), and the halo vectors one per thread
        const int rows = R + 3;
        const int nseg = (c.nx / halo + 63) / 64;
        if ((rows + waves - 1) / waves * nseg > kPrefetchVecs) return false;
        if (2 * rows > 64 * waves) return false;
    }
    c.cx = cx;
    c.rl = rl;
    c.waves = waves;
    c.units = units;
    c.P = P;
    c.rpw = rpw;
    c.R = R;
    c.wl = 0;
    c.split = false;
    c.bands = (c.ny + R - 1) / R;
    c.pitch = pitch;
    c.ldsA = lds;
    if (c.dim == 2)
        c.bpmA = (c.bands + units - 1) / units;
    else
        c.bpmA = (int64_t)c.bands * ((c.nz + units - 1) / units);
    c.bpmP = c.bpmA;
    c.nblocksA = class_size(c) * c.bpmA;
    return c.nblocksA < kMaxBlocks;
}

bool planCol(ClassPlan& c, int prec, int axis, int cy, int b)
{
    ColPlan& p = c.col[axis];
    const int n = axis == 1 ? c.ny : c.nz;
    if (!col_has(prec, cy) || n % cy) return false;
    const int P = n / cy;
    // a block's b columns must be contiguous in memory: y-lines (and 2D) run
    // along x only, z-lines along the whole x-y plane
    const int64_t run = axis == 1 ? c.nx : (int64_t)c.nx * c.ny;
    if (P > (1 << kMaxScanLevels)) return false;  // the chunk scan has kMaxScanLevels levels
    if (b < 1 || (b & (b - 1)) || run % b || b * P > kColMaxThreads) return false;
    p.cy = cy;
    p.b = b;
    p.P = P;
    p.run = run;
    if (axis == 1) {
        p.stride = c.nx;
        p.cols = (int64_t)c.nx * c.nz;
        p.outer = (int64_t)c.nx * c.ny;
    } else {
        p.stride = (int64_t)c.nx * c.ny;
        p.cols = (int64_t)c.nx * c.ny;
        p.outer = run;
    }
    p.nblocks = class_size(c) * (p.cols / b);
    return p.nblocks < kMaxBlocks;
}

bool default_A(ClassPlan& c, int prec)
{
    const int prefs[][2] = {{16, 2}, {16, 1}, {8, 2}, {8, 1}, {32, 1}, {4, 2}, {4, 1}, {32, 2},
                            {64, 1}, {4, 4}, {8, 4}, {16, 4}};
    const int units = c.dim == 3 ? 8 : 1;
    for (int waves : {4, 2, 1})
        for (auto& p : prefs)
            if (planA(c, prec, p[0], p[1], waves, units) || planA(c, prec, p[0], p[1], waves, 1))
                return true;
    // lines longer than 64 chunks of 64 (2D): the widest chunks that fit,
    // staged whole or (FP64) in the split form
    for (int cx : {32, 16, 8, 4})
        if (planA(c, prec, cx, 1, kPassAThreads / 64, 1) || planA(c, prec, cx, 1, kPassAThreads / 64, 0))
            return true;
    return false;
}

int best_b(int64_t run, int P)
{
    int b = 1;
    for (int t = 2; t <= 64; t *= 2)
        if (run % t == 0 && t * P <= kColMaxThreads) b = t;
    return b;
}

bool default_col(ClassPlan& c, int prec, int axis)
{
    const int n = axis == 1 ? c.ny : c.nz;
    const int prefs[] = {16, 32, 8, 64, 4};
    int bestcy = 0, bestb = 0, bestscore = -1;
    for (int cy : prefs) {
        if (!col_has(prec, cy) || n % cy) continue;
        const int P = n / cy;
        if (P > (1 << kMaxScanLevels)) continue;
        const int b = best_b(axis == 1 ? (int64_t)c.nx : (int64_t)c.nx * c.ny, P);
        if (b * P > kColMaxThreads) continue;
        const int score = std::min(b * elem_size(prec), 256);
        if (score > bestscore) {
            bestscore = score;
            bestcy = cy;
            bestb = b;
        }
    }
    return bestcy && planCol(c, prec, axis, bestcy, bestb);
}

// Grid sizes with a line-solve shape: x-lines of n = c P with P <= 64 chunks
// in one wavefront, or (2D) P = 128 or 256 over several; y- and z-lines of up
// to 256 chunks of a column-sweep chunk length.
bool axis_ok(int n, int axis, int dim, int prec)
{
    if (n < 8 || n > 8192 || n % 4) return false;
    if (axis == 0) {
        for (int c : {4, 8, 16, 32, 64})
            if (n % c == 0 && n / c <= 64 && n <= 4096) return true;
        if (dim == 2)
            for (int c : {4, 8, 16, 32, 64})
                for (int wl : {2, 4})
                    if (n == 64 * wl * c && (passA_wide_has(prec, c, wl, false) || passA_wide_has(prec, c, wl, true)))
                        return true;
        return false;
    }
    for (int c : {4, 8, 16, 32, 64})
        if (col_has(prec, c) && n % c == 0 && n / c <= (1 << kMaxScanLevels)) return true;
    return false;
}

ch_status validate(const ch_member_desc* members, int32_t m, int prec, int32_t cadence,
                   int64_t max_samples, std::string& err)
{
    if (!members || m < 1) {
        err = "members must be non-NULL and m >= 1";
        return CH_EINVAL;
    }
    if (prec != CH_F64 && prec != CH_F32_BULK) {
        err = "unknown precision";
        return CH_EINVAL;
    }
    if (cadence < 1) {
        err = "cadence must be >= 1";
        return CH_EINVAL;
    }
    if (max_samples < 1) {
        err = "max_samples must be >= 1";
        return CH_EINVAL;
    }
    for (int i = 0; i < m; ++i) {
        const ch_member_desc& d = members[i];
        char buf[320];
        if (d.dim != 2 && d.dim != 3) {
            snprintf(buf, sizeof buf, "member %d: dim must be 2 or 3", i);
            err = buf;
            return CH_EINVAL;
        }
        if (d.dim == 2 && d.n[2] != 1) {
            snprintf(buf, sizeof buf, "member %d: n[2] must be 1 in 2D", i);
            err = buf;
            return CH_EINVAL;
        }
        for (int a = 0; a < d.dim; ++a) {
            if (d.n[a] < 1 || !(d.L[a] > 0.0) || !std::isfinite(d.L[a])) {
                snprintf(buf, sizeof buf, "member %d: axis %d needs n >= 1 and finite L > 0", i, a);
                err = buf;
                return CH_EINVAL;
            }
        }
        if (!(d.gamma > 0.0) || !std::isfinite(d.gamma) || !(d.dt > 0.0) || !std::isfinite(d.dt) ||
            !std::isfinite(d.c0) || !std::isfinite(d.noise)) {
            snprintf(buf, sizeof buf, "member %d: gamma, dt must be finite and > 0; c0, noise finite", i);
            err = buf;
            return CH_EINVAL;
        }
        for (int a = 0; a < d.dim; ++a) {
            if (!axis_ok(d.n[a], a, d.dim, prec)) {
                snprintf(buf, sizeof buf,
                         "member %d: n[%d] = %d unsupported (need 8..8192, a multiple of 4; x: n = c*P with "
                         "c in {4,..,64}, P <= 64 (n <= 4096), or in 2D P = 128 or 256 chunks of 4..32; "
                         "y, z: n = c*P, P <= 256)",
                         i, a, d.n[a]);
                err = buf;
                return CH_EUNSUPPORTED;
            }
        }
    }
    return CH_OK;
}

// Root p of rho (z-1)^4 + z^2 inside the unit disk, and the derived recursion
// coefficients, chunk transfer matrices and ring-closure matrix.
void axis_coef(double rho, int n, int chunk, int prec, AxisCoef& out)
{
    typedef long double LD;
    typedef std::complex<LD> CX;
    const LD s = 1.0L / std::sqrt((LD)rho);
    const CX b(2.0L, s);                      // z^2 - (2 + i s) z + 1 = 0
    const CX disc = std::sqrt(b * b - (LD)4.0L);
    const CX big = (std::abs(b + disc) >= std::abs(b - disc)) ? (b + disc) / (LD)2 : (b - disc) / (LD)2;
    const CX p = (LD)1 / big;                 // roots multiply to 1
    LD a1 = 2.0L * p.real(), a2 = -std::norm(p);
    if (prec == 1) {
        a1 = (LD)(float)a1;
        a2 = (LD)(float)a2;
    } else {
        a1 = (LD)(double)a1;
        a2 = (LD)(double)a2;
    }
    const LD q1 = 1.0L - a1 - a2;
    out.a1 = (double)a1;
    out.a2 = (double)a2;
    out.ikappa = (double)(q1 * q1);
    out.inv_n = (double)(1.0L / n);
    {
        LD s0 = 0, s1 = 0;  // zero-state recursion over a chunk of ones
        for (int k = 0; k < chunk; ++k) {
            const LD u = 1.0L + a1 * s0 + a2 * s1;
            s1 = s0;
            s0 = u;
        }
        out.E1[0] = (double)s0;
        out.E1[1] = (double)s1;
    }
    auto mul = [](const LD* A, const LD* B, LD* C) {
        LD c0 = A[0] * B[0] + A[1] * B[2], c1 = A[0] * B[1] + A[1] * B[3];
        LD c2 = A[2] * B[0] + A[3] * B[2], c3 = A[2] * B[1] + A[3] * B[3];
        C[0] = c0;
        C[1] = c1;
        C[2] = c2;
        C[3] = c3;
    };
    const LD A[4] = {a1, a2, 1.0L, 0.0L};
    LD Mc[4] = {1, 0, 0, 1};
    for (int k = 0; k < chunk; ++k) mul(A, Mc, Mc);
    LD pw[4] = {Mc[0], Mc[1], Mc[2], Mc[3]};
    for (int l = 0; l < kMaxScanLevels; ++l) {
        for (int i = 0; i < 4; ++i) out.Mp[l][i] = (double)pw[i];
        mul(pw, pw, pw);
    }
    for (int i = 0; i < 4; ++i) out.M[i] = (double)Mc[i];
    LD An[4] = {1, 0, 0, 1};
    for (int k = 0; k < n; ++k) mul(A, An, An);
    const LD B0 = 1 - An[0], B1 = -An[1], B2 = -An[2], B3 = 1 - An[3];
    const LD det = B0 * B3 - B1 * B2;
    out.W[0] = (double)(B3 / det);
    out.W[1] = (double)(-B1 / det);
    out.W[2] = (double)(-B2 / det);
    out.W[3] = (double)(B0 / det);
}

void build_classes(const ch_member_desc* members, int32_t m, std::vector<ClassPlan>& classes)
{
    std::map<std::vector<int>, int> idx;
    for (int i = 0; i < m; ++i) {
        const ch_member_desc& d = members[i];
        std::vector<int> key = {d.dim, d.n[0], d.n[1], d.dim == 3 ? d.n[2] : 1};
        auto it = idx.find(key);
        if (it == idx.end()) {
            ClassPlan c;
            c.dim = d.dim;
            c.nx = d.n[0];
            c.ny = d.n[1];
            c.nz = d.dim == 3 ? d.n[2] : 1;
            idx[key] = (int)classes.size();
            classes.push_back(c);
            it = idx.find(key);
        }
        classes[it->second].members.push_back(i);
    }
    // Split the largest classes into consecutive runs of members, so that the
    // classes of a step can overlap on separate streams: one class's
    // latency-bound RHS pass with another's bandwidth-bound column sweeps.
    // Largest means most sites, which evens out the streams' work.
    auto sites = [](const ClassPlan& c) { return (double)c.members.size() * c.nx * c.ny * c.nz; };
    while ((int)classes.size() < kMaxStreams) {
        int big = -1;
        for (int c = 0; c < (int)classes.size(); ++c)
            if (classes[c].members.size() >= 2 * (size_t)kMinSplit &&
                (big < 0 || sites(classes[c]) > sites(classes[big])))
                big = c;
        if (big < 0) break;
        ClassPlan second = classes[big];
        const size_t half = classes[big].members.size() / 2;
        second.members.assign(classes[big].members.begin() + half, classes[big].members.end());
        classes[big].members.resize(half);
        classes.insert(classes.begin() + big + 1, second);
    }
}

bool default_plans(std::vector<ClassPlan>& classes, int prec)
{
    for (auto& c : classes) {
        if (!default_A(c, prec)) return false;
        if (!default_col(c, prec, 1)) return false;
        if (c.dim == 3 && !default_col(c, prec, 2)) return false;
    }
    return true;
}

void layout(const ch_member_desc* members, int32_t m, int prec, int64_t max_samples,
            std::vector<ClassPlan>& classes, Layout& L)
{
    size_t o = 0;
    L.off_mem = o;
    o = align_up(o + sizeof(MemberDev) * m);
    for (auto& c : classes) {
        c.off_mids = o;
        o = align_up(o + sizeof(int32_t) * c.members.size());
    }
    L.moff.assign(m, 0);
    int64_t e = 0;
    for (int i = 0; i < m; ++i) {
        const ch_member_desc& d = members[i];
        const int64_t sites = (int64_t)d.n[0] * d.n[1] * (d.dim == 3 ? d.n[2] : 1);
        L.moff[i] = e;
        e += (sites + 63) / 64 * 64;
    }
    L.total_elems = e;
    L.off_C = o;
    o = align_up(o + (size_t)e * elem_size(prec));
    L.off_W = o;
    o = align_up(o + (size_t)e * elem_size(prec));
    for (auto& c : classes) {
        // enough partial slots for the smallest tile (one x-line per block)
        // and for the RHS tiles of the split form
        c.partial_cap = (int64_t)c.members.size() * std::max<int64_t>((int64_t)c.nz * c.ny, split_tiles(c.nx, c.ny));
        c.off_partials = o;
        o = align_up(o + sizeof(double) * 3 * (size_t)c.partial_cap);
    }
    L.off_steps = o;
    o = align_up(o + sizeof(int64_t) * classes.size());
    L.off_nstamp = o;
    o = align_up(o + sizeof(int64_t) * classes.size());
    L.off_flags = o;
    o = align_up(o + sizeof(int32_t) * m);
    L.off_series = o;
    o = align_up(o + sizeof(double) * kSeriesSlots * (size_t)m * max_samples);
    L.off_energy = o;
    o = align_up(o + sizeof(double) * 4 * (size_t)m);
    L.off_beta = o;
    o = align_up(o + sizeof(double) * 6 * (size_t)max_samples);
    L.off_statm = o;
    o = align_up(o + sizeof(int32_t) * m);
    L.off_stat = o;
    o = align_up(o + sizeof(double) * (kMaxMoments * (size_t)max_samples + 2));
    L.off_hist = o;
    o = align_up(o + sizeof(uint64_t) * (kMaxHistBins + 2));
    L.total = o;
}

}  // namespace

struct ch_ctx {
    std::vector<ch_member_desc> desc;
    int prec = 0, conv = 0, K = 10;
    double theta = 1.0;  // 1: implicit ADI; 1/2: Crank-Nicolson ADI (2D)
    int64_t max_samples = 1;
    hipStream_t stream = nullptr;
    // streams of the other size classes (class ci runs on stream ci mod
    // (1 + aux.size()), stream 0 being `stream`), forked from and joined back
    // into `stream` in every step
    std::vector<hipStream_t> aux;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    int device = 0;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout L;
    std::vector<ClassPlan> classes;
    std::vector<MemberDev> mem;
    int64_t step = 0;
    int graph_steps = 16;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int gexec_steps = 0;
    std::string err;
    std::string arch;

    MemberDev* d_mem() { return reinterpret_cast<MemberDev*>(ws + L.off_mem); }
    void* d_C() { return ws + L.off_C; }
    void* d_W() { return ws + L.off_W; }
    int64_t* d_steps() { return reinterpret_cast<int64_t*>(ws + L.off_steps); }
    int64_t* d_nstamp() { return reinterpret_cast<int64_t*>(ws + L.off_nstamp); }
    int32_t* d_flags() { return reinterpret_cast<int32_t*>(ws + L.off_flags); }
    double* d_series() { return reinterpret_cast<double*>(ws + L.off_series); }
    double* d_energy() { return reinterpret_cast<double*>(ws + L.off_energy); }
    double* d_beta() { return reinterpret_cast<double*>(ws + L.off_beta); }
    int32_t* d_statm() { return reinterpret_cast<int32_t*>(ws + L.off_statm); }
    double* d_stat() { return reinterpret_cast<double*>(ws + L.off_stat); }
    uint64_t* d_hist() { return reinterpret_cast<uint64_t*>(ws + L.off_hist); }
};

namespace {

ch_status fail(ch_ctx* ctx, ch_status st, const char* fmt, ...)
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

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, CH_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// Device-table entry of one member: spacings, parameters and the line-solve
// coefficients of every used axis for the chunk lengths of its class plan.
void fill_member(const ch_member_desc& d, int64_t off, const ClassPlan& c, int prec, double theta,
                 MemberDev& md)
{
    md = MemberDev{};
    md.off = off;
    md.sites = (int64_t)d.n[0] * d.n[1] * (d.dim == 3 ? d.n[2] : 1);
    md.vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        const bool used = a < d.dim;
        md.h[a] = used ? d.L[a] / d.n[a] : 1.0;
        md.ih2[a] = used ? 1.0 / (md.h[a] * md.h[a]) : 0.0;
        if (used) md.vol *= md.h[a];
    }
    md.gamma = d.gamma;
    md.dt = d.dt;
    for (int a = 0; a < d.dim; ++a) {
        const double h2 = md.h[a] * md.h[a];
        const double rho = theta * d.gamma * d.dt / (h2 * h2);  // the solves are (I + theta gamma dt D^2)
        const int chunk = a == 0 ? c.cx : c.col[a].cy;
        axis_coef(rho, d.n[a], chunk, prec, md.ax[a]);
        const AxisCoef& x = md.ax[a];
        AxisCoefF& f = md.axf[a];
        f.a1 = (float)x.a1;
        f.a2 = (float)x.a2;
        f.ikappa = (float)x.ikappa;
        f.inv_n = (float)x.inv_n;
        for (int i = 0; i < 2; ++i) f.E1[i] = (float)x.E1[i];
        for (int i = 0; i < 4; ++i) {
            f.M[i] = (float)x.M[i];
            f.W[i] = (float)x.W[i];
            for (int l = 0; l < kMaxScanLevels; ++l) f.Mp[l][i] = (float)x.Mp[l][i];
        }
    }
    const double* ih2 = md.ih2;
    double* rc = md.rc;
    rc[RC_DX] = md.dt * ih2[0];
    rc[RC_DY] = md.dt * ih2[1];
    rc[RC_DZ] = md.dt * ih2[2];
    rc[RC_GXY] = 2.0 * md.gamma * md.dt * ih2[0] * ih2[1];
    rc[RC_GXZ] = 2.0 * md.gamma * md.dt * ih2[0] * ih2[2];
    rc[RC_GYZ] = 2.0 * md.gamma * md.dt * ih2[1] * ih2[2];
    rc[RC_AX4] = md.gamma * md.dt * ih2[0] * ih2[0];
    rc[RC_AY4] = md.gamma * md.dt * ih2[1] * ih2[1];
    rc[RC_IHX2] = ih2[0];
    rc[RC_IHY2] = ih2[1];
    rc[RC_DT] = md.dt;
    rc[RC_TG] = 2.0 * md.gamma * md.dt;
    rc[RC_CXY] = ih2[0] * ih2[1];
    for (int i = 0; i < RC_N; ++i) md.rcf[i] = (float)rc[i];
}

void fill_member_table(ch_ctx* ctx)
{
    const int m = (int)ctx->desc.size();
    ctx->mem.assign(m, MemberDev{});
    for (auto& c : ctx->classes)
        for (int gi : c.members)
            fill_member(ctx->desc[gi], ctx->L.moff[gi], c, ctx->prec, ctx->theta, ctx->mem[gi]);
}

ch_status upload_tables(ch_ctx* ctx)
{
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_mem(), ctx->mem.data(), sizeof(MemberDev) * ctx->mem.size(),
                               hipMemcpyHostToDevice, ctx->stream));
    for (auto& c : ctx->classes) {
        std::vector<int32_t> mids(c.members.begin(), c.members.end());
        HIPCHK(ctx, hipMemcpyAsync(ctx->ws + c.off_mids, mids.data(), sizeof(int32_t) * mids.size(),
                                   hipMemcpyHostToDevice, ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

// The class's members as one arithmetic run (consecutive ids at equally
// spaced offsets), or mid0 = -1.
MemberRun member_run(const ch_ctx* ctx, const ClassPlan& c)
{
    MemberRun r{-1, 0, 0};
    const auto& mv = c.members;
    if (mv.empty()) return r;
    const int64_t off0 = ctx->L.moff[mv[0]];
    const int64_t stride = mv.size() > 1 ? ctx->L.moff[mv[1]] - off0 : 0;
    for (size_t i = 0; i < mv.size(); ++i)
        if (mv[i] != mv[0] + (int)i || ctx->L.moff[mv[i]] != off0 + (int64_t)i * stride) return r;
    r.mid0 = mv[0];
    r.off0 = off0;
    r.stride = stride;
    return r;
}

PassAArgs passA_args(ch_ctx* ctx, int ci, int mode)
{
    ClassPlan& c = ctx->classes[ci];
    PassAArgs a{};
    a.C = ctx->d_C();
    a.W = ctx->d_W();
    a.mem = ctx->d_mem();
    a.mids = reinterpret_cast<const int32_t*>(ctx->ws + c.off_mids);
    a.nmem = (int32_t)c.members.size();
    a.run = member_run(ctx, c);
    a.nx = c.nx;
    a.ny = c.ny;
    a.nz = c.nz;
    a.P = c.P;
    a.rows_per_wave = c.rpw;
    a.waves = c.waves;
    a.R = c.R;
    a.bands_y = c.bands;
    a.units = c.units;
    a.blocks_per_member = c.bpmA;
    a.nblocks = c.nblocksA;
    a.pitch = c.pitch;
    a.mode = mode;
    a.conv = ctx->conv;
    a.K = ctx->K;
    a.cn = c.cn ? 1 : 0;
    a.step = ctx->d_steps() + ci;
    a.partials = reinterpret_cast<double*>(ctx->ws + c.off_partials);
    a.nstamp = ctx->d_nstamp() + ci;
    return a;
}

FinArgs fin_args(ch_ctx* ctx, int ci, int mode)
{
    ClassPlan& c = ctx->classes[ci];
    FinArgs f{};
    f.enabled = 1;
    f.mode = mode;
    f.mem = ctx->d_mem();
    f.mids = reinterpret_cast<const int32_t*>(ctx->ws + c.off_mids);
    f.nmem = (int32_t)c.members.size();
    f.K = ctx->K;
    f.blocks_per_member = c.bpmP;
    f.partials = reinterpret_cast<const double*>(ctx->ws + c.off_partials);
    f.nstamp = ctx->d_nstamp() + ci;
    f.G = (int32_t)std::min<int64_t>(c.members.size(), 1024);
    f.max_samples = ctx->max_samples;
    f.step = ctx->d_steps() + ci;
    f.series = ctx->d_series();
    f.energy_now = ctx->d_energy();
    f.flags = ctx->d_flags();
    return f;
}

ColArgs col_args(ch_ctx* ctx, int ci, int axis, const void* src, void* dst, bool closes_step)
{
    ClassPlan& c = ctx->classes[ci];
    const ColPlan& p = c.col[axis];
    ColArgs a{};
    a.src = src;
    a.dst = dst;
    a.mem = ctx->d_mem();
    a.mids = reinterpret_cast<const int32_t*>(ctx->ws + c.off_mids);
    a.mrun = member_run(ctx, c);
    a.axis = axis;
    a.n = axis == 1 ? c.ny : c.nz;
    a.stride = p.stride;
    a.run = p.run;
    a.outer = p.outer;
    a.cols = p.cols;
    a.msites = (int64_t)c.nx * c.ny * c.nz;
    a.b = p.b;
    a.bshift = __builtin_ctz((unsigned)p.b);
    a.P = p.P;
    a.nblocks = p.nblocks;
    if (closes_step) {
        a.fin = fin_args(ctx, ci, MODE_STEP);
        a.fin.G = (int32_t)std::min<int64_t>(a.fin.G, p.nblocks);
    }
    return a;
}

hipError_t launch_A(ch_ctx* ctx, int ci, int mode, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                    hipStream_t s = nullptr)
{
    ClassPlan& c = ctx->classes[ci];
    PassAArgs a = passA_args(ctx, ci, mode);
    return launch_passA(ctx->prec, c.dim, c.cx, c.rl, c.units, a, c.ldsA, s ? s : ctx->stream, ev0, ev1);
}

// the column sweeps of one step: 2D  w -> C ;  3D  w -> w (y), w -> C (z)
hipError_t launch_cols(ch_ctx* ctx, int ci, int axis, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr, hipStream_t s = nullptr)
{
    ClassPlan& c = ctx->classes[ci];
    void* W = ctx->d_W();
    void* C = ctx->d_C();
    const bool last = (axis == c.dim - 1);
    return launch_col(ctx->prec, c.col[axis].cy, col_args(ctx, ci, axis, W, last ? C : W, last),
                      s ? s : ctx->stream, ev0, ev1);
}

void release_streams(ch_ctx* ctx)
{
    for (hipStream_t s : ctx->aux) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t ev : ctx->ev_join) (void)hipEventDestroy(ev);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    ctx->aux.clear();
    ctx->ev_join.clear();
    ctx->ev_fork = nullptr;
}

// nsteps steps.  Classes are independent (own members, partials, step
// counter), so each class runs all its steps in order on its own stream; the
// other streams are forked from the context stream first and joined back into
// it at the end.  Classes on different streams drift apart in phase, so one
// class's latency-bound RHS pass overlaps another's bandwidth-bound sweeps.
hipError_t enqueue_steps(ch_ctx* ctx, int64_t nsteps)
{
    const int nc = (int)ctx->classes.size();
    const int ns = 1 + (int)ctx->aux.size();
    hipError_t e;
    if (ns > 1) {
        if ((e = hipEventRecord(ctx->ev_fork, ctx->stream)) != hipSuccess) return e;
        for (hipStream_t s : ctx->aux)
            if ((e = hipStreamWaitEvent(s, ctx->ev_fork, 0)) != hipSuccess) return e;
    }
    // step-major order: the launches (and a captured graph's nodes) of the
    // classes interleave, so every stream has work from the first step on
    for (int64_t i = 0; i < nsteps; ++i) {
        for (int ci = 0; ci < nc; ++ci) {
            hipStream_t s = (ci % ns == 0) ? ctx->stream : ctx->aux[ci % ns - 1];
            if ((e = launch_A(ctx, ci, MODE_STEP, nullptr, nullptr, s)) != hipSuccess) return e;
            if ((e = launch_cols(ctx, ci, 1, nullptr, nullptr, s)) != hipSuccess) return e;
            if (ctx->classes[ci].dim == 3 && (e = launch_cols(ctx, ci, 2, nullptr, nullptr, s)) != hipSuccess)
                return e;
        }
    }
    for (int i = 0; i + 1 < ns; ++i) {
        if ((e = hipEventRecord(ctx->ev_join[i], ctx->aux[i])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ctx->stream, ctx->ev_join[i], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// nsteps stand-in steps for tuning, with the stream structure of
// enqueue_steps: pass A in timing mode (reads C, writes the scratch field w,
// no diagnostics) and the column sweeps in place on w.  The state, the step
// counters and the series are untouched.
hipError_t enqueue_timing_steps(ch_ctx* ctx, int nsteps)
{
    const int nc = (int)ctx->classes.size();
    const int ns = 1 + (int)ctx->aux.size();
    void* W = ctx->d_W();
    hipError_t e;
    if (ns > 1) {
        if ((e = hipEventRecord(ctx->ev_fork, ctx->stream)) != hipSuccess) return e;
        for (hipStream_t s : ctx->aux)
            if ((e = hipStreamWaitEvent(s, ctx->ev_fork, 0)) != hipSuccess) return e;
    }
    for (int i = 0; i < nsteps; ++i) {
        for (int ci = 0; ci < nc; ++ci) {
            hipStream_t s = (ci % ns == 0) ? ctx->stream : ctx->aux[ci % ns - 1];
            const ClassPlan& c = ctx->classes[ci];
            if ((e = launch_A(ctx, ci, MODE_TIMING, nullptr, nullptr, s)) != hipSuccess) return e;
            for (int axis = 1; axis < c.dim; ++axis)
                if ((e = launch_col(ctx->prec, c.col[axis].cy, col_args(ctx, ci, axis, W, W, false), s)) !=
                    hipSuccess)
                    return e;
        }
    }
    for (int i = 0; i + 1 < ns; ++i) {
        if ((e = hipEventRecord(ctx->ev_join[i], ctx->aux[i])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ctx->stream, ctx->ev_join[i], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t enqueue_diag(ch_ctx* ctx)
{
    hipError_t e;
    for (int ci = 0; ci < (int)ctx->classes.size(); ++ci) {
        if ((e = launch_A(ctx, ci, MODE_DIAG)) != hipSuccess) return e;
        if ((e = launch_fin(fin_args(ctx, ci, MODE_DIAG), ctx->stream)) != hipSuccess) return e;
    }
    return hipSuccess;
}

void drop_graph(ch_ctx* ctx)
{
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    ctx->gexec_steps = 0;
}

ch_status ensure_graph(ch_ctx* ctx, int steps)
{
    if (ctx->gexec && ctx->gexec_steps == steps) return CH_OK;
    drop_graph(ctx);
    HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_steps(ctx, steps);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(ctx, CH_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    // upload it now, so that its first replay costs no more than later ones
    if (e == hipSuccess) e = hipGraphUpload(ex, ctx->stream);
    if (e != hipSuccess) {
        if (ex) (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return fail(ctx, CH_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    ctx->graph = g;
    ctx->gexec = ex;
    ctx->gexec_steps = steps;
    return CH_OK;
}

bool need_diag(int64_t n, int K)
{
    return (n % K) == 0 || (n >= 1 && ((n - 1) % K) == 0) || (((n + 1) % K) == 0);
}

ch_status check_ctx(ch_ctx* ctx)
{
    if (!ctx) return fail(nullptr, CH_EINVAL, "ctx is NULL");
    if (!is_live(ctx)) return fail(nullptr, CH_ESTATE, "unknown or destroyed context");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(ctx, CH_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    return CH_OK;
}

std::string plan_text(const ch_ctx* ctx)
{
    std::string s;
    char buf[320];
    for (const auto& c : ctx->classes) {
        snprintf(buf, sizeof buf,
                 "%dD %dx%dx%d %s%s x%zu: A cx=%d rl=%d P=%d waves=%d units=%d R=%d blocks=%lld lds=%zu%s",
                 c.dim, c.nx, c.ny, c.nz, ctx->prec ? "f32" : "f64", c.cn ? " cn" : "", c.members.size(), c.cx, c.rl, c.P,
                 c.waves, c.units, c.R, (long long)c.nblocksA, c.ldsA,
                 c.split ? " split" : (c.wl ? " wide" : ""));
        s += buf;
        for (int a = 1; a < c.dim; ++a) {
            snprintf(buf, sizeof buf, " | %c cy=%d P=%d b=%d blocks=%lld", a == 1 ? 'y' : 'z',
                     c.col[a].cy, c.col[a].P, c.col[a].b, (long long)c.col[a].nblocks);
            s += buf;
        }
        s += "\n";
    }
    return s;
}

std::string class_key(const ch_ctx* ctx, const ClassPlan& c)
{
    char buf[128];
    snprintf(buf, sizeof buf, "%s:%s:%dD:%dx%dx%d:m%zu%s", ctx->arch.c_str(), ctx->prec ? "f32" : "f64",
             c.dim, c.nx, c.ny, c.nz, c.members.size(), c.cn ? ":cn" : "");
    return buf;
}

// The fastest few shapes of one class key in isolation: [0] pass A
// (cx, rl, waves, units), [1] y sweep (cy, b), [2] z sweep (cy, b).
struct Shortlist {
    static constexpr size_t kKeep[3] = {3, 2, 2};
    std::vector<std::pair<float, std::vector<int>>> c[3];
    void add(int k, float ms, std::vector<int> shape)
    {
        auto& v = c[k];
        v.emplace_back(ms, std::move(shape));
        std::sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
        if (v.size() > kKeep[k]) v.resize(kKeep[k]);
    }
};

// Validate a member selection (NULL = all members), require a common dt, copy
// the list to the workspace and report the recorded sample count.
ch_status stat_setup(ch_ctx* ctx, const int32_t* members, int32_t nm, int32_t& M, double& dt, int64_t& J)
{
    const int m = (int)ctx->desc.size();
    std::vector<int32_t> sel;
    if (members) {
        // the device list holds m entries (indices may repeat, e.g. a
        // bootstrap resample of the ensemble's own size)
        if (nm < 1 || nm > m) return fail(ctx, CH_EINVAL, "member selection needs 1 <= nm <= %d, got %d", m, nm);
        sel.assign(members, members + nm);
    } else {
        sel.resize(m);
        for (int i = 0; i < m; ++i) sel[i] = i;
    }
    for (int32_t i : sel)
        if (i < 0 || i >= m) return fail(ctx, CH_EINVAL, "member index %d out of range", i);
    dt = ctx->desc[sel[0]].dt;
    for (int32_t i : sel)
        if (ctx->desc[i].dt != dt) return fail(ctx, CH_EINVAL, "selected members have different dt");
    M = (int32_t)sel.size();
    J = std::min<int64_t>(ctx->step / ctx->K + 1, ctx->max_samples);
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_statm(), sel.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice,
                               ctx->stream));
    // the host list must outlive the copy; also the non-finite flags
    std::vector<int32_t> flags(m);
    HIPCHK(ctx, hipMemcpyAsync(flags.data(), ctx->d_flags(), sizeof(int32_t) * m, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int32_t i : sel)
        if (flags[i]) return fail(ctx, CH_ENONFINITE, "non-finite free energy in member %d", i);
    return CH_OK;
}

// first and last recorded samples with t1 <= t_j <= t2, t_j = (jK) dt
bool window_range(const ch_ctx* ctx, double dt, int64_t J, double t1, double t2, int64_t& j0, int64_t& j1)
{
    j0 = -1;
    j1 = -1;
    for (int64_t j = 0; j < J; ++j) {
        const double t = (double)(j * ctx->K) * dt;
        if (t >= t1 && t <= t2) {
            if (j0 < 0) j0 = j;
            j1 = j;
        }
    }
    return j0 >= 0;
}

}  // namespace

// ===========================================================================
// Allocation-free stepping (ch_step_static): its scratch is one static device
// array per GPU.  Host code never passes `scratch` itself to a kernel (in host
// code the name is only a stand-in for the device symbol): the device address
// is taken once per device with hipGetSymbolAddress and kept in
// g_static_ptr, and only that address is used.
// ===========================================================================
static __device__ __align__(256) unsigned char scratch[CH_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;  // guards the per-device addresses and the host staging tables
void* g_static_ptr[kStaticMaxDevices] = {};
// host staging of the member table and class member list (no heap use per call)
MemberDev g_static_mem[CH_STATIC_MAX_MEMBERS];
int32_t g_static_mids[CH_STATIC_MAX_MEMBERS];

// Offsets (bytes) of the parts of the static scratch for one call.
struct StaticLayout {
    size_t mem = 0, mids = 0, W = 0, partials = 0, steps = 0, nstamp = 0, flags = 0, series = 0,
           energy = 0, total = 0;
};

StaticLayout static_layout(const ClassPlan& c, int prec, int32_t m, int64_t sites)
{
    StaticLayout S;
    size_t o = 0;
    S.mem = o;
    o = align_up(o + sizeof(MemberDev) * m);
    S.mids = o;
    o = align_up(o + sizeof(int32_t) * m);
    S.W = o;
    o = align_up(o + (size_t)elem_size(prec) * (size_t)sites * m);
    S.partials = o;
    o = align_up(o + sizeof(double) * 3 * (size_t)(class_size(c) * c.bpmP));
    S.steps = o;
    o = align_up(o + sizeof(int64_t));
    S.nstamp = o;
    o = align_up(o + sizeof(int64_t));
    S.flags = o;
    o = align_up(o + sizeof(int32_t) * m);
    S.series = o;
    o = align_up(o + sizeof(double) * kSeriesSlots * m);  // one sample per member
    S.energy = o;
    o = align_up(o + sizeof(double) * 4 * m);
    S.total = o;
    return S;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ch_version(void) { return "ch-mi355x 0.1"; }

const char* ch_last_error(const ch_ctx* ctx)
{
    if (ctx && is_live(ctx)) return ctx->err.c_str();
    return g_err.c_str();
}

size_t ch_workspace_bytes(const ch_member_desc* members, int32_t m, ch_precision prec,
                          int32_t cadence, int64_t max_samples)
{
    std::string err;
    if (validate(members, m, prec, cadence, max_samples, err) != CH_OK) {
        g_err = err;
        return 0;
    }
    std::vector<ClassPlan> classes;
    build_classes(members, m, classes);
    if (!default_plans(classes, prec)) {
        g_err = "no tile shape fits a size class in LDS";
        return 0;
    }
    Layout L;
    layout(members, m, prec, max_samples, classes, L);
    return L.total;
}

ch_status ch_create(const ch_member_desc* members, int32_t m, ch_precision prec,
                    ch_energy_conv conv, int32_t cadence, int64_t max_samples, void* d_workspace,
                    size_t ws_bytes, void* hip_stream, ch_ctx** out)
{
    if (!out) return fail(nullptr, CH_EINVAL, "out is NULL");
    *out = nullptr;
    std::string err;
    ch_status st = validate(members, m, prec, cadence, max_samples, err);
    if (st != CH_OK) return fail(nullptr, st, "%s", err.c_str());
    if (conv != CH_ENERGY_QUARTER && conv != CH_ENERGY_PAPER_PRINTED)
        return fail(nullptr, CH_EINVAL, "unknown energy convention");
    if (!d_workspace) return fail(nullptr, CH_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return fail(nullptr, CH_EINVAL, "workspace must be 256-byte aligned");

    ch_ctx* ctx = new (std::nothrow) ch_ctx;
    if (!ctx) return fail(nullptr, CH_ENOMEM, "host allocation failed");
    ctx->desc.assign(members, members + m);
    ctx->prec = prec;
    ctx->conv = conv;
    ctx->K = cadence;
    ctx->max_samples = max_samples;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx->ws = reinterpret_cast<char*>(d_workspace);
    ctx->ws_bytes = ws_bytes;
    build_classes(members, m, ctx->classes);
    if (!default_plans(ctx->classes, prec)) {
        delete ctx;
        return fail(nullptr, CH_EUNSUPPORTED, "no tile shape fits a size class in LDS");
    }
    layout(members, m, prec, max_samples, ctx->classes, ctx->L);
    if (ws_bytes < ctx->L.total) {
        size_t need = ctx->L.total;
        delete ctx;
        return fail(nullptr, CH_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    }
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) {
        delete ctx;
        return fail(nullptr, CH_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
        ctx->arch = prop.gcnArchName;
        size_t colon = ctx->arch.find(':');
        if (colon != std::string::npos) ctx->arch.resize(colon);
    }
    const int nstreams = std::min<int>((int)ctx->classes.size(), kMaxStreams);
    if (nstreams > 1) {
        e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
        for (int i = 1; i < nstreams && e == hipSuccess; ++i) {
            hipStream_t s = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e == hipSuccess) ctx->aux.push_back(s);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) ctx->ev_join.push_back(ev);
        }
        if (e != hipSuccess) {
            release_streams(ctx);
            delete ctx;
            return fail(nullptr, CH_EDEVICE, "stream creation failed: %s", hipGetErrorString(e));
        }
    }
    fill_member_table(ctx);
    st = upload_tables(ctx);
    if (st != CH_OK) {
        g_err = ctx->err;
        release_streams(ctx);
        delete ctx;
        return st;
    }
    // zero fields, reset counters and series
    for (int i = 0; i < m; ++i) {
        e = launch_init_member(prec, static_cast<char*>(ctx->d_C()) + ctx->L.moff[i] * elem_size(prec),
                               ctx->mem[i].sites, 0, 0.0, 0.0, ctx->stream);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess)
        e = launch_reset(ctx->d_steps(), (int)ctx->classes.size(), 0, ctx->d_flags(), m,
                         ctx->d_series(), (int64_t)kSeriesSlots * m * max_samples, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        release_streams(ctx);
        delete ctx;
        return fail(nullptr, CH_EDEVICE, "initialisation failed: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(ctx);
    }
    *out = ctx;
    return CH_OK;
}

ch_status ch_init_random(ch_ctx* ctx)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    const int m = (int)ctx->desc.size();
    for (int i = 0; i < m; ++i) {
        const ch_member_desc& d = ctx->desc[i];
        HIPCHK(ctx, launch_init_member(ctx->prec,
                                       static_cast<char*>(ctx->d_C()) + ctx->L.moff[i] * elem_size(ctx->prec),
                                       ctx->mem[i].sites, d.seed, d.c0, d.noise, ctx->stream));
    }
    HIPCHK(ctx, launch_reset(ctx->d_steps(), (int)ctx->classes.size(), 0, ctx->d_flags(), m,
                             ctx->d_series(), (int64_t)kSeriesSlots * m * ctx->max_samples,
                             ctx->stream));
    ctx->step = 0;
    return CH_OK;
}

ch_status ch_set_field(ch_ctx* ctx, int32_t member, const double* src)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (member < 0 || member >= (int)ctx->desc.size() || !src)
        return fail(ctx, CH_EINVAL, "bad member index or NULL source");
    const int64_t sites = ctx->mem[member].sites;
    char* dst = static_cast<char*>(ctx->d_C()) + ctx->L.moff[member] * elem_size(ctx->prec);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->prec == CH_F64) {
        HIPCHK(ctx, hipMemcpyAsync(dst, src, sizeof(double) * sites, hipMemcpyHostToDevice, ctx->stream));
    } else {
        std::vector<float> tmp(sites);
        for (int64_t i = 0; i < sites; ++i) tmp[i] = (float)src[i];
        HIPCHK(ctx, hipMemcpyAsync(dst, tmp.data(), sizeof(float) * sites, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return CH_OK;
}

ch_status ch_get_field(ch_ctx* ctx, int32_t member, double* dst)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (member < 0 || member >= (int)ctx->desc.size() || !dst)
        return fail(ctx, CH_EINVAL, "bad member index or NULL destination");
    const int64_t sites = ctx->mem[member].sites;
    const char* src = static_cast<const char*>(ctx->d_C()) + ctx->L.moff[member] * elem_size(ctx->prec);
    if (ctx->prec == CH_F64) {
        HIPCHK(ctx, hipMemcpyAsync(dst, src, sizeof(double) * sites, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    } else {
        std::vector<float> tmp(sites);
        HIPCHK(ctx, hipMemcpyAsync(tmp.data(), src, sizeof(float) * sites, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int64_t i = 0; i < sites; ++i) dst[i] = (double)tmp[i];
    }
    return CH_OK;
}

ch_status ch_get_step(const ch_ctx* ctx, int64_t* n)
{
    if (!ctx || !n) return fail(nullptr, CH_EINVAL, "NULL argument");
    if (!is_live(ctx)) return fail(nullptr, CH_ESTATE, "unknown or destroyed context");
    *n = ctx->step;
    return CH_OK;
}

ch_status ch_set_step(ch_ctx* ctx, int64_t n)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (n < 0) return fail(ctx, CH_EINVAL, "step must be >= 0");
    if (n / ctx->K >= ctx->max_samples) return fail(ctx, CH_ESTATE, "step beyond the sample capacity");
    const int m = (int)ctx->desc.size();
    HIPCHK(ctx, launch_reset(ctx->d_steps(), (int)ctx->classes.size(), n, ctx->d_flags(), 0,
                             ctx->d_series(), (int64_t)kSeriesSlots * m * ctx->max_samples,
                             ctx->stream));
    ctx->step = n;
    return CH_OK;
}

ch_status ch_sync_step(ch_ctx* ctx, int64_t* n)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    int64_t dev = 0;
    HIPCHK(ctx, hipMemcpyAsync(&dev, ctx->d_steps(), sizeof dev, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (dev < 0 || dev / ctx->K >= ctx->max_samples)
        return fail(ctx, CH_ESTATE, "device step counter %lld out of range", (long long)dev);
    ctx->step = dev;
    if (n) *n = dev;
    return CH_OK;
}

ch_status ch_step(ch_ctx* ctx, int64_t nsteps)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (nsteps < 0) return fail(ctx, CH_EINVAL, "nsteps must be >= 0");
    const int64_t target = ctx->step + nsteps;
    if (target / ctx->K >= ctx->max_samples)
        return fail(ctx, CH_ESTATE, "step %lld would exceed max_samples = %lld at cadence %d",
                    (long long)target, (long long)ctx->max_samples, ctx->K);
    int64_t left = nsteps;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHK(ctx, hipStreamIsCapturing(ctx->stream, &cap));
    // the legacy null stream cannot be captured: launch directly there
    const bool use_graph =
        ctx->graph_steps > 0 && cap == hipStreamCaptureStatusNone && ctx->stream != nullptr;
    if (use_graph && left >= ctx->graph_steps) {
        st = ensure_graph(ctx, ctx->graph_steps);
        if (st != CH_OK) return st;
        while (left >= ctx->graph_steps) {
            HIPCHK(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
            left -= ctx->graph_steps;
        }
    }
    if (left > 0) HIPCHK(ctx, enqueue_steps(ctx, left));
    ctx->step = target;
    if (nsteps > 0 && need_diag(target, ctx->K)) HIPCHK(ctx, enqueue_diag(ctx));
    return CH_OK;
}

ch_status ch_energy(ch_ctx* ctx, double* F, double* meanC)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    const int m = (int)ctx->desc.size();
    HIPCHK(ctx, enqueue_diag(ctx));
    std::vector<double> en(4 * (size_t)m);
    std::vector<int32_t> flags(m);
    HIPCHK(ctx, hipMemcpyAsync(en.data(), ctx->d_energy(), sizeof(double) * en.size(),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(flags.data(), ctx->d_flags(), sizeof(int32_t) * m,
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    bool bad = false;
    for (int i = 0; i < m; ++i) {
        if (F) F[i] = en[4 * i + 0];
        if (meanC) meanC[i] = en[4 * i + 1];
        bad |= flags[i] != 0;
    }
    if (bad) return fail(ctx, CH_ENONFINITE, "non-finite free energy in at least one member");
    return CH_OK;
}

ch_status ch_beta_series(ch_ctx* ctx, int32_t member, double* t, double* F, double* dFdt,
                         double* dFdt_identity, double* beta, double* meanC, int64_t cap,
                         int64_t* count)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (member < 0 || member >= (int)ctx->desc.size() || cap < 0 || !count)
        return fail(ctx, CH_EINVAL, "bad member, cap or NULL count");
    int64_t J = std::min<int64_t>(ctx->step / ctx->K + 1, ctx->max_samples);
    J = std::min<int64_t>(J, cap);
    *count = J;
    const double dt = ctx->desc[member].dt;
    HIPCHK(ctx, launch_beta(ctx->d_series(), ctx->max_samples, member, ctx->K, ctx->step, dt,
                            ctx->d_beta(), J, ctx->stream));
    std::vector<double> buf(6 * (size_t)J);
    int32_t flag = 0;
    if (J > 0)
        HIPCHK(ctx, hipMemcpyAsync(buf.data(), ctx->d_beta(), sizeof(double) * buf.size(),
                                   hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(&flag, ctx->d_flags() + member, sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double* cols[6] = {t, F, dFdt, dFdt_identity, beta, meanC};
    for (int c = 0; c < 6; ++c)
        if (cols[c])
            for (int64_t j = 0; j < J; ++j) cols[c][j] = buf[6 * j + c];
    if (flag) return fail(ctx, CH_ENONFINITE, "non-finite free energy in member %d", member);
    return CH_OK;
}

ch_status ch_set_graph_steps(ch_ctx* ctx, int32_t graph_steps)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (graph_steps < 0) return fail(ctx, CH_EINVAL, "graph_steps must be >= 0");
    ctx->graph_steps = graph_steps;
    drop_graph(ctx);
    // capture, instantiate and upload the graph now (nothing runs), so that
    // the first ch_step that replays it pays for none of that
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHK(ctx, hipStreamIsCapturing(ctx->stream, &cap));
    if (graph_steps > 0 && ctx->stream != nullptr && cap == hipStreamCaptureStatusNone)
        return ensure_graph(ctx, graph_steps);
    return CH_OK;
}

ch_status ch_set_theta(ch_ctx* ctx, double theta)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (theta != 1.0 && theta != 0.5) return fail(ctx, CH_EINVAL, "theta must be 1 or 1/2");
    const bool cn = theta == 0.5;
    std::vector<ClassPlan> plans = ctx->classes;
    for (auto& c : plans) {
        if (cn && c.dim != 2)
            return fail(ctx, CH_EUNSUPPORTED, "the Crank-Nicolson variant needs 2D members only");
        c.cn = cn;
        // keep the class's shape where it is valid for the new variant
        if (!planA(c, ctx->prec, c.cx, c.rl, c.waves, c.units) && !default_A(c, ctx->prec))
            return fail(ctx, CH_EUNSUPPORTED, "no tile shape fits a size class in LDS");
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->classes = plans;
    ctx->theta = theta;
    fill_member_table(ctx);
    st = upload_tables(ctx);
    drop_graph(ctx);
    return st;
}

ch_status ch_describe(const ch_ctx* ctx, char* buf, size_t cap)
{
    if (!ctx || !buf || cap == 0) return fail(nullptr, CH_EINVAL, "NULL argument");
    if (!is_live(ctx)) return fail(nullptr, CH_ESTATE, "unknown or destroyed context");
    std::string s = plan_text(ctx);
    snprintf(buf, cap, "%s", s.c_str());
    return CH_OK;
}

ch_status ch_time_kernels(ch_ctx* ctx, int64_t nsteps, double* ms)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (nsteps < 1 || !ms) return fail(ctx, CH_EINVAL, "nsteps >= 1 and ms required");
    if ((ctx->step + nsteps) / ctx->K >= ctx->max_samples)
        return fail(ctx, CH_ESTATE, "sample capacity exceeded");
    // real steps, launched directly; every kernel carries a pair of events
    // that take its own start and end timestamps
    const int nc = (int)ctx->classes.size();
    std::vector<hipEvent_t> ev(2 * 3 * (size_t)nc * nsteps, nullptr);
    for (auto& x : ev) HIPCHK(ctx, hipEventCreate(&x));
    auto E = [&](int64_t s, int ci, int k) { return &ev[2 * ((size_t)(s * nc + ci) * 3 + k)]; };
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) {
        for (int ci = 0; ci < nc && e == hipSuccess; ++ci)
            e = launch_A(ctx, ci, MODE_STEP, E(s, ci, 0)[0], E(s, ci, 0)[1]);
        for (int ci = 0; ci < nc && e == hipSuccess; ++ci)
            e = launch_cols(ctx, ci, 1, E(s, ci, 1)[0], E(s, ci, 1)[1]);
        for (int ci = 0; ci < nc && e == hipSuccess; ++ci)
            if (ctx->classes[ci].dim == 3) e = launch_cols(ctx, ci, 2, E(s, ci, 2)[0], E(s, ci, 2)[1]);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    double acc[3] = {0, 0, 0};
    for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s)
        for (int ci = 0; ci < nc && e == hipSuccess; ++ci)
            for (int k = 0; k < ctx->classes[ci].dim && e == hipSuccess; ++k) {
                float f = 0;
                e = hipEventElapsedTime(&f, E(s, ci, k)[0], E(s, ci, k)[1]);
                acc[k] += f;
            }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return fail(ctx, CH_EDEVICE, "kernel timing failed: %s", hipGetErrorString(e));
    ctx->step += nsteps;
    if (need_diag(ctx->step, ctx->K)) HIPCHK(ctx, enqueue_diag(ctx));
    for (int k = 0; k < 3; ++k) ms[k] = acc[k] / nsteps;
    return CH_OK;
}

ch_status ch_autotune(ch_ctx* ctx, const char* cache_path)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    // cached choices: one line per class "key cx rl waves units cy_y b_y cy_z b_z"
    constexpr int NV = 8;
    std::map<std::string, std::vector<int>> cache;
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "r")) {
            char key[256];
            int v[NV];
            while (fscanf(f, "%255s %d %d %d %d %d %d %d %d", key, &v[0], &v[1], &v[2], &v[3], &v[4],
                          &v[5], &v[6], &v[7]) == NV + 1)
                cache[key] = std::vector<int>(v, v + NV);
            fclose(f);
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    // best of 3 batches of 8 launches after 2 warm-up launches
    auto time_it = [&](auto&& launch, float& ms) -> hipError_t {
        hipError_t e;
        for (int w = 0; w < 2; ++w)
            if ((e = launch()) != hipSuccess) return e;
        const int reps = 8;
        ms = 1e30f;
        for (int b = 0; b < 3; ++b) {
            if ((e = hipEventRecord(e0, ctx->stream)) != hipSuccess) return e;
            for (int r = 0; r < reps; ++r)
                if ((e = launch()) != hipSuccess) return e;
            if ((e = hipEventRecord(e1, ctx->stream)) != hipSuccess) return e;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
            float t = 0;
            if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
            ms = std::min(ms, t / reps);
        }
        return hipSuccess;
    };
    // whole stand-in steps of all classes (one graph of 16, best of 3 replays)
    auto time_steps = [&](float& ms) -> hipError_t {
        const int n = 16;
        hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        e = enqueue_timing_steps(ctx, n);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
        if (e == hipSuccess) e = e2;
        hipGraphExec_t ex = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphLaunch(ex, ctx->stream);
        ms = 1e30f;
        for (int b = 0; b < 3 && e == hipSuccess; ++b) {
            if ((e = hipEventRecord(e0, ctx->stream)) != hipSuccess) break;
            if ((e = hipGraphLaunch(ex, ctx->stream)) != hipSuccess) break;
            if ((e = hipEventRecord(e1, ctx->stream)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float t = 0;
            if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
            ms = std::min(ms, t / n);
        }
        if (ex) (void)hipGraphExecDestroy(ex);
        if (g) (void)hipGraphDestroy(g);
        return e;
    };
    std::map<std::string, Shortlist> shortlist;  // keys tuned in this call
    hipError_t err = hipSuccess;
    for (int ci = 0; ci < (int)ctx->classes.size() && err == hipSuccess; ++ci) {
        ClassPlan& c = ctx->classes[ci];
        const std::string key = class_key(ctx, c);
        auto hit = cache.find(key);
        if (hit != cache.end()) {
            const std::vector<int>& v = hit->second;
            ClassPlan t = c;
            bool ok = planA(t, ctx->prec, v[0], v[1], v[2], v[3]) &&
                      planCol(t, ctx->prec, 1, v[4], v[5]) &&
                      (c.dim == 2 || planCol(t, ctx->prec, 2, v[6], v[7]));
            if (ok) {
                c = t;
                continue;
            }
        }
        // pass A candidates (timing mode: reads C, writes the scratch field)
        float best = 1e30f;
        int bcx = c.cx, brl = c.rl, bw = c.waves, bu = c.units;
        Shortlist& sl = shortlist[key];
        const int unit_opts_2d[] = {1, 2, 4, 0};  // 0: split form (lines beyond 64 chunks)
        const int unit_opts_3d[] = {1, 4, 8, 16, 32};
        const int* uo = c.dim == 3 ? unit_opts_3d : unit_opts_2d;
        const int nuo = c.dim == 3 ? 5 : 4;
        for (int waves : {4, 2, 1})
            for (int rl : {1, 2, 4})
                for (int cx : {4, 8, 16, 32, 64})
                    for (int ui = 0; ui < nuo; ++ui) {
                        const int units = uo[ui];
                        ClassPlan t = c;
                        if (!planA(t, ctx->prec, cx, rl, waves, units)) continue;
                        ctx->classes[ci] = t;
                        fill_member_table(ctx);
                        if ((st = upload_tables(ctx)) != CH_OK) {
                            ctx->classes[ci] = c;
                            return st;
                        }
                        float ms = 0;
                        err = time_it([&] { return launch_A(ctx, ci, MODE_TIMING); }, ms);
                        if (err != hipSuccess) break;
                        sl.add(0, ms, {cx, rl, waves, units});
                        if (ms < best) {
                            best = ms;
                            bcx = cx;
                            brl = rl;
                            bw = waves;
                            bu = units;
                        }
                    }
        ctx->classes[ci] = c;
        if (err != hipSuccess) break;
        planA(c, ctx->prec, bcx, brl, bw, bu);
        ctx->classes[ci] = c;
        // column sweeps, in place on the scratch field
        for (int axis = 1; axis < c.dim && err == hipSuccess; ++axis) {
            const int n = axis == 1 ? c.ny : c.nz;
            float bestc = 1e30f;
            int bcy = c.col[axis].cy, bb = c.col[axis].b;
            for (int cy : {4, 8, 16, 32, 64}) {
                if (!col_has(ctx->prec, cy) || n % cy) continue;
                for (int b = 1; b <= kColMaxThreads; b *= 2) {
                    ClassPlan t = c;
                    if (!planCol(t, ctx->prec, axis, cy, b)) continue;
                    ClassPlan wider = c;
                    if (b * t.col[axis].P < 64 && planCol(wider, ctx->prec, axis, cy, 2 * b))
                        continue;  // a wider block fills the wavefront better
                    ctx->classes[ci] = t;
                    fill_member_table(ctx);
                    if ((st = upload_tables(ctx)) != CH_OK) {
                        ctx->classes[ci] = c;
                        return st;
                    }
                    float ms = 0;
                    void* W = ctx->d_W();
                    err = time_it(
                        [&] {
                            return launch_col(ctx->prec, cy, col_args(ctx, ci, axis, W, W, false),
                                              ctx->stream);
                        },
                        ms);
                    if (err != hipSuccess) break;
                    sl.add(axis, ms, {cy, b});
                    if (ms < bestc) {
                        bestc = ms;
                        bcy = cy;
                        bb = b;
                    }
                }
                if (err != hipSuccess) break;
            }
            planCol(c, ctx->prec, axis, bcy, bb);
            ctx->classes[ci] = c;
        }
        cache[key] = {c.cx, c.rl, c.waves, c.units, c.col[1].cy, c.col[1].b,
                      c.dim == 3 ? c.col[2].cy : 0, c.dim == 3 ? c.col[2].b : 0};
    }
    // Stage 2.  With several classes the steps of different classes overlap
    // on separate streams, and the fastest shapes in isolation need not be
    // the fastest together.  For each newly tuned class key in turn, every
    // combination of its short-listed shapes is applied to all classes with
    // that key and whole stand-in steps of all classes are timed together.
    // (the legacy null stream cannot be captured: no stage 2 there)
    if (err == hipSuccess && ctx->classes.size() > 1 && !shortlist.empty() && ctx->stream != nullptr) {
        for (auto& kv : shortlist) {
            const std::string& key = kv.first;
            const Shortlist& sl = kv.second;
            std::vector<int> idx;
            for (int ci = 0; ci < (int)ctx->classes.size(); ++ci)
                if (class_key(ctx, ctx->classes[ci]) == key) idx.push_back(ci);
            const int dim = ctx->classes[idx[0]].dim;
            const size_t nz = dim == 3 ? sl.c[2].size() : 1;
            float bestj = 1e30f;
            std::vector<ClassPlan> bestp;
            for (size_t ia = 0; ia < sl.c[0].size() && err == hipSuccess; ++ia)
                for (size_t iy = 0; iy < sl.c[1].size() && err == hipSuccess; ++iy)
                    for (size_t iz = 0; iz < nz && err == hipSuccess; ++iz) {
                        const std::vector<int>& A = sl.c[0][ia].second;
                        const std::vector<int>& Y = sl.c[1][iy].second;
                        std::vector<ClassPlan> saved, trial;
                        bool ok = true;
                        for (int ci : idx) {
                            ClassPlan t = ctx->classes[ci];
                            ok = ok && planA(t, ctx->prec, A[0], A[1], A[2], A[3]) &&
                                 planCol(t, ctx->prec, 1, Y[0], Y[1]) &&
                                 (dim == 2 || planCol(t, ctx->prec, 2, sl.c[2][iz].second[0],
                                                      sl.c[2][iz].second[1]));
                            trial.push_back(t);
                            saved.push_back(ctx->classes[ci]);
                        }
                        if (!ok) continue;
                        for (size_t k = 0; k < idx.size(); ++k) ctx->classes[idx[k]] = trial[k];
                        fill_member_table(ctx);
                        if ((st = upload_tables(ctx)) != CH_OK) return st;
                        float ms = 0;
                        err = time_steps(ms);
                        if (err == hipSuccess && ms < bestj) {
                            bestj = ms;
                            bestp = trial;
                        }
                        for (size_t k = 0; k < idx.size(); ++k) ctx->classes[idx[k]] = saved[k];
                    }
            if (err != hipSuccess) break;
            if (!bestp.empty()) {
                for (size_t k = 0; k < idx.size(); ++k) ctx->classes[idx[k]] = bestp[k];
                const ClassPlan& c = bestp[0];
                cache[key] = {c.cx, c.rl, c.waves, c.units, c.col[1].cy, c.col[1].b,
                              c.dim == 3 ? c.col[2].cy : 0, c.dim == 3 ? c.col[2].b : 0};
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    fill_member_table(ctx);
    st = upload_tables(ctx);
    drop_graph(ctx);
    if (err != hipSuccess) return fail(ctx, CH_EDEVICE, "autotune: %s", hipGetErrorString(err));
    if (st != CH_OK) return st;
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "w")) {
            for (auto& kv : cache)
                fprintf(f, "%s %d %d %d %d %d %d %d %d\n", kv.first.c_str(), kv.second[0], kv.second[1],
                        kv.second[2], kv.second[3], kv.second[4], kv.second[5], kv.second[6],
                        kv.second[7]);
            fclose(f);
        }
    }
    return CH_OK;
}

ch_status ch_num_classes(const ch_ctx* ctx, int32_t* nclasses)
{
    if (!ctx || !nclasses) return fail(nullptr, CH_EINVAL, "NULL argument");
    if (!is_live(ctx)) return fail(nullptr, CH_ESTATE, "unknown or destroyed context");
    *nclasses = (int32_t)ctx->classes.size();
    return CH_OK;
}

ch_status ch_set_tiles(ch_ctx* ctx, int32_t cls, int32_t cx, int32_t rl, int32_t waves,
                       int32_t units, int32_t cy, int32_t by, int32_t cz, int32_t bz)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (cls < 0 || cls >= (int)ctx->classes.size()) return fail(ctx, CH_EINVAL, "bad class index");
    ClassPlan t = ctx->classes[cls];
    if (!planA(t, ctx->prec, cx, rl, waves, units) || !planCol(t, ctx->prec, 1, cy, by) ||
        (t.dim == 3 && !planCol(t, ctx->prec, 2, cz, bz)))
        return fail(ctx, CH_EUNSUPPORTED, "tile shape not valid for class %d", cls);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->classes[cls] = t;
    fill_member_table(ctx);
    st = upload_tables(ctx);
    drop_graph(ctx);
    return st;
}

ch_status ch_destroy(ch_ctx* ctx)
{
    if (!ctx) return fail(nullptr, CH_EINVAL, "ctx is NULL");
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!g_live.erase(ctx)) return fail(nullptr, CH_ESTATE, "unknown or destroyed context");
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    release_streams(ctx);
    delete ctx;
    return CH_OK;
}

// ---- ensemble statistics of beta ---------------------------------------------

ch_status ch_ensemble_moments(ch_ctx* ctx, const int32_t* members, int32_t nm, int32_t pmax, double* t,
                              double* mu, int64_t cap, int64_t* count)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (pmax < 1 || pmax > kMaxMoments || cap < 0 || !mu || !count)
        return fail(ctx, CH_EINVAL, "need 1 <= pmax <= %d, cap >= 0, mu and count", kMaxMoments);
    int32_t M;
    double dt;
    int64_t J;
    if ((st = stat_setup(ctx, members, nm, M, dt, J)) != CH_OK) return st;
    J = std::min<int64_t>(J, cap);
    *count = J;
    if (J == 0) return CH_OK;
    HIPCHK(ctx, launch_moments(ctx->d_series(), ctx->max_samples, ctx->d_statm(), M, ctx->K, ctx->step, dt,
                               pmax, ctx->d_stat(), J, ctx->stream));
    std::vector<double> buf(kMaxMoments * (size_t)J);
    HIPCHK(ctx, hipMemcpyAsync(buf.data(), ctx->d_stat(), sizeof(double) * buf.size(), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t j = 0; j < J; ++j) {
        if (t) t[j] = (double)(j * ctx->K) * dt;
        for (int p = 0; p < pmax; ++p) mu[j * pmax + p] = buf[j * kMaxMoments + p];
    }
    return CH_OK;
}

ch_status ch_ensemble_window(ch_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2,
                             double* beta0, double* k)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (!(t1 <= t2)) return fail(ctx, CH_EINVAL, "need t1 <= t2");
    int32_t M;
    double dt;
    int64_t J;
    if ((st = stat_setup(ctx, members, nm, M, dt, J)) != CH_OK) return st;
    int64_t j0, j1;
    double out[2] = {std::nan(""), std::nan("")};
    if (window_range(ctx, dt, J, t1, t2, j0, j1)) {
        double* d_out = ctx->d_stat() + kMaxMoments * (size_t)ctx->max_samples;
        HIPCHK(ctx, launch_moments(ctx->d_series(), ctx->max_samples, ctx->d_statm(), M, ctx->K, ctx->step,
                                   dt, 2, ctx->d_stat(), J, ctx->stream));
        HIPCHK(ctx, launch_window(ctx->d_stat(), j0, j1, ctx->K, dt, d_out, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(out, d_out, sizeof out, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (beta0) *beta0 = out[0];
    if (k) *k = out[1];
    return CH_OK;
}

ch_status ch_beta_histogram(ch_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2,
                            double lo, double hi, int32_t nbins, uint64_t* counts)
{
    ch_status st = check_ctx(ctx);
    if (st != CH_OK) return st;
    if (!counts || nbins < 1 || nbins > kMaxHistBins || !(lo < hi) || !(t1 <= t2))
        return fail(ctx, CH_EINVAL, "need counts, 1 <= nbins <= %d, lo < hi, t1 <= t2", kMaxHistBins);
    int32_t M;
    double dt;
    int64_t J;
    if ((st = stat_setup(ctx, members, nm, M, dt, J)) != CH_OK) return st;
    std::vector<uint64_t> h(nbins + 2, 0);
    int64_t j0, j1;
    if (window_range(ctx, dt, J, t1, t2, j0, j1)) {
        HIPCHK(ctx, launch_hist(ctx->d_series(), ctx->max_samples, ctx->d_statm(), M, ctx->K, ctx->step, dt,
                                j0, j1, lo, hi, nbins,
                                reinterpret_cast<unsigned long long*>(ctx->d_hist()), ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(h.data(), ctx->d_hist(), sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    std::copy(h.begin(), h.end(), counts);
    return CH_OK;
}

ch_status ch_solver_coefficients(double rho, int32_t n, int32_t chunk, int32_t prec, double* out)
{
    if (!out || !(rho > 0.0) || n < 1 || chunk < 1 || (prec != 0 && prec != 1))
        return fail(nullptr, CH_EINVAL, "bad arguments");
    AxisCoef c;
    axis_coef(rho, n, chunk, prec, c);
    out[0] = c.a1;
    out[1] = c.a2;
    out[2] = c.ikappa;
    for (int i = 0; i < 4; ++i) out[3 + i] = c.M[i];
    for (int i = 0; i < 4; ++i) out[7 + i] = c.W[i];
    return CH_OK;
}

ch_status ch_step_static(const ch_member_desc* members, int32_t m, ch_precision prec, void* d_field,
                         int64_t nsteps, double* d_energy, void* hip_stream)
{
    // Diagnostics cadence of the step kernels: only step 0 is a sample step
    // (its partials are reduced into the one-sample series in scratch); the
    // energies of the final state come from a diagnostics pass at the end.
    constexpr int32_t kNoCadence = 1 << 30;
    std::string err;
    if (m < 1 || m > CH_STATIC_MAX_MEMBERS)
        return fail(nullptr, CH_EINVAL, "m = %d outside 1..%d", m, CH_STATIC_MAX_MEMBERS);
    ch_status st = validate(members, m, prec, kNoCadence, 1, err);
    if (st != CH_OK) return fail(nullptr, st, "%s", err.c_str());
    for (int i = 1; i < m; ++i)
        if (members[i].dim != members[0].dim || members[i].n[0] != members[0].n[0] ||
            members[i].n[1] != members[0].n[1] || members[i].n[2] != members[0].n[2])
            return fail(nullptr, CH_EINVAL, "member %d: every member needs the grid of member 0", i);
    if (!d_field) return fail(nullptr, CH_EINVAL, "d_field is NULL");
    if (reinterpret_cast<uintptr_t>(d_field) % 16)
        return fail(nullptr, CH_EINVAL, "d_field must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(d_energy) % 8) return fail(nullptr, CH_EINVAL, "d_energy must be 8-byte aligned");
    if (nsteps < 0) return fail(nullptr, CH_EINVAL, "nsteps must be >= 0");

    const ch_member_desc& d0 = members[0];
    ClassPlan c;
    c.dim = d0.dim;
    c.nx = d0.n[0];
    c.ny = d0.n[1];
    c.nz = d0.dim == 3 ? d0.n[2] : 1;
    c.nfixed = m;
    if (!default_A(c, prec) || !default_col(c, prec, 1) || (c.dim == 3 && !default_col(c, prec, 2)))
        return fail(nullptr, CH_EUNSUPPORTED, "no tile shape fits this grid in LDS");
    const int64_t sites = (int64_t)c.nx * c.ny * c.nz;
    const StaticLayout S = static_layout(c, prec, m, sites);
    if (S.total > CH_STATIC_SCRATCH_BYTES)
        return fail(nullptr, CH_ENOMEM,
                    "%d members of %lld sites need %zu bytes of static scratch; the maximum is %zu "
                    "(use ch_create with a workspace instead)",
                    m, (long long)sites, S.total, (size_t)CH_STATIC_SCRATCH_BYTES);

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, CH_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(nullptr, CH_EDEVICE, "device %d not supported", dev);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);

    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        // first call on this device (it is current): the device address of its
        // copy of the static array
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, CH_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    char* base = static_cast<char*>(g_static_ptr[dev]);
    for (int i = 0; i < m; ++i) {
        fill_member(members[i], (int64_t)i * sites, c, prec, 1.0, g_static_mem[i]);
        g_static_mids[i] = i;
    }
    // pageable host-to-device copies: the staging tables are read before the
    // calls return, so the next call may refill them
    if ((e = hipMemcpyAsync(base + S.mem, g_static_mem, sizeof(MemberDev) * m, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(base + S.mids, g_static_mids, sizeof(int32_t) * m, hipMemcpyHostToDevice, s)) !=
            hipSuccess)
        return fail(nullptr, CH_EDEVICE, "table upload: %s", hipGetErrorString(e));

    int64_t* steps = reinterpret_cast<int64_t*>(base + S.steps);
    int64_t* nstamp = reinterpret_cast<int64_t*>(base + S.nstamp);
    int32_t* flags = reinterpret_cast<int32_t*>(base + S.flags);
    double* series = reinterpret_cast<double*>(base + S.series);
    // the scratch keeps the previous call's contents: counter, flags and series start afresh
    if ((e = launch_reset(steps, 1, 0, flags, m, series, (int64_t)kSeriesSlots * m, s)) != hipSuccess)
        return fail(nullptr, CH_EDEVICE, "reset: %s", hipGetErrorString(e));

    PassAArgs a{};
    a.C = d_field;
    a.W = base + S.W;
    a.mem = reinterpret_cast<const MemberDev*>(base + S.mem);
    a.mids = reinterpret_cast<const int32_t*>(base + S.mids);
    a.nmem = m;
    a.run = MemberRun{0, 0, sites};  // members i at i * sites
    a.nx = c.nx;
    a.ny = c.ny;
    a.nz = c.nz;
    a.P = c.P;
    a.rows_per_wave = c.rpw;
    a.waves = c.waves;
    a.R = c.R;
    a.bands_y = c.bands;
    a.units = c.units;
    a.blocks_per_member = c.bpmA;
    a.nblocks = c.nblocksA;
    a.pitch = c.pitch;
    a.conv = CH_ENERGY_QUARTER;
    a.K = kNoCadence;
    a.step = steps;
    a.partials = reinterpret_cast<double*>(base + S.partials);
    a.nstamp = nstamp;

    FinArgs f{};
    f.enabled = 1;
    f.mem = a.mem;
    f.mids = a.mids;
    f.nmem = m;
    f.K = kNoCadence;
    f.blocks_per_member = c.bpmP;
    f.partials = a.partials;
    f.nstamp = nstamp;
    f.max_samples = 1;
    f.step = steps;
    f.series = series;
    f.energy_now = d_energy ? d_energy : reinterpret_cast<double*>(base + S.energy);
    f.flags = flags;

    auto col = [&](int axis, const void* src, void* dst, bool last) {
        const ColPlan& p = c.col[axis];
        ColArgs ca{};
        ca.src = src;
        ca.dst = dst;
        ca.mem = a.mem;
        ca.mids = a.mids;
        ca.mrun = a.run;
        ca.msites = sites;
        ca.axis = axis;
        ca.n = axis == 1 ? c.ny : c.nz;
        ca.stride = p.stride;
        ca.run = p.run;
        ca.outer = p.outer;
        ca.cols = p.cols;
        ca.b = p.b;
        ca.bshift = __builtin_ctz((unsigned)p.b);
        ca.P = p.P;
        ca.nblocks = p.nblocks;
        if (last) {
            ca.fin = f;
            ca.fin.mode = MODE_STEP;
            ca.fin.G = (int32_t)std::min<int64_t>(std::min<int64_t>(m, 1024), p.nblocks);
        }
        return launch_col(prec, p.cy, ca, s);
    };
    for (int64_t i = 0; i < nsteps; ++i) {
        a.mode = MODE_STEP;
        if ((e = launch_passA(prec, c.dim, c.cx, c.rl, c.units, a, c.ldsA, s)) != hipSuccess) break;
        if ((e = col(1, a.W, c.dim == 2 ? d_field : a.W, c.dim == 2)) != hipSuccess) break;
        if (c.dim == 3 && (e = col(2, a.W, d_field, true)) != hipSuccess) break;
    }
    if (e == hipSuccess && d_energy) {
        // F, <C> and G_id of the final state, and the step count
        a.mode = MODE_DIAG;
        f.mode = MODE_DIAG;
        f.G = (int32_t)std::min<int32_t>(m, 1024);
        e = launch_passA(prec, c.dim, c.cx, c.rl, c.units, a, c.ldsA, s);
        if (e == hipSuccess) e = launch_fin(f, s);
    }
    if (e != hipSuccess) return fail(nullptr, CH_EDEVICE, "launch: %s", hipGetErrorString(e));
    return CH_OK;
}

}  // extern "C"
