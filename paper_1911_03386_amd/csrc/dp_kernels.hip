// Model 1 of the paper (Sections 2-3): ensembles of mean-field droplet
// populations, dR_i/dt = H(R_i) (-1/R_i^2 + ubar/R_i) with
// ubar = sum H(R_i) / sum H(R_i) R_i (eq. (dRi), eq. (uval)), integrated in the
// volumes V_i = R_i^3:  dV_i/dt = 3 (ubar R_i - 1) while V_i > 0, 0 after.
//
// One workgroup integrates one member with the Dormand-Prince 5(4) pair
// (Dormand & Prince 1980; the pair inside ode45, which the paper used) under
// adaptive error control.  Every droplet's stage value depends on the other
// droplets only through the stage's mean field, a scalar: each stage is an
// elementwise pass over the member's droplets plus one block reduction of
// (live count, sum of radii).  Thread tid holds slots p*T + tid,
// p = 0..P-1: their stage increments live in registers, the state V and the
// error accumulator in LDS (private slots, so no barriers), and the
// integrator's scalars are uniform over the block.  Slots hold the live
// droplets in their original order: when deaths free a whole row of T slots,
// the live droplets are packed to the front (the dead ones' final volumes go
// back to global memory), so the work per stage follows the live count.  The
// slot -> droplet map is kept in global memory, so the layout, and with it
// every rounding, does not depend on how the run is split into launches.
//
// Error control, identical for every member:
//   err = max_i |h sum_s e_s k_{s,i}| / (atol + rtol max(|V_i|, |V_i^new|)),
//   accept iff err <= 1;  h *= clamp(0.9 err^(-1/5), 0.2, 5) (5 at err = 0),
//   no growth right after a rejection;  a step that would pass the next
//   sample time j*dts ends exactly on it.
// Samples: F = (1/2) sum H R^2 (eq. (Fdef)), dF/dt = -sum H (1/R)(1 - ubar R)^2
// (eq. (dFdt)), beta = -t (dF/dt)/F (eq. (betaN)).
#include "dp_internal.h"
#include "ensemble_stats.h"

#include <hip/hip_runtime.h>

namespace dp {
namespace {

// Dormand-Prince 5(4): stage matrix a[s][j] (row 6 = the order-5 weights,
// first same as last) and e = b5 - b4 (order-5 minus order-4 weights).
constexpr double kA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
constexpr double kE[7] = {71.0 / 57600.0,  0.0,          -71.0 / 16695.0, 71.0 / 1920.0,
                          -17253.0 / 339200.0, 22.0 / 525.0, -1.0 / 40.0};

// Lane exchange within rows of 16 lanes by DPP (a register move, no LDS
// round trip), on the two 32-bit halves of a double.  The patterns used are
// involutions: quad_perm [1,0,3,2] (0xB1) and [2,3,0,1] (0x4E), half-row
// mirror (0x141) and row mirror (0x140).
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double lane_value(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Wave sum, the same bits on every lane: a butterfly within each row of 16
// (each step adds the same two values on both lanes of a pair), then the
// four row sums in fixed order.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_swap<0xB1>(v);
    v += dpp_swap<0x4E>(v);
    v += dpp_swap<0x141>(v);
    v += dpp_swap<0x140>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_swap<0xB1>(v));
    v = fmax(v, dpp_swap<0x4E>(v));
    v = fmax(v, dpp_swap<0x141>(v));
    v = fmax(v, dpp_swap<0x140>(v));
    return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

// Block-wide sums of two values (or max of one), the same on every thread:
// the wave sums above, then every thread adds the wave totals in wave order.  The two halves of `red` alternate between calls, so one barrier per
// reduction suffices: a buffer is rewritten only after the barrier of the
// next reduction, which every reader of the previous contents has passed.
template <int T>
struct Reducer {
    static constexpr int W = T / 64;
    double (*red)[2][W];
    int buf = 0;

    __device__ void sum2(double& x, double& y)
    {
        x = wave_sum(x);
        y = wave_sum(y);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[buf][0][w] = x;
            red[buf][1][w] = y;
        }
        __syncthreads();
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            sx += red[buf][0][i];
            sy += red[buf][1][i];
        }
        x = sx;
        y = sy;
        buf ^= 1;
    }

    __device__ double max1(double x)
    {
        x = wave_max(x);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[buf][0][w] = x;
        __syncthreads();
        double m = red[buf][0][0];
#pragma unroll
        for (int i = 1; i < W; ++i) m = fmax(m, red[buf][0][i]);
        buf ^= 1;
        return m;
    }
};

__device__ __forceinline__ double radius(double v) { return v > 0.0 ? cbrt(v) : 0.0; }

// (live droplets, sum R) of the radii r -> ubar
__device__ __forceinline__ double mean_field(double cnt, double sr) { return cnt > 0.0 ? cnt / sr : 0.0; }

// Sample j of a member from its radii (r > 0 alive): F, dF/dt, beta.
template <int T, int P>
__device__ void record(Reducer<T>& rd, const double (&r)[P], int pm, double ubar, double cnt, double t,
                       double* row)
{
    double f2 = 0.0, g = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double R = r[p];
        if (p < pm && R > 0.0) {
            const double q = 1.0 - ubar * R;
            f2 += R * R;
            g += q * q / R;
        }
    }
    rd.sum2(f2, g);
    if (threadIdx.x == 0) {
        const double F = 0.5 * f2, dF = -g;
        row[0] = t;
        row[1] = F;
        row[2] = dF;
        row[3] = (t == 0.0) ? 0.0 : -t * dF / F;
        row[4] = ubar;
        row[5] = cnt;
    }
}

template <int T, int P>
__global__ void __launch_bounds__(T) init_kernel(Args a)
{
    __shared__ double red[2][2][T / 64];
    Reducer<T> rd{red};
    const int mi = a.order[blockIdx.x];
    const Member mb = a.mem[mi];
    const int pm = (mb.n + T - 1) / T;
    double* V = a.V + mb.off;  // holds the radii on entry, the volumes on exit
    double r[P];
    double cnt = 0.0, sr = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        r[p] = 0.0;
        const int i = p * T + threadIdx.x;
        if (p < pm && i < mb.n) {
            const double R0 = V[i];
            const double v = (R0 * R0) * R0;
            V[i] = v;
            r[p] = radius(v);
        }
        if (r[p] > 0.0) {
            cnt += 1.0;
            sr += r[p];
        }
    }
    rd.sum2(cnt, sr);
    const double ubar = mean_field(cnt, sr);
    record<T, P>(rd, r, pm, ubar, cnt, 0.0, a.series + (int64_t)mi * a.J * kSlots);
    for (int i = threadIdx.x; i < mb.n; i += T) a.slot[mb.off + i] = i;
    if (threadIdx.x == 0) {
        State s{};
        s.t = 0.0;
        s.h = a.h0;
        s.ubar = ubar;
        s.jn = 1;
        s.status = (a.J <= 1) ? kDone : kRunning;
        s.nslot = mb.n;
        s.live = (int32_t)cnt;
        a.st[mi] = s;
    }
}

// Pack the live droplets (V > 0) of slots [0, nslot) to slots [0, live) in
// slot order; dead droplets' volumes are final and go back to V.  Ranks come
// from wave ballots: slot p*T + tid precedes every slot of a later row p and,
// within row p, the slots of lower threads.  The old values are staged in
// `stage` (LDS) and the droplet indices in registers, so that every old slot
// is read before the barrier and written only after it.  Slots from
// live_total on are cleared (V = 0: no droplet).
template <int T, int P>
__device__ __noinline__ void compact(double* yl, double* stage, int32_t* slot, double* V, int pm, int32_t nslot,
                                     int32_t live_total, int32_t (*wcnt)[T / 64])
{
    constexpr int W = T / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned live = 0u;
    int32_t g[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int j = p * T + tid;
        const bool in = p < pm && j < nslot;
        const bool lv = in && yl[j] > 0.0;
        live |= (lv ? 1u : 0u) << p;
        const unsigned long long mask = __ballot(lv);
        if (lane == 0 && p < pm) wcnt[p][w] = __popcll(mask);
        g[p] = in ? slot[j] : -1;
        if (in) stage[j] = yl[j];
    }
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (p < pm) {
            const int j = p * T + tid;
            const bool lv = (live >> p) & 1u;
            const unsigned long long mask = __ballot(lv);
            int inrow = 0, row = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                row += wcnt[p][q];
                if (q < w) inrow += wcnt[p][q];
            }
            if (lv) {
                const int d = base + inrow + __popcll(mask & below);
                yl[d] = stage[j];
                slot[d] = g[p];
            } else if (g[p] >= 0) {
                V[g[p]] = stage[j];
            }
            // slots past the live ones are no droplet's (no live droplet lands there)
            if (j >= live_total) yl[j] = 0.0;
            base += row;
        }
    }
    __syncthreads();
}

// Up to `attempts` step attempts of one member per block; the state goes back
// to global memory at the end, so launches can be repeated until every
// member is done.  Each attempt ends in a uniform accept / reject decision.
template <int T, int P>
__global__ void __launch_bounds__(T) step_kernel(Args a, int64_t attempts)
{
    extern __shared__ double lds[];
    __shared__ double red[2][2][T / 64];
    __shared__ int32_t wcnt[P][T / 64];
    Reducer<T> rd{red};
    double* yl = lds;           // V, slot p*T + tid
    double* el = lds + P * T;   // sum_s e_s k_s
    const int tid = threadIdx.x;
    const int mi = a.order[blockIdx.x];
    const Member mb = a.mem[mi];
    State st = a.st[mi];
    if (st.status != kRunning) return;  // uniform
    int pm = (st.nslot + T - 1) / T;  // rows in use (uniform)
    double* V = a.V + mb.off;
    int32_t* slot = a.slot + mb.off;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int j = p * T + tid;
        if (p < pm) yl[j] = j < st.nslot ? V[slot[j]] : 0.0;
    }
    double* ser = a.series + (int64_t)mi * a.J * kSlots;
    double r[P];          // radii of the current stage's values
    bool fresh = false;   // r holds the radii of the state (after an accepted step)

    for (int64_t it = 0; it < attempts; ++it) {
        if (st.acc + st.rej >= a.max_total) {
            st.status = kAttemptLimit;
            break;
        }
        st.evals += 6.0 * st.live;  // first same as last: six new stages per attempt
        const double t_next = (double)st.jn * a.dts;
        const bool land = st.h >= t_next - st.t;
        const double h = land ? t_next - st.t : st.h;

        double S[6][P];  // S[s-1] = sum_{j<s} a[s][j] k_j, the increment of stage s
        double ub = st.ubar, cnt = 0.0;
        if (!fresh) {
#pragma unroll
            for (int p = 0; p < P; ++p) r[p] = p < pm ? radius(yl[p * T + tid]) : 0.0;
        }
        double errmax = 0.0;
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            // k_s from the stage radii and mean field, folded into the later
            // stages' increments and the error estimate
            double c2 = 0.0, sr = 0.0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (p >= pm) continue;  // uniform; keeps the loop single-exit for full unrolling
                const double k = r[p] > 0.0 ? 3.0 * (ub * r[p] - 1.0) : 0.0;
#pragma unroll
                for (int q = s + 1; q < 7; ++q) S[q - 1][p] = (s == 0) ? kA[q][0] * k : S[q - 1][p] + kA[q][s] * k;
                const int li = p * T + tid;
                el[li] = (s == 0) ? kE[0] * k : el[li] + kE[s] * k;
                const double y = yl[li];
                if (s < 6) {
                    const double Y = y + h * S[s][p];
                    r[p] = radius(Y);
                    if (r[p] > 0.0) {
                        c2 += 1.0;
                        sr += r[p];
                    }
                } else {
                    const double y5 = y + h * S[5][p];
                    const double sc = a.atol + a.rtol * fmax(fabs(y), fabs(y5));
                    errmax = fmax(errmax, fabs(h * el[li]) / sc);
                }
            }
            if (s < 6) {
                rd.sum2(c2, sr);
                ub = mean_field(c2, sr);
                cnt = c2;
            }
        }
        const double err = rd.max1(errmax);
        if (!(err <= 1.0) && !isfinite(err)) {
            st.status = kNonFinite;
            break;
        }
        if (err <= 1.0) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int li = p * T + tid;
                if (p < pm) yl[li] = yl[li] + h * S[5][p];
            }
            st.t = land ? t_next : st.t + h;
            double fac = err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
            if (st.rej_last) fac = fmin(fac, 1.0);
            st.rej_last = 0;
            st.acc += 1;
            st.h = h * fac;
            st.ubar = ub;  // the last stage is the new state (first same as last)
            if (land) {
                // r holds the radii of the new state
                record<T, P>(rd, r, pm, ub, cnt, st.t, ser + st.jn * kSlots);
                st.jn += 1;
                if (st.jn >= a.J) st.status = kDone;
            }
            // the last stage was evaluated at the new state: its radii are the
            // next attempt's first-stage radii (first same as last)
            fresh = true;
            const int live = (int)cnt;
            st.live = live;
            if ((live + T - 1) / T < pm) {
                compact<T, P>(yl, el, slot, V, pm, st.nslot, live, wcnt);
                st.nslot = live;
                pm = (live + T - 1) / T;
                fresh = false;
            }
        } else {
            st.h = h * fmax(0.2, 0.9 * pow(err, -0.2));
            st.rej_last = 1;
            st.rej += 1;
            fresh = false;
        }
        if (st.status == kRunning && st.t + st.h == st.t) st.status = kUnderflow;
        if (st.status != kRunning) break;
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int j = p * T + tid;
        if (p < pm && j < st.nslot) V[slot[j]] = yl[j];
    }
    if (tid == 0) a.st[mi] = st;
}

// --------------------------------------------------------------------------
// ensemble statistics of the recorded beta (the same definitions as for the
// Cahn-Hilliard ensembles: eq. (mup), eq. (beta0_stats), mu_2 = k t)
// --------------------------------------------------------------------------
constexpr int kStatThreads = ens_stats::kThreads;
static_assert(ens_stats::kMaxMoments == kMaxMoments, "one moment layout");

// beta of selected member i at sample j from the recorded series
struct SeriesBeta {
    const double* series;
    int64_t J;
    const int32_t* members;
    __device__ double operator()(int i, int64_t j) const
    {
        return series[((int64_t)members[i] * J + j) * kSlots + 3];
    }
};

__global__ void __launch_bounds__(kStatThreads) moments_kernel(const double* series, int64_t J,
                                                               const int32_t* members, int32_t nm,
                                                               int64_t count, int32_t pmax, double* out)
{
    ens_stats::moments(SeriesBeta{series, J, members}, nm, count, pmax, out);
}

__global__ void __launch_bounds__(kStatThreads) window_kernel(const double* mom, int64_t j0, int64_t j1,
                                                              double dts, double* out)
{
    ens_stats::window(mom, j0, j1, dts, [=](int64_t j) { return (double)j * dts; }, out);
}

__global__ void __launch_bounds__(kStatThreads) hist_kernel(const double* series, int64_t J,
                                                            const int32_t* members, int32_t nm, int64_t j0,
                                                            int64_t j1, double lo, double hi, int32_t nbins,
                                                            unsigned long long* counts)
{
    ens_stats::histogram(SeriesBeta{series, J, members}, nm, j0, j1, lo, hi, nbins, counts);
}

__global__ void zero_kernel(unsigned long long* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

template <int P>
hipError_t run_init(const Args& a, int32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((init_kernel<kThreads, P>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <int P>
hipError_t run_steps(const Args& a, int32_t blocks, int64_t attempts, hipStream_t s)
{
    const size_t lds = sizeof(double) * 2 * P * kThreads;
    hipLaunchKernelGGL((step_kernel<kThreads, P>), dim3((unsigned)blocks), dim3(kThreads), lds, s, a, attempts);
    return hipGetLastError();
}

}  // namespace

int per_thread(int32_t nmax)
{
    int p = 1;
    while (p < kMaxPerThread && (int64_t)p * kThreads < nmax) p *= 2;
    return p;
}

hipError_t launch_init(const Args& a, int32_t blocks, int per, hipStream_t s)
{
    switch (per) {
    case 1: return run_init<1>(a, blocks, s);
    case 2: return run_init<2>(a, blocks, s);
    case 4: return run_init<4>(a, blocks, s);
    case 8: return run_init<8>(a, blocks, s);
    case 16: return run_init<16>(a, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_steps(const Args& a, int32_t blocks, int per, int64_t attempts, hipStream_t s)
{
    switch (per) {
    case 1: return run_steps<1>(a, blocks, attempts, s);
    case 2: return run_steps<2>(a, blocks, attempts, s);
    case 4: return run_steps<4>(a, blocks, attempts, s);
    case 8: return run_steps<8>(a, blocks, attempts, s);
    case 16: return run_steps<16>(a, blocks, attempts, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_moments(const double* series, int64_t J, const int32_t* members, int32_t nm, int64_t count,
                          int32_t pmax, double* out, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = count < 4096 ? count : 4096;
    hipLaunchKernelGGL(moments_kernel, dim3((unsigned)blocks), dim3(kStatThreads), 0, s, series, J, members, nm,
                       count, pmax, out);
    return hipGetLastError();
}

hipError_t launch_window(const double* mom, int64_t j0, int64_t j1, double dts, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(window_kernel, dim3(1), dim3(kStatThreads), 0, s, mom, j0, j1, dts, out);
    return hipGetLastError();
}

hipError_t launch_hist(const double* series, int64_t J, const int32_t* members, int32_t nm, int64_t j0,
                       int64_t j1, double lo, double hi, int32_t nbins, unsigned long long* counts,
                       hipStream_t s)
{
    const int64_t total = (j1 - j0 + 1) * (int64_t)nm;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + kStatThreads - 1) / kStatThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)blocks), dim3(kStatThreads), 0, s, series, J, members, nm, j0,
                       j1, lo, hi, nbins, counts);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned long long* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace dp
