// HIP kernels (gfx950) of the Cahn-Hilliard ensemble step.
//
// One step of the semi-implicit ADI scheme (paper: Section 4.1 and Appendix A;
// the paper names the scheme but not its equations, so the form below is the
// reading this library adopts):
//
//   RHS     = C + dt lap_h(C^3 - C) - 2 gamma dt sum_{d<e} D_d D_e C
//   w       = (I + gamma dt D_x^2)^{-1} RHS            on every x-line
//   C^{n+1} = (I + gamma dt D_z^2)^{-1} (I + gamma dt D_y^2)^{-1} w
//
// and its Crank-Nicolson variant (2D), with a = gamma dt, X = I + a D_x^2 / 2,
// Y = I + a D_y^2 / 2:  X Y C^{n+1} = (I - a D_x^2 / 2)(I - a D_y^2 / 2) C
// + (RHS - C), computed as
//
//   G       = dt lap_h(C^3 - C) - 2 a D_x D_y C - a (D_x^2 + D_y^2) C
//   w       = (C + a D_y^2 C / 2) + X^{-1} G            on every x-line
//   C^{n+1} = Y^{-1} w
//
// (X and Y commute, so X Y C^{n+1} = X Y C + G, which is the scheme: the
// a^2 D_x^2 D_y^2 C terms of the two products cancel.)
//
// Kernels:
//   passA_kernel  x-lines.  A block stages R x-lines of C plus halo rows (and,
//                 in 3D, the neighbouring z-planes) in LDS, forms the RHS in
//                 registers (lane = contiguous chunk of one line), solves the
//                 periodic pentadiagonal system of every x-line and writes w.
//                 On cadence steps it also forms per-block FP64 partial sums
//                 of F, sum C and the dF/dt identity; the first blocks of the
//                 step's last line sweep reduce them per member in a fixed
//                 order.
//   passA_multi_kernel  the same with one block walking several work units
//                 (y-bands in 2D, z-planes of a y-band through a ring of
//                 staged planes in 3D), the next unit's rows loading while
//                 the current one is computed.
//   passA_wide_kernel  2D x-lines of 128 or 256 chunks, a line held by 2 or
//                 4 wavefronts whose chunk scans combine through LDS; in the
//                 split form (rows too long for LDS) it solves lines whose
//                 RHS rhs_tile_kernel formed over 8 x 256 tiles.
//   col_kernel    y- or z-lines.  A block owns b adjacent columns; lane
//                 (column, chunk) holds a contiguous chunk of one line in
//                 registers, loads are coalesced across columns.
//
// Line solve.  (I + rho [1,-4,6,-4,1]) is circulant with symbol
// 1 + rho (z - 2 + 1/z)^2 = kappa Q(z) Q(1/z), Q(z) = (1 - p/z)(1 - conj(p)/z),
// |p| < 1.  So the inverse is a causal second-order recursion followed by the
// mirrored anti-causal one, each applied to the periodic sequence.  Every
// chunk first runs the recursion from a zero state to get its end state
// (a pair of values), the chunk end states are combined by a scan with the
// chunk transfer matrix A^c (closing the ring with (I - A^n)^{-1}), and every
// chunk then reruns the recursion from its true incoming state.  Work per
// element and sweep: four two-term recursions and one scale.
#include "ch_internal.h"
#include "ensemble_stats.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

namespace chk {

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb)
{
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of logical tiles so that neighbouring tiles (which share
    // halo rows and planes) hit the same L2.  A bijection for any nb.
    // Block indices are 32-bit throughout (grids stay below 2^31 blocks, which
    // the planner checks): 64-bit divisions expand to long scalar sequences
    // that delay a block's first loads.
    const uint32_t q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Member id and element offset of class member mloc: arithmetic for a run of
// consecutive members, else from the member tables.
__device__ __forceinline__ int member_id(const MemberRun& r, const int32_t* mids, int mloc)
{
    return r.mid0 >= 0 ? r.mid0 + mloc : mids[mloc];
}
__device__ __forceinline__ int64_t member_off(const MemberRun& r, const MemberDev* mem, int mid, int mloc)
{
    if (r.mid0 >= 0) return r.off0 + (int64_t)mloc * r.stride;
    return mem[mid].off;
}

// lane / P for the lanes of a line group (P a power of two in most plans)
__device__ __forceinline__ int lane_div(int lane, int P)
{
    return (P & (P - 1)) == 0 ? lane >> __builtin_ctz((unsigned)P) : lane / P;
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Raw buffer access: a buffer resource (base address and byte range in
// scalar registers) plus a 32-bit per-lane byte offset and a wave-uniform
// scalar byte offset, so that strided accesses need no per-lane 64-bit
// address arithmetic; accesses past the range read 0 and write nothing.
// (The third resource word is the gfx9-family raw-buffer format.)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// 16-byte vectors (float4 / double2)
template <typename VT>
__device__ __forceinline__ VT buf_load16(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <typename VT>
__device__ __forceinline__ void buf_store16(const VT& v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 0);
}

template <typename T>
struct LineCoef {
    T a1, a2, ik;
    T M[4];
    T Mp[kMaxScanLevels][4];
    T W[4];
};

// A member's coefficients in the kernel's precision (no conversions in the kernel)
template <typename T>
struct CoefOf;
template <>
struct CoefOf<double> {
    static __device__ __forceinline__ const AxisCoef& ax(const MemberDev& m, int a) { return m.ax[a]; }
    static __device__ __forceinline__ const double* rc(const MemberDev& m) { return m.rc; }
};
template <>
struct CoefOf<float> {
    static __device__ __forceinline__ const AxisCoefF& ax(const MemberDev& m, int a) { return m.axf[a]; }
    static __device__ __forceinline__ const float* rc(const MemberDev& m) { return m.rcf; }
};

template <typename T, typename AC>
__device__ __forceinline__ void load_coef(LineCoef<T>& c, const AC& s, int P)
{
    c.a1 = (T)s.a1;
    c.a2 = (T)s.a2;
    c.ik = (T)s.ikappa;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        c.M[i] = (T)s.M[i];
        c.W[i] = (T)s.W[i];
    }
#pragma unroll
    for (int l = 0; l < kWaveScanLevels; ++l)
        if ((1 << l) < P)
#pragma unroll
            for (int i = 0; i < 4; ++i) c.Mp[l][i] = (T)s.Mp[l][i];
}

template <typename T>
__device__ __forceinline__ void mv(const T* M, T& x0, T& x1)
{
    T y0 = M[0] * x0 + M[1] * x1;
    T y1 = M[2] * x0 + M[3] * x1;
    x0 = y0;
    x1 = y1;
}

// causal recursion over a chunk from a zero state: end state (u_last, u_last-1)
template <typename T, int CL>
__device__ __forceinline__ void fwd_zero(const T (&v)[CL], T a1, T a2, T& e0, T& e1)
{
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int k = 0; k < CL; ++k) {
        T u = fma(a1, s0, fma(a2, s1, v[k]));
        s1 = s0;
        s0 = u;
    }
    e0 = s0;
    e1 = s1;
}

template <typename T, int CL>
__device__ __forceinline__ void fwd_true(T (&v)[CL], T a1, T a2, T s0, T s1, T m)
{
#pragma unroll
    for (int k = 0; k < CL; ++k) {
        T u = fma(a1, s0, fma(a2, s1, v[k] - m));
        s1 = s0;
        s0 = u;
        v[k] = u;
    }
}

// anti-causal recursion from a zero state: state at the chunk start (v_0, v_1)
template <typename T, int CL>
__device__ __forceinline__ void bwd_zero(const T (&v)[CL], T a1, T a2, T& e0, T& e1)
{
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int k = CL - 1; k >= 0; --k) {
        T u = fma(a1, s0, fma(a2, s1, v[k]));
        s1 = s0;
        s0 = u;
    }
    e0 = s0;
    e1 = s1;
}

template <typename T, int CL>
__device__ __forceinline__ void bwd_true(T (&v)[CL], T a1, T a2, T s0, T s1, T ik, T m)
{
#pragma unroll
    for (int k = CL - 1; k >= 0; --k) {
        T u = fma(a1, s0, fma(a2, s1, v[k]));
        s1 = s0;
        s0 = u;
        v[k] = fma(u, ik, m);
    }
}

// Cross-lane moves with precomputed ds_bpermute byte addresses (lane * 4).
__device__ __forceinline__ float lane_get(int addr, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_get(int addr, double v)
{
    const int2 w = *reinterpret_cast<int2*>(&v);
    int2 r;
    r.x = __builtin_amdgcn_ds_bpermute(addr, w.x);
    r.y = __builtin_amdgcn_ds_bpermute(addr, w.y);
    return *reinterpret_cast<double*>(&r);
}

// Sum over each aligned group of P lanes (P a power of two, at most 64) by
// butterflies: DPP lane exchanges inside rows of 16 (xor 1, xor 2, then the
// half-row and row mirrors, which pair the group halves in the same way), a
// swizzle across rows for 32 and a permute across halves for 64.  Each level
// adds a lane's value and its partner's, so every lane of the group ends with
// the same bits.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float lane_x(float v)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double lane_x(double v)
{
    int2 w = *reinterpret_cast<int2*>(&v);
    w.x = dpp_i<CTRL>(w.x);
    w.y = dpp_i<CTRL>(w.y);
    return *reinterpret_cast<double*>(&w);
}
__device__ __forceinline__ float swz16(float v)
{
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));  // lane ^ 16 within 32
}
__device__ __forceinline__ double swz16(double v)
{
    int2 w = *reinterpret_cast<int2*>(&v);
    w.x = __builtin_amdgcn_ds_swizzle(w.x, 0x401F);
    w.y = __builtin_amdgcn_ds_swizzle(w.y, 0x401F);
    return *reinterpret_cast<double*>(&w);
}
template <typename T>
__device__ __forceinline__ T group_sum(T x, int P, int lane)
{
    if (P >= 2) x += lane_x<0xB1>(x);   // quad_perm [1,0,3,2]
    if (P >= 4) x += lane_x<0x4E>(x);   // quad_perm [2,3,0,1]
    if (P >= 8) x += lane_x<0x141>(x);  // row_half_mirror
    if (P >= 16) x += lane_x<0x140>(x); // row_mirror
    if (P >= 32) x += swz16(x);
    if (P >= 64) x += lane_get(((lane ^ 32) & 63) << 2, x);
    return x;
}

// Source addresses of the wavefront scans: up[s] = lane - 2^s, dn[s] = lane + 2^s
// (wrapped; only read where the source lies in the same line), and the first
// and last lane of the line.
struct ScanLanes {
    int up[kWaveScanLevels], dn[kWaveScanLevels];
    int first, last;
};

__device__ __forceinline__ void make_lanes(ScanLanes& L, int lane, int gbase, int P)
{
#pragma unroll
    for (int s = 0; s < kWaveScanLevels; ++s) {
        L.up[s] = ((lane - (1 << s)) & 63) << 2;
        L.dn[s] = ((lane + (1 << s)) & 63) << 2;
    }
    L.first = (gbase & 63) << 2;
    L.last = ((gbase + P - 1) & 63) << 2;
}

// Scans of chunk end states over the P lanes of a line inside a wavefront
// (chunk j = lane - first lane of the line), for RL independent lines held by
// the same lanes.  On return (e0[q], e1[q]) is the true state entering chunk
// j of line q.  All 64 lanes must call them (P is uniform).
template <typename T, int RL>
__device__ __forceinline__ void scan_fwd_wave(T (&e0)[RL], T (&e1)[RL], int j, int P,
                                              const ScanLanes& L, const LineCoef<T>& c)
{
#pragma unroll
    for (int s = 0; s < kWaveScanLevels; ++s) {
        const int d = 1 << s;
        if (d < P) {
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                T y0 = lane_get(L.up[s], e0[q]);
                T y1 = lane_get(L.up[s], e1[q]);
                if (j >= d) {
                    mv(c.Mp[s], y0, y1);
                    e0[q] += y0;
                    e1[q] += y1;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RL; ++q) {
        const T z0 = lane_get(L.last, e0[q]);
        const T z1 = lane_get(L.last, e1[q]);
        T r0 = c.W[0] * z0 + c.W[1] * z1;  // state after the whole line = entering chunk 0
        T r1 = c.W[2] * z0 + c.W[3] * z1;
        T p0 = lane_get(L.up[0], e0[q]);
        T p1 = lane_get(L.up[0], e1[q]);
        if (j == 0) {
            p0 = T(0);
            p1 = T(0);
        }
#pragma unroll
        for (int s = 0; s < kWaveScanLevels; ++s)
            if (((1 << s) < P) && (j & (1 << s))) mv(c.Mp[s], r0, r1);
        e0[q] = p0 + r0;
        e1[q] = p1 + r1;
    }
}

template <typename T, int RL>
__device__ __forceinline__ void scan_bwd_wave(T (&e0)[RL], T (&e1)[RL], int j, int P,
                                              const ScanLanes& L, const LineCoef<T>& c)
{
#pragma unroll
    for (int s = 0; s < kWaveScanLevels; ++s) {
        const int d = 1 << s;
        if (d < P) {
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                T y0 = lane_get(L.dn[s], e0[q]);
                T y1 = lane_get(L.dn[s], e1[q]);
                if (j + d < P) {
                    mv(c.Mp[s], y0, y1);
                    e0[q] += y0;
                    e1[q] += y1;
                }
            }
        }
    }
    const int qq = P - 1 - j;
#pragma unroll
    for (int q = 0; q < RL; ++q) {
        const T z0 = lane_get(L.first, e0[q]);
        const T z1 = lane_get(L.first, e1[q]);
        T r0 = c.W[0] * z0 + c.W[1] * z1;  // state at the line start = entering chunk P-1
        T r1 = c.W[2] * z0 + c.W[3] * z1;
        T p0 = lane_get(L.dn[0], e0[q]);
        T p1 = lane_get(L.dn[0], e1[q]);
        if (j == P - 1) {
            p0 = T(0);
            p1 = T(0);
        }
#pragma unroll
        for (int s = 0; s < kWaveScanLevels; ++s)
            if (((1 << s) < P) && (qq & (1 << s))) mv(c.Mp[s], r0, r1);
        e0[q] = p0 + r0;
        e1[q] = p1 + r1;
    }
}

// Diagnostics step n needs (n >= 0): F at n = jK - 1, jK, jK + 1 (the centred
// difference of eq. (dFdt)) and the gradient of mu at n = jK.  One remainder,
// in 32 bits while n fits.
__device__ __forceinline__ void step_needs(int64_t n, int K, bool& needF, bool& needG)
{
    const int r = (n < 0x7fffffff) ? (int)((uint32_t)n % (uint32_t)K) : (int)(n % K);
    needG = r == 0;
    needF = needG || (n >= 1 && r == 1) || r == K - 1;
}

// Per-member reduction of the pass-A partials into the series.  Each thread of
// the block sums a strided subset of the member's partials (Neumaier), the
// wavefronts reduce with a fixed shuffle tree and thread 0 combines the
// wavefront sums in order: the result is deterministic.  blockDim.x must be a
// multiple of 64 (<= 512).  Called by the whole block.
__device__ void finalize_block(const FinArgs& f, int b, int G, double (*sred)[3])
{
    const int tid = threadIdx.x, nthreads = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = *f.nstamp;
    const int K = f.K;
    bool needF = true, needG = true;
    if (f.mode == MODE_STEP) step_needs(n, K, needF, needG);
    if (!needF) return;
    for (int ml = b; ml < f.nmem; ml += G) {
        double s[3] = {0.0, 0.0, 0.0}, cmp[3] = {0.0, 0.0, 0.0};
        const double* pp = f.partials + (int64_t)ml * f.blocks_per_member * 3;
        for (int64_t i = tid; i < f.blocks_per_member; i += nthreads) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double x = pp[i * 3 + q];
                const double t = s[q] + x;
                cmp[q] += (fabs(s[q]) >= fabs(x)) ? (s[q] - t) + x : (x - t) + s[q];
                s[q] = t;
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] += cmp[q];
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int q = 0; q < 3; ++q) s[q] += __shfl_down(s[q], off, 64);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 3; ++q) sred[wave][q] = s[q];
        __syncthreads();
        if (tid == 0) {
            double t[3] = {0.0, 0.0, 0.0};
            for (int w = 0; w < nthreads / 64; ++w)
#pragma unroll
                for (int q = 0; q < 3; ++q) t[q] += sred[w][q];
            const int gm = f.mids[ml];
            const MemberDev& mm = f.mem[gm];
            const double F = mm.vol * t[0];
            const double mC = t[1] / (double)mm.sites;
            const double Gid = -mm.vol * t[2];
            double* ser = f.series + (int64_t)gm * f.max_samples * kSeriesSlots;
            const int64_t ms = f.max_samples;
            if (n % K == 0 && n / K < ms) {
                ser[(n / K) * kSeriesSlots + 1] = F;
                if (needG) {
                    ser[(n / K) * kSeriesSlots + 3] = mC;
                    ser[(n / K) * kSeriesSlots + 4] = Gid;
                }
            }
            if (n >= 1 && (n - 1) % K == 0 && (n - 1) / K < ms) ser[((n - 1) / K) * kSeriesSlots + 2] = F;
            if ((n + 1) % K == 0 && (n + 1) / K < ms) ser[((n + 1) / K) * kSeriesSlots + 0] = F;
            if (f.mode == MODE_DIAG) {
                double* en = f.energy_now + (int64_t)gm * 4;
                en[0] = F;
                en[1] = mC;
                en[2] = Gid;
                en[3] = (double)n;
            }
            if (!isfinite(F)) f.flags[gm] = 1;
        }
        __syncthreads();  // sred is reused by the next member
    }
}

__global__ void __launch_bounds__(256) fin_kernel(FinArgs f)
{
    __shared__ double sred[4][3];
    finalize_block(f, blockIdx.x, gridDim.x, sred);
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};

template <typename T>
__device__ __forceinline__ void vec_get(const typename Vec16<T>::type& v, T* out);
template <>
__device__ __forceinline__ void vec_get<double>(const double2& v, double* out)
{
    out[0] = v.x;
    out[1] = v.y;
}
template <>
__device__ __forceinline__ void vec_get<float>(const float4& v, float* out)
{
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
}
template <typename T>
__device__ __forceinline__ typename Vec16<T>::type vec_make(const T* in);
template <>
__device__ __forceinline__ double2 vec_make<double>(const double* in)
{
    return make_double2(in[0], in[1]);
}
template <>
__device__ __forceinline__ float4 vec_make<float>(const float* in)
{
    return make_float4(in[0], in[1], in[2], in[3]);
}

template <typename T>
struct PadOf;
// LDS row layout of pass A: HALO periodic halo columns on each side (the
// 16-byte vector width, so a staged vector never straddles a chunk) and one
// element of padding after every chunk of CX elements, so that the lanes of a
// line, which read chunk-strided addresses, fall into different banks.
template <>
struct PadOf<double> {
    static constexpr int v = 1;
};
template <>
struct PadOf<float> {
    static constexpr int v = 1;
};

// --------------------------------------------------------------------------
// pass A: RHS + diagnostics + x-line solves
// --------------------------------------------------------------------------
// Stages rows y0 - ylo + r (r < nrows, periodic in y) of the planes
// z - 1 + pl (pl < npl; 3D, periodic in z) of a member's field into LDS row
// pl * planeStride + r * pitch: element x at HALO + x in the chunk layout, and
// (halos) one vector of periodic halo on either side of every row.
// Interior: a wavefront stages whole rows (rows of all planes go to the
// wavefronts round-robin), its lanes take consecutive 16-byte vectors of a
// row in segments of 64, and each lane issues NB loads before it writes any
// of them to LDS.  Row bases are wave-uniform (scalar registers).  Halos: one
// vector on each side of every row, one per thread.
template <typename T, int DIM, int CX>
__device__ __forceinline__ void stage_rows(T* sC, __amdgpu_buffer_rsrc_t rC, int nrows, int npl, int ylo,
                                           int y0, int z, int nx, int ny, int nz, int pitch, int planeStride,
                                           bool halos)
{
    constexpr int PADE = PadOf<T>::v;
    constexpr int VEC = Vec16<T>::n;
    constexpr int HALO = VEC;
    using VT = typename Vec16<T>::type;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nthreads = blockDim.x;  // 64 * waves
    const int nwaves = nthreads >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nvec = nx / VEC;
    const int nrows_all = npl * nrows;
    const int nseg = (nvec + 63) >> 6;
    constexpr int NB = 8;
    // a segment of 64 vectors holds whole chunks: its LDS span is SEGW, and a
    // lane's vector sits at the same offset `ll` in every segment
    constexpr int SEGW = 64 * VEC + (64 * VEC / CX) * PADE;
    static_assert((64 * VEC) % CX == 0, "segments hold whole chunks");
    const int lx = lane * VEC + HALO;
    const int ll = lx + (lx / CX) * PADE;
    const int lv = lane * VEC * (int)sizeof(T);
    if (DIM == 2 && (nvec & 63) == 0) {
        // one plane, every lane has a vector in every segment: per vector only
        // the wave-uniform row and segment advance
        int r = wv, seg = 0;  // wave-uniform cursor (row, segment)
        while (r < nrows) {
            VT val[NB];
            int dst[NB];
            bool use[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                use[i] = r < nrows;
                dst[i] = r * pitch + seg * SEGW;
                if (use[i]) {
                    const int rowo = wrapi(y0 - ylo + r, ny) * nx + seg * 64 * VEC;  // wave-uniform
                    val[i] = buf_load16<VT>(rC, lv, rowo * (int)sizeof(T));
                    if (++seg == nseg) {
                        seg = 0;
                        r += nwaves;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (use[i]) {
                    T e[VEC];
                    vec_get<T>(val[i], e);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) sC[dst[i] + ll + q] = e[q];
                }
        }
    } else if constexpr (DIM == 2) {
        // one plane: the wavefront's rows are wv, wv + nwaves, ...
        int r = wv, seg = 0;  // wave-uniform cursor (row, segment)
        while (r < nrows) {
            VT val[NB];
            int dst[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                dst[i] = -1;
                if (r < nrows) {
                    const int rowo = wrapi(y0 - ylo + r, ny) * nx;  // wave-uniform
                    const int xi = seg * 64 + lane;
                    if (xi < nvec) {
                        const uint32_t xs = (uint32_t)xi * VEC, xx = xs + HALO;
                        val[i] = buf_load16<VT>(rC, (int)xs * (int)sizeof(T), rowo * (int)sizeof(T));
                        dst[i] = r * pitch + (int)(xx + xx / CX * PADE);
                    }
                    if (++seg == nseg) {
                        seg = 0;
                        r += nwaves;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (dst[i] >= 0) {
                    T e[VEC];
                    vec_get<T>(val[i], e);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) sC[dst[i] + q] = e[q];
                }
        }
    } else {
        int pl = 0, r = wv, seg = 0;  // wave-uniform cursor (plane, row, segment)
        while (r >= nrows) {
            r -= nrows;
            ++pl;
        }
        while (pl < npl) {
            VT val[NB];
            int dst[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                dst[i] = -1;
                if (pl < npl) {
                    const int zz = (DIM == 3) ? wrapi(z - 1 + pl, nz) : 0;
                    const int yy = wrapi(y0 - ylo + r, ny);
                    const int rowo = (zz * ny + yy) * nx;  // wave-uniform
                    const int xi = seg * 64 + lane;
                    if (xi < nvec) {
                        const uint32_t xs = (uint32_t)xi * VEC, xx = xs + HALO;
                        val[i] = buf_load16<VT>(rC, (int)xs * (int)sizeof(T), rowo * (int)sizeof(T));
                        dst[i] = pl * planeStride + r * pitch + (int)(xx + xx / CX * PADE);
                    }
                    if (++seg == nseg) {
                        seg = 0;
                        r += nwaves;
                        while (r >= nrows) {
                            r -= nrows;
                            ++pl;
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (dst[i] >= 0) {
                    T e[VEC];
                    vec_get<T>(val[i], e);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) sC[dst[i] + q] = e[q];
                }
        }
    }
    {
        if (halos)
            for (int h = tid; h < 2 * nrows_all; h += nthreads) {
                const int rid = h >> 1, pl = rid / nrows, r = rid - pl * nrows;
                const int zz = (DIM == 3) ? wrapi(z - 1 + pl, nz) : 0;
                const int yy = wrapi(y0 - ylo + r, ny);
                // left halo: the last vector of the row; right halo: the first
                const int xs = (h & 1) ? 0 : nx - HALO;
                const int xx = (h & 1) ? nx + HALO : 0;
                const VT val = buf_load16<VT>(rC, ((zz * ny + yy) * nx + xs) * (int)sizeof(T), 0);
                T e[VEC];
                vec_get<T>(val, e);
                const int d = pl * planeStride + r * pitch + xx + (xx / CX) * PADE;
#pragma unroll
                for (int q = 0; q < VEC; ++q) sC[d + q] = e[q];
            }
    }
}

// Per-lane partial sums of the diagnostics over the lane's chunk of its RL
// lines (FP64): F (bulk + gradient energy, forward differences), sum C, and
// sum |grad_h mu|^2 with mu = C^3 - C - gamma lap_h C.  `at(dz, dy, m)`
// reads the staged field at plane offset dz, line dy of the lane's lines and
// element m of its chunk (the halo included); bit q of rowmask marks line q
// as inside the grid.
template <typename T, int DIM, int CX, int RL, typename At>
__device__ __forceinline__ void diag_sums(const At& at, unsigned rowmask, const MemberDev& md, int conv,
                                          bool needF, bool needG, double& pF, double& pS, double& pG)
{
    constexpr int HALO = Vec16<T>::n;
#define AT(dz, dy, m) at(dz, dy, m)
    if (needF) {
        const double cbulk = conv ? 0.5 : 0.25;
        const double hg = 0.5 * md.gamma;
        const double dx2 = md.ih2[0], dy2 = md.ih2[1], dz2 = md.ih2[2];
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            if (!((rowmask >> q) & 1)) continue;
#pragma unroll
            for (int k = 0; k < CX; ++k) {
                const int m0 = k + HALO;
                const double c = (double)AT(0, q, m0);
                const double ex = (double)AT(0, q, m0 + 1) - c;
                const double ey = (double)AT(0, q + 1, m0) - c;
                double gr = ex * ex * dx2 + ey * ey * dy2;
                if (DIM == 3) {
                    const double ez = (double)AT(1, q, m0) - c;
                    gr += ez * ez * dz2;
                }
                const double qq = c * c - 1.0;
                pF += cbulk * qq * qq + hg * gr;
                pS += c;
            }
        }
    }
    if (needG) {
        const double gam = md.gamma;
        const double dx2 = md.ih2[0], dy2 = md.ih2[1], dz2 = md.ih2[2];
        // chemical potential mu = C^3 - C - gamma lap_h C at (dz, dy, m)
        auto MU = [&](int dz, int dy, int m) -> double {
            const double u = (double)AT(dz, dy, m);
            double l = ((double)AT(dz, dy, m + 1) - 2.0 * u + (double)AT(dz, dy, m - 1)) * dx2 +
                       ((double)AT(dz, dy + 1, m) - 2.0 * u + (double)AT(dz, dy - 1, m)) * dy2;
            if (DIM == 3)
                l += ((double)AT(dz + 1, dy, m) - 2.0 * u + (double)AT(dz - 1, dy, m)) * dz2;
            return u * u * u - u - gam * l;
        };
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            if (!((rowmask >> q) & 1)) continue;
#pragma unroll
            for (int k = 0; k < CX; ++k) {
                const int m0 = k + HALO;
                const double mu = MU(0, q, m0);
                const double gx = MU(0, q, m0 + 1) - mu;
                const double gy = MU(0, q + 1, m0) - mu;
                double qq = gx * gx * dx2 + gy * gy * dy2;
                if (DIM == 3) {
                    const double gz = MU(1, q, m0) - mu;
                    qq += gz * gz * dz2;
                }
                pG += qq;
            }
        }
    }
#undef AT
}

// A lane's results (lines rl0 .. rl0+RL-1, chunk j) go to LDS rows of `so`
// in the staging layout, and each wavefront then stores the lines it holds
// itself (lines wv*rpw .. wv*rpw+rpw-1 of the unit) with coalesced 16-byte
// stores, lanes along the line.  The rows a wavefront reads back are the rows
// it wrote, and a wavefront's LDS operations complete in order, so only a
// wavefront-scope fence sits between the two.  The caller ends every read of
// these LDS rows (a block barrier) first.
template <typename T, int CX, int RL>
__device__ __forceinline__ void write_back(T* so, int pitch, const T (&v)[RL][CX], const bool (&rowok)[RL],
                                           int rl0, int j, int wv, int lane, int rpw, int Ract, int nvec,
                                           __amdgpu_buffer_rsrc_t rout, int out0, int nx)
{
    constexpr int PADE = PadOf<T>::v;
    constexpr int VEC = Vec16<T>::n;
    constexpr int HALO = VEC;
    using VT = typename Vec16<T>::type;
#pragma unroll
    for (int q = 0; q < RL; ++q) {
        if (!rowok[q]) continue;
        T* sr = so + (rl0 + q) * pitch + j * (CX + PADE);
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            const int m = k + HALO;
            sr[m + (m / CX) * PADE] = v[q][k];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nseg = (nvec + 63) >> 6;
    const int l1 = min(wv * rpw + rpw, Ract);
    constexpr int NB = 8;
    constexpr int SEGW = 64 * VEC + (64 * VEC / CX) * PADE;  // LDS span of a segment of 64 vectors
    static_assert((64 * VEC) % CX == 0, "segments hold whole chunks");
    if ((nvec & 63) == 0) {
        // every lane has a vector in every segment (see stage_rows)
        const int lx = lane * VEC + HALO;
        const int ll = lx + (lx / CX) * PADE;
        const int lv = lane * VEC * (int)sizeof(T);
        int l = wv * rpw, seg = 0;  // wave-uniform cursor (line, segment)
        while (l < l1) {
            VT val[NB];
            int row[NB];  // byte offset of the line's segment in the output (wave-uniform)
            bool use[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                use[i] = l < l1;
                row[i] = (out0 + l * nx + seg * 64 * VEC) * (int)sizeof(T);
                if (use[i]) {
                    val[i] = vec_make<T>(so + l * pitch + seg * SEGW + ll);
                    if (++seg == nseg) {
                        seg = 0;
                        ++l;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (use[i]) buf_store16<VT>(val[i], rout, lv, row[i]);
        }
        return;
    }
    int l = wv * rpw, seg = 0;  // wave-uniform cursor (line, segment)
    while (l < l1) {
        VT val[NB];
        int row[NB];  // element offset of the line in the output (wave-uniform)
        int off[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            off[i] = -1;
            row[i] = out0 + l * nx;
            if (l < l1) {
                const int xv = seg * 64 + lane;
                if (xv < nvec) {
                    const uint32_t xo = (uint32_t)xv * VEC, xx = xo + HALO;
                    val[i] = vec_make<T>(so + l * pitch + (int)(xx + xx / CX * PADE));
                    off[i] = (int)xo;
                }
                if (++seg == nseg) {
                    seg = 0;
                    ++l;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (off[i] >= 0) buf_store16<VT>(val[i], rout, off[i] * (int)sizeof(T), row[i] * (int)sizeof(T));
    }
}


// RHS of the scheme at line q, element m of a lane's staged rows:
//   C + dt lap_h(C^3 - C) - 2 gamma dt sum_{d<e} D_d D_e C
// with the coefficients folded: dx = dt / h_x^2 (etc.) and
// gxy = 2 gamma dt / (h_x^2 h_y^2) (etc.), so that each second difference
// costs one add and one fma and enters with one fma.
// `at(dz, dy, m)` reads the staged field.  A mixed term D_d D_e C is formed
// as the d-second difference of e-second differences; the inner differences
// and the values of C^3 - C at neighbouring sites are the same expressions a
// neighbouring element or line of the lane forms, so the unrolled loops
// compute each of them once.
template <typename T, int DIM, typename At>
__device__ __forceinline__ T rhs_site(const At& at, int q, int m, T dx, T dy, T dz, T gxy, T gxz, T gyz)
{
    auto N = [](T c) { return c * c * c - c; };
    auto d2 = [](T a, T b, T c) { return fma(T(-2), b, a + c); };  // a - 2 b + c
    auto dyy = [&](int dzz, int mm) { return d2(at(dzz, q + 1, mm), at(dzz, q, mm), at(dzz, q - 1, mm)); };
    const T c = at(0, q, m);
    const T Nc = N(c);
    T r = fma(dx, d2(N(at(0, q, m + 1)), Nc, N(at(0, q, m - 1))), c);
    r = fma(dy, d2(N(at(0, q + 1, m)), Nc, N(at(0, q - 1, m))), r);
    r = fma(-gxy, d2(dyy(0, m + 1), dyy(0, m), dyy(0, m - 1)), r);
    if (DIM == 3) {
        auto dzz = [&](int ddy, int mm) {
            return d2(at(1, q + ddy, mm), at(0, q + ddy, mm), at(-1, q + ddy, mm));
        };
        r = fma(dz, d2(N(at(1, q, m)), Nc, N(at(-1, q, m))), r);
        r = fma(-gxz, d2(dzz(0, m + 1), dzz(0, m), dzz(0, m - 1)), r);
        r = fma(-gyz, d2(dzz(1, m), dzz(0, m), dzz(-1, m)), r);
    }
    return r;
}


// Crank-Nicolson variant (2D): g = dt lap_h(C^3 - C) - 2 gamma dt D_x D_y C
// - gamma dt (D_x^2 + D_y^2) C at line q, element m, and b = C + gamma dt
// D_y^2 C / 2, the part of the x-solve's output that bypasses the solve.
template <typename T, typename At>
__device__ __forceinline__ void rhs_cn_site(const At& at, int q, int m, T ihx2, T ihy2, T dt, T tg, T cxy,
                                            T ax4, T ay4, T& g, T& b)
{
    auto N = [](T c) { return c * c * c - c; };
    auto dyy = [&](int mm) { return at(0, q + 1, mm) + at(0, q - 1, mm) - T(2) * at(0, q, mm); };
    const T c = at(0, q, m);
    const T Nc = N(c);
    const T lapN = (N(at(0, q, m + 1)) + N(at(0, q, m - 1)) - T(2) * Nc) * ihx2 +
                   (N(at(0, q + 1, m)) + N(at(0, q - 1, m)) - T(2) * Nc) * ihy2;
    const T cross = (dyy(m + 1) + dyy(m - 1) - T(2) * dyy(m)) * cxy;
    const T d4x = (at(0, q, m - 2) + at(0, q, m + 2)) - T(4) * (at(0, q, m - 1) + at(0, q, m + 1)) + T(6) * c;
    const T d4y = (at(0, q - 2, m) + at(0, q + 2, m)) - T(4) * (at(0, q - 1, m) + at(0, q + 1, m)) + T(6) * c;
    g = dt * lapN - tg * cross - ax4 * d4x - ay4 * d4y;
    b = c + T(0.5) * ay4 * d4y;
}


// The second launch bound is the wavefronts per SIMD the compiler must leave
// room for.  The FP32 2D shapes with at most 16 elements per lane fit 80
// registers without spilling (the unconstrained build takes 83 for c = 16,
// one wavefront per SIMD fewer than the LDS of a block allows); the others
// keep the compiler's choice.
template <typename T, int DIM, int CX, int RL, bool CN>
__global__ void __launch_bounds__(kPassAThreads, (sizeof(T) == 4 && DIM == 2 && !CN && CX * RL <= 16) ? 6 : 1)
    passA_kernel(PassAArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* sC = reinterpret_cast<T*>(lds_raw);
    __shared__ double red[kPassAThreads / 64][3];

    constexpr int PADE = PadOf<T>::v;
    constexpr int VEC = Vec16<T>::n;
    constexpr int HALO = VEC;
    static_assert(CX % VEC == 0, "LDS layout assumes vector-aligned chunks");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    const uint32_t blk = xcd_remap(blockIdx.x, (uint32_t)a.nblocks);
    const uint32_t per_member = (uint32_t)a.bands_y * (uint32_t)nz;
    const int mloc = (int)(blk / per_member);
    const uint32_t rem = blk - (uint32_t)mloc * per_member;
    const int z = (int)(rem / (uint32_t)a.bands_y);
    const int y0 = (int)(rem - (uint32_t)z * (uint32_t)a.bands_y) * a.R;
    const int mid = member_id(a.run, a.mids, mloc);
    const MemberDev& md = a.mem[mid];
    const int64_t moff = member_off(a.run, a.mem, mid, mloc);
    const uint32_t bytes = (uint32_t)((int64_t)nx * ny * nz * (int64_t)sizeof(T));
    const T* C = reinterpret_cast<const T*>(a.C) + moff;
    T* Wout = reinterpret_cast<T*>(a.W) + moff;
    // the member's field as a buffer: rows are wave-uniform scalar offsets
    const __amdgpu_buffer_rsrc_t rC = buffer_of(C, bytes);

    const int64_t n = *a.step;
    const int K = a.K;
    bool needF = a.mode == MODE_DIAG, needG = a.mode == MODE_DIAG;
    if (a.mode == MODE_STEP) step_needs(n, K, needF, needG);
    const bool solve = (a.mode != MODE_DIAG);

    // ---- stage C rows (with periodic halos) in LDS --------------------------
    // staged rows: y0 - YLO .. y0 + Ract - 1 + (rows below); the
    // Crank-Nicolson variant reads two rows on either side (D_y^2)
    constexpr int YLO = CN ? 2 : 1;
    const int rowsAlloc = a.R + (CN ? 4 : 3);
    const int pitch = a.pitch;
    const int planeStride = rowsAlloc * pitch;
    const int Ract = min(a.R, ny - y0);  // x-lines of this block inside the grid
    const int nrows = Ract + (CN ? 4 : (needG ? 3 : 2));
    const int npl = (DIM == 3) ? (needG ? 4 : 3) : 1;
    const int nvec = nx / VEC;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int nthreads = blockDim.x;  // 64 * waves
    stage_rows<T, DIM, CX>(sC, rC, nrows, npl, YLO, y0, z, nx, ny, nz, pitch, planeStride, true);
    __syncthreads();

    // ---- per-lane work: one chunk of CX elements of RL adjacent x-lines ------
    // Lanes j = 0..P-1 of a group hold consecutive chunks of the same RL lines;
    // sharing rows between the RL lines of a lane saves stencil work, and the
    // RL independent recursions interleave.
    const int P = a.P;
    const int g = lane_div(lane, P);          // line group within the wavefront
    const int j = lane - g * P;               // chunk index along the line
    const int groups = a.rows_per_wave / RL;  // line groups per wavefront
    const int rl0 = (wave * groups + g) * RL; // first x-line of this lane in the block
    const bool lane_ok = g < groups;
    bool rowok[RL];
#pragma unroll
    for (int q = 0; q < RL; ++q) rowok[q] = lane_ok && (rl0 + q < Ract);
    const bool active = rowok[0];
    constexpr int PL0 = (DIM == 3) ? 1 : 0;
    const T* cb = sC + PL0 * planeStride + (rl0 + YLO) * pitch + j * (CX + PADE);
#define AT(dz, dy, m) cb[(dz) * planeStride + (dy) * pitch + (m) + ((m) / CX) * PADE]

    // folded coefficients of the RHS
    const T* rc = CoefOf<T>::rc(md);
    const T ihx2 = rc[RC_IHX2], ihy2 = rc[RC_IHY2], dt = rc[RC_DT], tg = rc[RC_TG], cxy = rc[RC_CXY];
    const T cdx = rc[RC_DX], cdy = rc[RC_DY], cdz = rc[RC_DZ];
    const T gxy = rc[RC_GXY], gxz = rc[RC_GXZ], gyz = rc[RC_GYZ];

    // The RHS is formed on every lane: lines past the end of a ragged last
    // band read staged rows that exist (R + 3 are allocated) and their
    // results are never stored or summed.
    T v[RL][CX];
    T bypass[CN ? RL : 1][CN ? CX : 1];  // Crank-Nicolson: C + a D_y^2 C / 2, added after the x-solve
    if (solve) {
        auto at = [&](int dz, int dy, int m) { return AT(dz, dy, m); };
        if (CN) {
            const T ax4 = rc[RC_AX4], ay4 = rc[RC_AY4];
#pragma unroll
            for (int k = 0; k < CX; ++k)
#pragma unroll
                for (int q = 0; q < RL; ++q)
                    rhs_cn_site<T>(at, q, k + HALO, ihx2, ihy2, dt, tg, cxy, ax4, ay4, v[q][k],
                                   bypass[CN ? q : 0][CN ? k : 0]);
        } else {
#pragma unroll
            for (int k = 0; k < CX; ++k)
#pragma unroll
                for (int q = 0; q < RL; ++q)
                    v[q][k] = rhs_site<T, DIM>(at, q, k + HALO, cdx, cdy, cdz, gxy, gxz, gyz);
        }
    }

    double pF = 0.0, pS = 0.0, pG = 0.0;
    if (active) {
        unsigned rm = 0;
#pragma unroll
        for (int q = 0; q < RL; ++q) rm |= rowok[q] ? (1u << q) : 0u;
        auto at = [&](int dz, int dy, int m) { return AT(dz, dy, m); };
        diag_sums<T, DIM, CX, RL>(at, rm, md, a.conv, needF, needG, pF, pS, pG);
    }
#undef AT

    // ---- x-line solves (lanes of one line are contiguous in the wavefront) ---
    T mean[RL];
    if (solve) {
        LineCoef<T> cf;
        load_coef(cf, CoefOf<T>::ax(md, 0), P);
        ScanLanes SL;
        make_lanes(SL, lane, g * P, P);
        // the line mean passes through (I + rho D^4)^{-1} unchanged: take it out
        // before the recursions and add it back at the end
        T csum[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            csum[q] = T(0);
#pragma unroll
            for (int k = 0; k < CX; ++k) csum[q] += v[q][k];
        }
        if ((P & (P - 1)) == 0) {
#pragma unroll
            for (int q = 0; q < RL; ++q) csum[q] = group_sum(csum[q], P, lane);
        } else {
#pragma unroll
            for (int s = 0; s < kWaveScanLevels; ++s) {
                const int d = 1 << s;
                if (d < P) {
#pragma unroll
                    for (int q = 0; q < RL; ++q) {
                        const T y = lane_get(SL.up[s], csum[q]);
                        if (j >= d) csum[q] += y;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RL; ++q) csum[q] = lane_get(SL.last, csum[q]);
        }
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            mean[q] = csum[q] * CoefOf<T>::ax(md, 0).inv_n;
#pragma unroll
            for (int k = 0; k < CX; ++k) v[q][k] -= mean[q];
        }
        T e0[RL], e1[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) fwd_zero(v[q], cf.a1, cf.a2, e0[q], e1[q]);
        scan_fwd_wave<T, RL>(e0, e1, j, P, SL, cf);
#pragma unroll
        for (int q = 0; q < RL; ++q) fwd_true(v[q], cf.a1, cf.a2, e0[q], e1[q], T(0));
#pragma unroll
        for (int q = 0; q < RL; ++q) bwd_zero(v[q], cf.a1, cf.a2, e0[q], e1[q]);
        scan_bwd_wave<T, RL>(e0, e1, j, P, SL, cf);
#pragma unroll
        for (int q = 0; q < RL; ++q) bwd_true(v[q], cf.a1, cf.a2, e0[q], e1[q], cf.ik, mean[q]);
        if (CN)
#pragma unroll
            for (int q = 0; q < RL; ++q)
#pragma unroll
                for (int k = 0; k < CX; ++k) v[q][k] += bypass[CN ? q : 0][CN ? k : 0];
    }

    // ---- diagnostics partials -------------------------------------------------
    if (needF) {
        for (int off = 32; off > 0; off >>= 1) {
            pF += __shfl_down(pF, off, 64);
            pS += __shfl_down(pS, off, 64);
            pG += __shfl_down(pG, off, 64);
        }
        if (lane == 0) {
            red[wave][0] = pF;
            red[wave][1] = pS;
            red[wave][2] = pG;
        }
    }
    __syncthreads();  // LDS stencil reads done; wave partials visible

    // ---- write w through LDS (coalesced) -------------------------------------
    // (the __syncthreads above ended every read of the staged rows)
    if (solve)
        write_back<T, CX, RL>(sC + pitch, pitch, v, rowok, rl0, j, wv, lane, a.rows_per_wave, Ract, nvec,
                              buffer_of(Wout, bytes), (z * ny + y0) * nx, nx);

    // ---- block partials of F, sum C, sum |grad mu|^2 (reduced by finalize) ----
    if (blk == 0 && tid == 0 && a.mode != MODE_TIMING) *a.nstamp = n;
    if (needF && tid == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int w = 0; w < nthreads / 64; ++w) {
            s0 += red[w][0];
            s1 += red[w][1];
            s2 += red[w][2];
        }
        a.partials[(size_t)blk * 3 + 0] = s0;
        a.partials[(size_t)blk * 3 + 1] = s1;
        a.partials[(size_t)blk * 3 + 2] = s2;
    }
}

// --------------------------------------------------------------------------
// pass A for lines longer than one wavefront (2D)
// --------------------------------------------------------------------------
// A line of P = 64 WL chunks is held by WL wavefronts (lane = chunk within
// the wavefront's segment of 64 chunks); a block of 4 wavefronts holds
// R = 4 / WL lines.  The chunk scans run inside each wavefront as in pass A
// and are then combined over the line's wavefronts through LDS.  With T_w the
// end state of segment w from a zero start and A64 = (A^c)^64 the transfer
// over one segment, the zero-start state entering segment w is
// S_w = A64 S_{w-1} + T_{w-1} (S_0 = 0), the ring closes with
// r = (I - A^n)^{-1} S_WL, and chunk j = 64 w + lane enters with
// (A^c)^lane (A64^w r + S_w) plus the exclusive prefix inside the segment.
// The anti-causal recursion mirrors this from the right end.
// XONLY: the RHS is already in W (rhs_tile_kernel formed it and took the
// diagnostics); only the block's lines are staged, then solved in place.
template <typename T, int CX, int WL, bool XONLY>
__global__ void __launch_bounds__(kPassAThreads) passA_wide_kernel(PassAArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* sC = reinterpret_cast<T*>(lds_raw);
    __shared__ double red[kPassAThreads / 64][3];
    // per wavefront: chunk-sum total, and the end states of the two scans
    // (separate arrays, so that no barrier guards their reuse)
    __shared__ T ssum[kPassAThreads / 64];
    __shared__ T sfw[kPassAThreads / 64][2];
    __shared__ T sbw[kPassAThreads / 64][2];

    constexpr int PADE = PadOf<T>::v;
    constexpr int VEC = Vec16<T>::n;
    constexpr int HALO = VEC;
    constexpr int R = (kPassAThreads / 64) / WL;  // lines per block
    static_assert(CX % VEC == 0 && R >= 1 && (kPassAThreads / 64) % WL == 0, "wide pass A shape");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = wv / WL, wl = wv - li * WL;  // line of the block, wavefront within the line
    const int nx = a.nx, ny = a.ny;

    const uint32_t blk = xcd_remap(blockIdx.x, (uint32_t)a.nblocks);
    const int mloc = (int)(blk / (uint32_t)a.bands_y);
    const int y0 = (int)(blk - (uint32_t)mloc * (uint32_t)a.bands_y) * R;
    const int mid = member_id(a.run, a.mids, mloc);
    const MemberDev& md = a.mem[mid];
    const int64_t moff = member_off(a.run, a.mem, mid, mloc);
    const uint32_t bytes = (uint32_t)((int64_t)nx * ny * (int64_t)sizeof(T));
    T* Wout = reinterpret_cast<T*>(a.W) + moff;
    const T* src = XONLY ? Wout : reinterpret_cast<const T*>(a.C) + moff;

    const int64_t n = *a.step;
    const int K = a.K;
    bool needF = !XONLY && a.mode == MODE_DIAG, needG = needF;
    if (!XONLY && a.mode == MODE_STEP) step_needs(n, K, needF, needG);
    const bool solve = (a.mode != MODE_DIAG);

    constexpr int YLO = XONLY ? 0 : 1;
    const int pitch = a.pitch;
    const int Ract = min(R, ny - y0);
    const int nrows = XONLY ? Ract : Ract + (needG ? 3 : 2);
    stage_rows<T, 2, CX>(sC, buffer_of(src, bytes), nrows, 1, YLO, y0, 0, nx, ny, 1, pitch, 0, !XONLY);
    __syncthreads();

    // lines past the end of a ragged last band compute on rows that exist
    // (R + 3 are allocated; R in the XONLY form) and are never stored or summed
    const int j = wl * 64 + lane;  // chunk of the line
    const bool active = li < Ract;
    const T* cb = sC + (li + YLO) * pitch + j * (CX + PADE);
    T v[1][CX];
    if (XONLY) {
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            const int m = k + HALO;
            v[0][k] = cb[m + (m / CX) * PADE];
        }
    } else if (solve) {
        const T* rc = CoefOf<T>::rc(md);
        const T cdx = rc[RC_DX], cdy = rc[RC_DY], gxy = rc[RC_GXY];
        auto at = [&](int, int dy, int m) { return cb[dy * pitch + m + (m / CX) * PADE]; };
#pragma unroll
        for (int k = 0; k < CX; ++k) v[0][k] = rhs_site<T, 2>(at, 0, k + HALO, cdx, cdy, T(0), gxy, T(0), T(0));
    }
    double pF = 0.0, pS = 0.0, pG = 0.0;
    if (!XONLY && active) {
        auto at = [&](int, int dy, int m) { return cb[dy * pitch + m + (m / CX) * PADE]; };
        diag_sums<T, 2, CX, 1>(at, 1u, md, a.conv, needF, needG, pF, pS, pG);
    }

    // ---- x-line solves across the line's wavefronts ------------------------
    T mean = T(0);
    if (solve) {
        const auto& ac = CoefOf<T>::ax(md, 0);
        LineCoef<T> cf;
        load_coef(cf, ac, 64);
        T A64[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) A64[i] = ac.Mp[kWaveScanLevels][i];
        ScanLanes SL;
        make_lanes(SL, lane, 0, 64);
        // the line mean: chunk sums added up inside the wavefront, the
        // wavefront totals added in order (the same order for every wavefront
        // of the line)
        T cs = T(0);
#pragma unroll
        for (int k = 0; k < CX; ++k) cs += v[0][k];
        cs = group_sum(cs, 64, lane);
        if (lane == 63) ssum[wv] = cs;
        __syncthreads();
        T tot = T(0);
        for (int w = 0; w < WL; ++w) tot += ssum[li * WL + w];
        mean = tot * ac.inv_n;
#pragma unroll
        for (int k = 0; k < CX; ++k) v[0][k] -= mean;

        // causal recursion
        T e0, e1;
        fwd_zero(v[0], cf.a1, cf.a2, e0, e1);
#pragma unroll
        for (int s = 0; s < kWaveScanLevels; ++s) {
            T y0v = lane_get(SL.up[s], e0), y1v = lane_get(SL.up[s], e1);
            if (lane >= (1 << s)) {
                mv(cf.Mp[s], y0v, y1v);
                e0 += y0v;
                e1 += y1v;
            }
        }
        if (lane == 63) {
            sfw[wv][0] = e0;
            sfw[wv][1] = e1;
        }
        __syncthreads();
        {
            T S0 = T(0), S1 = T(0), U0 = T(0), U1 = T(0);
            for (int w = 0; w < WL; ++w) {
                if (w == wl) {
                    U0 = S0;
                    U1 = S1;
                }
                mv(A64, S0, S1);
                S0 += sfw[li * WL + w][0];
                S1 += sfw[li * WL + w][1];
            }
            T r0 = cf.W[0] * S0 + cf.W[1] * S1, r1 = cf.W[2] * S0 + cf.W[3] * S1;
            for (int w = 0; w < wl; ++w) mv(A64, r0, r1);
            r0 += U0;
            r1 += U1;
#pragma unroll
            for (int s = 0; s < kWaveScanLevels; ++s)
                if (lane & (1 << s)) mv(cf.Mp[s], r0, r1);
            T p0 = lane_get(SL.up[0], e0), p1 = lane_get(SL.up[0], e1);
            if (lane == 0) {
                p0 = T(0);
                p1 = T(0);
            }
            fwd_true(v[0], cf.a1, cf.a2, p0 + r0, p1 + r1, T(0));
        }

        // anti-causal recursion
        bwd_zero(v[0], cf.a1, cf.a2, e0, e1);
#pragma unroll
        for (int s = 0; s < kWaveScanLevels; ++s) {
            T y0v = lane_get(SL.dn[s], e0), y1v = lane_get(SL.dn[s], e1);
            if (lane + (1 << s) < 64) {
                mv(cf.Mp[s], y0v, y1v);
                e0 += y0v;
                e1 += y1v;
            }
        }
        if (lane == 0) {
            sbw[wv][0] = e0;
            sbw[wv][1] = e1;
        }
        __syncthreads();
        {
            T S0 = T(0), S1 = T(0), U0 = T(0), U1 = T(0);
            for (int w = WL - 1; w >= 0; --w) {
                if (w == wl) {
                    U0 = S0;
                    U1 = S1;
                }
                mv(A64, S0, S1);
                S0 += sbw[li * WL + w][0];
                S1 += sbw[li * WL + w][1];
            }
            T r0 = cf.W[0] * S0 + cf.W[1] * S1, r1 = cf.W[2] * S0 + cf.W[3] * S1;
            for (int w = WL - 1; w > wl; --w) mv(A64, r0, r1);
            r0 += U0;
            r1 += U1;
#pragma unroll
            for (int s = 0; s < kWaveScanLevels; ++s)
                if ((63 - lane) & (1 << s)) mv(cf.Mp[s], r0, r1);
            T p0 = lane_get(SL.dn[0], e0), p1 = lane_get(SL.dn[0], e1);
            if (lane == 63) {
                p0 = T(0);
                p1 = T(0);
            }
            bwd_true(v[0], cf.a1, cf.a2, p0 + r0, p1 + r1, cf.ik, mean);
        }
    }

    // ---- diagnostics partials -------------------------------------------------
    if (needF) {
        for (int off = 32; off > 0; off >>= 1) {
            pF += __shfl_down(pF, off, 64);
            pS += __shfl_down(pS, off, 64);
            pG += __shfl_down(pG, off, 64);
        }
        if (lane == 0) {
            red[wv][0] = pF;
            red[wv][1] = pS;
            red[wv][2] = pG;
        }
    }
    __syncthreads();  // LDS stencil reads done; wavefront partials visible

    // ---- each wavefront stores its own segment of its line through LDS -------
    if (solve) {
        const bool ok[1] = {active};
        const int seg0 = wl * 64 * CX;  // first element of the segment
        write_back<T, CX, 1>(sC + YLO * pitch + seg0 + (seg0 / CX) * PADE, pitch, v, ok, li, lane, li, lane, 1,
                             Ract, 64 * CX / VEC, buffer_of(Wout, bytes), y0 * nx + seg0, nx);
    }

    if (!XONLY) {
        if (blk == 0 && tid == 0 && a.mode != MODE_TIMING) *a.nstamp = n;
        if (needF && tid == 0) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int w = 0; w < kPassAThreads / 64; ++w) {
                s0 += red[w][0];
                s1 += red[w][1];
                s2 += red[w][2];
            }
            a.partials[(size_t)blk * 3 + 0] = s0;
            a.partials[(size_t)blk * 3 + 1] = s1;
            a.partials[(size_t)blk * 3 + 2] = s2;
        }
    }
}

// RHS pass of the split form (2D): the RHS of the scheme over a tile of
// kTileY x kTileX sites into W, and the tile's diagnostics partials; the
// XONLY wide pass A then solves the x-lines of W in place.  It serves lines
// whose staged rows do not fit LDS.  Threads: kTileY rows x 32 lanes, a lane
// a chunk of kTileX / 32 sites, in the padded chunk layout of pass A (so the
// stencil and diagnostics helpers apply unchanged).
template <typename T>
__global__ void __launch_bounds__(kPassAThreads) rhs_tile_kernel(PassAArgs a)
{
    constexpr int TY = kTileY, TX = kTileX, CT = kTileX / 32;
    constexpr int PADE = PadOf<T>::v;
    constexpr int VEC = Vec16<T>::n;
    constexpr int HALO = VEC;
    constexpr int RW = TX + 2 * HALO;  // staged row: x0 - HALO .. x0 + TX + HALO - 1
    constexpr int PITCH = RW + ((RW - 1) / CT) * PADE + 1;
    constexpr int NVR = RW / VEC;
    static_assert(TY * 32 == kPassAThreads && CT % VEC == 0, "tile shape");
    using VT = typename Vec16<T>::type;
    __shared__ __align__(16) T sT[(TY + 3) * PITCH];
    __shared__ double red[kPassAThreads / 64][3];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = a.nx, ny = a.ny;
    const int tiles_x = nx / TX;
    const uint32_t per_member = (uint32_t)tiles_x * (uint32_t)((ny + TY - 1) / TY);
    const uint32_t blk = xcd_remap(blockIdx.x, (uint32_t)a.nblocks);
    const int mloc = (int)(blk / per_member);
    const int t = (int)(blk - (uint32_t)mloc * per_member);
    const int y0 = (t / tiles_x) * TY, x0 = (t % tiles_x) * TX;
    const int mid = member_id(a.run, a.mids, mloc);
    const MemberDev& md = a.mem[mid];
    const int64_t moff = member_off(a.run, a.mem, mid, mloc);
    const uint32_t bytes = (uint32_t)((int64_t)nx * ny * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rC = buffer_of(reinterpret_cast<const T*>(a.C) + moff, bytes);

    const int64_t n = *a.step;
    const int K = a.K;
    bool needF = a.mode == MODE_DIAG, needG = a.mode == MODE_DIAG;
    if (a.mode == MODE_STEP) step_needs(n, K, needF, needG);
    const bool store = (a.mode != MODE_DIAG);

    // stage rows y0 - 1 .. y0 + Tact (+1 for the gradient of mu), periodic
    const int Tact = min(TY, ny - y0);
    const int nrows = Tact + (needG ? 3 : 2);
    for (int i = tid; i < nrows * NVR; i += kPassAThreads) {
        const int r = i / NVR, vi = i - r * NVR;
        const int yy = wrapi(y0 - 1 + r, ny);
        const int xs = wrapi(x0 - HALO + vi * VEC, nx);  // a whole vector: nx and x0 are multiples of VEC
        const VT val = buf_load16<VT>(rC, (yy * nx + xs) * (int)sizeof(T), 0);
        T e[VEC];
        vec_get<T>(val, e);
        const int xx = vi * VEC;
#pragma unroll
        for (int q = 0; q < VEC; ++q) sT[r * PITCH + (xx + q) + ((xx + q) / CT) * PADE] = e[q];
    }
    __syncthreads();

    const int row = tid >> 5, jx = tid & 31;
    const bool ok = row < Tact;
    const T* cb = sT + (row + 1) * PITCH + jx * (CT + PADE);
    double pF = 0.0, pS = 0.0, pG = 0.0;
    if (ok) {
        auto at = [&](int, int dy, int m) { return cb[dy * PITCH + m + (m / CT) * PADE]; };
        diag_sums<T, 2, CT, 1>(at, 1u, md, a.conv, needF, needG, pF, pS, pG);
    }
    if (store && ok) {
        const T* rc = CoefOf<T>::rc(md);
        const T cdx = rc[RC_DX], cdy = rc[RC_DY], gxy = rc[RC_GXY];
        auto at = [&](int, int dy, int m) { return cb[dy * PITCH + m + (m / CT) * PADE]; };
        T v[CT];
#pragma unroll
        for (int k = 0; k < CT; ++k) v[k] = rhs_site<T, 2>(at, 0, k + HALO, cdx, cdy, T(0), gxy, T(0), T(0));
        const __amdgpu_buffer_rsrc_t rW = buffer_of(reinterpret_cast<T*>(a.W) + moff, bytes);
        const int o = ((y0 + row) * nx + x0 + jx * CT) * (int)sizeof(T);
#pragma unroll
        for (int k = 0; k < CT; k += VEC) buf_store16<VT>(vec_make<T>(v + k), rW, o + k * (int)sizeof(T), 0);
    }
    if (needF) {
        for (int off = 32; off > 0; off >>= 1) {
            pF += __shfl_down(pF, off, 64);
            pS += __shfl_down(pS, off, 64);
            pG += __shfl_down(pG, off, 64);
        }
        if (lane == 0) {
            red[wave][0] = pF;
            red[wave][1] = pS;
            red[wave][2] = pG;
        }
    }
    __syncthreads();
    if (blk == 0 && tid == 0 && a.mode != MODE_TIMING) *a.nstamp = n;
    if (needF && tid == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int w = 0; w < kPassAThreads / 64; ++w) {
            s0 += red[w][0];
            s1 += red[w][1];
            s2 += red[w][2];
        }
        a.partials[(size_t)blk * 3 + 0] = s0;
        a.partials[(size_t)blk * 3 + 1] = s1;
        a.partials[(size_t)blk * 3 + 2] = s2;
    }
}

// --------------------------------------------------------------------------
// pass A, several work units per block
// --------------------------------------------------------------------------
// A block walks `units` work units and loads the next unit's rows into
// registers while it computes the current one; they go to LDS once every read
// of the rows they replace is done.
//   2D: a unit is a y-band of R x-lines; the block takes consecutive bands of
//       one member.  Results leave through LDS with coalesced stores.
//   3D: a unit is one z-plane of a y-band; the block takes consecutive planes
//       of one band.  LDS holds a ring of 4 staged planes, so every plane is
//       read from memory once per block instead of three or four times, and a
//       unit adds one plane.  Results are stored from registers (each lane
//       writes its contiguous chunk), so the ring needs no output space.
template <typename T, int DIM, int CX, int RL>
__global__ void __launch_bounds__(kPassAThreads) passA_multi_kernel(PassAArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* sC = reinterpret_cast<T*>(lds_raw);
    __shared__ double red[kPassAThreads / 64][3];

    constexpr int PADE = PadOf<T>::v;
    constexpr int VEC = Vec16<T>::n;
    constexpr int HALO = VEC;
    constexpr int NPF = kPrefetchVecs;
    static_assert(CX % VEC == 0, "LDS layout assumes vector-aligned chunks");
    using VT = typename Vec16<T>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    const uint32_t blk = xcd_remap(blockIdx.x, (uint32_t)a.nblocks);
    const uint32_t bpm = (uint32_t)a.blocks_per_member;
    const int mloc = (int)(blk / bpm);
    const uint32_t rem = blk - (uint32_t)mloc * bpm;
    // 2D: bands band0 .. band0 + nunits - 1;  3D: planes zbase .. zbase + nunits - 1 of band0
    const int band0 = (DIM == 2) ? (int)rem * a.units : (int)(rem % a.bands_y);
    const int zbase = (DIM == 2) ? 0 : (int)(rem / (uint32_t)a.bands_y) * a.units;
    const int nunits = (DIM == 2) ? min(a.units, a.bands_y - band0) : min(a.units, nz - zbase);
    const int mid = member_id(a.run, a.mids, mloc);
    const MemberDev& md = a.mem[mid];
    const int64_t moff = member_off(a.run, a.mem, mid, mloc);
    const T* C = reinterpret_cast<const T*>(a.C) + moff;
    T* Wout = reinterpret_cast<T*>(a.W) + moff;

    const int64_t n = *a.step;
    const int K = a.K;
    bool needF = a.mode == MODE_DIAG, needG = a.mode == MODE_DIAG;
    if (a.mode == MODE_STEP) step_needs(n, K, needF, needG);
    const bool solve = (a.mode != MODE_DIAG);

    const int pitch = a.pitch;
    const int planeStride = (a.R + 3) * pitch;
    const int nvec = nx / VEC;
    const int nseg = (nvec + 63) >> 6;     // 64-vector segments of a row
    const int xhi = needG ? 2 : 1;           // highest plane offset the stencils read
    const int nwaves = nthreads >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);

    // lines of unit u: y0 .. y0 + Ract - 1, staged rows y0 - 1 .. y0 - 1 + nrows - 1
    auto unit_y0 = [&](int u) { return (DIM == 2 ? band0 + u : band0) * a.R; };
    auto unit_rows = [&](int u) { return min(a.R, ny - unit_y0(u)) + (needG ? 3 : 2); };

    // Staging follows the single-unit kernel: a wavefront takes whole rows
    // (round-robin), its lanes consecutive 16-byte vectors of the row in
    // segments of 64; halos are one vector per thread.  In 3D a plane goes
    // to ring slot (z - zbase + 1) mod 4.
    auto slot_of = [&](int zz) { return (DIM == 3) ? ((zz - zbase + 1) & 3) * planeStride : 0; };
    auto row_of = [&](int zz, int yfirst, int r) {
        const int zw = (DIM == 3) ? wrapi(zz, nz) : 0;
        return C + ((int64_t)zw * ny + wrapi(yfirst - 1 + r, ny)) * nx;
    };
    auto put = [&](const VT& val, int dst) {
        T e[VEC];
        vec_get<T>(val, e);
#pragma unroll
        for (int q = 0; q < VEC; ++q) sC[dst + q] = e[q];
    };
    // interior vector seg*64+lane of staged row r (plane zz, first line
    // yfirst), if the lane has one
    auto load_vec = [&](int zz, int yfirst, int r, int seg, VT& val, int& dst) {
        const int xi = seg * 64 + lane;
        if (xi < nvec) {
            const uint32_t xs = (uint32_t)xi * VEC, xx = xs + HALO;
            val = *reinterpret_cast<const VT*>(row_of(zz, yfirst, r) + xs);
            dst = slot_of(zz) + r * pitch + (int)(xx + xx / CX * PADE);
        }
    };
    // halo vector h (row h / 2; left side for even h)
    auto load_halo = [&](int zz, int yfirst, int h, VT& val, int& dst) {
        const int r = h >> 1;
        const int xs = (h & 1) ? 0 : nx - HALO;
        const int xx = (h & 1) ? nx + HALO : 0;
        val = *reinterpret_cast<const VT*>(row_of(zz, yfirst, r) + xs);
        dst = slot_of(zz) + r * pitch + xx + (xx / CX) * PADE;
    };

    // first unit: its rows (2D) or planes zbase-1 .. zbase+xhi (3D), in
    // batches of NPF loads
    {
        const int yf = unit_y0(0), nrows = unit_rows(0);
        for (int p = 0; p < (DIM == 3 ? xhi + 2 : 1); ++p) {
            const int zz = zbase - 1 + p;
            int r = wv, seg = 0;  // wave-uniform cursor (row, segment)
            while (r < nrows) {
                VT pv[NPF];
                int pd[NPF];
#pragma unroll
                for (int i = 0; i < NPF; ++i) {
                    pd[i] = -1;
                    if (r < nrows) {
                        load_vec(zz, yf, r, seg, pv[i], pd[i]);
                        if (++seg == nseg) {
                            seg = 0;
                            r += nwaves;
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < NPF; ++i)
                    if (pd[i] >= 0) put(pv[i], pd[i]);
            }
            for (int h = tid; h < 2 * nrows; h += nthreads) {
                VT v;
                int d;
                load_halo(zz, yf, h, v, d);
                put(v, d);
            }
        }
    }
    __syncthreads();

    const int P = a.P;
    const int g = lane_div(lane, P);
    const int j = lane - g * P;
    const int groups = a.rows_per_wave / RL;
    const int rl0 = (wave * groups + g) * RL;
    const bool lane_ok = g < groups;
    const int cb_off = (rl0 + 1) * pitch + j * (CX + PADE);

    // folded coefficients of the RHS
    const T* rc = CoefOf<T>::rc(md);
    const T cdx = rc[RC_DX], cdy = rc[RC_DY], cdz = rc[RC_DZ];
    const T gxy = rc[RC_GXY], gxz = rc[RC_GXZ], gyz = rc[RC_GYZ];

    double pF = 0.0, pS = 0.0, pG = 0.0;
    for (int u = 0; u < nunits; ++u) {
        const int z = zbase + u;
        const int y0 = unit_y0(u);
        const int Ract = min(a.R, ny - y0);
        const bool has_next = u + 1 < nunits;
        bool rowok[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) rowok[q] = lane_ok && (rl0 + q < Ract);
        const bool active = rowok[0];
        // the rows the next unit adds start loading now (the host guarantees
        // that a wavefront's share of them fits NPF vectors per lane and the
        // halos one vector per thread); their LDS places are recomputed when
        // they are written, from the same wave-uniform cursor
        const int pf_z = (DIM == 3) ? z + 1 + xhi : 0;
        const int pf_y = has_next ? unit_y0(u + 1) : 0;
        const int pf_rows = has_next ? unit_rows(u + 1) : 0;
        VT pv[NPF], ph;
        {
            int r = wv, seg = 0;  // wave-uniform cursor (row, segment)
#pragma unroll
            for (int i = 0; i < NPF; ++i) {
                if (r < pf_rows) {
                    const int xi = seg * 64 + lane;
                    if (xi < nvec)
                        pv[i] = *reinterpret_cast<const VT*>(row_of(pf_z, pf_y, r) + (uint32_t)xi * VEC);
                    if (++seg == nseg) {
                        seg = 0;
                        r += nwaves;
                    }
                }
            }
            if (tid < 2 * pf_rows) {
                int d;
                load_halo(pf_z, pf_y, tid, ph, d);
            }
        }

        // staged planes z-1 .. z+2 (3D ring slots); 2D uses slot 0 only
        const int s0 = (DIM == 3 ? (u & 3) * planeStride : 0) + cb_off;
        const int s1 = (DIM == 3 ? ((u + 1) & 3) * planeStride : 0) + cb_off;
        const int s2 = (DIM == 3 ? ((u + 2) & 3) * planeStride : 0) + cb_off;
        const int s3 = (DIM == 3 ? ((u + 3) & 3) * planeStride : 0) + cb_off;
#define AT(dz, dy, m) \
    sC[((dz) < 0 ? s0 : (dz) == 0 ? s1 : (dz) == 1 ? s2 : s3) + (dy) * pitch + (m) + ((m) / CX) * PADE]

        // every lane forms the RHS (see the single-unit kernel)
        T v[RL][CX];
        if (solve) {
            auto at = [&](int dz, int dy, int m) { return AT(dz, dy, m); };
#pragma unroll
            for (int k = 0; k < CX; ++k)
#pragma unroll
                for (int q = 0; q < RL; ++q)
                    v[q][k] = rhs_site<T, DIM>(at, q, k + HALO, cdx, cdy, cdz, gxy, gxz, gyz);
        }
        if (active) {
            unsigned rm = 0;
#pragma unroll
            for (int q = 0; q < RL; ++q) rm |= rowok[q] ? (1u << q) : 0u;
            auto at = [&](int dz, int dy, int m) { return AT(dz, dy, m); };
            diag_sums<T, DIM, CX, RL>(at, rm, md, a.conv, needF, needG, pF, pS, pG);
        }
#undef AT

        if (solve) {
            LineCoef<T> cf;
            load_coef(cf, CoefOf<T>::ax(md, 0), P);
            ScanLanes SL;
            make_lanes(SL, lane, g * P, P);
            T mean[RL], csum[RL];
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                csum[q] = T(0);
#pragma unroll
                for (int k = 0; k < CX; ++k) csum[q] += v[q][k];
            }
            if ((P & (P - 1)) == 0) {
#pragma unroll
                for (int q = 0; q < RL; ++q) csum[q] = group_sum(csum[q], P, lane);
            } else {
#pragma unroll
                for (int s = 0; s < kWaveScanLevels; ++s) {
                    const int d = 1 << s;
                    if (d < P) {
#pragma unroll
                        for (int q = 0; q < RL; ++q) {
                            const T y = lane_get(SL.up[s], csum[q]);
                            if (j >= d) csum[q] += y;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < RL; ++q) csum[q] = lane_get(SL.last, csum[q]);
            }
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                mean[q] = csum[q] * CoefOf<T>::ax(md, 0).inv_n;
#pragma unroll
                for (int k = 0; k < CX; ++k) v[q][k] -= mean[q];
            }
            T e0[RL], e1[RL];
#pragma unroll
            for (int q = 0; q < RL; ++q) fwd_zero(v[q], cf.a1, cf.a2, e0[q], e1[q]);
            scan_fwd_wave<T, RL>(e0, e1, j, P, SL, cf);
#pragma unroll
            for (int q = 0; q < RL; ++q) fwd_true(v[q], cf.a1, cf.a2, e0[q], e1[q], T(0));
#pragma unroll
            for (int q = 0; q < RL; ++q) bwd_zero(v[q], cf.a1, cf.a2, e0[q], e1[q]);
            scan_bwd_wave<T, RL>(e0, e1, j, P, SL, cf);
#pragma unroll
            for (int q = 0; q < RL; ++q) bwd_true(v[q], cf.a1, cf.a2, e0[q], e1[q], cf.ik, mean[q]);
            if (DIM == 3) {
                // each lane stores its own chunk of every line it holds
#pragma unroll
                for (int q = 0; q < RL; ++q) {
                    if (!rowok[q]) continue;
                    T* dst = Wout + ((int64_t)z * ny + y0 + rl0 + q) * nx + j * CX;
#pragma unroll
                    for (int k = 0; k < CX; k += VEC)
                        *reinterpret_cast<VT*>(dst + k) = vec_make<T>(&v[q][k]);
                }
            }
        }
        if (DIM == 2 && solve) {
            __syncthreads();  // every read of the staged rows is done
            write_back<T, CX, RL>(sC + pitch, pitch, v, rowok, rl0, j, wv, lane, a.rows_per_wave, Ract, nvec,
                                  buffer_of(Wout, (uint32_t)((int64_t)nx * ny * (int64_t)sizeof(T))), y0 * nx, nx);
        }

        if (has_next) {
            __syncthreads();  // every read of the rows the new ones replace is done
            const int base = slot_of(pf_z);
            int r = wv, seg = 0;  // the cursor of the loads above
#pragma unroll
            for (int i = 0; i < NPF; ++i) {
                if (r < pf_rows) {
                    const int xi = seg * 64 + lane;
                    if (xi < nvec) {
                        const uint32_t xx = (uint32_t)xi * VEC + HALO;
                        put(pv[i], base + r * pitch + (int)(xx + xx / CX * PADE));
                    }
                    if (++seg == nseg) {
                        seg = 0;
                        r += nwaves;
                    }
                }
            }
            if (tid < 2 * pf_rows) {
                const int hr = tid >> 1;
                const int xx = (tid & 1) ? nx + HALO : 0;
                put(ph, base + hr * pitch + xx + (xx / CX) * PADE);
            }
            __syncthreads();
        }
    }

    if (blk == 0 && tid == 0 && a.mode != MODE_TIMING) *a.nstamp = n;
    if (needF) {
        for (int off = 32; off > 0; off >>= 1) {
            pF += __shfl_down(pF, off, 64);
            pS += __shfl_down(pS, off, 64);
            pG += __shfl_down(pG, off, 64);
        }
        if (lane == 0) {
            red[wave][0] = pF;
            red[wave][1] = pS;
            red[wave][2] = pG;
        }
        __syncthreads();
        if (tid == 0) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int w = 0; w < nthreads / 64; ++w) {
                s0 += red[w][0];
                s1 += red[w][1];
                s2 += red[w][2];
            }
            a.partials[(size_t)blk * 3 + 0] = s0;
            a.partials[(size_t)blk * 3 + 1] = s1;
            a.partials[(size_t)blk * 3 + 2] = s2;
        }
    }
}

// --------------------------------------------------------------------------
// y- / z-line solves
// --------------------------------------------------------------------------
template <typename T, int CY>
__global__ void __launch_bounds__(kColMaxThreads) col_kernel(ColArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int bP = a.b * a.P;
    T* sE0 = reinterpret_cast<T*>(lds_raw);
    T* sE1 = sE0 + bP;
    T* sF0 = sE1 + bP;
    T* sF1 = sF0 + bP;
    T* sS = sF1 + bP;  // chunk sums

    __shared__ double sred[kColMaxThreads / 64][3];
    const int tid = threadIdx.x;
    const int P = a.P;
    // blockDim.x is b * P rounded up to whole wavefronts; threads beyond b * P
    // only take part in the barriers
    const int j0 = tid >> a.bshift;  // b is a power of two
    const bool colok = j0 < P;
    const int j = colok ? j0 : 0;
    const int c = tid & (a.b - 1);
    const uint32_t blk = xcd_remap(blockIdx.x, (uint32_t)a.nblocks);
    const uint32_t bpm = (uint32_t)(a.cols >> a.bshift);
    const int mloc = (int)(blk / bpm);
    // the block's b columns are consecutive elements of one run (b divides the
    // run length): its first column's element offset is block-uniform
    const uint32_t col0 = (blk - (uint32_t)mloc * bpm) << a.bshift;
    const uint32_t run = col0 / (uint32_t)a.run;
    const int64_t base0 = (int64_t)(col0 - run * (uint32_t)a.run) + (int64_t)run * a.outer;
    const int mid = member_id(a.mrun, a.mids, mloc);
    const MemberDev& md = a.mem[mid];
    const int64_t moff = member_off(a.mrun, a.mem, mid, mloc);
    const int64_t st = a.stride;
    // lane offset: column c, first element of chunk j; element k of the chunk
    // adds the uniform k * stride
    const uint32_t span = (uint32_t)((a.msites - base0) * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rsrc = buffer_of(reinterpret_cast<const T*>(a.src) + moff + base0, span);
    const __amdgpu_buffer_rsrc_t rdst = buffer_of(reinterpret_cast<T*>(a.dst) + moff + base0, span);
    const int voff = (int)(((int64_t)j * CY * st + c) * (int64_t)sizeof(T));
    const int sstep = (int)(st * (int64_t)sizeof(T));

    // every thread loads (a thread past the block's columns reads chunk 0 of
    // column c, in range, and its values are never summed, scanned or stored)
    T v[CY];
#pragma unroll
    for (int k = 0; k < CY; ++k) v[k] = buf_load<T>(rsrc, voff, k * sstep);

    const auto& ac = CoefOf<T>::ax(md, a.axis);
    const T a1 = ac.a1, a2 = ac.a2, ik = ac.ikappa;
    // the scan's 2x2 matrices live in LDS (read as broadcasts where they are
    // used), which keeps them out of the scalar registers
    __shared__ T sco[(kMaxScanLevels + 1) * 4];  // Mp[0..6], then W
    if (tid < kMaxScanLevels * 4)
        sco[tid] = ac.Mp[tid >> 2][tid & 3];
    else if (tid < (kMaxScanLevels + 1) * 4)
        sco[tid] = ac.W[tid - kMaxScanLevels * 4];
    const T* W = sco + kMaxScanLevels * 4;

    // causal recursion.  The line mean m passes through the solve unchanged;
    // the recursions run on v - m (chunk end states corrected by m * E1, the
    // end state of a chunk of ones) and m is added back at the end.
    //
    // The chunk end states of a column are combined by a Kogge-Stone scan over
    // its P chunks in LDS (log2 P levels, ping-pong buffers, one barrier per
    // level) with the powers M^(2^s) of the chunk transfer matrix; the ring is
    // closed with (I - A^n)^{-1} as in the x-solve.
    const T E10 = ac.E1[0], E11 = ac.E1[1];
    auto Mp = [&](int l) -> const T* { return sco + 4 * l; };
    T e0, e1, csum = T(0);
#pragma unroll
    for (int k = 0; k < CY; ++k) csum += v[k];
    fwd_zero(v, a1, a2, e0, e1);
    const int me = j * a.b + c;
    if (colok) sS[me] = csum;
    __syncthreads();
    // the line mean: every thread of the column sums the P chunk sums in order
    T tot = T(0);
    for (int q = 0; q < P; ++q) tot += sS[q * a.b + c];
    const T m = tot * ac.inv_n;
    e0 -= m * E10;
    e1 -= m * E11;
    // inclusive scan S_j = f_j + M S_{j-1} over the chunks of the column
    // ping-pong buffers (a select, not an indexed pointer array: no scratch)
    auto B0 = [&](int q) { return q ? sF0 : sE0; };
    auto B1 = [&](int q) { return q ? sF1 : sE1; };
    int pp = 0;
#pragma unroll
    for (int l = 0; l < kMaxScanLevels; ++l) {
        const int d = 1 << l;
        if (d >= P) break;  // uniform
        if (colok) {
            B0(pp)[me] = e0;
            B1(pp)[me] = e1;
        }
        __syncthreads();
        if (colok && j >= d) {
            T y0 = B0(pp)[me - d * a.b], y1 = B1(pp)[me - d * a.b];
            mv(Mp(l), y0, y1);
            e0 += y0;
            e1 += y1;
        }
        pp ^= 1;
    }
    if (colok) {
        B0(pp)[me] = e0;
        B1(pp)[me] = e1;
    }
    __syncthreads();
    {
        // state after the whole column = entering chunk 0, carried to chunk j
        const T z0 = B0(pp)[(P - 1) * a.b + c], z1 = B1(pp)[(P - 1) * a.b + c];
        T r0 = W[0] * z0 + W[1] * z1, r1 = W[2] * z0 + W[3] * z1;
#pragma unroll
        for (int l = 0; l < kMaxScanLevels; ++l)
            if (((1 << l) < P) && (j & (1 << l))) mv(Mp(l), r0, r1);
        if (j > 0) {
            r0 += B0(pp)[me - a.b];
            r1 += B1(pp)[me - a.b];
        }
        fwd_true(v, a1, a2, r0, r1, m);
    }
    __syncthreads();  // the scan buffers are reused below

    // anti-causal recursion: the same scan over the reversed chunk order
    bwd_zero(v, a1, a2, e0, e1);
    const int jr = P - 1 - j;
    pp = 0;
#pragma unroll
    for (int l = 0; l < kMaxScanLevels; ++l) {
        const int d = 1 << l;
        if (d >= P) break;  // uniform
        if (colok) {
            B0(pp)[me] = e0;
            B1(pp)[me] = e1;
        }
        __syncthreads();
        if (colok && jr >= d) {
            T y0 = B0(pp)[me + d * a.b], y1 = B1(pp)[me + d * a.b];
            mv(Mp(l), y0, y1);
            e0 += y0;
            e1 += y1;
        }
        pp ^= 1;
    }
    if (colok) {
        B0(pp)[me] = e0;
        B1(pp)[me] = e1;
    }
    __syncthreads();
    {
        // state at the column start = entering chunk P-1 (from above), carried down
        const T z0 = B0(pp)[c], z1 = B1(pp)[c];
        T r0 = W[0] * z0 + W[1] * z1, r1 = W[2] * z0 + W[3] * z1;
#pragma unroll
        for (int l = 0; l < kMaxScanLevels; ++l)
            if (((1 << l) < P) && (jr & (1 << l))) mv(Mp(l), r0, r1);
        if (j < P - 1) {
            r0 += B0(pp)[me + a.b];
            r1 += B1(pp)[me + a.b];
        }
        bwd_true(v, a1, a2, r0, r1, ik, m);
    }

    if (colok)
#pragma unroll
        for (int k = 0; k < CY; ++k) buf_store(v[k], rdst, voff, k * sstep);

    // last sweep of the step: the first G blocks reduce the pass-A partials (pass
    // A ran to completion before this launch) and one thread advances the step
    if (a.fin.enabled) {
        if ((int)blockIdx.x < a.fin.G) finalize_block(a.fin, blockIdx.x, a.fin.G, sred);
        if (blockIdx.x == 0 && tid == 0 && a.fin.mode == MODE_STEP) *a.fin.step = *a.fin.nstamp + 1;
    }
}

// --------------------------------------------------------------------------
// initial condition, resets, beta series
// --------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    // k-th output of SplitMix64 (Steele, Lea & Flood 2014)
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void init_kernel(T* C, int64_t sites, uint64_t seed, double c0, double noise)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < sites;
         s += (int64_t)gridDim.x * blockDim.x) {
        const double u = (double)(splitmix64_at(seed, (uint64_t)s + 1) >> 11) * 0x1.0p-53;
        C[s] = (T)(c0 + noise * (2.0 * u - 1.0));
    }
}

__global__ void reset_kernel(int64_t* steps, int nsteps, int64_t value, int32_t* flags, int m,
                             double* series, int64_t series_len)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = t; i < series_len; i += stride) series[i] = __builtin_nan("");
    for (int64_t i = t; i < nsteps; i += stride) steps[i] = value;
    for (int64_t i = t; i < m; i += stride) flags[i] = 0;
}

// Sample j (n = jK): t, F, G_fd, G_id, beta, <C>.  G_fd is the central
// difference of the recorded F where both neighbours exist, else one-sided.
// G_fd and beta of sample jj (step n = jj K) of one member's series: the
// central difference of F around n, one-sided at the ends of the recorded run.
__device__ __forceinline__ void beta_at(const double* ser, int64_t jj, int32_t K, int64_t ncur, double dt,
                                        double& G, double& beta)
{
    const int64_t n = jj * K;
    const double Fm = ser[jj * kSeriesSlots + 0], F0 = ser[jj * kSeriesSlots + 1];
    const double Fp = ser[jj * kSeriesSlots + 2];
    const bool hasm = n >= 1 && !isnan(Fm);
    const bool hasp = n + 1 <= ncur && !isnan(Fp);
    if (hasm && hasp)
        G = (Fp - Fm) / (2.0 * dt);
    else if (hasp)
        G = (Fp - F0) / dt;
    else if (hasm)
        G = (F0 - Fm) / dt;
    else
        G = __builtin_nan("");
    const double t = (double)n * dt;
    beta = (n == 0) ? 0.0 : -t * G / F0;
}

__global__ void beta_kernel(const double* series, int64_t max_samples, int32_t member, int32_t K,
                            int64_t ncur, double dt, double* out, int64_t J)
{
    const double* ser = series + (int64_t)member * max_samples * kSeriesSlots;
    for (int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; jj < J;
         jj += (int64_t)gridDim.x * blockDim.x) {
        double G, beta;
        beta_at(ser, jj, K, ncur, dt, G, beta);
        double* o = out + jj * 6;
        o[0] = (double)(jj * K) * dt;
        o[1] = ser[jj * kSeriesSlots + 1];
        o[2] = G;
        o[3] = ser[jj * kSeriesSlots + 4];
        o[4] = beta;
        o[5] = ser[jj * kSeriesSlots + 3];
    }
}

// --------------------------------------------------------------------------
// ensemble statistics of beta
// --------------------------------------------------------------------------
constexpr int kStatThreads = ens_stats::kThreads;
static_assert(ens_stats::kMaxMoments == kMaxMoments, "one moment layout");

// beta_m(t_j) of the selected members from the recorded F slots (the same
// formula as the beta series)
struct SeriesBeta {
    const double* series;
    int64_t max_samples;
    const int32_t* members;
    int32_t K;
    int64_t ncur;
    double dt;
    __device__ double operator()(int i, int64_t j) const
    {
        double G, b;
        beta_at(series + (int64_t)members[i] * max_samples * kSeriesSlots, j, K, ncur, dt, G, b);
        return b;
    }
};

__global__ void __launch_bounds__(kStatThreads) moments_kernel(const double* series, int64_t max_samples,
                                                               const int32_t* members, int32_t nm,
                                                               int32_t K, int64_t ncur, double dt,
                                                               int32_t pmax, double* out, int64_t J)
{
    ens_stats::moments(SeriesBeta{series, max_samples, members, K, ncur, dt}, nm, J, pmax, out);
}

__global__ void __launch_bounds__(kStatThreads) window_kernel(const double* mom, int64_t j0, int64_t j1,
                                                              int32_t K, double dt, double* out)
{
    ens_stats::window(mom, j0, j1, (double)K * dt, [=](int64_t j) { return (double)(j * K) * dt; }, out);
}

__global__ void __launch_bounds__(kStatThreads) hist_kernel(const double* series, int64_t max_samples,
                                                            const int32_t* members, int32_t nm, int32_t K,
                                                            int64_t ncur, double dt, int64_t j0, int64_t j1,
                                                            double lo, double hi, int32_t nbins,
                                                            unsigned long long* counts)
{
    ens_stats::histogram(SeriesBeta{series, max_samples, members, K, ncur, dt}, nm, j0, j1, lo, hi, nbins,
                         counts);
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
// With a pair of events, the events take the kernel's own start and end
// timestamps (hipExtLaunchKernel), so no extra packets sit between kernels.
template <typename K, typename A>
static hipError_t launch_k(K k, unsigned blocks, unsigned threads, size_t lds, hipStream_t s,
                           const A& a, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ev0 && ev1)
        hipExtLaunchKernelGGL(k, dim3(blocks), dim3(threads), (std::uint32_t)lds, s, ev0, ev1, 0, a);
    else
        hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int DIM, int CX, int RL, bool CN = false>
static hipError_t launchA(const PassAArgs& a, size_t lds, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1)
{
    auto k = passA_kernel<T, DIM, CX, RL, CN>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(k, (unsigned)a.nblocks, 64 * a.waves, lds, s, a, ev0, ev1);
}

template <typename T, int DIM, int CX, int RL>
static hipError_t launchMulti(const PassAArgs& a, size_t lds, hipStream_t s, hipEvent_t ev0,
                              hipEvent_t ev1)
{
    auto k = passA_multi_kernel<T, DIM, CX, RL>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(k, (unsigned)a.nblocks, 64 * a.waves, lds, s, a, ev0, ev1);
}

// (chunk length, lines per lane) pairs that are compiled
#define CH_PASSA_SHAPES(X) \
    X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(4, 2) X(8, 2) X(16, 2) X(32, 2) X(4, 4) X(8, 4) X(16, 4)
// ... and those of the several-units variant
#define CH_MULTI_SHAPES(X) X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(4, 2) X(8, 2) X(16, 2)
// ... and of the Crank-Nicolson variant (2D, one unit per block)
#define CH_CN_SHAPES(X) X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(64, 1)

template <typename T, int DIM>
static hipError_t launchA_shape(int cx, int rl, int units, const PassAArgs& a, size_t lds,
                                hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (a.cn) {
        if (DIM != 2 || units != 1) return hipErrorInvalidValue;
#define X(C, R) \
    if (cx == C && rl == R) return launchA<T, 2, C, R, true>(a, lds, s, ev0, ev1);
        CH_CN_SHAPES(X)
#undef X
        return hipErrorInvalidValue;
    }
    if (units > 1) {
#define X(C, R) \
    if (cx == C && rl == R) return launchMulti<T, DIM, C, R>(a, lds, s, ev0, ev1);
        CH_MULTI_SHAPES(X)
#undef X
        return hipErrorInvalidValue;
    }
    if (units != 1) return hipErrorInvalidValue;
#define X(C, R) \
    if (cx == C && rl == R) return launchA<T, DIM, C, R>(a, lds, s, ev0, ev1);
    CH_PASSA_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

bool passA_has(int dim, int cx, int rl, int units, bool cn)
{
    if (dim != 2 && dim != 3) return false;
    if (cn) {
        if (dim != 2 || units != 1) return false;
#define X(C, R) \
    if (cx == C && rl == R) return true;
        CH_CN_SHAPES(X)
#undef X
        return false;
    }
    if (units > 1) {
#define X(C, R) \
    if (cx == C && rl == R) return true;
        CH_MULTI_SHAPES(X)
#undef X
        return false;
    }
    if (units != 1) return false;
#define X(C, R) \
    if (cx == C && rl == R) return true;
    CH_PASSA_SHAPES(X)
#undef X
    return false;
}

// (chunk length, wavefronts per line) of lines longer than one wavefront
#define CH_WIDE_SHAPES(X) X(4, 4) X(8, 2) X(8, 4) X(16, 2) X(16, 4) X(32, 2) X(32, 4)
// ... and of the split form (FP64 lines whose staged rows exceed LDS)
#define CH_SPLIT_SHAPES(X) X(4, 4) X(32, 4)

template <typename T, int CX, int WL, bool XONLY>
static hipError_t launchW(const PassAArgs& a, size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    auto k = passA_wide_kernel<T, CX, WL, XONLY>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(k, (unsigned)a.nblocks, kPassAThreads, lds, s, a, ev0, ev1);
}

bool passA_wide_has(int prec, int cx, int wl, bool split)
{
    if (split) {
        if (prec != 0) return false;
#define X(C, W) \
    if (cx == C && wl == W) return true;
        CH_SPLIT_SHAPES(X)
#undef X
        return false;
    }
#define X(C, W) \
    if (cx == C && wl == W) return true;
    CH_WIDE_SHAPES(X)
#undef X
    return false;
}

// Lines longer than one wavefront (a.P > 64).  units == 0 selects the split
// form: the RHS tile pass, then (unless only diagnostics are asked for) the
// x-solve in place on W.  With events, ev0 and ev1 bracket both launches.
template <typename T>
static hipError_t launch_wide(int cx, int units, const PassAArgs& a, size_t lds, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1)
{
    const int wl = a.P / 64;
    if (a.P % 64 || !passA_wide_has(sizeof(T) == 8 ? 0 : 1, cx, wl, units == 0)) return hipErrorInvalidValue;
    if (units != 0) {
#define X(C, W) \
    if (cx == C && wl == W) return launchW<T, C, W, false>(a, lds, s, ev0, ev1);
        CH_WIDE_SHAPES(X)
#undef X
        return hipErrorInvalidValue;
    }
    if constexpr (sizeof(T) == 8) {
        hipError_t e;
        if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
        PassAArgs t = a;
        t.blocks_per_member = (int64_t)(a.nx / kTileX) * ((a.ny + kTileY - 1) / kTileY);
        t.nblocks = t.blocks_per_member * a.nmem;
        if ((e = launch_k(rhs_tile_kernel<T>, (unsigned)t.nblocks, kPassAThreads, 0, s, t, nullptr, nullptr)) !=
            hipSuccess)
            return e;
        if (a.mode != MODE_DIAG) {
            e = hipErrorInvalidValue;
#define X(C, W) \
    if (cx == C && wl == W) e = launchW<T, C, W, true>(a, lds, s, nullptr, nullptr);
            CH_SPLIT_SHAPES(X)
#undef X
            if (e != hipSuccess) return e;
        }
        if (ev1 && (e = hipEventRecord(ev1, s)) != hipSuccess) return e;
        return hipSuccess;
    }
    return hipErrorInvalidValue;
}

int passA_pad(int prec) { return prec == 0 ? PadOf<double>::v : PadOf<float>::v; }
int passA_halo(int prec) { return prec == 0 ? Vec16<double>::n : Vec16<float>::n; }

hipError_t launch_passA(int prec, int dim, int cx, int rl, int units, const PassAArgs& a,
                        size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (a.nblocks <= 0) return hipSuccess;
    if (a.P > 64) {
        if (dim != 2 || rl != 1 || a.cn) return hipErrorInvalidValue;
        return prec == 0 ? launch_wide<double>(cx, units, a, lds, s, ev0, ev1)
                         : launch_wide<float>(cx, units, a, lds, s, ev0, ev1);
    }
    if (prec == 0)
        return dim == 2 ? launchA_shape<double, 2>(cx, rl, units, a, lds, s, ev0, ev1)
                        : launchA_shape<double, 3>(cx, rl, units, a, lds, s, ev0, ev1);
    return dim == 2 ? launchA_shape<float, 2>(cx, rl, units, a, lds, s, ev0, ev1)
                    : launchA_shape<float, 3>(cx, rl, units, a, lds, s, ev0, ev1);
}

template <typename T, int CY>
static hipError_t launchC(const ColArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    const size_t lds = (size_t)5 * a.b * a.P * sizeof(T);
    const int threads = (a.b * a.P + 63) / 64 * 64;
    return launch_k(col_kernel<T, CY>, (unsigned)a.nblocks, threads, lds, s, a, ev0, ev1);
}

template <typename T>
static hipError_t launchC_cy(int cy, const ColArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    switch (cy) {
    case 4: return launchC<T, 4>(a, s, ev0, ev1);
    case 8: return launchC<T, 8>(a, s, ev0, ev1);
    case 16: return launchC<T, 16>(a, s, ev0, ev1);
    case 32: return launchC<T, 32>(a, s, ev0, ev1);
    case 64:
        // 64 doubles per lane exceed the register file: FP32 only
        if constexpr (sizeof(T) == 4) return launchC<T, 64>(a, s, ev0, ev1);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

bool col_has(int prec, int cy)
{
    if (prec == 0) return cy == 4 || cy == 8 || cy == 16 || cy == 32;
    return cy == 4 || cy == 8 || cy == 16 || cy == 32 || cy == 64;
}

hipError_t launch_col(int prec, int cy, const ColArgs& a, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1)
{
    if (a.nblocks <= 0) return hipSuccess;
    if (!col_has(prec, cy)) return hipErrorInvalidValue;
    return prec == 0 ? launchC_cy<double>(cy, a, s, ev0, ev1) : launchC_cy<float>(cy, a, s, ev0, ev1);
}

hipError_t launch_init_member(int prec, void* C, int64_t sites, uint64_t seed, double c0,
                              double noise, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((sites + 255) / 256, 65536);
    if (prec == 0)
        hipLaunchKernelGGL(init_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<double*>(C), sites, seed, c0, noise);
    else
        hipLaunchKernelGGL(init_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<float*>(C), sites, seed, c0, noise);
    return hipGetLastError();
}

hipError_t launch_reset(int64_t* steps, int nsteps, int64_t value, int32_t* flags, int m,
                        double* series, int64_t series_len, hipStream_t s)
{
    const int64_t big = std::max<int64_t>(series_len, std::max<int64_t>(m, nsteps));
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((big + 255) / 256, 4096));
    hipLaunchKernelGGL(reset_kernel, dim3((unsigned)blocks), dim3(256), 0, s, steps, nsteps, value,
                       flags, m, series, series_len);
    return hipGetLastError();
}

hipError_t launch_fin(const FinArgs& f, hipStream_t s)
{
    hipLaunchKernelGGL(fin_kernel, dim3((unsigned)std::max(1, f.G)), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_beta(const double* series, int64_t max_samples, int32_t member, int32_t K,
                       int64_t ncur, double dt, double* out, int64_t J, hipStream_t s)
{
    if (J <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((J + 255) / 256, 1024);
    hipLaunchKernelGGL(beta_kernel, dim3((unsigned)blocks), dim3(256), 0, s, series, max_samples,
                       member, K, ncur, dt, out, J);
    return hipGetLastError();
}

hipError_t launch_moments(const double* series, int64_t max_samples, const int32_t* members, int32_t nm,
                          int32_t K, int64_t ncur, double dt, int32_t pmax, double* out, int64_t J,
                          hipStream_t s)
{
    if (J <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(J, 4096);
    hipLaunchKernelGGL(moments_kernel, dim3((unsigned)blocks), dim3(kStatThreads), 0, s, series,
                       max_samples, members, nm, K, ncur, dt, pmax, out, J);
    return hipGetLastError();
}

hipError_t launch_window(const double* mom, int64_t j0, int64_t j1, int32_t K, double dt, double* out,
                         hipStream_t s)
{
    hipLaunchKernelGGL(window_kernel, dim3(1), dim3(kStatThreads), 0, s, mom, j0, j1, K, dt, out);
    return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long* p, int32_t n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

hipError_t launch_hist(const double* series, int64_t max_samples, const int32_t* members, int32_t nm,
                       int32_t K, int64_t ncur, double dt, int64_t j0, int64_t j1, double lo, double hi,
                       int32_t nbins, unsigned long long* counts, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3((nbins + 2 + 255) / 256), dim3(256), 0, s, counts, nbins + 2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (j1 - j0 + 1) * (int64_t)nm;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + kStatThreads - 1) / kStatThreads, 4096);
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)blocks), dim3(kStatThreads), 0, s, series, max_samples,
                       members, nm, K, ncur, dt, j0, j1, lo, hi, nbins, counts);
    return hipGetLastError();
}

}  // namespace chk
