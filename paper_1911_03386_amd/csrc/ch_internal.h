// Internal types shared by the host runtime (ch_host.cpp) and the kernels
// (ch_kernels.hip).  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chk {

constexpr int kMaxScanLevels = 8;  // (A^c)^(2^s), s < 8: enough for P <= 256 chunks
constexpr int kWaveScanLevels = 6; // lanes of one line inside a wavefront: P <= 64
constexpr int kSeriesSlots = 5;    // F(jK-1), F(jK), F(jK+1), <C>(jK), G_id(jK)
constexpr int kPassAThreads = 256; // 4 wavefronts
constexpr int kColMaxThreads = 512;
constexpr int kMaxMoments = 8;     // ensemble statistics: mu_1 .. mu_8
constexpr int kPrefetchVecs = 12;  // several-unit pass A: 16-byte vectors per lane prefetched for the next unit
constexpr int kTileY = 8;          // RHS pass of the split form: tile rows (4 wavefronts x 2 rows of 32 lanes)
constexpr int kTileX = 256;        //   ... and tile columns (8 per lane)

// Coefficients of the periodic solve (I + rho [1,-4,6,-4,1]) y = x along one
// axis of one member, factored as y = ikappa * Qa^{-1} Qc^{-1} x with the
// causal recursion Qc^{-1}: u_i = x_i + a1 u_{i-1} + a2 u_{i-2} and its
// mirror image Qa^{-1} (a1 = 2 Re p, a2 = -|p|^2, p the root of
// rho (z-1)^4 + z^2 inside the unit circle).  A recursion state is the pair
// (u_i, u_{i-1}); one element advances it by the companion matrix
// A = [[a1, a2], [1, 0]].
struct AxisCoef {
    double a1, a2, ikappa;
    double inv_n;                    // 1 / line length (the line mean is passed around
                                     // the recursions, which then see zero-mean data)
    double E1[2];                    // zero-state end state of a chunk of ones
    double M[4];                     // A^c, c = chunk length (row-major)
    double Mp[kMaxScanLevels][4];    // (A^c)^(2^s)
    double W[4];                     // (I - A^n)^{-1}, n = line length
};

// The same coefficients rounded to FP32 once on the host, for the FP32
// kernels (no conversions in a kernel's prologue).
struct AxisCoefF {
    float a1, a2, ikappa, inv_n;
    float E1[2];
    float M[4];
    float Mp[kMaxScanLevels][4];
    float W[4];
};

// Products of the member's parameters that the RHS uses, formed once on the
// host in FP64 (in the order written) and also rounded to FP32.
enum : int {
    RC_DX, RC_DY, RC_DZ,     // dt / h_d^2
    RC_GXY, RC_GXZ, RC_GYZ,  // 2 gamma dt / (h_d^2 h_e^2)
    RC_AX4, RC_AY4,          // gamma dt / h_x^4, gamma dt / h_y^4 (Crank-Nicolson)
    RC_IHX2, RC_IHY2,        // 1 / h_x^2, 1 / h_y^2
    RC_DT, RC_TG,            // dt, 2 gamma dt
    RC_CXY,                  // 1 / (h_x^2 h_y^2)
    RC_N
};

struct MemberDev {
    int64_t off;       // element offset of this member in the field arrays
    int64_t sites;
    double h[3];
    double ih2[3];     // 1 / h^2
    double gamma, dt;
    double vol;        // prod h
    AxisCoef ax[3];
    AxisCoefF axf[3];
    double rc[RC_N];
    float rcf[RC_N];
};

// A class whose members have consecutive ids (every class of a uniform
// ensemble) is also described arithmetically: member mloc is id mid0 + mloc
// at element offset off0 + mloc * stride.  Kernels then form a member's
// buffer without a dependent load of the member tables.  mid0 < 0: look the
// members up.
struct MemberRun {
    int32_t mid0 = -1;
    int64_t off0 = 0, stride = 0;
};

// Step kernel modes.
enum : int { MODE_STEP = 0, MODE_DIAG = 1, MODE_TIMING = 2 };

// Per-member reduction of the pass-A partial sums (F, sum C, sum |grad mu|^2)
// into the sample series.  Blocks 0..G-1 of the step's last sweep do it
// (block b takes members b, b+G, ...), or a G-block kernel after a
// diagnostics-only pass A.  The step index comes from the stamp pass A wrote,
// so the step counter itself is only read by pass A and advanced by one
// thread of the last sweep.
struct FinArgs {
    int32_t enabled;           // 0: nothing to do
    int32_t mode;              // MODE_STEP: record what step n needs; the last sweep then
                               //   advances the counter.  MODE_DIAG: record everything.
    int32_t G;                 // blocks taking part in the reduction
    const MemberDev* mem;
    const int32_t* mids;       // member ids of the class
    int32_t nmem;
    int32_t K;                 // cadence
    int64_t blocks_per_member; // pass-A blocks (= partial triples) per member
    const double* partials;    // [member][blocks_per_member][3]
    const int64_t* nstamp;     // step index of the partials (written by pass A)
    int64_t max_samples;
    int64_t* step;             // step counter of the class
    double* series;            // [member][max_samples][kSeriesSlots]
    double* energy_now;        // [member][4]
    int32_t* flags;            // [member] sticky non-finite flags
};

struct PassAArgs {
    const void* C;             // T*, state C^n (all members)
    void* W;                   // T*, output of the x-solve
    const MemberDev* mem;      // member table (global ids)
    const int32_t* mids;       // member ids of this class
    int32_t nmem;              // members in this class
    MemberRun run;             // the class's members as one arithmetic run, where they are
    int32_t nx, ny, nz;
    int32_t P;                 // chunks per x-line (lanes; above 64 a line spans P / 64 wavefronts)
    int32_t rows_per_wave;     // x-lines per wavefront (line groups x lines per lane; 0 above 64 chunks)
    int32_t waves;             // wavefronts per block (1, 2 or 4)
    int32_t R;                 // x-lines per block (= waves * rows_per_wave)
    int32_t bands_y;           // y-bands per (member, z) = ceil(ny / R)
    int32_t units;             // work units per block: y-bands (2D) or z-planes of a y-band (3D)
    int64_t blocks_per_member;
    int64_t nblocks;           // blocks of this launch
    int32_t pitch;             // LDS row pitch (elements)
    int32_t mode;
    int32_t conv;              // energy convention
    int32_t K;                 // cadence
    int32_t cn;                // 1: Crank-Nicolson variant (theta = 1/2, 2D, one unit per block)
    const int64_t* step;       // step counter of this class (read only)
    double* partials;          // [nblocks][3]
    int64_t* nstamp;           // block 0 records the step index of the partials here
};

struct ColArgs {
    const void* src;           // T*
    void* dst;                 // T* (may equal src)
    const MemberDev* mem;
    const int32_t* mids;
    MemberRun mrun;            // the class's members as one arithmetic run, where they are
    int32_t axis;              // 1 = y, 2 = z
    int32_t n;                 // line length
    int64_t stride;            // element distance between line neighbours
    int64_t run;               // columns come in runs of `run` consecutive elements
    int64_t outer;             // element distance between runs
    int64_t cols;              // columns per member
    int64_t msites;            // sites per member
    int32_t b;                 // columns per block (a power of two dividing run)
    int32_t bshift;            // log2 b
    int32_t P;                 // chunks per column
    int64_t nblocks;
    FinArgs fin;               // enabled on the last sweep of a step
};

// Kernel launchers (ch_kernels.hip).  prec: 0 = double, 1 = float.  They
// return hipErrorInvalidValue for an uninstantiated chunk length.
// ev0/ev1 (optional): events that take the kernel's own start/end timestamps
hipError_t launch_passA(int prec, int dim, int cx, int rl, int units, const PassAArgs& a,
                        size_t lds_bytes, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
hipError_t launch_col(int prec, int cy, const ColArgs& a, hipStream_t s, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
hipError_t launch_init_member(int prec, void* C, int64_t sites, uint64_t seed, double c0,
                              double noise, hipStream_t s);
hipError_t launch_reset(int64_t* steps, int nsteps, int64_t value, int32_t* flags, int m,
                        double* series, int64_t series_len, hipStream_t s);
hipError_t launch_fin(const FinArgs& f, hipStream_t s);
hipError_t launch_beta(const double* series, int64_t max_samples, int32_t member, int32_t K,
                       int64_t ncur, double dt, double* out, int64_t J, hipStream_t s);
hipError_t launch_moments(const double* series, int64_t max_samples, const int32_t* members, int32_t nm,
                          int32_t K, int64_t ncur, double dt, int32_t pmax, double* out, int64_t J,
                          hipStream_t s);
hipError_t launch_window(const double* mom, int64_t j0, int64_t j1, int32_t K, double dt, double* out,
                         hipStream_t s);
// zeroes counts[0 .. nbins+1] first
hipError_t launch_hist(const double* series, int64_t max_samples, const int32_t* members, int32_t nm,
                       int32_t K, int64_t ncur, double dt, int64_t j0, int64_t j1, double lo, double hi,
                       int32_t nbins, unsigned long long* counts, hipStream_t s);

bool passA_has(int dim, int cx, int rl, int units, bool cn = false);  // units > 1: several units per block
// lines of 64 wl chunks of cx (2D): split = RHS pass (kTileY x kTileX tiles) then the x-solve in place
bool passA_wide_has(int prec, int cx, int wl, bool split);
bool col_has(int prec, int cy);
int passA_pad(int prec);       // LDS padding (elements) after every chunk
int passA_halo(int prec);      // periodic halo columns on each side of an LDS row

}  // namespace chk
