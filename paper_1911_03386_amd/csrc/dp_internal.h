// Internal interface between the droplet-ensemble host runtime (dp_host.cpp)
// and its kernels (dp_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dp {

constexpr int kSlots = 6;           // t, F, dF/dt, beta, ubar, live droplets
constexpr int kThreads = 512;       // threads per member (one workgroup)
constexpr int kMaxPerThread = 16;   // droplets per thread at most
constexpr int kMaxN = kThreads * kMaxPerThread;
constexpr int kMaxMoments = 8;      // stride of the moments table

enum MemberStatus : int32_t {
    kRunning = 0,
    kDone = 1,
    kUnderflow = 2,   // t + h == t
    kNonFinite = 3,   // the error estimate is not finite
    kAttemptLimit = 4,
};

struct Member {
    int64_t off;   // first droplet in the volume array
    int32_t n;     // droplets
    int32_t pad;
};

// Integrator state of one member between launches.
struct State {
    double t, h, ubar;   // time, next trial step, mean field of the state
    int64_t jn;          // next sample index
    int64_t acc, rej;    // accepted and rejected step attempts
    int32_t rej_last;    // the last attempt was rejected
    int32_t status;      // MemberStatus
    int32_t nslot;       // slots in use: slot j < nslot holds droplet slot[j]
    int32_t live;        // live droplets of the state
    double evals;        // live-droplet stage evaluations so far (6 per live droplet and attempt)
};

struct Args {
    const Member* mem;
    const int32_t* order;   // block b integrates member order[b]
    State* st;
    double* V;              // volumes, all members concatenated
    int32_t* slot;          // per member (offset Member::off): droplet held by each slot
    double* series;         // [member][J][kSlots]
    int64_t J;              // samples per member: t_j = j dts
    double dts, rtol, atol, h0;
    int64_t max_total;      // attempts per member over the whole run
};

// droplets per thread that a launch is compiled for, given the largest member
int per_thread(int32_t nmax);
hipError_t launch_init(const Args& a, int32_t blocks, int per, hipStream_t s);
hipError_t launch_steps(const Args& a, int32_t blocks, int per, int64_t attempts, hipStream_t s);
hipError_t launch_moments(const double* series, int64_t J, const int32_t* members, int32_t nm, int64_t count,
                          int32_t pmax, double* out, hipStream_t s);
hipError_t launch_hist(const double* series, int64_t J, const int32_t* members, int32_t nm, int64_t j0,
                       int64_t j1, double lo, double hi, int32_t nbins, unsigned long long* counts,
                       hipStream_t s);
hipError_t launch_window(const double* mom, int64_t j0, int64_t j1, double dts, double* out, hipStream_t s);
hipError_t launch_zero(unsigned long long* p, int64_t n, hipStream_t s);

}  // namespace dp
