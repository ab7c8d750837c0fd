// Host-only build of the runtimes for the sanitizer test: the kernel
// launchers are not linked, every launch fails, and the shape predicates
// mirror the compiled shape tables closely enough for the validation paths.
#include "../../paper_1911_03386_amd/csrc/ch_internal.h"
#include "../../paper_1911_03386_amd/csrc/dp_internal.h"

namespace chk {
hipError_t launch_passA(int, int, int, int, int, const PassAArgs&, size_t, hipStream_t, hipEvent_t, hipEvent_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_col(int, int, const ColArgs&, hipStream_t, hipEvent_t, hipEvent_t) { return hipErrorInvalidValue; }
hipError_t launch_init_member(int, void*, int64_t, uint64_t, double, double, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_reset(int64_t*, int, int64_t, int32_t*, int, double*, int64_t, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_fin(const FinArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_beta(const double*, int64_t, int32_t, int32_t, int64_t, double, double*, int64_t, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_moments(const double*, int64_t, const int32_t*, int32_t, int32_t, int64_t, double, int32_t, double*,
                          int64_t, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_window(const double*, int64_t, int64_t, int32_t, double, double*, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_hist(const double*, int64_t, const int32_t*, int32_t, int32_t, int64_t, double, int64_t, int64_t,
                       double, double, int32_t, unsigned long long*, hipStream_t)
{
    return hipErrorInvalidValue;
}
bool passA_has(int dim, int cx, int rl, int units, bool cn)
{
    const bool c = cx == 4 || cx == 8 || cx == 16 || cx == 32 || cx == 64;
    return (dim == 2 || dim == 3) && c && rl >= 1 && units >= 1 && (!cn || (dim == 2 && units == 1));
}
bool passA_wide_has(int prec, int cx, int wl, bool split)
{
    if (split) return prec == 0 && wl == 4 && (cx == 4 || cx == 32);
    return (wl == 2 && (cx == 8 || cx == 16 || cx == 32)) || (wl == 4 && (cx == 4 || cx == 8 || cx == 16 || cx == 32));
}
bool col_has(int prec, int cy) { return cy == 4 || cy == 8 || cy == 16 || cy == 32 || (prec == 1 && cy == 64); }
int passA_pad(int) { return 1; }
int passA_halo(int prec) { return prec == 0 ? 2 : 4; }
}  // namespace chk

namespace dp {
int per_thread(int32_t nmax) { return nmax <= 512 ? 1 : nmax <= 1024 ? 2 : nmax <= 2048 ? 4 : nmax <= 4096 ? 8 : 16; }
hipError_t launch_init(const Args&, int32_t, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_steps(const Args&, int32_t, int, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_moments(const double*, int64_t, const int32_t*, int32_t, int64_t, int32_t, double*, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_hist(const double*, int64_t, const int32_t*, int32_t, int64_t, int64_t, double, double, int32_t,
                       unsigned long long*, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_window(const double*, int64_t, int64_t, double, double*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_zero(unsigned long long*, int64_t, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace dp
