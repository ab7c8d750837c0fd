/*
 * dp.h -- C ABI of the droplet-population ensembles in libch.so: Model 1 of
 * the paper (Sections 2 and 3).
 *
 * Each ensemble member is a population of N droplets with radii R_i:
 *
 *     dR_i/dt = H(R_i) (-1/R_i^2 + ubar/R_i),
 *     ubar    = sum_i H(R_i) / sum_i H(R_i) R_i        (paper: eq. (dRi), eq. (uval))
 *
 * started from given radii (the paper draws them from U(0, 1): eq.
 * (dRi_init)).  The library integrates the volumes V_i = (R_i R_i) R_i, for
 * which the law reads dV_i/dt = 3 (ubar R_i - 1), R_i = cbrt(V_i), while
 * V_i > 0 and dV_i/dt = 0 once V_i <= 0 (the droplet has died).  This is the
 * paper's regularisation H(R_i + eps) (Section 3.1) in the limit eps -> 0;
 * in V the rates stay bounded where dR/dt is singular.
 *
 * Time integration: the Dormand-Prince 5(4) Runge-Kutta pair (the pair inside
 * ode45, which the paper used), advancing with the order-5 solution, with
 *
 *     err = max_i |h sum_s e_s k_{s,i}| / (atol + rtol max(|V_i|, |V_i new|)),
 *
 * e = order-5 minus order-4 weights; a step is accepted iff err <= 1; the
 * next trial step is h * clamp(0.9 err^(-1/5), 0.2, 5) (5 when err = 0), with
 * no growth right after a rejection; a step that would pass the next sample
 * time t_j = j dt_sample is shortened to end on it.  The first trial step is
 * h0.
 *
 * Samples j = 0..J-1, J = round(t_end / dt_sample) + 1, of every member:
 *
 *     t, F = (1/2) sum H(R) R^2                       (eq. (Fdef), volume constraint held)
 *     dF/dt = -sum H(R) (1/R) (1 - ubar R)^2          (eq. (dFdt))
 *     beta = -t (dF/dt) / F                           (eq. (betaN)); 0 at t = 0
 *     ubar, live droplets
 *
 * stored as 6 doubles per sample in that order.
 *
 * Conventions: as in ch.h.  Functions return ch_status and never throw; the
 * caller owns one device workspace of dp_workspace_bytes() bytes (256-byte
 * aligned) that must outlive the context; work runs on the caller's stream;
 * calls returning data to the host synchronise it; a context is not
 * re-entrant.  Until dp_set_radii has run, the other calls on the context
 * (except dp_destroy and dp_last_error) return CH_ESTATE; so do calls on a
 * destroyed or unknown context.
 */
#ifndef DP_H_
#define DP_H_

#include <stddef.h>
#include <stdint.h>

#include "ch.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dp_ctx dp_ctx;

typedef struct {
    double t_end;          /* >= 0; samples at j * dt_sample up to t_end */
    double dt_sample;      /* > 0 */
    double rtol, atol;     /* > 0: the error control above */
    double h0;             /* > 0: first trial step */
    int64_t max_attempts;  /* > 0: step attempts (accepted + rejected) per member over the run */
} dp_params;

/* Member states reported by dp_member_info. */
enum { DP_RUNNING = 0, DP_DONE = 1, DP_UNDERFLOW = 2, DP_NONFINITE = 3, DP_ATTEMPT_LIMIT = 4 };

/* Largest population per member. */
#define DP_MAX_DROPLETS 8192

/* Bytes of device workspace for m members of n[0..m-1] droplets
 * (1 <= n[i] <= DP_MAX_DROPLETS); 0 if the arguments are invalid. */
size_t dp_workspace_bytes(const int32_t* n, int32_t m, const dp_params* prm);

/* Create a context over the caller's workspace and stream (hipStream_t or
 * NULL).  Errors: CH_EINVAL (arguments, workspace too small or misaligned),
 * CH_EDEVICE. */
ch_status dp_create(const int32_t* n, int32_t m, const dp_params* prm, void* d_workspace, size_t ws_bytes,
                    void* hip_stream, dp_ctx** out);

/* Initial radii of all members, concatenated in member order (sum n values,
 * host memory).  V = (R R) R; radii <= 0 are dead from the start.  Records
 * sample 0 and resets every member to t = 0, h = h0.  Enqueued on the
 * stream; the host buffer may be reused when the call returns. */
ch_status dp_set_radii(dp_ctx* ctx, const double* host_radii);

/* One launch: up to `attempts` step attempts (> 0) for every member still
 * running.  Asynchronous. */
ch_status dp_advance(dp_ctx* ctx, int64_t attempts);

/* Launch dp_advance with `attempts` per launch until no member is running
 * (synchronising after each launch); *launches (may be NULL) receives the
 * launch count and *kernel_ms (may be NULL) the summed device time of those
 * launches, from events around them.  Returns CH_OK when every member is
 * done, CH_ENONFINITE if a member's error estimate was not finite,
 * CH_ESTATE on a step-size underflow or the attempt limit. */
ch_status dp_run(dp_ctx* ctx, int64_t attempts, int64_t* launches, double* kernel_ms);

/* Progress of one member (synchronises): time reached, accepted and
 * rejected attempts, state (DP_*), samples recorded, and the live-droplet
 * stage evaluations so far (each attempt evaluates six new stages of every
 * droplet alive at its start: the pair's last stage is the next step's
 * first).  Every output pointer may be NULL. */
ch_status dp_member_info(dp_ctx* ctx, int32_t member, double* t, int64_t* accepted, int64_t* rejected,
                         int32_t* state, int64_t* samples, double* evals);

/* Current volumes of one member (n values, host memory; synchronises). */
ch_status dp_get_volumes(dp_ctx* ctx, int32_t member, double* host_dst);

/* Recorded samples of one member: out holds cap*6 doubles (row j: t, F,
 * dF/dt, beta, ubar, live); *count = min(cap, samples recorded).
 * Synchronises. */
ch_status dp_series(dp_ctx* ctx, int32_t member, double* out, int64_t cap, int64_t* count);

/* Ensemble statistics of beta over the listed members (members = NULL: all;
 * otherwise 1 <= nm <= m, the ensemble size, else CH_EINVAL before anything
 * is enqueued; indices may repeat), over the samples every listed member has recorded, with the
 * definitions of ch.h: mu_1, central moments mu_p (eq. (mup); 1 <= pmax <= 8;
 * mu holds cap*pmax doubles, t may be NULL), the window mean beta0 of mu_1
 * and the slope k of mu_2 = k t (eq. (beta0_stats)), and the histogram of
 * beta (1 <= nbins <= 4096; counts holds nbins + 2 values).  Synchronise. */
ch_status dp_ensemble_moments(dp_ctx* ctx, const int32_t* members, int32_t nm, int32_t pmax, double* t,
                              double* mu, int64_t cap, int64_t* count);
ch_status dp_ensemble_window(dp_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2,
                             double* beta0, double* k);
ch_status dp_beta_histogram(dp_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2, double lo,
                            double hi, int32_t nbins, uint64_t* counts);

/* Release the context (synchronises the stream). */
ch_status dp_destroy(dp_ctx* ctx);

/* Message of the last failed call on ctx (thread-local when ctx is NULL). */
const char* dp_last_error(const dp_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DP_H_ */
