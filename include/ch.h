/*
 * ch.h -- C ABI of the MI355X Cahn-Hilliard ensemble library (libch.so).
 *
 * The library time-steps a batch ("ensemble") of independent periodic
 * realisations of the constant-mobility Cahn-Hilliard equation
 *
 *     dC/dt = lap(C^3 - C - gamma lap C)                 (paper: eq. (ch))
 *
 * with the semi-implicit ADI finite-difference scheme (paper: Section 4.1,
 * Appendix A), and records the free energy F, its rate dF/dt and the
 * coarsening rate beta = -(t/F) dF/dt                 (paper: eq. (dFdt_ch),
 * eq. (betadef)).  The discrete scheme, exactly:
 *
 *   RHS     = C^n + dt lap_h(C^3 - C) - 2 gamma dt sum_{d<e} D_d D_e C^n
 *   w^0     = RHS;  (I + gamma dt D_d^2) w^d = w^{d-1} on every d-line, d = x,y(,z)
 *   C^{n+1} = w^D
 *
 * with D_d the periodic second difference on a vertex grid x_i = i h_d,
 * h_d = L_d / n_d.  Diagnostics of the state C^n:
 *
 *   F      = prod(h) sum [ e(C) + gamma/2 sum_d ((C_{+d} - C)/h_d)^2 ],
 *            e(C) = (C^2-1)^2/4 (CH_ENERGY_QUARTER) or (C^2-1)^2/2 (as printed)
 *   <C>    = sum C / #sites                  (conserved; paper Section 4)
 *   G_id   = -prod(h) sum_d |(mu_{+d} - mu)/h_d|^2, mu = C^3 - C - gamma lap_h C
 *   G_fd   = (F^{n+1} - F^{n-1}) / (2 dt)     (one-sided where a neighbour is
 *                                               missing: the run's start/end)
 *   beta   = -(n dt) G_fd / F^n,  beta = 0 at n = 0
 *
 * Samples are taken at n = jK (K = cadence), j = 0, 1, ..., max_samples-1.
 *
 * Conventions
 *  - Every function returns ch_status; nothing throws or aborts across the ABI.
 *  - Fields are x-fastest: site (i1, i2, i3) is element i1 + n1*(i2 + n2*i3).
 *  - Device memory is owned by the caller: one workspace of
 *    ch_workspace_bytes() bytes, 256-byte aligned, that must outlive the
 *    context.  The library keeps only host metadata (and, when enabled, HIP
 *    graphs that reference the workspace).
 *  - Work is enqueued on the caller's HIP stream given to ch_create (NULL =
 *    the null stream).  Calls that return data to the host synchronise it.
 *    With several size classes, ch_step runs the classes on up to four
 *    streams: up to three more streams (default priority, created by
 *    ch_create, destroyed by ch_destroy) are forked from the caller's stream
 *    at the start of each ch_step call or graph replay and joined back into
 *    it at the end, so the caller's stream orders all work as usual.
 *  - Asynchronous device faults surface at the next synchronising call as
 *    CH_EDEVICE.  A non-finite F sets a sticky per-member flag reported as
 *    CH_ENONFINITE by ch_energy, ch_beta_series and the ensemble-statistics
 *    calls.
 *  - A context is bound to one stream and is not re-entrant.
 */
#ifndef CH_H_
#define CH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ch_ctx ch_ctx; /* opaque */

/* The enums are int-sized, and any int may be passed for them: the library
 * checks the values (in C++ the fixed underlying type makes every int a
 * valid value of the type). */
#ifdef __cplusplus
#define CH_ENUM_INT : int
#else
#define CH_ENUM_INT
#endif

typedef enum CH_ENUM_INT {
    CH_OK = 0,
    CH_EINVAL = 1,       /* bad argument; nothing was enqueued */
    CH_ENOMEM = 2,       /* workspace too small, or host allocation failed */
    CH_EDEVICE = 3,      /* a HIP call failed (message in ch_last_error) */
    CH_ESTATE = 4,       /* call not valid in the current state (e.g. sample
                            capacity exceeded, destroyed context) */
    CH_ENONFINITE = 5,   /* F became NaN/Inf for at least one member */
    CH_EUNSUPPORTED = 6  /* valid but unsupported shape (see ch_member_desc) */
} ch_status;

typedef enum CH_ENUM_INT {
    CH_F64 = 0,      /* state, stencils and line solves in FP64 */
    CH_F32_BULK = 1  /* state, stencils and line solves in FP32; F, <C>, G and
                        beta are always reduced and reported in FP64 */
} ch_precision;

typedef enum CH_ENUM_INT {
    CH_ENERGY_QUARTER = 0,       /* e(C) = (C^2-1)^2/4, consistent with eq. (ch) */
    CH_ENERGY_PAPER_PRINTED = 1  /* e(C) = (C^2-1)^2/2, the prefactor printed
                                    with eq. (dFdt_ch) */
} ch_energy_conv;

/* One ensemble member.
 *  dim      2 or 3
 *  n[3]     points per axis (x, y, z); n[2] must be 1 when dim == 2.  Each
 *           used axis needs 8 <= n <= 8192 and n a multiple of 4.  x: n = c * P
 *           with c in {4, 8, 16, 32, 64} and P <= 64 chunks (n <= 4096), or,
 *           in 2D, P = 128 or 256 chunks of c in {4, 8, 16, 32} (lines held
 *           by 2 or 4 wavefronts).  y, z: n = c * P with P <= 256 chunks of a
 *           column-sweep chunk length (4..32; FP32 also 64).  Every power of
 *           two from 8 to 8192 qualifies in 2D, to 4096 along x in 3D;
 *           otherwise CH_EUNSUPPORTED.
 *  L[3]     domain lengths (> 0); L[2] ignored in 2D
 *  gamma    interface parameter (> 0);  dt  time step (> 0)
 *  c0, noise  initial condition C = c0 + noise (2u - 1), u in [0,1) from the
 *           (site+1)-th output of SplitMix64 seeded with `seed`:
 *           u = (out >> 11) * 2^-53 (computed in FP64, rounded to FP32 in
 *           CH_F32_BULK mode). */
typedef struct {
    int32_t dim;
    int32_t n[3];
    double L[3];
    double gamma;
    double dt;
    double c0;
    double noise;
    uint64_t seed;
} ch_member_desc;

/* Bytes of device workspace needed for this ensemble (0 if the arguments are
 * invalid; ch_last_error(NULL) then says why). */
size_t ch_workspace_bytes(const ch_member_desc* members, int32_t m, ch_precision prec,
                          int32_t cadence, int64_t max_samples);

/* Create a context over a caller-owned device workspace.  Fields start at 0;
 * call ch_init_random or ch_set_field before stepping.  cadence K >= 1 is the
 * sample spacing in steps; max_samples >= 1 bounds the number of samples
 * (n <= K (max_samples - 1) steps may be taken).  hip_stream is a hipStream_t
 * (NULL = null stream).  *out receives the context. */
ch_status ch_create(const ch_member_desc* members, int32_t m, ch_precision prec,
                    ch_energy_conv conv, int32_t cadence, int64_t max_samples,
                    void* d_workspace, size_t ws_bytes, void* hip_stream, ch_ctx** out);

/* Fill every member's field with its seeded initial condition (on device) and
 * reset the step counter, the sample series and the non-finite flags. */
ch_status ch_init_random(ch_ctx* ctx);

/* Copy one member's field from/to host memory (FP64, x-fastest, #sites
 * values).  In CH_F32_BULK mode set rounds to nearest FP32 and get widens.
 * Both synchronise the stream. */
ch_status ch_set_field(ch_ctx* ctx, int32_t member, const double* host_src);
ch_status ch_get_field(ch_ctx* ctx, int32_t member, double* host_dst);

/* Step counter n (time t = n dt per member).  ch_set_step also clears the
 * recorded series, so a run restored from saved fields continues from n
 * with fresh samples (the first restored sample takes a one-sided
 * difference). */
ch_status ch_get_step(const ch_ctx* ctx, int64_t* n);
ch_status ch_set_step(ch_ctx* ctx, int64_t n);

/* Advance every member by nsteps steps (asynchronous on the context stream).
 * Records F on steps n = -1, 0, +1 (mod K) and <C>, G_id on n = 0 (mod K).
 * CH_ESTATE if the sample capacity would be exceeded. */
ch_status ch_step(ch_ctx* ctx, int64_t nsteps);

/* F and <C> of the current state of every member (arrays of m doubles; either
 * pointer may be NULL).  Synchronises. */
ch_status ch_energy(ch_ctx* ctx, double* F, double* meanC);

/* The sample series of one member: for j = 0..count-1 (n = jK <= current
 * step), t, F, G_fd, G_id, beta and <C> (any pointer may be NULL; each holds
 * at least cap doubles).  *count = min(cap, floor(n_current/K) + 1).
 * Synchronises. */
ch_status ch_beta_series(ch_ctx* ctx, int32_t member, double* t, double* F, double* dFdt,
                         double* dFdt_identity, double* beta, double* meanC, int64_t cap,
                         int64_t* count);

/* Time scheme.  theta = 1 (default): the implicit ADI step above.
 * theta = 1/2 (every member 2D): its Crank-Nicolson variant
 *
 *   (I + a D_x^2/2)(I + a D_y^2/2) C^{n+1}
 *       = (I - a D_x^2/2)(I - a D_y^2/2) C^n + (RHS - C^n),   a = gamma dt,
 *
 * second order in dt where only the pure fourth derivatives act (paper:
 * Appendix A, the scheme for hyper-diffusion alone) and first order once the
 * explicit nonlinear and mixed terms act, as for theta = 1.  Its stiff axis
 * modes are not damped: their growth factors approach -1 as gamma dt / h^4
 * grows (about -0.99 for 512^2 grids at dt = 1e-3), where theta = 1 removes
 * them within a step.  Applies from the next step; the state, the step
 * counter and the series are kept; tile shapes are re-planned (the variant
 * reads two halo lines on either side in y).  CH_EINVAL for any other theta,
 * CH_EUNSUPPORTED if a member is 3D. */
ch_status ch_set_theta(ch_ctx* ctx, double theta);

/* Tile shapes.  ch_autotune times every valid tile shape of every size class
 * on the device (using the workspace's scratch field only: the state and the
 * series are untouched) and keeps the fastest.  With several classes it then
 * times the best few shapes of each class together, as whole steps of all
 * classes running concurrently, and keeps the fastest combination.
 * cache_path (may be NULL) is a text file of earlier choices keyed by GPU
 * architecture, shape, member count and precision; it is read first and
 * rewritten with the results. */
ch_status ch_autotune(ch_ctx* ctx, const char* cache_path);

/* Number of size classes and explicit tile shapes for one class.  Members
 * are grouped by dimension and grid shape, in order of first appearance; while
 * there are fewer than four classes, the class with the most sites among
 * those of at least 8 members is split into two classes of consecutive
 * members.  Classes are
 * independent and run concurrently on separate streams.  The
 * RHS + x-solve pass: cx = elements per lane of an x-line, rl = x-lines per
 * lane, waves = wavefronts per block, units = work units a block walks
 * through, loading the next one while it computes the current one (y-bands
 * in 2D; z-planes of one y-band in 3D, with a ring of staged planes).  The
 * y-solve: cy = elements per
 * lane, by = columns per block; cz/bz the same for the z-solve (ignored in
 * 2D).  x-lines of more than 64 chunks (nx / cx = 128 or 256; 2D) take
 * rl = 1, waves = 4 and units = 1, or units = 0 for the split form: the RHS
 * is formed over 8 x 256 tiles into the scratch field first and the x-lines
 * are then solved in place there (FP64, nx a multiple of 256; the form used
 * where a line's staged rows exceed LDS).  CH_EUNSUPPORTED if the shape is
 * not valid for the class (nothing changes then). */
ch_status ch_num_classes(const ch_ctx* ctx, int32_t* nclasses);
ch_status ch_set_tiles(ch_ctx* ctx, int32_t cls, int32_t cx, int32_t rl, int32_t waves,
                       int32_t units, int32_t cy, int32_t by, int32_t cz, int32_t bz);

/* HIP graphs: with graph_steps > 0, ch_step replays a captured graph of
 * graph_steps steps (default 16); 0 launches every kernel directly.
 * ch_set_graph_steps captures, instantiates and uploads that graph at once
 * (nothing runs), so the first ch_step that replays it costs no more than
 * later ones; ch_autotune and ch_set_tiles drop it, and the next ch_step
 * that needs it builds it again.  Kernels
 * are always launched directly on the legacy null stream (it cannot be
 * captured) and while the caller is capturing the stream itself.  A graph the
 * caller captures advances the device step counter on every replay, while the
 * host keeps the count it had at capture: ch_sync_step reads the device
 * counter back (synchronising the stream) so that later calls see the true
 * step; it changes neither the state nor the series. */
ch_status ch_set_graph_steps(ch_ctx* ctx, int32_t graph_steps);
ch_status ch_sync_step(ch_ctx* ctx, int64_t* n);

/* Describe the chosen tile shapes as text (for logs), NUL-terminated. */
ch_status ch_describe(const ch_ctx* ctx, char* buf, size_t cap);

/* Mean device duration (ms) per launch of each kernel kind over nsteps real
 * steps, launched directly on the context stream, each kernel with a pair of
 * HIP events that take its own start and end timestamps
 * (hipExtLaunchKernel): ms[0] = RHS + x-solve pass, ms[1] = y-solve pass,
 * ms[2] = z-solve pass (0 in 2D), summed over size classes.  The steps include
 * the sample-step diagnostics like any other steps; the state advances by
 * nsteps. */
ch_status ch_time_kernels(ch_ctx* ctx, int64_t nsteps, double* ms);

/* Ensemble statistics of beta (the paper's eq. (mup) and eq. (beta0_stats),
 * and the fit of the variance growth E(dbeta^2) = k t; Sections 3.3 and 4).
 * members: nm member indices (NULL = all members; otherwise 1 <= nm <= m, the
 * ensemble size, else CH_EINVAL before anything is enqueued; indices may
 * repeat, e.g. a bootstrap resample); the selected members must
 * share dt, so that sample j is at t_j = jK dt for all of them.  All three
 * are computed on the device in FP64 with fixed-order sums (deterministic),
 * from the recorded F series with the same beta as ch_beta_series, and
 * synchronise.  CH_ENONFINITE if a selected member has a non-finite F.
 *
 * ch_ensemble_moments: for every recorded sample j = 0..count-1,
 *   mu[j*pmax + 0]     = mu_1(t_j) = (1/M) sum_m beta_m(t_j),
 *   mu[j*pmax + p - 1] = mu_p(t_j) = (1/M) sum_m (beta_m(t_j) - mu_1(t_j))^p,
 * 1 <= pmax <= 8; t (may be NULL) receives t_j; mu holds cap*pmax doubles;
 * *count = min(cap, floor(n_current/K) + 1).
 *
 * ch_ensemble_window: over the recorded samples with t1 <= t_j <= t2,
 *   beta0 = (trapezoid integral of mu_1) / (t_last - t_first),
 *   k     = sum t_j mu_2(t_j) / sum t_j^2 (least squares through the origin);
 * NaN when the window holds fewer than two samples (beta0) or none (k).
 *
 * ch_beta_histogram: beta_m(t_j) over the members and the recorded samples
 * with t1 <= t_j <= t2: counts[0] = values below lo, counts[1..nbins] = nbins
 * equal bins of [lo, hi), counts[nbins+1] = values at or above hi (NaN not
 * counted); 1 <= nbins <= 4096, counts holds nbins + 2 values. */
ch_status ch_ensemble_moments(ch_ctx* ctx, const int32_t* members, int32_t nm, int32_t pmax, double* t,
                              double* mu, int64_t cap, int64_t* count);
ch_status ch_ensemble_window(ch_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2,
                             double* beta0, double* k);
ch_status ch_beta_histogram(ch_ctx* ctx, const int32_t* members, int32_t nm, double t1, double t2,
                            double lo, double hi, int32_t nbins, uint64_t* counts);

/* Release the context (synchronises its stream).  Later calls with the same
 * pointer return CH_ESTATE. */
ch_status ch_destroy(ch_ctx* ctx);

/* Coefficients of the factorised periodic line solve used by the kernels, for
 * host-side checks: out[0..2] = a1, a2, ikappa; out[3..6] = A^chunk and
 * out[7..10] = (I - A^n)^{-1} (row-major 2x2), A = [[a1, a2], [1, 0]].  The
 * solve of (I + rho [1,-4,6,-4,1]) y = x on a periodic line of n points is
 * y = ikappa * (anti-causal recursion)(causal recursion) x with
 * u_i = x_i + a1 u_{i-1} + a2 u_{i-2}.  prec 1 gives the FP32-rounded a1, a2
 * (and ikappa, A^chunk, W derived from them). */
ch_status ch_solver_coefficients(double rho, int32_t n, int32_t chunk, int32_t prec, double* out);

/* ---- Allocation-free stepping ----------------------------------------------
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): no context and no workspace.  Advances
 * fields the caller owns by nsteps steps of the scheme above (the same kernels
 * as ch_step, with the default tile shapes).  The scratch these kernels need
 * (the x-solve output field, the coefficient table, the diagnostic partials,
 * the step counter) lives in one static device array of
 * CH_STATIC_SCRATCH_BYTES bytes per GPU, which each GPU the library runs on
 * holds from the library's first use there until the process ends.  The call
 * performs no hipMalloc, hipFree or other allocation.
 *
 *  members   m host descriptors, 1 <= m <= CH_STATIC_MAX_MEMBERS, as for
 *            ch_create, all with the dimension and grid (n[]) of member 0;
 *            seed, c0 and noise are not used.
 *  d_field   device array, 16-byte aligned: member i's field starts at element
 *            i * S, S = n[0] n[1] n[2], x-fastest; double (CH_F64) or float
 *            (CH_F32_BULK).  Advanced in place.
 *  d_energy  device array of 4 m doubles, or NULL.  After the last step:
 *            [4i] = F (quarter prefactor), [4i+1] = <C>, [4i+2] = G_id,
 *            [4i+3] = nsteps; a non-finite state gives a non-finite F.
 *  hip_stream  everything is enqueued on it, asynchronously (NULL = null stream).
 *
 * CH_EINVAL / CH_EUNSUPPORTED for bad descriptors, differing grids, m out of
 * range, a NULL or misaligned d_field, or nsteps < 0; CH_ENOMEM when the
 * scratch of this ensemble (about S m bytes per byte of element, plus tables)
 * exceeds CH_STATIC_SCRATCH_BYTES.  Nothing is enqueued on an error; the
 * message is in ch_last_error(NULL).
 *
 * Every call on a GPU shares that GPU's scratch array, and the array keeps the
 * last call's contents (each call resets the counter, flags and series it
 * uses).  Calls that overlap on one GPU (other streams, or other host threads
 * without ordering between them) race on the array and give wrong results:
 * serialise them.  The coefficient table goes up with a host-to-device copy
 * from library memory, so the call cannot be captured into a graph. */
#define CH_STATIC_SCRATCH_BYTES ((size_t)80 << 20)
#define CH_STATIC_MAX_MEMBERS 64
ch_status ch_step_static(const ch_member_desc* members, int32_t m, ch_precision prec, void* d_field,
                         int64_t nsteps, double* d_energy, void* hip_stream);

/* Last error message of ctx, or of the calling thread when ctx == NULL. */
const char* ch_last_error(const ch_ctx* ctx);

/* Library version string. */
const char* ch_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CH_H_ */
