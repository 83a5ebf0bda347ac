/*
 * gp_ssm -- exact O(N) Gaussian-process likelihood, gradient and posterior for
 * exposure-integrated, possibly overlapping measurements of a sum of SHO
 * (stochastically driven damped harmonic oscillator) processes, computed by a
 * Kalman filter and smoother (the RTS posterior, in adjoint form) over the
 * augmented state-space model of
 * "Scalable Gaussian Processes for Integrated and Overlapping Measurements via
 * Augmented State-Space Models" (Sec. 3.2: an integrator state per instrument,
 * reset when an exposure opens and read out when it closes), on AMD MI355X
 * (gfx950) in FP64.
 *
 * Problem statement (Sec. 3.2, exposure-averaged measurement model):
 *   y_n = (1/delta_n) int_{t^s_n}^{t^e_n} f(t) dt + eps_n,
 *   eps_n ~ N(0, yerr_n^2 + jitter^2),   delta_n = t^e_n - t^s_n,
 *   f = sum_{m=1..M} SHO_m,  SHO covariance with (sigma_m, omega0_m, Q_m)
 *   as in Appendix B (k(0) = sigma^2, omega0 in rad per time unit).
 * A zero-length exposure (t^e_n == t^s_n) is an instantaneous sample of f.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A batch holds B independent series.  offsets[B+1] (int64, ascending,
 *    offsets[0] = 0) delimits each series' measurements in the flat arrays
 *    t_start, t_end, y, yerr (length offsets[B]).  Within a series t_start
 *    must be non-decreasing; t_end >= t_start; yerr >= 0; all finite.  A
 *    series may be empty: its log-likelihood is 0, its gradient 0 and its
 *    posterior at any test time the prior.
 *  - Hyperparameters are series-major: sigma[b*M + m], omega0[b*M + m],
 *    quality[b*M + m] (all > 0, finite), jitter[b] (>= 0) or NULL for zero.
 *    They may be device or host arrays (host arrays are copied on the
 *    stream).  Output arrays must be device memory (hipMalloc'd or managed);
 *    so must every other array argument unless stated otherwise.  The
 *    caller owns all buffers.  `stream` is a hipStream_t (NULL = the
 *    default stream); kernels are enqueued on it and outputs are valid once
 *    it has synchronised.  Plan creation and the smoother read some inputs
 *    on the host (the data, test times) and synchronise with `stream` to do
 *    so; gp_ssm_plan_loglik and gp_ssm_plan_loglik_grad do not: they only
 *    enqueue work, replayed from a graph the plan captures on its first such
 *    call (again after its workspace grows).  Calls on one plan share its
 *    workspace and must be issued on one stream, or ordered by the caller.
 *  - At most GP_SSM_MAX_TERMS terms and GP_SSM_MAX_SLOTS simultaneously open
 *    exposures per series (the overlap depth; instrument labels are assigned
 *    internally, Sec. 3.2.3).
 *  - Return value: 0 on success, else a negative GP_SSM_E* code with a
 *    message from gp_ssm_last_error().  Pointers, sizes and the data are
 *    validated on the host before any device work.  The hyperparameters are
 *    validated on the device, per series, before any other kernel reads
 *    them: per-series status[b] (int32, may be NULL) receives 0,
 *    GP_SSM_EPARAM for a series whose hyperparameters are out of range, or
 *    GP_SSM_ENUMERIC for a series whose likelihood is not finite (a
 *    non-positive innovation variance, an overflow or a singular summary);
 *    the outputs of such a series are NaN and other series are unaffected.
 *    The plan forms return 0 in that case (they do not wait for the device);
 *    the one-shot forms, which do, return GP_SSM_EPARAM or GP_SSM_ENUMERIC
 *    when any series failed.
 */
#ifndef GP_SSM_H
#define GP_SSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GP_SSM_MAX_TERMS 4
#define GP_SSM_MAX_SLOTS 4
#define GP_SSM_MAX_INSTRUMENTS 8

/* term kinds (gp_ssm_plan_set_term_kinds) */
#define GP_SSM_TERM_SHO 0  /* stochastically driven damped harmonic oscillator (sigma, omega0, Q) */
#define GP_SSM_TERM_REAL 1 /* real exponential term sigma^2 exp(-omega0 |tau|); Q unused */

#define GP_SSM_OK 0
#define GP_SSM_EINVAL (-1)   /* null pointer, B < 1, M out of range, bad offsets */
#define GP_SSM_EDATA (-2)    /* non-finite data, t_end < t_start, unsorted t_start, yerr < 0 */
#define GP_SSM_EPARAM (-3)   /* sigma, omega0, Q or an amplitude <= 0 or non-finite; jitter < 0 or
                                non-finite; an offset non-finite */
#define GP_SSM_EOVERLAP (-4) /* more than GP_SSM_MAX_SLOTS exposures open at once */
#define GP_SSM_ENUMERIC (-5) /* some series had a non-finite result; see status[] */
#define GP_SSM_EDEVICE (-6)  /* no usable gfx950 device or a HIP error */
#define GP_SSM_ENOMEM (-7)   /* device or host allocation failed */

/* Opaque, hyperparameter-independent description of a batch: the event
 * stream of every series (starts and ends of exposures, Sec. 3.2, ordered in
 * time with ends first at ties), instrument slots, and the split of each
 * series into chunks at instants where no exposure is open.  Lives on the
 * device that was current at creation. */
typedef struct gp_ssm_plan gp_ssm_plan;

typedef struct {
  int32_t chunk_min;     /* shortest chunk in events (default 24) */
  int32_t chunk_target;  /* target chunk length in events; 0 = derived from the batch */
  int64_t target_chunks; /* wanted number of chunks when deriving (default 131072) */
  int32_t single_chunk;  /* 1 = never split a series in time (each series then
                          * fills one lane of a 64-lane work wave; a batch
                          * whose layout would pad its events more than
                          * 16-fold beyond 2^24 events is refused with
                          * GP_SSM_ENOMEM) */
  int32_t threads;       /* host threads used to build the plan; 0 = all */
  /* device bytes for the per-event filter states that the gradient and the
   * smoother keep between their forward and backward sweeps (default
   * 32 GiB; <= 0 = default).  Past it they run in rounds of work waves that
   * reuse one buffer (at least one slot per workgroup the GPU holds at once),
   * so memory stays bounded whatever the size of the batch. */
  int64_t record_budget;
} gp_ssm_plan_options;

/* n_events_padded: events in the interleaved device layout, the real ones and
 * the no-op padding of chunks shorter than the longest of their wavefront;
 * n_segments: runs of up to 64 consecutive chunks combined by one wavefront
 * of the time-parallel scan; device_bytes: device memory the plan holds now
 * (its event layout and tables, and the workspace its calls have grown);
 * record_bytes: the part of it that holds per-event filter states for the
 * backward passes (one slot per resident workgroup, bounded by the number of
 * workgroups the GPU runs at once times the longest work wave, not by the
 * size of the batch). */
typedef struct {
  int64_t n_series, n_meas, n_events, n_events_padded;
  int32_t n_chunks, n_segments, max_slots, max_chunk_len;
  int64_t device_bytes, record_bytes;
} gp_ssm_plan_stats;

/* Fills *opt with the defaults. */
void gp_ssm_plan_default_options(gp_ssm_plan_options* opt);

/* Builds a plan for the batch.  offsets may be a host or device pointer; the
 * measurement arrays are device pointers (copied to the host to plan).  The
 * plan keeps its own copy of the data in event order; the inputs may be
 * freed afterwards.  opt may be NULL (defaults).  Returns GP_SSM_EINVAL,
 * GP_SSM_EDATA, GP_SSM_EOVERLAP, GP_SSM_ENOMEM or GP_SSM_EDEVICE on failure,
 * with *out set to NULL. */
int gp_ssm_plan_create(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                       const double* y, const double* yerr, const gp_ssm_plan_options* opt, void* stream,
                       gp_ssm_plan** out);

/* Kinds of the n_terms terms of later calls (kinds: host array, every
 * series the same; NULL or n_terms = 0: all SHO, the default).  An SHO term
 * has the kernel of Appendix B (sigma, omega0, Q); with Q = 1/2 it is the
 * Matern-3/2 kernel sigma^2 (1 + sqrt(3) tau / rho) exp(-sqrt(3) tau / rho)
 * at omega0 = sqrt(3) / rho.  A real term (GP_SSM_TERM_REAL) has the kernel
 * sigma^2 exp(-omega0 |tau|), the real celerite term of Appendix A (b = d =
 * 0) with rate c = omega0, as a one-state process with its integrator: its
 * quality entries are not read (any value; not validated) and its Q
 * derivative is 0.  Calls with another number of terms fail with
 * GP_SSM_EINVAL.  Synchronises the device. */
int gp_ssm_plan_set_term_kinds(gp_ssm_plan* plan, int32_t n_terms, const int32_t* kinds);

/* Instrument of every measurement, for the observation model with one
 * amplitude a_i and one offset c_i per instrument i (Sec. 2.2: the
 * observation matrix of a measurement, scaled per instrument; Sec. 3.2.3:
 * instrument labels; Sec. 1: combining instruments of different
 * calibration):
 *   y_n = a_{i(n)} (1/delta_n) int f dt + c_{i(n)} + eps_n,
 * the noise not scaled.  instrument[offsets[B]] (host or device int32, in
 * the order of the plan's measurements) holds labels 0..n_inst-1, n_inst <=
 * GP_SSM_MAX_INSTRUMENTS; NULL or n_inst = 0 removes the labels.  These
 * labels are the caller's calibration groups, unrelated to the integrator
 * slots the plan assigns to overlapping exposures.  The *_inst entry points
 * then take the per-series amplitudes and offsets; the other entry points
 * use a = 1, c = 0.  Synchronises the device.  GP_SSM_EINVAL for a label
 * out of range. */
int gp_ssm_plan_set_instruments(gp_ssm_plan* plan, int32_t n_inst, const int32_t* instrument, void* stream);

/* Releases the plan and its device memory (and any workspace it grew). */
void gp_ssm_plan_destroy(gp_ssm_plan* plan);

/* Sizes of the plan (host output). */
int gp_ssm_plan_get_stats(const gp_ssm_plan* plan, gp_ssm_plan_stats* out);

/* Log-likelihood of every series (Sec. 2.4 with the augmented filter of
 * Sec. 3.2), including -N/2 log 2 pi.  loglik[B] (device), status[B] (device,
 * may be NULL). */
int gp_ssm_plan_loglik(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                       const double* quality, const double* jitter, double* loglik, int32_t* status, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the log-likelihood
 * of gp_ssm_plan_loglik, computed by the same kernels, with its workspace
 * taken from a static device array of 64 MiB that the library holds on each
 * GPU it runs on until the process ends.  Calls no hipMalloc, hipFree or
 * other allocating routine, does not synchronise and captures no graph.
 * Every array argument must be device memory (GP_SSM_EINVAL otherwise), and
 * the plan must live on the current device.  A batch whose workspace (about
 * 2.5 KB per chunk and 4.4 KB per series and term at three terms) exceeds
 * 64 MiB is refused with GP_SSM_ENOMEM before any device work.  All calls on
 * one GPU share the array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller. */
int gp_ssm_plan_loglik_noalloc(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                               const double* quality, const double* jitter, double* loglik, int32_t* status,
                               void* stream);

/* Log-likelihood and its gradient by a reverse-mode adjoint of the filter.
 * grad[b*(3M+1) + k] holds d loglik_b / d(sigma_1..M, omega0_1..M,
 * Q_1..M, jitter) in that order. */
int gp_ssm_plan_loglik_grad(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, double* loglik, double* grad, int32_t* status,
                            void* stream);

/* Log-likelihood with per-instrument amplitudes and offsets (after
 * gp_ssm_plan_set_instruments): amp[b*n_inst + i] (> 0, finite) and
 * off[b*n_inst + i] (finite) of series b, host or device; either may be
 * NULL (1, resp. 0).  A series with an amplitude or offset out of range gets
 * status GP_SSM_EPARAM.  GP_SSM_EINVAL when the plan has no instruments.
 * Other arguments as for gp_ssm_plan_loglik. */
int gp_ssm_plan_loglik_inst(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, const double* amp, const double* off,
                            double* loglik, int32_t* status, void* stream);

/* Its gradient as well: grad[b*G + k], G = 3M + 1 + 2 n_inst, holds d
 * loglik_b / d(sigma_1..M, omega0_1..M, Q_1..M, jitter, amp_0..n_inst-1,
 * off_0..n_inst-1).  The amplitude derivative comes from the adjoint of the
 * observation vector (h = a h0), the offset derivative is minus the
 * adjoint of the innovation. */
int gp_ssm_plan_loglik_grad_inst(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                                 const double* quality, const double* jitter, const double* amp, const double* off,
                                 double* loglik, double* grad, int32_t* status, void* stream);

/* Posterior (the RTS smoother's result, Sec. 3.2.2, and prediction at
 * arbitrary times, Sec. 2.5 Algorithm 1).  test_offsets[B+1] (host or device int64) delimits
 * each series' test times in t_test (device, any order within a series).
 * mean_test/var_test[test_offsets[B]] receive the posterior mean and
 * variance of the latent instantaneous f(t*).  mean_data/var_data[N] (may be
 * NULL) receive the posterior of the exposure-averaged f at each measurement.
 * loglik[B] may be NULL. */
int gp_ssm_plan_smooth(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                       const double* quality, const double* jitter, const int64_t* test_offsets, const double* t_test,
                       double* mean_test, double* var_test, double* mean_data, double* var_data, double* loglik,
                       int32_t* status, void* stream);

/* The same posterior with, in addition, each SHO term's own latent process
 * at the test times (Appendix C, component-wise predictive means and
 * variances: the observation vector restricted to term m, applied to the
 * smoothed state).  term_mean/term_var[test_offsets[B] * n_terms] (device,
 * both required when there are test times) hold row i = test time i of
 * t_test, column m = term m; the row sums of term_mean equal mean_test.
 * Other arguments as for gp_ssm_plan_smooth. */
int gp_ssm_plan_smooth_terms(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                             const double* quality, const double* jitter, const int64_t* test_offsets,
                             const double* t_test, double* mean_test, double* var_test, double* term_mean,
                             double* term_var, double* mean_data, double* var_data, double* loglik, int32_t* status,
                             void* stream);

/* The posterior with per-instrument amplitudes and offsets (amp, off as for
 * gp_ssm_plan_loglik_inst).  mean_test/var_test (and the per-term outputs,
 * when term_mean and term_var are given) are the latent process;
 * mean_data/var_data are the noise-free measured quantity a_i (1/delta_n)
 * int f dt + c_i.  Other arguments as for gp_ssm_plan_smooth_terms. */
int gp_ssm_plan_smooth_inst(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, const double* amp, const double* off,
                            const int64_t* test_offsets, const double* t_test, double* mean_test, double* var_test,
                            double* term_mean, double* term_var, double* mean_data, double* var_data, double* loglik,
                            int32_t* status, void* stream);

/* Log-likelihood by the square-root (Cholesky-factor) form of the filter, the
 * remedy Sec. 3.2.3 and Sec. 5 name for the covariance form's loss of
 * accuracy on nearly noise-free data: the covariance of the augmented state is
 * carried as a triangular factor (time update: Householder reflections of
 * the transition applied to the factor beside the process noise's factor;
 * measurement update: the array form, by plane rotations), so that it stays
 * positive semidefinite.  The same model, term kinds and instrument labels as
 * gp_ssm_plan_loglik_inst (amp and off may be NULL; with a plan without
 * instrument labels both must be NULL).  Whole series, 16 GPU lanes each
 * (one row of the factor per lane), no time splitting: a robust alternative,
 * not the batched path's speed.
 * loglik[B] and status[B] (optional) in device memory, NaN and a nonzero
 * status for a failed series as for gp_ssm_plan_loglik.  Asynchronous on
 * `stream`. */
int gp_ssm_plan_loglik_sqrt(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, const double* amp, const double* off,
                            double* loglik, int32_t* status, void* stream);

/* The square-root filter's log-likelihood with the series split in time at
 * the plan's chunks (Sec. 3.2.4's time-parallel idea in factor form): for
 * every chunk at once, the filter conditioned on the chunk's first SHO state
 * x0, in factor form (16 GPU lanes per chunk, one row of the factor each),
 * summarised as the end state's x0-affine mean A x0 + b and covariance
 * factor U, and the chunk's density of its measurements as a function of x0,
 * exp(-c0 - |R x0 - rho|^2 / 2 - eps^2 / 2) with [[R, rho], [0, eps]] a
 * triangular factor of the measurements' whitened rows
 * (rank-one updates by rotations); then, per series, the summaries combined
 * pairwise in a tree (one GPU lane per pair, one launch per level), each
 * combination taking the second summary as a measurement of the first's end
 * state in array form, so that no covariance is formed from a difference.
 * The same model and arguments as gp_ssm_plan_loglik_sqrt; device memory
 * for two levels of summaries, about 2 x 92 doubles per chunk at three terms,
 * is allocated on the first call. */
int gp_ssm_plan_loglik_sqrt_split(gp_ssm_plan* plan, int32_t n_terms, const double* sigma, const double* omega0,
                                  const double* quality, const double* jitter, const double* amp, const double* off,
                                  double* loglik, int32_t* status, void* stream);

/* Reference "plain" GPU filter: the same per-event device code, one series at
 * a time, one lane, no time splitting, one launch per series.  Computes the
 * log-likelihood of series [first, first+count) of the plan.  Used as the
 * baseline that the batched launch is compared with. */
int gp_ssm_plan_plain_loglik(gp_ssm_plan* plan, int64_t first, int64_t count, int32_t n_terms, const double* sigma,
                             const double* omega0, const double* quality, const double* jitter, double* loglik,
                             void* stream);

/* One-shot forms: build a plan with default options, run it once, wait for
 * `stream`, destroy the plan.  Same arguments and outputs as the plan forms;
 * they return GP_SSM_EPARAM or GP_SSM_ENUMERIC when any series failed
 * (status[b] says which; status may be NULL).
 *
 * gp_ssm_loglik: the marginal log-likelihood of each series (the Gaussian
 * likelihood of Sec. 2.4, evaluated by the Kalman filter over the augmented
 * model of Sec. 3.2 with the per-event update of Sec. 3.2.2). */
int gp_ssm_loglik(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end, const double* y,
                  const double* yerr, int32_t n_terms, const double* sigma, const double* omega0, const double* quality,
                  const double* jitter, double* loglik, int32_t* status, void* stream);
/* gp_ssm_loglik_grad: the same log-likelihood and its gradient with respect
 * to every term's (sigma, omega0, Q) (Appendix B parameterisation) and the
 * jitter, grad[b*(3M+1) + k] ordered as for gp_ssm_plan_loglik_grad. */
int gp_ssm_loglik_grad(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                       const double* y, const double* yerr, int32_t n_terms, const double* sigma, const double* omega0,
                       const double* quality, const double* jitter, double* loglik, double* grad, int32_t* status,
                       void* stream);
/* gp_ssm_smooth: the posterior of Sec. 3.2.2 (the smoother over the
 * augmented model) at the data and, by the interpolation of Sec. 2.5
 * Algorithm 1, at the test times; arguments as for gp_ssm_plan_smooth. */
int gp_ssm_smooth(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                  const double* y, const double* yerr, int32_t n_terms, const double* sigma, const double* omega0,
                  const double* quality, const double* jitter, const int64_t* test_offsets, const double* t_test,
                  double* mean_test, double* var_test, double* mean_data, double* var_data, int32_t* status,
                  void* stream);

/* Autotuner of the batched launch.  The plan's chunk length sets how many
 * lanes each series gets (one lane per chunk, 64 lanes to a work wave) and
 * how long each lane's sequential run is; it follows from the target chunk
 * count over the batch.  gp_ssm_autotune builds a plan for each candidate
 * target chunk count (gp_ssm_autotune_candidates lists them), times three
 * replays of the log-likelihood (what = 0) or log-likelihood + gradient
 * (what = 1) call with HIP events on `stream`, and returns in *best the
 * default options with the fastest target, and in *best_ms (may be NULL) its
 * time per call.  Inputs as for gp_ssm_plan_create and the plan calls.
 * With cache_path (may be NULL) the choice is looked up first by the
 * workload's shape (series, measurements and events to two significant
 * digits, overlap depth, terms, kind of call, GPU architecture) and
 * appended to the file after tuning.  The environment variable
 * GP_SSM_TARGET_CHUNKS, when set to a positive count, overrides it all.
 * Every candidate is an ordinary plan: they compute the same results up to
 * rounding order.  Synchronises `stream`; allocates and frees its own
 * workspace. */
int gp_ssm_autotune(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                    const double* y, const double* yerr, int32_t n_terms, const double* sigma, const double* omega0,
                    const double* quality, const double* jitter, int32_t what, const char* cache_path,
                    gp_ssm_plan_options* best, double* best_ms, void* stream);
/* Copies up to cap candidate target chunk counts; returns their number. */
int gp_ssm_autotune_candidates(int64_t* target_chunks, int32_t cap);

/* Kernel timing.  While enabled, every kernel the library launches is
 * bracketed by HIP events on its stream and its duration is accumulated per
 * kernel name.  gp_ssm_profile_read copies up to `cap` entries (name, count,
 * total milliseconds) and returns the number of distinct kernels; names are
 * library-owned static strings.  Reading synchronises the device. */
int gp_ssm_profile_enable(int32_t on);
int gp_ssm_profile_reset(void);
int gp_ssm_profile_read(const char** names, int64_t* counts, double* total_ms, int32_t cap);

/* Message of the last error on the calling thread ("" if none). */
const char* gp_ssm_last_error(void);

/* Library version string. */
const char* gp_ssm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GP_SSM_H */
