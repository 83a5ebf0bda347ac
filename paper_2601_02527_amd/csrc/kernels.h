// Kernel-side data structures and the launch interface shared by the
// per-term-count translation units and the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "gp_ssm_filter.h"

namespace gpssm {

struct DevPlan {
  const double *dt, *t, *y, *r, *invd;
  const uint32_t* info;
  const int64_t* meas;
  const int32_t *seg_chunk0, *seg_nch;                    // scan segments
  const int32_t *wv_series, *wv_nch, *wv_len, *wv_chunk;  // work waves (see plan.h)
  const int64_t* wv_ev0;
  const int32_t *chunk_len, *chunk_series, *chunk_wv, *chunk_lane;
  const uint8_t* chunk_first;
  const int32_t *series_chunk0, *series_nch, *series_seg0, *series_nseg, *series_wv0, *series_nwv;
  const int32_t* wv_order;  // launch order of the work waves (null: natural order)
  int64_t n_series;
  int32_t n_chunks, n_seg, n_wv;
  int32_t max_series_nseg;  // the most segments (second level: groups) of one series
};

// hyperparameters prepared on the device: per (series, term) TermConst and the
// Taylor coefficients followed by their beta-derivatives (2*NCOEF doubles);
// bad[b] = 1 when series b's hyperparameters failed validation (its constants
// are then those of sigma = omega0 = Q = 1, jitter 0, and its outputs NaN).
// With instruments (ni > 0): itab[b] is series b's row of the instrument
// table (ITAB_W doubles, see ITAB_INVA), icnt[b] its number of measurements
// of each instrument (MAX_INST), and the gradient partials carry 2 ni more
// rows (amplitudes, then offsets).
struct DevParams {
  const TermConst* tc;
  const double* coef;
  const double* jit;
  const int32_t* bad;
  const double* itab = nullptr;
  const int32_t* icnt = nullptr;
  int32_t ni = 0;
};

// -sum over series b's measurements of log(amplitude): the density factor of
// the rescaled measurements the filter sees (0 without instruments)
__device__ __forceinline__ double inst_loglik(const DevParams& pr, int64_t b) {
  double s = 0.0;
  for (int i = 0; i < pr.ni; ++i) s -= (double)pr.icnt[b * MAX_INST + i] * pr.itab[b * ITAB_W + ITAB_LOGA + i];
  return s;
}

// the caller's pointers of one call, read by the kernels from device memory
// (written there on the call's stream before the kernels), so that a captured
// sequence of launches serves every later call with other buffers
struct CallArgs {
  const double *sigma, *omega0, *quality, *jitter;
  double *loglik, *grad;
  int32_t* status;
  // per-series instrument amplitudes and offsets [series][instrument] (null:
  // 1 and 0), and whether grad rows carry their derivatives
  const double *amp = nullptr, *off = nullptr;
  int32_t grad_inst = 0;
};

// test-time work of the smoother, assigned to chunks on the host
struct DevTests {
  const double* t;            // test times, grouped by chunk, sorted within a chunk
  const int64_t* out_index;   // where each result goes
  const int64_t* chunk_t0;    // first test of each chunk (n_chunks + 1 entries)
  const double* chunk_tprev;  // time of the previous chunk's last event
  double* term_mean;          // per-term latent posterior [test][term], or null
  double* term_var;
};

struct Launch {
  hipStream_t stream;
};

// Per-event record buffer of the backward kernels (k_adjoint, k_smooth).
// Within the plan's record budget every work wave keeps its records at its
// own place in the event layout (slot = 0, one launch over all waves).
// Beyond it the buffer holds `grid` slots of `slot` doubles (the longest work
// wave's events x 64 lanes x fields), and the kernels run in rounds of at
// most `grid` work waves taken in launch order, workgroup i of the round
// starting at entry `first` using slot i; memory is then bounded by the
// budget (at least the workgroups the GPU holds at once), not by the batch.
struct RecSlots {
  double* base;
  int64_t slot;
  int32_t grid;
  int32_t first;
  // the records of the work wave whose events start at ev0 (F fields each)
  __device__ __forceinline__ double* records(int64_t ev0, int F) const {
    return slot ? base + (int64_t)blockIdx.x * slot : base + ev0 * F;
  }
};

// per-(M, J) kernel launchers
struct KernelSet {
  void (*summaries)(const Launch&, const DevPlan&, const DevParams&, double* summ);
  void (*adjoint)(const Launch&, const DevPlan&, const DevParams&, const double* bstate, const double* badj,
                  const RecSlots& rec, double* gpart);
  void (*plain)(const Launch&, const DevPlan&, const DevParams&, int64_t series, double* loglik);
  void (*sqrt)(const Launch&, const DevPlan&, const DevParams&, const int32_t* order, const CallArgs* args);
  void (*sqrt_split)(const Launch&, const DevPlan&, const DevParams&, double* summ, double* tmp, int32_t levels,
                     const CallArgs* args);
  void (*smooth)(const Launch&, const DevPlan&, const DevParams&, const double* bstate, const double* bsmooth,
                 const RecSlots& rec, const DevTests& tests, double* mean_test, double* var_test, double* mean_data,
                 double* var_data);
  // workgroups of k_adjoint / k_smooth resident at once on one compute unit
  int (*adjoint_occupancy)();
  int (*smooth_occupancy)();
};

// per number of terms: the plain model, (i) the kernels that also take
// instrument tables, and (x) those that take real exponential terms as well
KernelSet kernels_m1(int J);
KernelSet kernels_m2(int J);
KernelSet kernels_m3(int J);
KernelSet kernels_m4(int J);
KernelSet kernels_m1i(int J);
KernelSet kernels_m2i(int J);
KernelSet kernels_m3i(int J);
KernelSet kernels_m4i(int J);
KernelSet kernels_m1x(int J);
KernelSet kernels_m2x(int J);
KernelSet kernels_m3x(int J);
KernelSet kernels_m4x(int J);

// kernel timing hooks (capi)
void prof_begin(const char* name, hipStream_t s);
void prof_end(const char* name, hipStream_t s);

// per-event record of the forward pass kept for the backward passes:
// the filtered state before the event (m, packed P)
template <class Dm>
constexpr int rec_fields() {
  return Dm::D + Dm::NP;
}

}  // namespace gpssm
