// C-ABI of the library (declared in include/gp_ssm.h): plans, workspace,
// hyperparameter validation and preparation on the device, the launch order
// of the work waves, the capture of a whole step in a graph, and the dispatch
// of the per-(terms, slots) kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gp_ssm.h"
#include "kernels.h"
#include "sqrt_filter.h"
#include "plan.h"
#include "scan.h"

using namespace gpssm;

static_assert(GP_SSM_MAX_INSTRUMENTS == MAX_INST, "instrument table width");

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(GP_SSM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
struct Prof {
  std::mutex mu;
  bool on = false;
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<int64_t, double>> total;
  std::vector<std::string> names;  // stable storage for returned names
  hipEvent_t cur_a = nullptr;
} g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_flush() {
  for (auto& p : g_prof.pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    auto& t = g_prof.total[p.name];
    t.first += 1;
    t.second += ms;
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
}

// ---------------------------------------------------------------------------
// small kernels that do not depend on the slot count
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool param_ok(double v) { return v > 0.0 && isfinite(v); }

// hyperparameters of series b valid: sigma, omega0 (the rate of a real
// term) and Q (SHO terms only) > 0 and finite for every term, jitter >= 0
// and finite (or absent)
// and finite (or absent); with ni instruments, their amplitudes > 0 and
// finite and offsets finite (when given)
__device__ __forceinline__ bool series_params_ok(const CallArgs& a, const int32_t* kinds, int64_t b, int M, int ni) {
  bool ok = true;
  for (int t = 0; t < M; ++t) {
    const int64_t i = b * M + t;
    const bool real = kinds && kinds[t] == GP_SSM_TERM_REAL;
    ok = ok && param_ok(a.sigma[i]) && param_ok(a.omega0[i]) && (real || param_ok(a.quality[i]));
  }
  if (a.jitter) ok = ok && a.jitter[b] >= 0.0 && isfinite(a.jitter[b]);
  for (int i = 0; i < ni; ++i) {
    if (a.amp) ok = ok && param_ok(a.amp[b * ni + i]);
    if (a.off) ok = ok && isfinite(a.off[b * ni + i]);
  }
  return ok;
}

// Validates the hyperparameters and prepares them: per (series, term) the
// step constants and the Taylor tables of one series interval per thread,
// per series the jitter, the instrument table (ni > 0) and the validation
// flag.  A series that fails validation is prepared with sigma = omega0 = Q
// = 1, jitter 0, amplitudes 1 and offsets 0, so that every kernel runs on
// finite, in-range values; its outputs are set to NaN and its status to
// GP_SSM_EPARAM where they are written.
__global__ void k_prep(int64_t B, int M, int ni, const CallArgs* __restrict__ args, const int32_t* __restrict__ kinds,
                       TermConst* __restrict__ tc, double* __restrict__ coef, double* __restrict__ jit,
                       int32_t* __restrict__ bad, double* __restrict__ itab) {
  const CallArgs a = *args;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < B * M * NI) {
    const int64_t i = j / NI;
    const int iv = (int)(j - i * NI);
    const bool ok = series_params_ok(a, kinds, i / M, M, ni);
    const bool real = kinds && kinds[i % M] == GP_SSM_TERM_REAL;
    const TermConst t = !ok ? make_term(1.0, 1.0, 1.0)
                            : (real ? make_real_term(a.sigma[i], a.omega0[i])
                                    : make_term(a.sigma[i], a.omega0[i], a.quality[i]));
    if (iv == 0) tc[i] = t;
    double* c = coef + i * 2 * NCOEF + iv * ISTRIDE;
    series_interval_table(t.beta, interval_centre(iv, t.b1ser, t.wser), c, c + NCOEF);
  }
  if (j < B) {
    const bool ok = series_params_ok(a, kinds, j, M, ni);
    jit[j] = (ok && a.jitter) ? a.jitter[j] : 0.0;
    bad[j] = ok ? 0 : 1;
    if (ni > 0) {
      double* row = itab + j * ITAB_W;
      for (int i = 0; i < MAX_INST; ++i) {
        const bool have = ok && i < ni;
        const double amp = (have && a.amp) ? a.amp[j * ni + i] : 1.0;
        row[ITAB_INVA + i] = 1.0 / amp;
        row[ITAB_OFF + i] = (have && a.off) ? a.off[j * ni + i] : 0.0;
        row[ITAB_AMP + i] = amp;
        row[ITAB_LOGA + i] = log(amp);
      }
    }
  }
}

// writes each measurement's instrument label into bits 16-18 of its event's
// encoding (ends and instantaneous measurements; other events keep 0)
__global__ void k_set_inst(int64_t n_ev, uint32_t* __restrict__ info, const int64_t* __restrict__ meas,
                           const int32_t* __restrict__ label) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_ev) return;
  uint32_t v = info[e] & ~(7u << EV_INST_SHIFT);
  const int64_t n = meas[e];
  const uint32_t k = v & 3u;
  if (label && n >= 0 && (k == EV_END || k == EV_INSTANT)) v |= (uint32_t)label[n] << EV_INST_SHIFT;
  info[e] = v;
}

// Launch order of the work waves, computed on the device each call (it
// depends on the hyperparameters).  A wave's cost varies with its series'
// terms: a wavefront pays for the Taylor branch of a term at a step when any
// of its lanes needs it, and for the closed-form branch when any lane needs
// that.  With p the fraction of the series' steps below the switch point, the
// expected cost per step and term is C_SER (1 - (1-p)^64) + C_CLO (1 - p^64)
// on top of W0 for the filter step; p comes from the series' step-length
// distribution (the plan's cumulative histogram over powers of two).
// Dispatching the costliest waves first (longest processing time first)
// evens out the SIMDs' loads.  One workgroup sorts the waves by a key of
// 64 levels per octave of cost (counting sort; the order within a level is
// arbitrary, and results do not depend on the order).
constexpr int ORDER_THREADS = 1024;
constexpr int ORDER_NB = 4096;

__device__ __forceinline__ int order_key(const DevPlan& p, int M, const TermConst* __restrict__ tc,
                                         const float* __restrict__ cdf_all, int32_t w) {
  constexpr double W0 = 4.0, C_SER = 1.0, C_CLO = 1.5;
  const int64_t b = p.wv_series[w];
  const float* cdf = cdf_all + b * DT_NE;
  double c = W0;
  for (int t = 0; t < M; ++t) {
    const TermConst& q = tc[b * M + t];
    const double thr = XSER / fmax(1.0, q.beta) / q.w0;  // steps with dt <= thr take the series
    int ex;
    const double fr = frexp(thr, &ex);  // thr = fr 2^ex, fr in [0.5, 1)
    const int k = ex - DT_KMIN;
    double pr;
    if (k <= 0)
      pr = cdf[0];
    else if (k >= DT_NE)
      pr = 1.0;
    else  // linear in log2(dt) between the edges 2^(ex-1) and 2^ex
      pr = cdf[k - 1] + (cdf[k] - cdf[k - 1]) * (log2(fr) + 1.0);
    c += C_SER * (1.0 - pow(1.0 - pr, (double)WAVE)) + C_CLO * (1.0 - pow(pr, (double)WAVE));
  }
  const double cost = (double)p.wv_len[w] * c;
  const int lvl = (int)(log2(fmax(cost, 1.0)) * 64.0);
  return ORDER_NB - 1 - min(max(lvl, 0), ORDER_NB - 1);  // costliest first
}

__global__ __launch_bounds__(ORDER_THREADS) void k_order(DevPlan p, int M, const TermConst* __restrict__ tc,
                                                         const float* __restrict__ cdf, int32_t* __restrict__ order) {
  __shared__ int32_t hist[ORDER_NB];
  __shared__ int32_t part[ORDER_THREADS];
  constexpr int PER = ORDER_NB / ORDER_THREADS;
  const int tid = threadIdx.x;
  for (int i = tid; i < ORDER_NB; i += ORDER_THREADS) hist[i] = 0;
  __syncthreads();
  for (int32_t w = tid; w < p.n_wv; w += ORDER_THREADS) atomicAdd(&hist[order_key(p, M, tc, cdf, w)], 1);
  __syncthreads();
  // exclusive prefix sum of the histogram: PER bins per thread, then a scan
  // of the per-thread sums
  int32_t loc = 0;
  for (int i = 0; i < PER; ++i) loc += hist[tid * PER + i];
  part[tid] = loc;
  __syncthreads();
  for (int d = 1; d < ORDER_THREADS; d <<= 1) {
    const int32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = part[tid] - loc;
  for (int i = 0; i < PER; ++i) {
    const int32_t h = hist[tid * PER + i];
    hist[tid * PER + i] = run;
    run += h;
  }
  __syncthreads();
  for (int32_t w = tid; w < p.n_wv; w += ORDER_THREADS) {
    const int32_t at = atomicAdd(&hist[order_key(p, M, tc, cdf, w)], 1);
    order[at] = w;
  }
}

// gradient partials of a series' work waves summed: one wavefront per series,
// lane l takes waves l, l + 64, ..., then a fixed-order wave reduction; NaN for
// a series whose status is not 0
// (with instruments the partials carry 2 ni more rows, written to grad only
// when the call asks for their derivatives; an amplitude's derivative gains
// -N_i/a_i from the -log(a_i) of each of the N_i measurements)
__global__ __launch_bounds__(WAVE) void k_reduce_grad(DevPlan p, DevParams pr, int M, const double* __restrict__ gpart,
                                                      const CallArgs* __restrict__ args) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t S = p.n_wv;
  const int32_t s0 = p.series_wv0[b], n = p.series_nwv[b];
  const int ni = pr.ni;
  const int G = 3 * M + 1 + (args->grad_inst ? 2 * ni : 0);
  double* const grad = args->grad;
  const bool good = args->status[b] == 0;
  for (int f = 0; f < G; ++f) {
    double s = 0.0;
    for (int32_t q = lane; q < n; q += WAVE) s += gpart[(int64_t)f * S + s0 + q];
    s = wave_sum(s);
    const int i = f - (3 * M + 1);
    if (i >= 0 && i < ni) s -= (double)pr.icnt[b * MAX_INST + i] * pr.itab[b * ITAB_W + ITAB_INVA + i];
    if (lane == 0) grad[b * G + f] = (good && isfinite(s)) ? s : __builtin_nan("");
  }
}

// test times of series without measurements: the prior (mean 0, variance
// sum_m sigma_m^2, each term's own variance sigma_m^2)
__global__ void k_prior_tests(int64_t n, const int64_t* __restrict__ idx, const int32_t* __restrict__ series, int M,
                              const TermConst* __restrict__ tc, const int32_t* __restrict__ bad,
                              double* __restrict__ mean_test, double* __restrict__ var_test,
                              double* __restrict__ term_mean, double* __restrict__ term_var) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = idx[i], b = series[i];
  const double poison = bad[b] ? __builtin_nan("") : 0.0;
  double v = 0.0;
  for (int t = 0; t < M; ++t) {
    const double s2 = tc[b * M + t].sigma * tc[b * M + t].sigma;
    v += s2;
    if (term_mean) {
      term_mean[o * M + t] = poison;
      term_var[o * M + t] = s2 + poison;
    }
  }
  mean_test[o] = poison;
  var_test[o] = v + poison;
}

// features: bit 0 the plan has real terms, bit 1 instrument labels
KernelSet kernel_set(int M, int J, int features) {
  J = std::max(1, J);
  if (features & 1) {
    switch (M) {
      case 1: return kernels_m1x(J);
      case 2: return kernels_m2x(J);
      case 3: return kernels_m3x(J);
      default: return kernels_m4x(J);
    }
  }
  if (features & 2) {
    switch (M) {
      case 1: return kernels_m1i(J);
      case 2: return kernels_m2i(J);
      case 3: return kernels_m3i(J);
      default: return kernels_m4i(J);
    }
  }
  switch (M) {
    case 1: return kernels_m1(J);
    case 2: return kernels_m2(J);
    case 3: return kernels_m3(J);
    default: return kernels_m4(J);
  }
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
// Every (re)allocation bumps *gen, the generation of the plan's workspace: a
// captured graph holds buffer addresses and is captured again when the
// generation it was captured at is no longer current.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  uint64_t* gen = nullptr;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  int ensure(size_t n) {
    if (n <= bytes) return 0;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (gen) ++*gen;
    if (hipMalloc(&p, n) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GP_SSM_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
    return 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

template <class T>
int upload(DBuf& d, const std::vector<T>& v) {
  if (int rc = d.ensure(std::max<size_t>(1, v.size()) * sizeof(T))) return rc;
  if (!v.empty()) HIP_TRY(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return 0;
}

// true for memory a kernel can read and write (device or managed)
bool device_memory(const void* ptr) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

int host_copy(const void* src, size_t bytes, void* dst, hipStream_t s) {
  if (bytes == 0) return 0;
  if (device_memory(src)) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    std::memcpy(dst, src, bytes);
  }
  return 0;
}

bool graphs_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("GP_SSM_GRAPH");
    return !(e && e[0] == '0');
  }();
  return on;
}

}  // namespace

namespace gpssm {
void prof_begin(const char* name, hipStream_t s) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.cur_a = prof_event();
  if (g_prof.cur_a) (void)hipEventRecord(g_prof.cur_a, s);
  (void)name;
}
void prof_end(const char* name, hipStream_t s) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  hipEvent_t b = prof_event();
  if (!b || !g_prof.cur_a) return;
  (void)hipEventRecord(b, s);
  g_prof.pending.push_back({name, g_prof.cur_a, b});
  g_prof.cur_a = nullptr;
  if (g_prof.pending.size() > 4096) prof_flush();
}
}  // namespace gpssm

namespace {
enum StepKind { STEP_LOGLIK = 0, STEP_GRAD = 1 };
constexpr int64_t DEFAULT_RECORD_BUDGET = int64_t(32) << 30;
constexpr int ARG_RING = 16;
}  // namespace

// ---------------------------------------------------------------------------
// the entry point that allocates nothing (gp_ssm_plan_loglik_noalloc) takes
// its workspace from this array: one copy per GPU the library runs on, held
// until the process ends, shared by every such call on that GPU
// ---------------------------------------------------------------------------
namespace {
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
}  // namespace
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_at;  // device -> address of its copy of `scratch`

// the device address of the current device's copy of `scratch` (looked up
// once per device, with that device current); host code uses this address,
// never the array's name
int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_at.find(device);
  if (it != g_scratch_at.end()) {
    *out = it->second;
    return 0;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(GP_SSM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_at[device] = ptr;
  *out = ptr;
  return 0;
}

// writes the call's pointers (a kernel argument) to the argument block
__global__ void k_set_args(CallArgs a, CallArgs* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = a;
}
}  // namespace

struct gp_ssm_plan {
  int device = 0;
  int n_cu = 1;
  int64_t record_budget = 0;  // bytes of per-event records before the backward kernels run in rounds
  int32_t kinds_M = 0;        // number of terms gp_ssm_plan_set_term_kinds described (0: all SHO)
  int32_t n_inst = 0;         // instruments gp_ssm_plan_set_instruments described (0: none)
  bool kinds_real = false;    // some term of the kinds is a real term
  std::vector<int64_t> offsets;  // the series' measurement ranges
  uint64_t gen = 0;  // workspace generation (see DBuf)
  HostPlan host;
  DBuf dt, t, y, r, invd, info, meas;
  DBuf seg_chunk0, seg_nch, grp_seg0, grp_nseg, series_grp0, series_ngrp;
  DBuf wv_series, wv_nch, wv_len, wv_chunk, wv_ev0;
  DBuf chunk_len, chunk_series, chunk_wv, chunk_lane, chunk_first;
  DBuf series_chunk0, series_nch, series_seg0, series_nseg, series_wv0, series_nwv, series_dt_cdf;
  // workspace
  DBuf tc, coef, jit, pbad, summ, bstate, badj, bsmooth, gpart, rec, status, llbuf, stage;
  DBuf pre, suf, segtot, segstate, segfut, segll, segok;
  DBuf pre2, suf2, grptot, grpstate, grpfut;
  DBuf tests_t, tests_idx, tests_c0, tests_before, prior_idx, prior_series;
  DBuf wv_order, args, kinds, itab, icnt;
  DBuf sqrt_order;  // series by decreasing event count (the square-root filter's groups)
  DBuf sqsumm, sqsumm2;  // chunk summaries of the time-split square-root filter (two tree levels)
  // the call's pointers go to `args` on the call's stream from a ring of
  // pinned host slots; an event per slot marks when its copy has been done
  CallArgs* args_host = nullptr;
  hipEvent_t args_ev[ARG_RING] = {};
  int args_next = 0;
  // one captured step per (kind, number of terms)
  struct Graph {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = 0;
  };
  std::map<int, Graph> graphs;
  hipStream_t cap = nullptr;

  std::vector<DBuf*> workspace() {
    return {&tc,       &coef,   &jit,     &pbad,      &summ,      &bstate,    &badj,         &bsmooth,
            &gpart,    &rec,    &status,  &llbuf,     &stage,     &pre,       &suf,          &segtot,
            &segstate, &segfut, &segll,   &segok,     &pre2,      &suf2,      &grptot,       &grpstate,
            &grpfut,   &wv_order, &args,  &kinds,     &itab,      &tests_t,   &tests_idx, &tests_c0,  &tests_before,
            &prior_idx, &prior_series};
  }
  std::vector<const DBuf*> all_buffers() const {
    auto* self = const_cast<gp_ssm_plan*>(this);
    std::vector<const DBuf*> v = {&dt, &t, &y, &r, &invd, &info, &meas, &seg_chunk0, &seg_nch, &grp_seg0, &grp_nseg,
                                  &series_grp0, &series_ngrp, &wv_series, &wv_nch, &wv_len, &wv_chunk, &wv_ev0,
                                  &chunk_len, &chunk_series, &chunk_wv, &chunk_lane, &chunk_first, &series_chunk0,
                                  &series_nch, &series_seg0, &series_nseg, &series_wv0, &series_nwv, &series_dt_cdf,
                                  &icnt, &sqrt_order, &sqsumm, &sqsumm2};
    for (DBuf* d : self->workspace()) v.push_back(d);
    return v;
  }

  gp_ssm_plan() {
    for (DBuf* d : workspace()) d->gen = &gen;
  }
  ~gp_ssm_plan() {
    (void)hipDeviceSynchronize();
    for (auto& kv : graphs)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (cap) (void)hipStreamDestroy(cap);
    for (hipEvent_t& e : args_ev)
      if (e) (void)hipEventDestroy(e);
    if (args_host) (void)hipHostFree(args_host);
  }

  DevPlan dev() const {
    DevPlan p;
    p.dt = dt.as<double>();
    p.t = t.as<double>();
    p.y = y.as<double>();
    p.r = r.as<double>();
    p.invd = invd.as<double>();
    p.info = info.as<uint32_t>();
    p.meas = meas.as<int64_t>();
    p.seg_chunk0 = seg_chunk0.as<int32_t>();
    p.seg_nch = seg_nch.as<int32_t>();
    p.wv_series = wv_series.as<int32_t>();
    p.wv_nch = wv_nch.as<int32_t>();
    p.wv_len = wv_len.as<int32_t>();
    p.wv_chunk = wv_chunk.as<int32_t>();
    p.wv_ev0 = wv_ev0.as<int64_t>();
    p.chunk_len = chunk_len.as<int32_t>();
    p.chunk_series = chunk_series.as<int32_t>();
    p.chunk_wv = chunk_wv.as<int32_t>();
    p.chunk_lane = chunk_lane.as<int32_t>();
    p.chunk_first = chunk_first.as<uint8_t>();
    p.series_chunk0 = series_chunk0.as<int32_t>();
    p.series_nch = series_nch.as<int32_t>();
    p.series_seg0 = series_seg0.as<int32_t>();
    p.series_nseg = series_nseg.as<int32_t>();
    p.series_wv0 = series_wv0.as<int32_t>();
    p.series_nwv = series_nwv.as<int32_t>();
    p.wv_order = wv_order.as<int32_t>();
    p.n_series = host.n_series;
    p.n_chunks = host.n_chunks;
    p.n_seg = host.n_seg;
    p.n_wv = host.n_wv;
    p.max_series_nseg = host.max_series_nseg;
    return p;
  }

  // the plan seen by the second scan level: groups of segments in the place
  // of segments, segments in the place of chunks
  DevPlan dev_groups() const {
    DevPlan p = dev();
    p.seg_chunk0 = grp_seg0.as<int32_t>();
    p.seg_nch = grp_nseg.as<int32_t>();
    p.series_seg0 = series_grp0.as<int32_t>();
    p.series_nseg = series_ngrp.as<int32_t>();
    p.n_chunks = host.n_seg;
    p.n_seg = host.n_grp;
    p.max_series_nseg = host.max_series_ngrp;
    return p;
  }

  DevParams params() const {
    DevParams pr;
    pr.tc = tc.as<TermConst>();
    pr.coef = coef.as<double>();
    pr.jit = jit.as<double>();
    pr.bad = pbad.as<int32_t>();
    pr.itab = n_inst ? itab.as<double>() : nullptr;
    pr.icnt = n_inst ? icnt.as<int32_t>() : nullptr;
    pr.ni = n_inst;
    return pr;
  }

  const CallArgs* dargs() const { return args.as<CallArgs>(); }
  // the optional features the kernels of calls with M terms must take
  int features(int32_t M) const { return (has_real(M) ? 1 : 0) | (n_inst > 0 ? 2 : 0); }
  bool has_real(int32_t M) const { return kinds_M == M && kinds_real; }
};

namespace {

int check_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return fail(GP_SSM_EDEVICE, "no HIP device available");
  }
  return 0;
}

// ---------------------------------------------------------------------------
// per-call arguments
// ---------------------------------------------------------------------------
// Checks the call's pointers and sends them to the plan's argument block on
// the call's stream.  Hyperparameters in host memory are first copied into
// the plan's staging buffer; outputs must be device memory.
int put_args(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
             const double* jitter, double* loglik, double* grad, int32_t* status, hipStream_t s,
             const double* amp = nullptr, const double* off = nullptr, int32_t grad_inst = 0) {
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  if (M < 1 || M > GP_SSM_MAX_TERMS) return fail(GP_SSM_EINVAL, "n_terms out of range");
  if (!sigma || !omega0 || !quality) return fail(GP_SSM_EINVAL, "null hyperparameter pointer");
  if (pl->kinds_M != 0 && pl->kinds_M != M)
    return fail(GP_SSM_EINVAL, "term kinds were set for " + std::to_string(pl->kinds_M) + " terms, the call has " +
                                   std::to_string(M));
  const int64_t B = pl->host.n_series;
  if ((loglik && !device_memory(loglik)) || (grad && !device_memory(grad)) || (status && !device_memory(status)))
    return fail(GP_SSM_EINVAL, "output arrays must be device memory");
  if ((amp || off || grad_inst) && pl->n_inst == 0)
    return fail(GP_SSM_EINVAL, "instrument parameters given, but the plan has no instrument labels "
                               "(gp_ssm_plan_set_instruments)");
  const int64_t NI_ = pl->n_inst;
  CallArgs a{sigma, omega0, quality, jitter, loglik, grad, status, amp, off, grad_inst};
  const bool host_in = !device_memory(sigma) || !device_memory(omega0) || !device_memory(quality) ||
                       (jitter && !device_memory(jitter)) || (amp && !device_memory(amp)) ||
                       (off && !device_memory(off));
  if (host_in) {
    // host hyperparameters: staged through device memory (the copies are
    // ordered on the stream before the kernels that read them)
    if (int rc = pl->stage.ensure(sizeof(double) * (3 * B * M + B + 2 * B * NI_))) return rc;
    double* d = pl->stage.as<double>();
    const double* src[6] = {sigma, omega0, quality, jitter, amp, off};
    const int64_t cnt[6] = {B * M, B * M, B * M, B, B * NI_, B * NI_};
    double* dst[6] = {d, d + B * M, d + 2 * B * M, d + 3 * B * M, d + 3 * B * M + B, d + 3 * B * M + B + B * NI_};
    for (int k = 0; k < 6; ++k) {
      if (!src[k] || cnt[k] == 0) continue;
      HIP_TRY(hipMemcpyAsync(dst[k], src[k], sizeof(double) * cnt[k],
                             device_memory(src[k]) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    }
    a.sigma = dst[0];
    a.omega0 = dst[1];
    a.quality = dst[2];
    a.jitter = jitter ? dst[3] : nullptr;
    a.amp = amp ? dst[4] : nullptr;
    a.off = off ? dst[5] : nullptr;
  }
  if (!pl->args_host) {
    HIP_TRY(hipHostMalloc((void**)&pl->args_host, sizeof(CallArgs) * ARG_RING, hipHostMallocDefault));
    for (hipEvent_t& e : pl->args_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (int rc = pl->args.ensure(sizeof(CallArgs))) return rc;
  const int k = pl->args_next;
  pl->args_next = (k + 1) % ARG_RING;
  HIP_TRY(hipEventSynchronize(pl->args_ev[k]));  // the slot's previous copy is done
  pl->args_host[k] = a;
  HIP_TRY(hipMemcpyAsync(pl->args.p, &pl->args_host[k], sizeof(CallArgs), hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(pl->args_ev[k], s));
  return 0;
}

// ---------------------------------------------------------------------------
// workspace (allocated before any launch, so that a captured step never
// allocates) and the launches of one step
// ---------------------------------------------------------------------------
int record_slots(gp_ssm_plan* pl, int32_t M, bool smooth, RecSlots& rs) {
  const KernelSet ks = kernel_set(M, pl->host.max_slots, pl->features(M));
  const int NX = 2 * M;
  const int J = std::max(1, pl->host.max_slots);
  const int D = NX + J;
  const int F = D + D * (D + 1) / 2;
  const int64_t n_wv = std::max<int64_t>(1, pl->host.n_wv);
  const int64_t whole = sizeof(double) * F * std::max<int64_t>(1, pl->host.n_ev_pad);
  if (whole <= pl->record_budget) {
    // every work wave at its own place in the event layout, one launch
    rs.grid = (int32_t)n_wv;
    rs.slot = 0;
    if (int rc = pl->rec.ensure(whole)) return rc;
  } else {
    // rounds of work waves, one slot per workgroup of a round: at least the
    // workgroups the GPU holds at once, more if the budget allows
    const int occ = smooth ? ks.smooth_occupancy() : ks.adjoint_occupancy();
    rs.slot = (int64_t)std::max(1, pl->host.max_chunk_len) * WAVE * F;
    const int64_t fit = pl->record_budget / (int64_t)(sizeof(double) * rs.slot);
    rs.grid = (int32_t)std::min<int64_t>(n_wv, std::max<int64_t>((int64_t)occ * pl->n_cu, fit));
    if (int rc = pl->rec.ensure(sizeof(double) * rs.slot * rs.grid)) return rc;
  }
  rs.base = pl->rec.as<double>();
  rs.first = 0;
  return 0;
}

int reserve(gp_ssm_plan* pl, int32_t M, int back, bool smooth) {
  const HostPlan& h = pl->host;
  const int64_t B = h.n_series;
  const int NX = 2 * M;
  const int NXP = NX * (NX + 1) / 2;
  const int64_t C = std::max<int64_t>(1, h.n_chunks);
  const int64_t S = std::max<int64_t>(1, h.n_seg);
  const int EF = elem_fields(NX);
  int rc = 0;
  if ((rc = pl->tc.ensure(sizeof(TermConst) * B * M)) || (rc = pl->coef.ensure(sizeof(double) * B * M * 2 * NCOEF)) ||
      (rc = pl->jit.ensure(sizeof(double) * B)) || (rc = pl->pbad.ensure(sizeof(int32_t) * B)) ||
      (rc = pl->itab.ensure(sizeof(double) * ITAB_W * std::max<int64_t>(1, B))) ||
      (rc = pl->wv_order.ensure(sizeof(int32_t) * std::max<int64_t>(1, h.n_wv))) ||
      (rc = pl->args.ensure(sizeof(CallArgs))) ||
      (rc = pl->summ.ensure(sizeof(double) * summary_size(NX) * C)) ||
      (rc = pl->bstate.ensure(sizeof(double) * (NX + NXP) * C)) || (rc = pl->pre.ensure(sizeof(double) * EF * C)) ||
      (rc = pl->suf.ensure(sizeof(double) * EF * C)) || (rc = pl->segtot.ensure(sizeof(double) * EF * S)) ||
      (rc = pl->segstate.ensure(sizeof(double) * (NX + NXP) * S)) ||
      (rc = pl->segfut.ensure(sizeof(double) * (NX + NXP) * S)) || (rc = pl->segll.ensure(sizeof(double) * S)) ||
      (rc = pl->segok.ensure(sizeof(int32_t) * S)) || (rc = pl->status.ensure(sizeof(int32_t) * B)) ||
      (rc = pl->llbuf.ensure(sizeof(double) * B)))
    return rc;
  if (h.max_series_nseg > WAVE) {
    const int64_t G = std::max<int64_t>(1, h.n_grp);
    if ((rc = pl->pre2.ensure(sizeof(double) * EF * S)) || (rc = pl->suf2.ensure(sizeof(double) * EF * S)) ||
        (rc = pl->grptot.ensure(sizeof(double) * EF * G)) ||
        (rc = pl->grpstate.ensure(sizeof(double) * (NX + NXP) * G)) ||
        (rc = pl->grpfut.ensure(sizeof(double) * (NX + NXP) * G)))
      return rc;
  }
  if (back) {
    if ((rc = pl->badj.ensure(sizeof(double) * (NX + NXP) * C))) return rc;
    if (smooth && (rc = pl->bsmooth.ensure(sizeof(double) * (NX + NXP) * C))) return rc;
    if (!smooth &&
        (rc = pl->gpart.ensure(sizeof(double) * (3 * M + 1 + 2 * pl->n_inst) * std::max<int64_t>(1, h.n_wv))))
      return rc;
    RecSlots rs;
    if ((rc = record_slots(pl, M, smooth, rs))) return rc;
  }
  return 0;
}

// device memory of the log-likelihood part of a call: the prepared
// hyperparameters, the launch order, the argument block and the scan's
// workspace (the plan's own buffers, or carved from the static scratch array
// by the entry point that allocates nothing)
struct FwdWork {
  TermConst* tc;
  double* coef;
  double* jit;
  int32_t* bad;
  double* itab;
  const int32_t* icnt;
  int32_t ni;
  int32_t* order;
  const CallArgs* args;
  double *summ, *bstate, *pre, *suf, *segtot, *segstate, *segfut, *segll;
  int32_t* segok;
  double *pre2, *suf2, *grptot, *grpstate, *grpfut;
  DevParams params() const { return DevParams{tc, coef, jit, bad, ni ? itab : nullptr, ni ? icnt : nullptr, ni}; }
};

FwdWork plan_work(gp_ssm_plan* pl) {
  FwdWork W;
  W.tc = pl->tc.as<TermConst>();
  W.coef = pl->coef.as<double>();
  W.jit = pl->jit.as<double>();
  W.bad = pl->pbad.as<int32_t>();
  W.itab = pl->itab.as<double>();
  W.icnt = pl->icnt.as<int32_t>();
  W.ni = pl->n_inst;
  W.order = pl->wv_order.as<int32_t>();
  W.args = pl->dargs();
  W.summ = pl->summ.as<double>();
  W.bstate = pl->bstate.as<double>();
  W.pre = pl->pre.as<double>();
  W.suf = pl->suf.as<double>();
  W.segtot = pl->segtot.as<double>();
  W.segstate = pl->segstate.as<double>();
  W.segfut = pl->segfut.as<double>();
  W.segll = pl->segll.as<double>();
  W.segok = pl->segok.as<int32_t>();
  W.pre2 = pl->pre2.as<double>();
  W.suf2 = pl->suf2.as<double>();
  W.grptot = pl->grptot.as<double>();
  W.grpstate = pl->grpstate.as<double>();
  W.grpfut = pl->grpfut.as<double>();
  return W;
}

// Lays the log-likelihood workspace of (plan, M) out from `base` (256-byte
// aligned pieces); returns the bytes it needs.  Nothing is written.
size_t carve_work(const gp_ssm_plan* pl, int32_t M, unsigned char* base, FwdWork& W) {
  const HostPlan& h = pl->host;
  const int64_t B = h.n_series;
  const int NX = 2 * M;
  const int NXP = NX * (NX + 1) / 2;
  const int64_t C = std::max<int64_t>(1, h.n_chunks);
  const int64_t S = std::max<int64_t>(1, h.n_seg);
  const int64_t G = std::max<int64_t>(1, h.n_grp);
  const int64_t EF = elem_fields(NX);
  size_t at = 0;
  auto take = [&](size_t bytes) {
    unsigned char* q = base + at;
    at += (bytes + 255) / 256 * 256;
    return q;
  };
  W.args = (const CallArgs*)take(sizeof(CallArgs));
  W.tc = (TermConst*)take(sizeof(TermConst) * B * M);
  W.coef = (double*)take(sizeof(double) * B * M * 2 * NCOEF);
  W.jit = (double*)take(sizeof(double) * B);
  W.bad = (int32_t*)take(sizeof(int32_t) * B);
  W.ni = pl->n_inst;
  W.itab = W.ni ? (double*)take(sizeof(double) * ITAB_W * B) : nullptr;
  W.icnt = pl->icnt.as<int32_t>();
  W.order = (int32_t*)take(sizeof(int32_t) * std::max<int64_t>(1, h.n_wv));
  W.summ = (double*)take(sizeof(double) * summary_size(NX) * C);
  W.bstate = (double*)take(sizeof(double) * (NX + NXP) * C);
  W.pre = (double*)take(sizeof(double) * EF * C);
  W.suf = W.pre;  // the suffixes serve the backward passes only
  W.segtot = (double*)take(sizeof(double) * EF * S);
  W.segstate = (double*)take(sizeof(double) * (NX + NXP) * S);
  W.segfut = (double*)take(sizeof(double) * (NX + NXP) * S);
  W.segll = (double*)take(sizeof(double) * S);
  W.segok = (int32_t*)take(sizeof(int32_t) * S);
  W.pre2 = W.suf2 = W.grptot = W.grpstate = W.grpfut = nullptr;
  if (h.max_series_nseg > WAVE) {
    W.pre2 = (double*)take(sizeof(double) * EF * S);
    W.suf2 = W.pre2;
    W.grptot = (double*)take(sizeof(double) * EF * G);
    W.grpstate = (double*)take(sizeof(double) * (NX + NXP) * G);
    W.grpfut = (double*)take(sizeof(double) * (NX + NXP) * G);
  }
  return at;
}

// validation, preparation and launch order of the hyperparameters
void enqueue_prep(gp_ssm_plan* pl, const FwdWork& W, int32_t M, hipStream_t s) {
  const int64_t B = pl->host.n_series;
  const int threads = 256;
  const int64_t n = std::max<int64_t>(B * M * NI, B);
  DevPlan p = pl->dev();
  p.wv_order = W.order;
  prof_begin("k_prep", s);
  const int32_t* kinds = pl->kinds_M == M ? pl->kinds.as<int32_t>() : nullptr;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, s, B, M, W.ni, W.args,
                     kinds, W.tc, W.coef, W.jit, W.bad, W.itab);
  prof_end("k_prep", s);
  prof_begin("k_order", s);
  hipLaunchKernelGGL(k_order, dim3(1), dim3(ORDER_THREADS), 0, s, p, M, W.tc, pl->series_dt_cdf.as<float>(),
                     W.order);
  prof_end("k_order", s);
}

void enqueue_forward(gp_ssm_plan* pl, const FwdWork& W, int32_t M, hipStream_t s, int back, bool need_smooth) {
  DevPlan p = pl->dev();
  p.wv_order = W.order;
  const DevParams pr = W.params();
  const KernelSet ks = kernel_set(M, pl->host.max_slots, pl->features(M));
  Launch L{s};
  ks.summaries(L, p, pr, W.summ);
  ScanWork w;
  w.summ = W.summ;
  w.pre = W.pre;
  w.suf = W.suf;
  w.segtot = W.segtot;
  w.segstate = W.segstate;
  w.segfut = W.segfut;
  w.bstate = W.bstate;
  w.badj = back ? pl->badj.as<double>() : nullptr;
  w.bsmooth = (back && need_smooth) ? pl->bsmooth.as<double>() : nullptr;
  w.segll = W.segll;
  w.segok = W.segok;
  w.p2 = nullptr;
  DevPlan p2;
  if (pl->host.max_series_nseg > WAVE) {
    p2 = pl->dev_groups();
    p2.wv_order = W.order;
    w.p2 = &p2;
    w.pre2 = W.pre2;
    w.suf2 = W.suf2;
    w.grptot = W.grptot;
    w.grpstate = W.grpstate;
    w.grpfut = W.grpfut;
  }
  run_scan(M, s, p, pr, w, W.args, back);
}

void enqueue_grad_tail(gp_ssm_plan* pl, int32_t M, hipStream_t s) {
  const DevPlan p = pl->dev();
  const KernelSet ks = kernel_set(M, pl->host.max_slots, pl->features(M));
  RecSlots rs;
  (void)record_slots(pl, M, false, rs);  // reserved: no allocation here
  Launch L{s};
  ks.adjoint(L, p, pl->params(), pl->bstate.as<double>(), pl->badj.as<double>(), rs, pl->gpart.as<double>());
  prof_begin("k_reduce_grad", s);
  hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)pl->host.n_series), dim3(WAVE), 0, s, p, pl->params(), M,
                     pl->gpart.as<double>(), pl->dargs());
  prof_end("k_reduce_grad", s);
}

void enqueue_step(gp_ssm_plan* pl, int32_t M, int kind, hipStream_t s) {
  const FwdWork W = plan_work(pl);
  enqueue_prep(pl, W, M, s);
  enqueue_forward(pl, W, M, s, kind == STEP_GRAD, false);
  if (kind == STEP_GRAD) enqueue_grad_tail(pl, M, s);
}

// One step (log-likelihood, or with its gradient) after put_args: replayed
// from a graph captured once per (plan, kind, number of terms) and workspace
// generation, or launched kernel by kernel while kernel timing is on (its
// events are per launch) or graphs are switched off (GP_SSM_GRAPH=0).
int run_step(gp_ssm_plan* pl, int32_t M, int kind, hipStream_t s) {
  if (int rc = reserve(pl, M, kind == STEP_GRAD, false)) return rc;
  if (g_prof.on || !graphs_enabled()) {
    enqueue_step(pl, M, kind, s);
    HIP_TRY(hipGetLastError());
    return 0;
  }
  auto& g = pl->graphs[kind * 16 + M];
  if (!g.exec || g.gen != pl->gen) {
    if (g.exec) {
      HIP_TRY(hipGraphExecDestroy(g.exec));
      g.exec = nullptr;
    }
    if (!pl->cap) HIP_TRY(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
    enqueue_step(pl, M, kind, pl->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e1 = hipStreamEndCapture(pl->cap, &graph);
    if (e1 != hipSuccess || !graph) return fail(GP_SSM_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e1));
    const hipError_t e2 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      g.exec = nullptr;
      return fail(GP_SSM_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(e2));
    }
    g.gen = pl->gen;
  }
  HIP_TRY(hipGraphLaunch(g.exec, s));
  return 0;
}

// waits for the stream and turns the per-series status into a return code
int sync_status(gp_ssm_plan* pl, const int32_t* status, hipStream_t s) {
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t B = pl->host.n_series;
  std::vector<int32_t> st(B);
  HIP_TRY(hipMemcpy(st.data(), status, sizeof(int32_t) * B, hipMemcpyDeviceToHost));
  int64_t nbad = 0, nparam = 0, first = -1;
  for (int64_t b = 0; b < B; ++b)
    if (st[b] != 0) {
      ++nbad;
      if (st[b] == GP_SSM_EPARAM) ++nparam;
      if (first < 0) first = b;
    }
  if (nparam) return fail(GP_SSM_EPARAM, "sigma, omega0 and Q must be positive and finite, jitter >= 0 and finite, "
                                             "instrument amplitudes positive and finite, offsets finite (" +
                                             std::to_string(nparam) + " series, first " + std::to_string(first) + ")");
  if (nbad)
    return fail(GP_SSM_ENUMERIC, "non-finite result in " + std::to_string(nbad) + " series (first " +
                                     std::to_string(first) + ")");
  return 0;
}

}  // namespace

extern "C" {

void gp_ssm_plan_default_options(gp_ssm_plan_options* opt) {
  if (!opt) return;
  PlanOptions d;
  opt->chunk_min = d.chunk_min;
  opt->chunk_target = d.chunk_target;
  opt->target_chunks = d.target_chunks;
  opt->single_chunk = d.single_chunk;
  opt->threads = d.threads;
  opt->record_budget = DEFAULT_RECORD_BUDGET;
}

int gp_ssm_plan_create(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                       const double* y, const double* yerr, const gp_ssm_plan_options* opt, void* stream,
                       gp_ssm_plan** out) {
  g_err.clear();
  if (!out) return fail(GP_SSM_EINVAL, "null output pointer");
  *out = nullptr;
  if (n_series < 1) return fail(GP_SSM_EINVAL, "n_series < 1");
  if (!offsets) return fail(GP_SSM_EINVAL, "null offsets");
  if (int rc = check_device()) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int64_t> off(n_series + 1);
  if (int rc = host_copy(offsets, sizeof(int64_t) * (n_series + 1), off.data(), s)) return rc;
  if (off[0] != 0) return fail(GP_SSM_EINVAL, "offsets[0] != 0");
  for (int64_t b = 0; b < n_series; ++b)
    if (off[b + 1] < off[b]) return fail(GP_SSM_EINVAL, "offsets not ascending");
  const int64_t N = off[n_series];
  if (N > 0 && (!t_start || !t_end || !y || !yerr)) return fail(GP_SSM_EINVAL, "null input pointer");
  std::vector<double> ts(N), te(N), yy(N), ye(N);
  if (int rc = host_copy(t_start, sizeof(double) * N, ts.data(), s)) return rc;
  if (int rc = host_copy(t_end, sizeof(double) * N, te.data(), s)) return rc;
  if (int rc = host_copy(y, sizeof(double) * N, yy.data(), s)) return rc;
  if (int rc = host_copy(yerr, sizeof(double) * N, ye.data(), s)) return rc;
  PlanOptions po;
  if (opt) {
    if (opt->chunk_min > 0) po.chunk_min = opt->chunk_min;
    po.chunk_target = opt->chunk_target;
    if (opt->target_chunks > 0) po.target_chunks = opt->target_chunks;
    po.single_chunk = opt->single_chunk;
    po.threads = opt->threads;
  }
  gp_ssm_plan* pl = new (std::nothrow) gp_ssm_plan();
  if (!pl) return fail(GP_SSM_ENOMEM, "host allocation failed");
  std::string err;
  int rc = build_plan(n_series, off.data(), ts.data(), te.data(), yy.data(), ye.data(), po, pl->host, err);
  if (rc) {
    delete pl;
    return fail(rc, err);
  }
  pl->record_budget = (opt && opt->record_budget > 0) ? opt->record_budget : DEFAULT_RECORD_BUDGET;
  pl->offsets = std::move(off);
  (void)hipGetDevice(&pl->device);
  if (hipDeviceGetAttribute(&pl->n_cu, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess ||
      pl->n_cu < 1) {
    (void)hipGetLastError();
    pl->n_cu = 1;
  }
  HostPlan& h = pl->host;
  if ((rc = upload(pl->dt, h.dt)) || (rc = upload(pl->t, h.t)) || (rc = upload(pl->y, h.y)) || (rc = upload(pl->r, h.r)) ||
      (rc = upload(pl->invd, h.invd)) || (rc = upload(pl->info, h.info)) || (rc = upload(pl->meas, h.meas)) ||
      (rc = upload(pl->seg_chunk0, h.seg_chunk0)) || (rc = upload(pl->seg_nch, h.seg_nch)) ||
      (rc = upload(pl->grp_seg0, h.grp_seg0)) || (rc = upload(pl->grp_nseg, h.grp_nseg)) ||
      (rc = upload(pl->series_grp0, h.series_grp0)) || (rc = upload(pl->series_ngrp, h.series_ngrp)) ||
      (rc = upload(pl->wv_series, h.wv_series)) || (rc = upload(pl->wv_nch, h.wv_nch)) ||
      (rc = upload(pl->wv_len, h.wv_len)) || (rc = upload(pl->wv_chunk, h.wv_chunk)) ||
      (rc = upload(pl->wv_ev0, h.wv_ev0)) || (rc = upload(pl->chunk_len, h.chunk_len)) ||
      (rc = upload(pl->chunk_series, h.chunk_series)) || (rc = upload(pl->chunk_wv, h.chunk_wv)) ||
      (rc = upload(pl->chunk_lane, h.chunk_lane)) || (rc = upload(pl->chunk_first, h.chunk_first)) ||
      (rc = upload(pl->series_chunk0, h.series_chunk0)) || (rc = upload(pl->series_nch, h.series_nch)) ||
      (rc = upload(pl->series_seg0, h.series_seg0)) || (rc = upload(pl->series_nseg, h.series_nseg)) ||
      (rc = upload(pl->series_wv0, h.series_wv0)) || (rc = upload(pl->series_nwv, h.series_nwv)) ||
      (rc = upload(pl->series_dt_cdf, h.series_dt_cdf))) {
    delete pl;
    return rc;
  }
  {
    // the square-root filter's order of the series, longest first, so that
    // the groups of a wavefront run series of similar length
    std::vector<int32_t> order(h.n_series);
    for (int64_t b = 0; b < h.n_series; ++b) order[b] = (int32_t)b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return h.series_nev[a] > h.series_nev[b]; });
    if ((rc = upload(pl->sqrt_order, order))) {
      delete pl;
      return rc;
    }
  }
  // the event arrays live on the device now; keep only the tables the host needs
  std::vector<double>().swap(h.dt);
  std::vector<double>().swap(h.y);
  std::vector<double>().swap(h.r);
  std::vector<double>().swap(h.invd);
  std::vector<uint32_t>().swap(h.info);
  std::vector<int64_t>().swap(h.meas);
  *out = pl;
  return 0;
}

void gp_ssm_plan_destroy(gp_ssm_plan* plan) { delete plan; }

int gp_ssm_plan_set_term_kinds(gp_ssm_plan* pl, int32_t n_terms, const int32_t* kinds) {
  g_err.clear();
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  if (n_terms == 0 || !kinds) {
    pl->kinds_M = 0;
    pl->kinds_real = false;
    ++pl->gen;
    return 0;
  }
  if (n_terms < 1 || n_terms > GP_SSM_MAX_TERMS) return fail(GP_SSM_EINVAL, "n_terms out of range");
  std::vector<int32_t> k(kinds, kinds + n_terms);
  for (int32_t v : k)
    if (v != GP_SSM_TERM_SHO && v != GP_SSM_TERM_REAL) return fail(GP_SSM_EINVAL, "unknown term kind");
  HIP_TRY(hipDeviceSynchronize());  // earlier calls may still read the kinds
  if (int rc = upload(pl->kinds, k)) return rc;
  pl->kinds_M = n_terms;
  pl->kinds_real = false;
  for (int32_t v : k) pl->kinds_real = pl->kinds_real || v == GP_SSM_TERM_REAL;
  ++pl->gen;  // captured steps hold the kernels of the term kinds
  return 0;
}

int gp_ssm_plan_set_instruments(gp_ssm_plan* pl, int32_t n_inst, const int32_t* instrument, void* stream) {
  g_err.clear();
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  const bool clear = n_inst == 0 || !instrument;
  if (!clear && (n_inst < 1 || n_inst > GP_SSM_MAX_INSTRUMENTS)) return fail(GP_SSM_EINVAL, "n_inst out of range");
  const int64_t N = pl->host.n_meas;
  std::vector<int32_t> lab;
  if (!clear) {
    lab.resize(N);
    if (int rc = host_copy(instrument, sizeof(int32_t) * N, lab.data(), (hipStream_t)stream)) return rc;
    for (int64_t i = 0; i < N; ++i)
      if (lab[i] < 0 || lab[i] >= n_inst)
        return fail(GP_SSM_EINVAL, "instrument label out of range at measurement " + std::to_string(i));
  }
  HIP_TRY(hipDeviceSynchronize());  // earlier calls may still read the event encoding
  DBuf d;
  if (!clear) {
    if (int rc = upload(d, lab)) return rc;
    // measurements of each instrument per series
    const int64_t B = pl->host.n_series;
    std::vector<int32_t> cnt(std::max<int64_t>(1, B) * MAX_INST, 0);
    for (int64_t b = 0; b < B; ++b)
      for (int64_t i = pl->offsets[b]; i < pl->offsets[b + 1]; ++i) ++cnt[b * MAX_INST + lab[i]];
    if (int rc = upload(pl->icnt, cnt)) return rc;
  }
  const int64_t n_ev = pl->host.n_ev_pad;
  if (n_ev > 0) {
    hipLaunchKernelGGL(k_set_inst, dim3((unsigned)((n_ev + 255) / 256)), dim3(256), 0, 0, n_ev, pl->info.as<uint32_t>(),
                       pl->meas.as<int64_t>(), clear ? nullptr : d.as<int32_t>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
  }
  pl->n_inst = clear ? 0 : n_inst;
  ++pl->gen;  // captured steps hold the instrument table's presence
  return 0;
}

int gp_ssm_plan_get_stats(const gp_ssm_plan* pl, gp_ssm_plan_stats* out) {
  if (!pl || !out) return fail(GP_SSM_EINVAL, "null pointer");
  out->n_series = pl->host.n_series;
  out->n_meas = pl->host.n_meas;
  out->n_events = pl->host.n_events;
  out->n_events_padded = pl->host.n_ev_pad;
  out->n_chunks = pl->host.n_chunks;
  out->n_segments = pl->host.n_seg;
  out->max_slots = pl->host.max_slots;
  out->max_chunk_len = pl->host.max_chunk_len;
  out->device_bytes = 0;
  for (const DBuf* d : pl->all_buffers()) out->device_bytes += (int64_t)d->bytes;
  out->record_bytes = (int64_t)pl->rec.bytes;
  return 0;
}

int gp_ssm_plan_loglik(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
                       const double* jitter, double* loglik, int32_t* status, void* stream) {
  g_err.clear();
  if (!loglik) return fail(GP_SSM_EINVAL, "null loglik");
  hipStream_t s = (hipStream_t)stream;
  if (int rc = put_args(pl, M, sigma, omega0, quality, jitter, loglik, nullptr, status, s)) return rc;
  return run_step(pl, M, STEP_LOGLIK, s);
}

int gp_ssm_plan_loglik_inst(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, const double* amp, const double* off,
                            double* loglik, int32_t* status, void* stream) {
  g_err.clear();
  if (!loglik) return fail(GP_SSM_EINVAL, "null loglik");
  hipStream_t s = (hipStream_t)stream;
  if (int rc = put_args(pl, M, sigma, omega0, quality, jitter, loglik, nullptr, status, s, amp, off, 0)) return rc;
  return run_step(pl, M, STEP_LOGLIK, s);
}

int gp_ssm_plan_loglik_noalloc(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                               const double* quality, const double* jitter, double* loglik, int32_t* status,
                               void* stream) {
  g_err.clear();
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  if (M < 1 || M > GP_SSM_MAX_TERMS) return fail(GP_SSM_EINVAL, "n_terms out of range");
  if (!sigma || !omega0 || !quality || !loglik) return fail(GP_SSM_EINVAL, "null pointer");
  if (pl->kinds_M != 0 && pl->kinds_M != M) return fail(GP_SSM_EINVAL, "term kinds were set for another number of terms");
  for (const void* q : {(const void*)sigma, (const void*)omega0, (const void*)quality, (const void*)jitter,
                        (const void*)loglik, (const void*)status})
    if (q && !device_memory(q)) return fail(GP_SSM_EINVAL, "every array must be device memory");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != pl->device) return fail(GP_SSM_EINVAL, "the plan lives on another device than the current one");
  void* base = nullptr;
  if (int rc = scratch_address(dev, &base)) return rc;
  FwdWork W;
  const size_t need = carve_work(pl, M, (unsigned char*)base, W);
  if (need > SCRATCH_BYTES)
    return fail(GP_SSM_ENOMEM, "the batch needs " + std::to_string(need) + " bytes of workspace; the static scratch "
                               "holds " + std::to_string(SCRATCH_BYTES) + " (use gp_ssm_plan_loglik)");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_set_args, dim3(1), dim3(WAVE), 0, s, CallArgs{sigma, omega0, quality, jitter, loglik, nullptr, status},
                     const_cast<CallArgs*>(W.args));
  enqueue_prep(pl, W, M, s);
  enqueue_forward(pl, W, M, s, 0, false);
  HIP_TRY(hipGetLastError());
  return 0;
}

static int plan_loglik_grad(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, const double* amp, const double* off,
                            int32_t grad_inst, double* loglik, double* grad, int32_t* status, void* stream) {
  g_err.clear();
  if (!loglik || !grad) return fail(GP_SSM_EINVAL, "null output");
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  hipStream_t s = (hipStream_t)stream;
  // the gradient reduction reads every series' status: the plan's own array
  // when the caller passes none
  if (int rc = pl->status.ensure(sizeof(int32_t) * pl->host.n_series)) return rc;
  int32_t* st = status ? status : pl->status.as<int32_t>();
  if (int rc = put_args(pl, M, sigma, omega0, quality, jitter, loglik, grad, st, s, amp, off, grad_inst)) return rc;
  return run_step(pl, M, STEP_GRAD, s);
}

int gp_ssm_plan_loglik_grad(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, double* loglik, double* grad,
                            int32_t* status, void* stream) {
  return plan_loglik_grad(pl, M, sigma, omega0, quality, jitter, nullptr, nullptr, 0, loglik, grad, status, stream);
}

int gp_ssm_plan_loglik_grad_inst(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                                 const double* quality, const double* jitter, const double* amp, const double* off,
                                 double* loglik, double* grad, int32_t* status, void* stream) {
  if (pl && pl->n_inst == 0) {
    g_err.clear();
    return fail(GP_SSM_EINVAL, "the plan has no instrument labels (gp_ssm_plan_set_instruments)");
  }
  return plan_loglik_grad(pl, M, sigma, omega0, quality, jitter, amp, off, 1, loglik, grad, status, stream);
}

// the smoother with optional per-term outputs at the test times
static int plan_smooth(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
                       const double* jitter, const double* amp, const double* off, const int64_t* test_offsets, const double* t_test, double* mean_test,
                       double* var_test, double* term_mean, double* term_var, bool want_terms, double* mean_data,
                       double* var_data, double* loglik, int32_t* status, void* stream) {
  g_err.clear();
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  if (!test_offsets) return fail(GP_SSM_EINVAL, "null test_offsets");
  hipStream_t s = (hipStream_t)stream;
  const HostPlan& h = pl->host;
  const int64_t B = h.n_series;
  std::vector<int64_t> to(B + 1);
  if (int rc = host_copy(test_offsets, sizeof(int64_t) * (B + 1), to.data(), s)) return rc;
  if (to[0] != 0) return fail(GP_SSM_EINVAL, "test_offsets[0] != 0");
  for (int64_t q = 0; q < B; ++q)
    if (to[q + 1] < to[q]) return fail(GP_SSM_EINVAL, "test_offsets not ascending");
  const int64_t T = to[B];
  if (T > 0 && (!t_test || !mean_test || !var_test)) return fail(GP_SSM_EINVAL, "null test arrays");
  if (want_terms && T > 0 && (!term_mean || !term_var)) return fail(GP_SSM_EINVAL, "null term arrays");
  for (const void* o : {(const void*)mean_test, (const void*)var_test, (const void*)term_mean, (const void*)term_var,
                        (const void*)mean_data, (const void*)var_data})
    if (o && !device_memory(o)) return fail(GP_SSM_EINVAL, "output arrays must be device memory");
  std::vector<double> tt(T);
  if (int rc = host_copy(t_test, sizeof(double) * T, tt.data(), s)) return rc;
  for (int64_t i = 0; i < T; ++i)
    if (!std::isfinite(tt[i])) return fail(GP_SSM_EDATA, "non-finite test time");
  // assign each test time to the chunk whose event interval holds it; test
  // times of a series without measurements take the prior
  const int64_t C = h.n_chunks;
  std::vector<int32_t> owner(T);
  std::vector<int64_t> cnt(C + 1, 0), prior_idx;
  std::vector<int32_t> prior_series;
  for (int64_t q = 0; q < B; ++q) {
    const int32_t c0 = h.series_chunk0[q], n = h.series_nch[q];
    for (int64_t i = to[q]; i < to[q + 1]; ++i) {
      if (n == 0) {
        owner[i] = -1;
        prior_idx.push_back(i);
        prior_series.push_back((int32_t)q);
        continue;
      }
      int32_t lo = c0, hi = c0 + n - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi) / 2;
        if (h.chunk_t1[mid] >= tt[i])
          hi = mid;
        else
          lo = mid + 1;
      }
      owner[i] = lo;
      ++cnt[lo + 1];
    }
  }
  std::vector<int64_t> c0v(C + 1, 0);
  for (int64_t c = 0; c < C; ++c) c0v[c + 1] = c0v[c] + cnt[c + 1];
  std::vector<int64_t> fillp(c0v.begin(), c0v.end() - 1), idx(std::max<int64_t>(0, c0v[C]));
  for (int64_t i = 0; i < T; ++i)
    if (owner[i] >= 0) idx[fillp[owner[i]]++] = i;
  for (int64_t c = 0; c < C; ++c) {
    std::stable_sort(idx.begin() + c0v[c], idx.begin() + c0v[c + 1], [&](int64_t x, int64_t y) { return tt[x] < tt[y]; });
  }
  std::vector<double> tsort(idx.size());
  for (size_t i = 0; i < idx.size(); ++i) tsort[i] = tt[idx[i]];
  std::vector<double> tprev(std::max<int64_t>(1, C), 0.0);
  for (int64_t c = 0; c < C; ++c) tprev[c] = h.chunk_first[c] ? 0.0 : h.chunk_t1[c - 1];
  // the smoother is not captured: make sure no earlier call still reads the
  // test tables before they are replaced
  HIP_TRY(hipStreamSynchronize(s));
  if (int rc = upload(pl->tests_t, tsort)) return rc;
  if (int rc = upload(pl->tests_idx, idx)) return rc;
  if (int rc = upload(pl->tests_c0, c0v)) return rc;
  if (int rc = upload(pl->tests_before, tprev)) return rc;
  if (int rc = upload(pl->prior_idx, prior_idx)) return rc;
  if (int rc = upload(pl->prior_series, prior_series)) return rc;

  if (int rc = reserve(pl, M, 1, true)) return rc;
  int32_t* st = status ? status : pl->status.as<int32_t>();
  double* ll = loglik ? loglik : pl->llbuf.as<double>();
  if (int rc = put_args(pl, M, sigma, omega0, quality, jitter, ll, nullptr, st, s, amp, off, 0)) return rc;
  const FwdWork W = plan_work(pl);
  enqueue_prep(pl, W, M, s);
  enqueue_forward(pl, W, M, s, 1, true);
  const DevPlan p = pl->dev();
  const KernelSet ks = kernel_set(M, h.max_slots, pl->features(M));
  RecSlots rs;
  if (int rc = record_slots(pl, M, true, rs)) return rc;
  DevTests dt;
  dt.t = pl->tests_t.as<double>();
  dt.out_index = pl->tests_idx.as<int64_t>();
  dt.chunk_t0 = pl->tests_c0.as<int64_t>();
  dt.chunk_tprev = pl->tests_before.as<double>();
  dt.term_mean = want_terms ? term_mean : nullptr;
  dt.term_var = want_terms ? term_var : nullptr;
  Launch L{s};
  ks.smooth(L, p, pl->params(), pl->bstate.as<double>(), pl->bsmooth.as<double>(), rs, dt, mean_test, var_test,
            mean_data, var_data);
  if (!prior_idx.empty()) {
    const int64_t n = (int64_t)prior_idx.size();
    hipLaunchKernelGGL(k_prior_tests, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       pl->prior_idx.as<int64_t>(), pl->prior_series.as<int32_t>(), M, pl->tc.as<TermConst>(),
                       pl->pbad.as<int32_t>(), mean_test, var_test, dt.term_mean, dt.term_var);
  }
  HIP_TRY(hipGetLastError());
  return 0;
}

int gp_ssm_plan_smooth(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
                       const double* jitter, const int64_t* test_offsets, const double* t_test, double* mean_test,
                       double* var_test, double* mean_data, double* var_data, double* loglik, int32_t* status,
                       void* stream) {
  return plan_smooth(pl, M, sigma, omega0, quality, jitter, nullptr, nullptr, test_offsets, t_test, mean_test,
                     var_test, nullptr, nullptr, false, mean_data, var_data, loglik, status, stream);
}

int gp_ssm_plan_smooth_terms(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                             const double* quality, const double* jitter, const int64_t* test_offsets,
                             const double* t_test, double* mean_test, double* var_test, double* term_mean,
                             double* term_var, double* mean_data, double* var_data, double* loglik, int32_t* status,
                             void* stream) {
  return plan_smooth(pl, M, sigma, omega0, quality, jitter, nullptr, nullptr, test_offsets, t_test, mean_test,
                     var_test, term_mean, term_var, true, mean_data, var_data, loglik, status, stream);
}

int gp_ssm_plan_smooth_inst(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, const double* amp, const double* off,
                            const int64_t* test_offsets, const double* t_test, double* mean_test, double* var_test,
                            double* term_mean, double* term_var, double* mean_data, double* var_data, double* loglik,
                            int32_t* status, void* stream) {
  return plan_smooth(pl, M, sigma, omega0, quality, jitter, amp, off, test_offsets, t_test, mean_test, var_test,
                     term_mean, term_var, term_mean || term_var, mean_data, var_data, loglik, status, stream);
}

int gp_ssm_plan_plain_loglik(gp_ssm_plan* pl, int64_t first, int64_t count, int32_t M, const double* sigma,
                             const double* omega0, const double* quality, const double* jitter, double* loglik,
                             void* stream) {
  g_err.clear();
  if (!loglik) return fail(GP_SSM_EINVAL, "null loglik");
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  if (first < 0 || count < 0 || first + count > pl->host.n_series) return fail(GP_SSM_EINVAL, "series range");
  hipStream_t s = (hipStream_t)stream;
  if (int rc = reserve(pl, M, 0, false)) return rc;
  if (int rc = put_args(pl, M, sigma, omega0, quality, jitter, loglik, nullptr, nullptr, s)) return rc;
  enqueue_prep(pl, plan_work(pl), M, s);
  const DevPlan p = pl->dev();
  const KernelSet ks = kernel_set(M, pl->host.max_slots, pl->features(M));
  Launch L{s};
  for (int64_t b = first; b < first + count; ++b) {
    ks.plain(L, p, pl->params(), b, loglik);
    HIP_TRY(hipGetLastError());
  }
  return 0;
}

int gp_ssm_plan_loglik_sqrt(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, const double* amp, const double* off,
                            double* loglik, int32_t* status, void* stream) {
  g_err.clear();
  if (!loglik) return fail(GP_SSM_EINVAL, "null loglik");
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  hipStream_t s = (hipStream_t)stream;
  if (int rc = put_args(pl, M, sigma, omega0, quality, jitter, loglik, nullptr, status, s, amp, off, 0)) return rc;
  if (int rc = reserve(pl, M, 0, false)) return rc;
  enqueue_prep(pl, plan_work(pl), M, s);
  const KernelSet ks = kernel_set(M, pl->host.max_slots, pl->features(M));
  Launch L{s};
  ks.sqrt(L, pl->dev(), pl->params(), pl->sqrt_order.as<int32_t>(), pl->dargs());
  HIP_TRY(hipGetLastError());
  return 0;
}

int gp_ssm_plan_loglik_sqrt_split(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                                  const double* quality, const double* jitter, const double* amp, const double* off,
                                  double* loglik, int32_t* status, void* stream) {
  g_err.clear();
  if (!loglik) return fail(GP_SSM_EINVAL, "null loglik");
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  hipStream_t s = (hipStream_t)stream;
  if (int rc = put_args(pl, M, sigma, omega0, quality, jitter, loglik, nullptr, status, s, amp, off, 0)) return rc;
  if (int rc = reserve(pl, M, 0, false)) return rc;
  const size_t sbytes = sizeof(double) * sq_fields(2 * M) * std::max<int64_t>(1, pl->host.n_chunks);
  if (int rc = pl->sqsumm.ensure(sbytes)) return rc;
  if (int rc = pl->sqsumm2.ensure(sbytes)) return rc;
  // levels of the tree: the most chunks of one series, halved until one
  int32_t most = 0, levels = 0;
  for (int32_t n : pl->host.series_nch) most = std::max(most, n);
  while ((int64_t(1) << levels) < most) ++levels;
  enqueue_prep(pl, plan_work(pl), M, s);
  const KernelSet ks = kernel_set(M, pl->host.max_slots, pl->features(M));
  Launch L{s};
  ks.sqrt_split(L, pl->dev(), pl->params(), pl->sqsumm.as<double>(), pl->sqsumm2.as<double>(), levels, pl->dargs());
  HIP_TRY(hipGetLastError());
  return 0;
}

// One-shot forms: plan with default options, run, wait, destroy.  They return
// GP_SSM_EPARAM or GP_SSM_ENUMERIC when any series failed (its outputs NaN).
static int one_shot_plan(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                         const double* y, const double* yerr, void* stream, gp_ssm_plan** pl) {
  return gp_ssm_plan_create(n_series, offsets, t_start, t_end, y, yerr, nullptr, stream, pl);
}

// ---------------------------------------------------------------------------
// autotuner: the chunk length (hence the lanes each series gets: its events
// over the chunk length, one lane per chunk, 64 lanes to a work wave) is
// picked by timing one call per candidate target chunk count
// ---------------------------------------------------------------------------
static const int64_t TUNE_CANDIDATES[] = {16384, 32768, 65536, 131072, 262144, 524288};
constexpr int N_TUNE = (int)(sizeof(TUNE_CANDIDATES) / sizeof(TUNE_CANDIDATES[0]));

static std::string tune_key(const gp_ssm_plan* pl, int32_t M, int32_t what) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) arch = prop.gcnArchName;
  else (void)hipGetLastError();
  // the workload's shape: series, measurements and events rounded to two
  // significant digits, overlap depth, terms, kind of call, device
  auto r2 = [](int64_t v) {
    if (v < 100) return v;
    int64_t p = 1;
    while (v / p >= 100) p *= 10;
    return (v / p) * p;
  };
  return "B=" + std::to_string(r2(pl->host.n_series)) + ",N=" + std::to_string(r2(pl->host.n_meas)) +
         ",E=" + std::to_string(r2(pl->host.n_events)) + ",J=" + std::to_string(pl->host.max_slots) +
         ",M=" + std::to_string(M) + ",kind=" + std::to_string(what) + ",arch=" + arch;
}

int gp_ssm_autotune_candidates(int64_t* target_chunks, int32_t cap) {
  for (int i = 0; i < N_TUNE && i < cap; ++i)
    if (target_chunks) target_chunks[i] = TUNE_CANDIDATES[i];
  return N_TUNE;
}

int gp_ssm_autotune(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                    const double* y, const double* yerr, int32_t n_terms, const double* sigma, const double* omega0,
                    const double* quality, const double* jitter, int32_t what, const char* cache_path,
                    gp_ssm_plan_options* best, double* best_ms, void* stream) {
  g_err.clear();
  if (!best) return fail(GP_SSM_EINVAL, "null output");
  if (what != 0 && what != 1) return fail(GP_SSM_EINVAL, "what must be 0 (log-likelihood) or 1 (with gradient)");
  gp_ssm_plan_default_options(best);
  if (best_ms) *best_ms = -1.0;
  hipStream_t s = (hipStream_t)stream;
  if (const char* e = std::getenv("GP_SSM_TARGET_CHUNKS")) {
    const long long v = std::atoll(e);
    if (v > 0) {
      best->target_chunks = v;
      return 0;
    }
  }
  const int64_t B = n_series;
  double* tmp = nullptr;  // log-likelihood, gradient and status of the timing calls
  const size_t tmp_bytes = sizeof(double) * B * (1 + 3 * (size_t)std::max(1, n_terms) + 1) + sizeof(int32_t) * B;
  std::string key;
  int rc = 0;
  double best_t = 1e300;
  for (int i = 0; i < N_TUNE && rc == 0; ++i) {
    gp_ssm_plan_options o;
    gp_ssm_plan_default_options(&o);
    o.target_chunks = TUNE_CANDIDATES[i];
    gp_ssm_plan* pl = nullptr;
    if ((rc = gp_ssm_plan_create(n_series, offsets, t_start, t_end, y, yerr, &o, stream, &pl))) break;
    if (i == 0) {
      key = tune_key(pl, n_terms, what);
      // a stored choice for this shape of workload
      if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
          char line[1024];
          long long tc = 0;
          double ms = -1.0;
          while (std::fgets(line, sizeof line, f)) {
            char k[900];
            long long v;
            double t;
            if (std::sscanf(line, "%899s %lld %lf", k, &v, &t) == 3 && key == k) {
              tc = v;
              ms = t;
            }
          }
          std::fclose(f);
          if (tc > 0) {
            gp_ssm_plan_destroy(pl);
            best->target_chunks = tc;
            if (best_ms) *best_ms = ms;
            return 0;
          }
        }
      }
      if (hipMalloc((void**)&tmp, tmp_bytes) != hipSuccess) {
        (void)hipGetLastError();
        gp_ssm_plan_destroy(pl);
        return fail(GP_SSM_ENOMEM, "autotune: hipMalloc failed");
      }
    }
    double* ll = tmp;
    double* gr = tmp + B;
    int32_t* st = (int32_t*)(tmp + B * (1 + 3 * (size_t)n_terms + 1));
    auto call = [&]() {
      return what ? gp_ssm_plan_loglik_grad(pl, n_terms, sigma, omega0, quality, jitter, ll, gr, st, stream)
                  : gp_ssm_plan_loglik(pl, n_terms, sigma, omega0, quality, jitter, ll, st, stream);
    };
    hipEvent_t a = nullptr, b = nullptr;
    if ((rc = call()) == 0 && (rc = call()) == 0) {  // the first call captures the step
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        rc = fail(GP_SSM_EDEVICE, "autotune: hipEventCreate failed");
      } else {
        (void)hipEventRecord(a, s);
        for (int k = 0; k < 3 && rc == 0; ++k) rc = call();
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (rc == 0 && ms / 3.0 < best_t) {
          best_t = ms / 3.0;
          best->target_chunks = TUNE_CANDIDATES[i];
        }
      }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    gp_ssm_plan_destroy(pl);
  }
  if (tmp) (void)hipFree(tmp);
  if (rc) return rc;
  if (best_ms) *best_ms = best_t;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s %lld %.6f\n", key.c_str(), (long long)best->target_chunks, best_t);
      std::fclose(f);
    }
  }
  return 0;
}

int gp_ssm_loglik(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end, const double* y,
                  const double* yerr, int32_t n_terms, const double* sigma, const double* omega0, const double* quality,
                  const double* jitter, double* loglik, int32_t* status, void* stream) {
  gp_ssm_plan* pl = nullptr;
  if (int rc = one_shot_plan(n_series, offsets, t_start, t_end, y, yerr, stream, &pl)) return rc;
  int rc = pl->status.ensure(sizeof(int32_t) * n_series);
  int32_t* st = status ? status : pl->status.as<int32_t>();
  if (rc == 0) rc = gp_ssm_plan_loglik(pl, n_terms, sigma, omega0, quality, jitter, loglik, st, stream);
  if (rc == 0) rc = sync_status(pl, st, (hipStream_t)stream);
  gp_ssm_plan_destroy(pl);
  return rc;
}

int gp_ssm_loglik_grad(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                       const double* y, const double* yerr, int32_t n_terms, const double* sigma, const double* omega0,
                       const double* quality, const double* jitter, double* loglik, double* grad, int32_t* status,
                       void* stream) {
  gp_ssm_plan* pl = nullptr;
  if (int rc = one_shot_plan(n_series, offsets, t_start, t_end, y, yerr, stream, &pl)) return rc;
  int rc = pl->status.ensure(sizeof(int32_t) * n_series);
  int32_t* st = status ? status : pl->status.as<int32_t>();
  if (rc == 0) rc = gp_ssm_plan_loglik_grad(pl, n_terms, sigma, omega0, quality, jitter, loglik, grad, st, stream);
  if (rc == 0) rc = sync_status(pl, st, (hipStream_t)stream);
  gp_ssm_plan_destroy(pl);
  return rc;
}

int gp_ssm_smooth(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                  const double* y, const double* yerr, int32_t n_terms, const double* sigma, const double* omega0,
                  const double* quality, const double* jitter, const int64_t* test_offsets, const double* t_test,
                  double* mean_test, double* var_test, double* mean_data, double* var_data, int32_t* status,
                  void* stream) {
  gp_ssm_plan* pl = nullptr;
  if (int rc = one_shot_plan(n_series, offsets, t_start, t_end, y, yerr, stream, &pl)) return rc;
  int rc = pl->status.ensure(sizeof(int32_t) * n_series);
  int32_t* st = status ? status : pl->status.as<int32_t>();
  if (rc == 0)
    rc = gp_ssm_plan_smooth(pl, n_terms, sigma, omega0, quality, jitter, test_offsets, t_test, mean_test, var_test,
                            mean_data, var_data, nullptr, st, stream);
  if (rc == 0) rc = sync_status(pl, st, (hipStream_t)stream);
  gp_ssm_plan_destroy(pl);
  return rc;
}

int gp_ssm_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  return 0;
}

int gp_ssm_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  prof_flush();
  g_prof.total.clear();
  return 0;
}

int gp_ssm_profile_read(const char** names, int64_t* counts, double* total_ms, int32_t cap) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  prof_flush();
  g_prof.names.clear();
  for (auto& kv : g_prof.total) g_prof.names.push_back(kv.first);
  int32_t i = 0;
  for (auto& kv : g_prof.total) {
    if (i < cap) {
      if (names) names[i] = g_prof.names[i].c_str();
      if (counts) counts[i] = kv.second.first;
      if (total_ms) total_ms[i] = kv.second.second;
    }
    ++i;
  }
  return (int)g_prof.total.size();
}

const char* gp_ssm_last_error(void) { return g_err.c_str(); }

const char* gp_ssm_version(void) { return "gp_ssm 0.1 (gfx950, fp64)"; }

}  // extern "C"
