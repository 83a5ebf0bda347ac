// C-ABI of the library (declared in include/gp_ssm.h): plans, workspace,
// hyperparameter preparation, the cross-chunk combination and the dispatch of
// the per-(terms, slots) kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gp_ssm.h"
#include "kernels.h"
#include "plan.h"
#include "scan.h"

using namespace gpssm;

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
__global__ void k_prep(int64_t B, int M, const double* __restrict__ sigma, const double* __restrict__ omega0,
                       const double* __restrict__ quality, const double* __restrict__ jitter, TermConst* __restrict__ tc,
                       double* __restrict__ coef, double* __restrict__ jit) {
  // one thread per (series, term, series interval)
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < B * M * NI) {
    const int64_t i = j / NI;
    const int iv = (int)(j - i * NI);
    const TermConst t = make_term(sigma[i], omega0[i], quality[i]);
    if (iv == 0) tc[i] = t;
    double* c = coef + i * 2 * NCOEF + iv * ISTRIDE;
    series_interval_table(t.beta, interval_centre(iv, t.b1ser, t.wser), c, c + NCOEF);
  }
  if (j < B) jit[j] = jitter ? jitter[j] : 0.0;
}

// gradient partials of a series' work waves summed: one wavefront per series,
// lane l takes waves l, l + 64, ..., then a fixed-order wave reduction
__global__ __launch_bounds__(WAVE) void k_reduce_grad(DevPlan p, int M, const double* __restrict__ gpart,
                                                      const int32_t* __restrict__ status, double* __restrict__ grad) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t S = p.n_wv;
  const int32_t s0 = p.series_wv0[b], n = p.series_nwv[b];
  const int G = 3 * M + 1;
  const bool good = status == nullptr || status[b] == 0;
  for (int f = 0; f < G; ++f) {
    double s = 0.0;
    for (int32_t q = lane; q < n; q += WAVE) s += gpart[(int64_t)f * S + s0 + q];
    s = wave_sum(s);
    if (lane == 0) grad[b * G + f] = (good && isfinite(s)) ? s : __builtin_nan("");
  }
}

KernelSet kernel_set(int M, int J) {
  J = std::max(1, J);
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
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  int ensure(size_t n) {
    if (n <= bytes) return 0;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, n) != hipSuccess) return fail(GP_SSM_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
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

int host_copy(const void* src, size_t bytes, void* dst, hipStream_t s) {
  if (bytes == 0) return 0;
  hipPointerAttribute_t attr;
  bool device = false;
  if (hipPointerGetAttributes(&attr, src) == hipSuccess) {
    device = (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
  } else {
    (void)hipGetLastError();
  }
  if (device) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    std::memcpy(dst, src, bytes);
  }
  return 0;
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

struct gp_ssm_plan {
  int device = 0;
  HostPlan host;
  DBuf dt, t, y, r, invd, info, meas;
  DBuf seg_chunk0, seg_nch, grp_seg0, grp_nseg, series_grp0, series_ngrp;
  DBuf wv_series, wv_nch, wv_len, wv_chunk, wv_ev0;
  DBuf chunk_len, chunk_series, chunk_wv, chunk_lane, chunk_first;
  DBuf series_chunk0, series_nch, series_seg0, series_nseg, series_wv0, series_nwv;
  // workspace
  DBuf tc, coef, jit, summ, bstate, badj, bsmooth, gpart, rec, status;
  DBuf pre, suf, segtot, segstate, segfut, segll, segok;
  DBuf pre2, suf2, grptot, grpstate, grpfut;
  DBuf tests_t, tests_idx, tests_c0, tests_before;
  // launch order of the work waves (most expensive first): written on the
  // host into pinned memory, copied on the call's stream; order_ev marks the
  // copy so the buffer is not rewritten before it is done
  DBuf wv_order;
  int32_t* order_host = nullptr;
  hipEvent_t order_ev = nullptr;

  ~gp_ssm_plan() {
    if (order_ev) {
      (void)hipEventSynchronize(order_ev);
      (void)hipEventDestroy(order_ev);
    }
    if (order_host) (void)hipHostFree(order_host);
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
    return p;
  }
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

// validates hyperparameters (host copies) and prepares them on the device
// Launch order of the work waves.  Two or so wavefronts share each SIMD over a
// launch, and a wave's cost varies with its series' terms: a
// wavefront pays for the Taylor branch of a term at a step when any of its
// lanes needs it, and for the closed-form branch when any lane needs that.
// With p the fraction of the series' steps below the switch point, the
// expected cost per step and term is C_SER (1 - (1-p)^64) + C_CLO (1 - p^64)
// on top of W0 for the filter step; p comes from the series' step-length
// distribution.  Dispatching the costliest waves first (longest processing
// time first) evens out the SIMDs' loads.
int set_launch_order(gp_ssm_plan* pl, int32_t M, const double* omega0, const double* quality, hipStream_t s) {
  constexpr double W0 = 4.0, C_SER = 1.0, C_CLO = 1.5;
  const HostPlan& h = pl->host;
  const int64_t S = h.n_wv;
  if (S == 0) return 0;
  if (!pl->order_host) {
    HIP_TRY(hipHostMalloc((void**)&pl->order_host, sizeof(int32_t) * S, hipHostMallocDefault));
    HIP_TRY(hipEventCreateWithFlags(&pl->order_ev, hipEventDisableTiming));
    if (int rc = pl->wv_order.ensure(sizeof(int32_t) * S)) return rc;
  } else {
    HIP_TRY(hipEventSynchronize(pl->order_ev));
  }
  std::vector<double> term_cost(h.n_series);
  for (int64_t b = 0; b < h.n_series; ++b) {
    const float* cdf = h.series_dt_cdf.data() + b * DT_NE;
    double c = W0;
    for (int t = 0; t < M; ++t) {
      const double w0 = omega0[b * M + t], beta = 0.5 / quality[b * M + t];
      const double thr = XSER / std::max(1.0, beta) / w0;  // steps with dt <= thr take the series
      int ex;
      const double fr = std::frexp(thr, &ex);  // thr = fr 2^ex, fr in [0.5, 1)
      const int k = ex - DT_KMIN;
      double p;
      if (k <= 0)
        p = cdf[0];
      else if (k >= DT_NE)
        p = 1.0;
      else  // linear in log2(dt) between the edges 2^(ex-1) and 2^ex
        p = cdf[k - 1] + (cdf[k] - cdf[k - 1]) * (std::log2(fr) + 1.0);
      c += C_SER * (1.0 - std::pow(1.0 - p, WAVE)) + C_CLO * (1.0 - std::pow(p, WAVE));
    }
    term_cost[b] = c;
  }
  std::vector<std::pair<double, int32_t>> key(S);
  for (int64_t q = 0; q < S; ++q) key[q] = {-(double)h.wv_len[q] * term_cost[h.wv_series[q]], (int32_t)q};
  std::sort(key.begin(), key.end());
  for (int64_t q = 0; q < S; ++q) pl->order_host[q] = key[q].second;
  HIP_TRY(hipMemcpyAsync(pl->wv_order.p, pl->order_host, sizeof(int32_t) * S, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(pl->order_ev, s));
  return 0;
}

int prepare_params(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
                   const double* jitter, hipStream_t s, DevParams& pr) {
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  if (M < 1 || M > GP_SSM_MAX_TERMS) return fail(GP_SSM_EINVAL, "n_terms out of range");
  if (!sigma || !omega0 || !quality) return fail(GP_SSM_EINVAL, "null hyperparameter pointer");
  const int64_t B = pl->host.n_series;
  std::vector<double> h(3 * B * M + B);
  if (int rc = host_copy(sigma, sizeof(double) * B * M, h.data(), s)) return rc;
  if (int rc = host_copy(omega0, sizeof(double) * B * M, h.data() + B * M, s)) return rc;
  if (int rc = host_copy(quality, sizeof(double) * B * M, h.data() + 2 * B * M, s)) return rc;
  if (jitter) {
    if (int rc = host_copy(jitter, sizeof(double) * B, h.data() + 3 * B * M, s)) return rc;
  }
  for (int64_t i = 0; i < 3 * B * M; ++i)
    if (!(h[i] > 0) || !std::isfinite(h[i]))
      return fail(GP_SSM_EPARAM, "sigma, omega0 and Q must be positive and finite (entry " + std::to_string(i % (B * M)) + ")");
  if (jitter)
    for (int64_t b = 0; b < B; ++b)
      if (!(h[3 * B * M + b] >= 0) || !std::isfinite(h[3 * B * M + b]))
        return fail(GP_SSM_EPARAM, "jitter must be >= 0 and finite (series " + std::to_string(b) + ")");
  if (int rc = set_launch_order(pl, M, h.data() + B * M, h.data() + 2 * B * M, s)) return rc;
  if (int rc = pl->tc.ensure(sizeof(TermConst) * B * M)) return rc;
  if (int rc = pl->coef.ensure(sizeof(double) * B * M * 2 * NCOEF)) return rc;
  if (int rc = pl->jit.ensure(sizeof(double) * B)) return rc;
  const int threads = 256;
  const int64_t n = std::max<int64_t>(B * M * NI, B);
  prof_begin("k_prep", s);
  hipLaunchKernelGGL(k_prep, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, s, B, M, sigma, omega0,
                     quality, jitter, pl->tc.as<TermConst>(), pl->coef.as<double>(), pl->jit.as<double>());
  prof_end("k_prep", s);
  HIP_TRY(hipGetLastError());
  pr.tc = pl->tc.as<TermConst>();
  pr.coef = pl->coef.as<double>();
  pr.jit = pl->jit.as<double>();
  return 0;
}

int run_forward(gp_ssm_plan* pl, int32_t M, const DevParams& pr, hipStream_t s, double* loglik, int32_t* status,
                int back, bool need_smooth) {
  const int NX = 2 * M;
  const int NXP = NX * (NX + 1) / 2;
  const int64_t C = std::max<int64_t>(1, pl->host.n_chunks);
  const int64_t S = std::max<int64_t>(1, pl->host.n_seg);
  const int EF = elem_fields(NX);
  if (int rc = pl->summ.ensure(sizeof(double) * summary_size(NX) * C)) return rc;
  if (int rc = pl->bstate.ensure(sizeof(double) * (NX + NXP) * C)) return rc;
  if (int rc = pl->pre.ensure(sizeof(double) * EF * C)) return rc;
  if (int rc = pl->suf.ensure(sizeof(double) * EF * C)) return rc;
  if (int rc = pl->segtot.ensure(sizeof(double) * EF * S)) return rc;
  if (int rc = pl->segstate.ensure(sizeof(double) * (NX + NXP) * S)) return rc;
  if (int rc = pl->segfut.ensure(sizeof(double) * (NX + NXP) * S)) return rc;
  if (int rc = pl->segll.ensure(sizeof(double) * S)) return rc;
  if (int rc = pl->segok.ensure(sizeof(int32_t) * S)) return rc;
  if (back) {
    if (int rc = pl->badj.ensure(sizeof(double) * (NX + NXP) * C)) return rc;
    if (need_smooth)
      if (int rc = pl->bsmooth.ensure(sizeof(double) * (NX + NXP) * C)) return rc;
  }
  const DevPlan p = pl->dev();
  const KernelSet ks = kernel_set(M, pl->host.max_slots);
  Launch L{s};
  ks.summaries(L, p, pr, pl->summ.as<double>());
  HIP_TRY(hipGetLastError());
  ScanWork w;
  w.summ = pl->summ.as<double>();
  w.pre = pl->pre.as<double>();
  w.suf = pl->suf.as<double>();
  w.segtot = pl->segtot.as<double>();
  w.segstate = pl->segstate.as<double>();
  w.segfut = pl->segfut.as<double>();
  w.bstate = pl->bstate.as<double>();
  w.badj = back ? pl->badj.as<double>() : nullptr;
  w.bsmooth = (back && need_smooth) ? pl->bsmooth.as<double>() : nullptr;
  w.segll = pl->segll.as<double>();
  w.segok = pl->segok.as<int32_t>();
  w.p2 = nullptr;
  DevPlan p2;
  if (pl->host.max_series_nseg > WAVE) {
    const int64_t G = std::max<int64_t>(1, pl->host.n_grp);
    if (int rc = pl->pre2.ensure(sizeof(double) * EF * S)) return rc;
    if (int rc = pl->suf2.ensure(sizeof(double) * EF * S)) return rc;
    if (int rc = pl->grptot.ensure(sizeof(double) * EF * G)) return rc;
    if (int rc = pl->grpstate.ensure(sizeof(double) * (NX + NXP) * G)) return rc;
    if (int rc = pl->grpfut.ensure(sizeof(double) * (NX + NXP) * G)) return rc;
    p2 = pl->dev_groups();
    w.p2 = &p2;
    w.pre2 = pl->pre2.as<double>();
    w.suf2 = pl->suf2.as<double>();
    w.grptot = pl->grptot.as<double>();
    w.grpstate = pl->grpstate.as<double>();
    w.grpfut = pl->grpfut.as<double>();
  }
  run_scan(M, s, p, pr, w, loglik, status, back);
  HIP_TRY(hipGetLastError());
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
}

int gp_ssm_plan_create(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                       const double* y, const double* yerr, const gp_ssm_plan_options* opt, void* stream,
                       gp_ssm_plan** out) {
  g_err.clear();
  if (!out) return fail(GP_SSM_EINVAL, "null output pointer");
  *out = nullptr;
  if (n_series < 1) return fail(GP_SSM_EINVAL, "n_series < 1");
  if (!offsets || !t_start || !t_end || !y || !yerr) return fail(GP_SSM_EINVAL, "null input pointer");
  if (int rc = check_device()) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int64_t> off(n_series + 1);
  if (int rc = host_copy(offsets, sizeof(int64_t) * (n_series + 1), off.data(), s)) return rc;
  if (off[0] != 0) return fail(GP_SSM_EINVAL, "offsets[0] != 0");
  for (int64_t b = 0; b < n_series; ++b)
    if (off[b + 1] < off[b]) return fail(GP_SSM_EINVAL, "offsets not ascending");
  const int64_t N = off[n_series];
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
  (void)hipGetDevice(&pl->device);
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
      (rc = upload(pl->series_wv0, h.series_wv0)) || (rc = upload(pl->series_nwv, h.series_nwv))) {
    delete pl;
    return rc;
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
  return 0;
}

int gp_ssm_plan_loglik(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
                       const double* jitter, double* loglik, int32_t* status, void* stream) {
  g_err.clear();
  if (!loglik) return fail(GP_SSM_EINVAL, "null loglik");
  hipStream_t s = (hipStream_t)stream;
  DevParams pr;
  if (int rc = prepare_params(pl, M, sigma, omega0, quality, jitter, s, pr)) return rc;
  return run_forward(pl, M, pr, s, loglik, status, 0, false);
}

int gp_ssm_plan_loglik_grad(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                            const double* quality, const double* jitter, double* loglik, double* grad,
                            int32_t* status, void* stream) {
  g_err.clear();
  if (!loglik || !grad) return fail(GP_SSM_EINVAL, "null output");
  hipStream_t s = (hipStream_t)stream;
  DevParams pr;
  if (int rc = prepare_params(pl, M, sigma, omega0, quality, jitter, s, pr)) return rc;
  const int64_t B = pl->host.n_series;
  int32_t* st = status;
  if (!st) {
    if (int rc = pl->status.ensure(sizeof(int32_t) * B)) return rc;
    st = pl->status.as<int32_t>();
  }
  if (int rc = run_forward(pl, M, pr, s, loglik, st, 1, false)) return rc;
  const int NX = 2 * M;
  const int J = std::max(1, pl->host.max_slots);
  const int D = NX + J;
  const int F = D + D * (D + 1) / 2;
  const int64_t C = pl->host.n_chunks;
  if (int rc = pl->rec.ensure(sizeof(double) * F * std::max<int64_t>(1, pl->host.n_ev_pad))) return rc;
  if (int rc = pl->gpart.ensure(sizeof(double) * (3 * M + 1) * std::max<int64_t>(1, pl->host.n_wv))) return rc;
  const DevPlan p = pl->dev();
  const KernelSet ks = kernel_set(M, pl->host.max_slots);
  Launch L{s};
  ks.adjoint(L, p, pr, pl->bstate.as<double>(), pl->badj.as<double>(), pl->rec.as<double>(), pl->gpart.as<double>());
  HIP_TRY(hipGetLastError());
  prof_begin("k_reduce_grad", s);
  hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)B), dim3(WAVE), 0, s, p, M, pl->gpart.as<double>(), st,
                     grad);
  prof_end("k_reduce_grad", s);
  HIP_TRY(hipGetLastError());
  return 0;
}

// the smoother with optional per-term outputs at the test times
static int plan_smooth(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
                const double* jitter, const int64_t* test_offsets, const double* t_test, double* mean_test,
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
  std::vector<double> tt(T);
  if (int rc = host_copy(t_test, sizeof(double) * T, tt.data(), s)) return rc;
  for (int64_t i = 0; i < T; ++i)
    if (!std::isfinite(tt[i])) return fail(GP_SSM_EDATA, "non-finite test time");
  // assign each test time to the chunk whose event interval holds it
  const int64_t C = h.n_chunks;
  std::vector<int32_t> owner(T);
  std::vector<int64_t> cnt(C + 1, 0);
  for (int64_t q = 0; q < B; ++q) {
    const int32_t c0 = h.series_chunk0[q], n = h.series_nch[q];
    if (to[q + 1] > to[q] && n == 0) return fail(GP_SSM_EINVAL, "test times for a series without measurements");
    for (int64_t i = to[q]; i < to[q + 1]; ++i) {
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
  std::vector<int64_t> fillp(c0v.begin(), c0v.end() - 1), idx(T);
  for (int64_t i = 0; i < T; ++i) idx[fillp[owner[i]]++] = i;
  std::vector<double> tsort(T);
  for (int64_t c = 0; c < C; ++c) {
    std::stable_sort(idx.begin() + c0v[c], idx.begin() + c0v[c + 1], [&](int64_t x, int64_t y) { return tt[x] < tt[y]; });
  }
  for (int64_t i = 0; i < T; ++i) tsort[i] = tt[idx[i]];
  std::vector<double> tprev(std::max<int64_t>(1, C), 0.0);
  for (int64_t c = 0; c < C; ++c) tprev[c] = h.chunk_first[c] ? 0.0 : h.chunk_t1[c - 1];
  if (int rc = upload(pl->tests_t, tsort)) return rc;
  if (int rc = upload(pl->tests_idx, idx)) return rc;
  if (int rc = upload(pl->tests_c0, c0v)) return rc;
  if (int rc = upload(pl->tests_before, tprev)) return rc;

  DevParams pr;
  if (int rc = prepare_params(pl, M, sigma, omega0, quality, jitter, s, pr)) return rc;
  int32_t* st = status;
  if (!st) {
    if (int rc = pl->status.ensure(sizeof(int32_t) * B)) return rc;
    st = pl->status.as<int32_t>();
  }
  double* ll = loglik;
  DBuf tmpll;
  if (!ll) {
    if (int rc = tmpll.ensure(sizeof(double) * B)) return rc;
    ll = tmpll.as<double>();
  }
  if (int rc = run_forward(pl, M, pr, s, ll, st, 1, true)) return rc;
  const int NX = 2 * M;
  const int J = std::max(1, h.max_slots);
  const int D = NX + J;
  const int F = D + D * (D + 1) / 2;
  if (int rc = pl->rec.ensure(sizeof(double) * F * std::max<int64_t>(1, h.n_ev_pad))) return rc;
  const DevPlan p = pl->dev();
  const KernelSet ks = kernel_set(M, h.max_slots);
  DevTests dt;
  dt.t = pl->tests_t.as<double>();
  dt.out_index = pl->tests_idx.as<int64_t>();
  dt.chunk_t0 = pl->tests_c0.as<int64_t>();
  dt.chunk_tprev = pl->tests_before.as<double>();
  dt.term_mean = want_terms ? term_mean : nullptr;
  dt.term_var = want_terms ? term_var : nullptr;
  Launch L{s};
  ks.smooth(L, p, pr, pl->bstate.as<double>(), pl->bsmooth.as<double>(), pl->rec.as<double>(), dt, mean_test, var_test,
            mean_data, var_data);
  HIP_TRY(hipGetLastError());
  if (!loglik) HIP_TRY(hipStreamSynchronize(s));  // the temporary log-likelihood buffer is freed on return
  return 0;
}

int gp_ssm_plan_smooth(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0, const double* quality,
                       const double* jitter, const int64_t* test_offsets, const double* t_test, double* mean_test,
                       double* var_test, double* mean_data, double* var_data, double* loglik, int32_t* status,
                       void* stream) {
  return plan_smooth(pl, M, sigma, omega0, quality, jitter, test_offsets, t_test, mean_test, var_test, nullptr,
                     nullptr, false, mean_data, var_data, loglik, status, stream);
}

int gp_ssm_plan_smooth_terms(gp_ssm_plan* pl, int32_t M, const double* sigma, const double* omega0,
                             const double* quality, const double* jitter, const int64_t* test_offsets,
                             const double* t_test, double* mean_test, double* var_test, double* term_mean,
                             double* term_var, double* mean_data, double* var_data, double* loglik, int32_t* status,
                             void* stream) {
  return plan_smooth(pl, M, sigma, omega0, quality, jitter, test_offsets, t_test, mean_test, var_test, term_mean,
                     term_var, true, mean_data, var_data, loglik, status, stream);
}

int gp_ssm_plan_plain_loglik(gp_ssm_plan* pl, int64_t first, int64_t count, int32_t M, const double* sigma,
                             const double* omega0, const double* quality, const double* jitter, double* loglik,
                             void* stream) {
  g_err.clear();
  if (!loglik) return fail(GP_SSM_EINVAL, "null loglik");
  if (!pl) return fail(GP_SSM_EINVAL, "null plan");
  if (first < 0 || count < 0 || first + count > pl->host.n_series) return fail(GP_SSM_EINVAL, "series range");
  hipStream_t s = (hipStream_t)stream;
  DevParams pr;
  if (int rc = prepare_params(pl, M, sigma, omega0, quality, jitter, s, pr)) return rc;
  const DevPlan p = pl->dev();
  const KernelSet ks = kernel_set(M, pl->host.max_slots);
  Launch L{s};
  for (int64_t b = first; b < first + count; ++b) {
    ks.plain(L, p, pr, b, loglik);
    HIP_TRY(hipGetLastError());
  }
  return 0;
}

static int one_shot_plan(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                         const double* y, const double* yerr, void* stream, gp_ssm_plan** pl) {
  return gp_ssm_plan_create(n_series, offsets, t_start, t_end, y, yerr, nullptr, stream, pl);
}

int gp_ssm_loglik(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end, const double* y,
                  const double* yerr, int32_t n_terms, const double* sigma, const double* omega0, const double* quality,
                  const double* jitter, double* loglik, int32_t* status, void* stream) {
  gp_ssm_plan* pl = nullptr;
  if (int rc = one_shot_plan(n_series, offsets, t_start, t_end, y, yerr, stream, &pl)) return rc;
  int rc = gp_ssm_plan_loglik(pl, n_terms, sigma, omega0, quality, jitter, loglik, status, stream);
  if (rc == 0 && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = fail(GP_SSM_EDEVICE, "stream sync failed");
  gp_ssm_plan_destroy(pl);
  return rc;
}

int gp_ssm_loglik_grad(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end,
                       const double* y, const double* yerr, int32_t n_terms, const double* sigma, const double* omega0,
                       const double* quality, const double* jitter, double* loglik, double* grad, int32_t* status,
                       void* stream) {
  gp_ssm_plan* pl = nullptr;
  if (int rc = one_shot_plan(n_series, offsets, t_start, t_end, y, yerr, stream, &pl)) return rc;
  int rc = gp_ssm_plan_loglik_grad(pl, n_terms, sigma, omega0, quality, jitter, loglik, grad, status, stream);
  if (rc == 0 && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = fail(GP_SSM_EDEVICE, "stream sync failed");
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
  int rc = gp_ssm_plan_smooth(pl, n_terms, sigma, omega0, quality, jitter, test_offsets, t_test, mean_test, var_test,
                              mean_data, var_data, nullptr, status, stream);
  if (rc == 0 && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = fail(GP_SSM_EDEVICE, "stream sync failed");
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
