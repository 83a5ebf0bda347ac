// Time-parallel combination of chunk summaries (the associative scan of the
// parallel Kalman filter, Sec. 3.2.4 following SG21, over chunk summaries
// instead of single events):
//
//  k_seg_scan   one wavefront per segment (<= 64 chunks of one series):
//               Kogge-Stone inclusive prefix and suffix compositions of the
//               chunk summaries across the lanes, and the segment total.
//  k_series_scan one wavefront per series: the filtered state at the start
//               of every segment (prefix over segment totals applied to the
//               prior) and the future information (eta~, J~) after every
//               segment (suffix over segment totals).
//  k_seg_fix    one wavefront per segment: the filtered state at every chunk
//               boundary, each chunk's log-likelihood contribution, and, for
//               the gradient and the smoother, the future information at each
//               chunk's end, from which follow the gradient of the future
//               likelihood with respect to the boundary moments and the
//               smoother's adjoint pair there.
//  k_series_finish  sums the per-segment log-likelihoods of each series (and,
//                   with instruments, its -log(amplitude) terms).
//
// When a series has more than 64 segments, the segment totals are treated as
// chunk summaries one level up: k_seg_scan over groups of 64 segments,
// k_series_scan over the group totals, and k_grp_fix gives the state entering
// every segment and the information after it, so that no lane walks more than
// a few totals in sequence.
#include <hip/hip_runtime.h>

#include "../../include/gp_ssm.h"
#include "kernels.h"
#include "plan.h"
#include "scan.h"

namespace gpssm {

namespace {

template <int N>
__device__ __forceinline__ void prior_state(const DevParams& pr, int64_t b, double* m, double* P) {
  constexpr int M = N / 2;
#pragma unroll
  for (int i = 0; i < N; ++i) m[i] = 0.0;
#pragma unroll
  for (int i = 0; i < N * (N + 1) / 2; ++i) P[i] = 0.0;
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const double s2 = pr.tc[b * M + t].sigma * pr.tc[b * M + t].sigma;
    P[sidx(2 * t, 2 * t, N)] = s2;
    P[sidx(2 * t + 1, 2 * t + 1, N)] = s2 * second_prior(pr.tc[b * M + t]);
  }
}

template <int N>
__device__ __forceinline__ void lds_put(double* lds, int lane, const Elem<N>& e, int stride = WAVE) {
  e.store([&](int f, double v) { lds[f * stride + lane] = v; });
}

template <int N>
__global__ __launch_bounds__(WAVE) void k_seg_scan(DevPlan p, const double* __restrict__ summ, double* __restrict__ pre,
                                                   double* __restrict__ suf, double* __restrict__ segtot, int want_back) {
  constexpr int EF = elem_fields(N);
  __shared__ double lds[EF * WAVE];
  const int s = blockIdx.x, lane = threadIdx.x;
  const int32_t nch = p.seg_nch[s];
  const int64_t C = p.n_chunks, S = p.n_seg;
  const int64_t c = p.seg_chunk0[s] + lane;
  const bool valid = lane < nch;
  bool ok = true;
  Elem<N> tmp;
  // The running compositions live in the LDS exchange area, so both operands
  // of a composition are read from LDS and only its result is held in
  // registers.  A lane composes only with lanes of the segment (Kogge-Stone
  // levels d < nch), so the lanes past the segment are never read.
  // inclusive prefix
  if (valid)
    for (int f = 0; f < EF; ++f) lds[f * WAVE + lane] = summ[(int64_t)f * C + c];
  __syncthreads();
#pragma unroll 1
  for (int d = 1; d < nch; d <<= 1) {
    const bool act = lane >= d && valid;
    if (act) compose<N>(ElemLds<N>(lds + lane - d), ElemLds<N>(lds + lane), tmp, ok);
    __syncthreads();
    if (act) lds_put<N>(lds, lane, tmp);
    __syncthreads();
  }
  if (valid)
    for (int f = 0; f < EF; ++f) pre[(int64_t)f * C + c] = lds[f * WAVE + lane];
  if (lane == nch - 1)
    for (int f = 0; f < EF; ++f) segtot[(int64_t)f * S + s] = lds[f * WAVE + lane];
  if (!want_back) return;  // the suffixes serve the backward passes only
  // inclusive suffix
  __syncthreads();
  if (valid)
    for (int f = 0; f < EF; ++f) lds[f * WAVE + lane] = summ[(int64_t)f * C + c];
  __syncthreads();
#pragma unroll 1
  for (int d = 1; d < nch; d <<= 1) {
    const bool act = lane + d < nch;
    if (act) compose<N>(ElemLds<N>(lds + lane), ElemLds<N>(lds + lane + d), tmp, ok);
    __syncthreads();
    if (act) lds_put<N>(lds, lane, tmp);
    __syncthreads();
  }
  if (valid)
    for (int f = 0; f < EF; ++f) suf[(int64_t)f * C + c] = lds[f * WAVE + lane];
  (void)ok;
}

template <int N, int SW>
__global__ __launch_bounds__(WAVE) void k_series_scan(DevPlan p, DevParams pr, const double* __restrict__ segtot,
                                                      double* __restrict__ segstate, double* __restrict__ segfut,
                                                      int want_back) {
  constexpr int EF = elem_fields(N);
  constexpr int NP = N * (N + 1) / 2;
  // xch: the exchange area of the lane scans; blk: each lane's block total;
  // SW lanes per field (the launch guarantees that no more lanes hold a block)
  __shared__ double lds[2 * EF * SW];
  double* const xch = lds;
  double* const blk = lds + EF * SW;
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t S = p.n_seg;
  const int32_t s0 = p.series_seg0[b], ns = p.series_nseg[b];
  if (ns == 0) return;
  const int32_t q = (ns + WAVE - 1) / WAVE;
  const int32_t nl = (ns + q - 1) / q;  // lanes holding a block of segments, each non-empty
  const int32_t lo = min(ns, lane * q), hi = min(ns, lo + q);
  const bool has = lane < nl;
  bool ok = true;
  auto tot = [&](int32_t k) { return [=](int f) { return segtot[(int64_t)f * S + s0 + k]; }; };
  Elem<N> tmp;
  // block total of this lane (a lane reads and writes only its own slots;
  // each segment total is staged in the lane's exchange slot, so that both
  // operands of the composition are LDS views at fixed offsets)
  if (has) {
    for (int f = 0; f < EF; ++f) blk[f * SW + lane] = segtot[(int64_t)f * S + s0 + lo];
    for (int32_t k = lo + 1; k < hi; ++k) {
      for (int f = 0; f < EF; ++f) xch[f * SW + lane] = segtot[(int64_t)f * S + s0 + k];
      compose<N>(ElemLds<N, SW>(blk + lane), ElemLds<N, SW>(xch + lane), tmp, ok);
      lds_put<N>(blk, lane, tmp, SW);
    }
    for (int f = 0; f < EF; ++f) xch[f * SW + lane] = blk[f * SW + lane];
  }
  __syncthreads();
  // inclusive prefix over the lanes holding a block
#pragma unroll 1
  for (int d = 1; d < nl; d <<= 1) {
    const bool act = lane >= d && has;
    if (act) compose<N>(ElemLds<N, SW>(xch + lane - d), ElemLds<N, SW>(xch + lane), tmp, ok);
    __syncthreads();
    if (act) lds_put<N>(xch, lane, tmp, SW);
    __syncthreads();
  }
  // the state entering this lane's block: the prior advanced through the
  // blocks of the lanes before it
  if (has) {
    double m[N], P[NP], mn[N], Pn[NP];
    prior_state<N>(pr, b, m, P);
    if (lane > 0) {
      combine_forward<N>(
          m, P, [&](int f) { return f == sum_c0(N) ? 0.0 : xch[f * SW + lane - 1]; }, mn, Pn, ok);
#pragma unroll
      for (int i = 0; i < N; ++i) m[i] = mn[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) P[i] = Pn[i];
    }
    for (int32_t k = lo; k < hi; ++k) {
#pragma unroll
      for (int i = 0; i < N; ++i) segstate[(int64_t)i * S + s0 + k] = m[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) segstate[(int64_t)(N + i) * S + s0 + k] = P[i];
      combine_forward<N>(m, P, tot(k), mn, Pn, ok);
#pragma unroll
      for (int i = 0; i < N; ++i) m[i] = mn[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) P[i] = Pn[i];
    }
  }
  if (!want_back) return;
  // inclusive suffix over the lanes holding a block; the future after this
  // lane's block is the information of the next lane's suffix
  __syncthreads();
  if (has)
    for (int f = 0; f < EF; ++f) xch[f * SW + lane] = blk[f * SW + lane];
  __syncthreads();
#pragma unroll 1
  for (int d = 1; d < nl; d <<= 1) {
    const bool act = lane + d < nl;
    if (act) compose<N>(ElemLds<N, SW>(xch + lane), ElemLds<N, SW>(xch + lane + d), tmp, ok);
    __syncthreads();
    if (act) lds_put<N>(xch, lane, tmp, SW);
    __syncthreads();
  }
  if (!has) return;
  double Jf[NP], ef[N];
  if (lane + 1 < nl) {
#pragma unroll
    for (int i = 0; i < NP; ++i) Jf[i] = xch[(sum_J(N) + i) * SW + lane + 1];
#pragma unroll
    for (int i = 0; i < N; ++i) ef[i] = xch[(sum_eta(N) + i) * SW + lane + 1];
  } else {
#pragma unroll
    for (int i = 0; i < NP; ++i) Jf[i] = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) ef[i] = 0.0;
  }
  for (int32_t k = hi - 1; k >= lo; --k) {
#pragma unroll
    for (int i = 0; i < NP; ++i) segfut[(int64_t)i * S + s0 + k] = Jf[i];
#pragma unroll
    for (int i = 0; i < N; ++i) segfut[(int64_t)(NP + i) * S + s0 + k] = ef[i];
    double Jn[NP], en[N];
    future_step<N>(tot(k), Jf, ef, Jn, en, ok);
#pragma unroll
    for (int i = 0; i < NP; ++i) Jf[i] = Jn[i];
#pragma unroll
    for (int i = 0; i < N; ++i) ef[i] = en[i];
  }
  (void)ok;
}

template <int N>
__global__ __launch_bounds__(WAVE) void k_seg_fix(DevPlan p, const double* __restrict__ summ,
                                                  const double* __restrict__ pre, const double* __restrict__ suf,
                                                  const double* __restrict__ segstate, const double* __restrict__ segfut,
                                                  double* __restrict__ bstate, double* __restrict__ badj,
                                                  double* __restrict__ bsmooth, double* __restrict__ segll,
                                                  int32_t* __restrict__ segok, int want_back) {
  constexpr int NP = N * (N + 1) / 2;
  const int s = blockIdx.x, lane = threadIdx.x;
  const int32_t nch = p.seg_nch[s];
  const int64_t C = p.n_chunks, S = p.n_seg;
  const int64_t c = p.seg_chunk0[s] + lane;
  const bool valid = lane < nch;
  bool ok = true;
  double ll = 0.0;
  if (valid) {
    double m[N], P[NP], mn[N], Pn[NP];
#pragma unroll
    for (int i = 0; i < N; ++i) m[i] = segstate[(int64_t)i * S + s];
#pragma unroll
    for (int i = 0; i < NP; ++i) P[i] = segstate[(int64_t)(N + i) * S + s];
    if (lane > 0) {
      combine_forward<N>(m, P, [&](int f) { return f == sum_c0(N) ? 0.0 : pre[(int64_t)f * C + c - 1]; }, mn, Pn, ok);
#pragma unroll
      for (int i = 0; i < N; ++i) m[i] = mn[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) P[i] = Pn[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) bstate[(int64_t)i * C + c] = m[i];
#pragma unroll
    for (int i = 0; i < NP; ++i) bstate[(int64_t)(N + i) * C + c] = P[i];
    ll = combine_forward<N>(m, P, [&](int f) { return summ[(int64_t)f * C + c]; }, mn, Pn, ok);
    if (want_back) {
      double Jf[NP], ef[N];
#pragma unroll
      for (int i = 0; i < NP; ++i) Jf[i] = segfut[(int64_t)i * S + s];
#pragma unroll
      for (int i = 0; i < N; ++i) ef[i] = segfut[(int64_t)(NP + i) * S + s];
      if (lane + 1 < nch) {
        double Jn[NP], en[N];
        future_step<N>([&](int f) { return suf[(int64_t)f * C + c + 1]; }, Jf, ef, Jn, en, ok);
#pragma unroll
        for (int i = 0; i < NP; ++i) Jf[i] = Jn[i];
#pragma unroll
        for (int i = 0; i < N; ++i) ef[i] = en[i];
      }
      double mb[N], Pb[NP], Lb[NP];
      boundary_adjoint<N>(mn, Pn, Jf, ef, mb, Pb, bsmooth ? Lb : nullptr, ok);
#pragma unroll
      for (int i = 0; i < N; ++i) badj[(int64_t)i * C + c] = mb[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) badj[(int64_t)(N + i) * C + c] = Pb[i];
      if (bsmooth) {
        // the smoother's adjoint pair (lambda, Lambda) after the chunk
#pragma unroll
        for (int i = 0; i < N; ++i) bsmooth[(int64_t)i * C + c] = mb[i];
#pragma unroll
        for (int i = 0; i < NP; ++i) bsmooth[(int64_t)(N + i) * C + c] = Lb[i];
      }
    }
  }
  const double tot = wave_sum(ll);
  const int bad = __any((!ok || !isfinite(ll)) && valid);
  if (lane == 0) {
    segll[s] = tot;
    segok[s] = bad ? 0 : 1;
  }
}

// one wavefront per series: lane l sums segments l, l + 64, ..., then a
// fixed-order wave reduction (the same result on every run).  The outputs go
// to the call's loglik and status (either may be null); a series whose
// hyperparameters failed validation gets NaN and GP_SSM_EPARAM.
__global__ __launch_bounds__(WAVE) void k_series_finish(DevPlan p, DevParams pr, const double* __restrict__ segll,
                                                        const int32_t* __restrict__ segok,
                                                        const CallArgs* __restrict__ args) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t s0 = p.series_seg0[b], ns = p.series_nseg[b];
  double ll = 0.0;
  bool bad = false;
  for (int32_t k = lane; k < ns; k += WAVE) {
    ll += segll[s0 + k];
    bad = bad || !segok[s0 + k];
  }
  ll = wave_sum(ll) + inst_loglik(pr, b);
  const bool good = !__any(bad) && isfinite(ll);
  if (lane == 0) {
    const bool pbad = pr.bad[b] != 0;
    double* const loglik = args->loglik;
    int32_t* const status = args->status;
    if (loglik) loglik[b] = (good && !pbad) ? ll : __builtin_nan("");
    if (status) status[b] = pbad ? GP_SSM_EPARAM : (good ? 0 : GP_SSM_ENUMERIC);
  }
}

// second scan level: from the state entering each group of segments and the
// information after it (grpstate, grpfut), and the prefixes and suffixes of
// the segment totals within the group (pre2, suf2), the state entering every
// segment and the information after it.  p2 sees groups as segments and
// segments as chunks; one wavefront per group, one segment per lane.
template <int N>
__global__ __launch_bounds__(WAVE) void k_grp_fix(DevPlan p2, const double* __restrict__ pre2,
                                                  const double* __restrict__ suf2, const double* __restrict__ grpstate,
                                                  const double* __restrict__ grpfut, double* __restrict__ segstate,
                                                  double* __restrict__ segfut, int want_back) {
  constexpr int NP = N * (N + 1) / 2;
  const int g = blockIdx.x, lane = threadIdx.x;
  const int32_t n = p2.seg_nch[g];
  if (lane >= n) return;
  const int64_t S = p2.n_chunks, G = p2.n_seg;
  const int64_t s = p2.seg_chunk0[g] + lane;
  bool ok = true;
  double m[N], P[NP];
#pragma unroll
  for (int i = 0; i < N; ++i) m[i] = grpstate[(int64_t)i * G + g];
#pragma unroll
  for (int i = 0; i < NP; ++i) P[i] = grpstate[(int64_t)(N + i) * G + g];
  if (lane > 0) {
    double mn[N], Pn[NP];
    combine_forward<N>(m, P, [&](int f) { return f == sum_c0(N) ? 0.0 : pre2[(int64_t)f * S + s - 1]; }, mn, Pn, ok);
#pragma unroll
    for (int i = 0; i < N; ++i) m[i] = mn[i];
#pragma unroll
    for (int i = 0; i < NP; ++i) P[i] = Pn[i];
  }
#pragma unroll
  for (int i = 0; i < N; ++i) segstate[(int64_t)i * S + s] = m[i];
#pragma unroll
  for (int i = 0; i < NP; ++i) segstate[(int64_t)(N + i) * S + s] = P[i];
  if (!want_back) return;
  double Jf[NP], ef[N];
#pragma unroll
  for (int i = 0; i < NP; ++i) Jf[i] = grpfut[(int64_t)i * G + g];
#pragma unroll
  for (int i = 0; i < N; ++i) ef[i] = grpfut[(int64_t)(NP + i) * G + g];
  if (lane + 1 < n) {
    double Jn[NP], en[N];
    future_step<N>([&](int f) { return suf2[(int64_t)f * S + s + 1]; }, Jf, ef, Jn, en, ok);
#pragma unroll
    for (int i = 0; i < NP; ++i) Jf[i] = Jn[i];
#pragma unroll
    for (int i = 0; i < N; ++i) ef[i] = en[i];
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) segfut[(int64_t)i * S + s] = Jf[i];
#pragma unroll
  for (int i = 0; i < N; ++i) segfut[(int64_t)(NP + i) * S + s] = ef[i];
  (void)ok;  // a failed combination leaves non-finite states, caught by the segment's check
}

template <int N>
void run_levels(hipStream_t st, const DevPlan& p, const DevParams& pr, const ScanWork& w, int back);

template <int N>
void run_scan_n(hipStream_t st, const DevPlan& p, const DevParams& pr, const ScanWork& w, const CallArgs* args,
                int back) {
  // series without measurements have no segment; k_series_finish still gives
  // them log-likelihood 0 and status 0
  if (p.n_seg > 0) run_levels<N>(st, p, pr, w, back);
  prof_begin("k_series_finish", st);
  hipLaunchKernelGGL(k_series_finish, dim3((unsigned)p.n_series), dim3(WAVE), 0, st, p, pr, w.segll, w.segok, args);
  prof_end("k_series_finish", st);
}

// k_series_scan with LDS for 16 lanes when no series has more than 16
// segments (the common case of many series): its exchange areas then take
// 23 KB instead of 93 KB at N = 6, and four workgroups fit in a CU instead
// of one
template <int N>
void launch_series_scan(hipStream_t st, const DevPlan& p, const DevParams& pr, const double* tot, double* state,
                        double* fut, int back) {
  prof_begin("k_series_scan", st);
  if (p.max_series_nseg <= 16)
    hipLaunchKernelGGL((k_series_scan<N, 16>), dim3((unsigned)p.n_series), dim3(WAVE), 0, st, p, pr, tot, state, fut,
                       back);
  else
    hipLaunchKernelGGL((k_series_scan<N, WAVE>), dim3((unsigned)p.n_series), dim3(WAVE), 0, st, p, pr, tot, state,
                       fut, back);
  prof_end("k_series_scan", st);
}

template <int N>
void run_levels(hipStream_t st, const DevPlan& p, const DevParams& pr, const ScanWork& w, int back) {
  prof_begin("k_seg_scan", st);
  hipLaunchKernelGGL(k_seg_scan<N>, dim3(p.n_seg), dim3(WAVE), 0, st, p, w.summ, w.pre, w.suf, w.segtot, back);
  prof_end("k_seg_scan", st);
  if (w.p2) {
    // series with more than WAVE segments: the segment totals are scanned in
    // groups of WAVE like the chunk summaries, the group totals per series
    const DevPlan& p2 = *w.p2;
    prof_begin("k_grp_scan", st);
    hipLaunchKernelGGL(k_seg_scan<N>, dim3(p2.n_seg), dim3(WAVE), 0, st, p2, w.segtot, w.pre2, w.suf2, w.grptot,
                       back);
    prof_end("k_grp_scan", st);
    launch_series_scan<N>(st, p2, pr, w.grptot, w.grpstate, w.grpfut, back);
    prof_begin("k_grp_fix", st);
    hipLaunchKernelGGL(k_grp_fix<N>, dim3(p2.n_seg), dim3(WAVE), 0, st, p2, w.pre2, w.suf2, w.grpstate, w.grpfut,
                       w.segstate, w.segfut, back);
    prof_end("k_grp_fix", st);
  } else {
    launch_series_scan<N>(st, p, pr, w.segtot, w.segstate, w.segfut, back);
  }
  prof_begin("k_seg_fix", st);
  hipLaunchKernelGGL(k_seg_fix<N>, dim3(p.n_seg), dim3(WAVE), 0, st, p, w.summ, w.pre, w.suf, w.segstate, w.segfut,
                     w.bstate, w.badj, w.bsmooth, w.segll, w.segok, back);
  prof_end("k_seg_fix", st);
}

}  // namespace

void run_scan(int M, hipStream_t st, const DevPlan& p, const DevParams& pr, const ScanWork& w, const CallArgs* args,
              int back) {
  switch (M) {
    case 1: run_scan_n<2>(st, p, pr, w, args, back); break;
    case 2: run_scan_n<4>(st, p, pr, w, args, back); break;
    case 3: run_scan_n<6>(st, p, pr, w, args, back); break;
    default: run_scan_n<8>(st, p, pr, w, args, back); break;
  }
}

}  // namespace gpssm
