// Kernels for one number of SHO terms (GPSSM_M, set by the including file)
// and every slot count J = 1..MAX_SLOTS.
//
// Work mapping: one wavefront per segment (up to 64 consecutive chunks of one
// series, one chunk per lane).  All lanes of a wavefront share the series, so
// its hyperparameters and Taylor tables are wavefront-uniform (scalar loads);
// events are stored interleaved so each step of the wavefront reads 64
// consecutive values.  Lanes whose chunk is shorter than the segment's
// longest read padding events (zero step, no measurement), which leave the
// state unchanged.
#pragma once

#include "kernels.h"
#include "plan.h"

#ifndef GPSSM_M
#error "define GPSSM_M before including kernels_impl.h"
#endif

namespace gpssm {
namespace GPSSM_NS {

constexpr int M = GPSSM_M;

template <class Dm>
__device__ __forceinline__ void load_terms(const DevParams& pr, int64_t b, TermConst* tc) {
#pragma unroll
  for (int t = 0; t < Dm::M; ++t) tc[t] = pr.tc[b * Dm::M + t];
}

template <class Dm>
__device__ __forceinline__ Obs load_event(const DevPlan& p, int64_t e, double jit2, double& dt, uint32_t& info) {
  dt = p.dt[e];
  info = p.info[e];
  return make_obs<Dm>(info, p.y[e], p.r[e], p.invd[e], jit2);
}

// one plain filter step; returns the log-likelihood term
template <class Dm>
__device__ __forceinline__ double plain_step(double* m, double* P, const TermQ* tq, uint32_t info, const Obs& o) {
  constexpr int D = Dm::D;
  const uint32_t open = ev_open(info);
  predict_mean<Dm>(m, tq, open);
  predict_cov<Dm>(P, tq, open);
  double u[D];
  obs_gain<Dm>(P, o, u);
  const double S = obs_dot<Dm>(u, o) + o.R;
  const double iS = 1.0 / S;
  const double v = o.y - obs_dot<Dm>(m, o);
  const double viS = v * iS;
#pragma unroll
  for (int i = 0; i < D; ++i) m[i] = fma(u[i], viS, m[i]);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double ui = u[i] * iS;
#pragma unroll
    for (int j = i; j < D; ++j) P[sidx(i, j, D)] = fma(-ui, u[j], P[sidx(i, j, D)]);
  }
  close_slot<Dm>(m, P, info);
  return o.has ? -0.5 * (LOG_2PI + log(S) + v * viS) : 0.0;
}

// ---------------------------------------------------------------------------
// chunk summaries (conditional filter), one chunk per lane
// ---------------------------------------------------------------------------
template <int J>
__global__ __launch_bounds__(WAVE) void k_summaries(DevPlan p, DevParams pr, double* __restrict__ summ) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, NXP = Dm::NXP;
  const int seg = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t b = p.seg_series[seg];
  const int32_t nch = p.seg_nch[seg], L = p.seg_len[seg];
  const int64_t ev0 = p.seg_ev0[seg];
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  const double* coef = pr.coef + b * M * 2 * NCOEF;
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  CondState<Dm> st;
  st.init();
  for (int32_t k = 0; k < L; ++k) {
    const int64_t e = ev0 + (int64_t)k * WAVE + lane;
    double dt;
    uint32_t info;
    const Obs o = load_event<Dm>(p, e, jit2, dt, info);
    TermQ tq[M];
    discretise<M>(tc, coef, dt, tq);
    st.step(tq, info, o);
  }
  if (lane < nch) {
    const int64_t c = p.seg_chunk0[seg] + lane;
    const int64_t C = p.n_chunks;
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int k = 0; k < NX; ++k) summ[(sum_A(NX) + i * NX + k) * C + c] = st.S[i * NX + k];
#pragma unroll
    for (int i = 0; i < NX; ++i) summ[(sum_b(NX) + i) * C + c] = st.mu[i];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int k = i; k < NX; ++k) summ[(sum_C(NX) + sidx(i, k, NX)) * C + c] = st.P[sidx(i, k, Dm::D)];
#pragma unroll
    for (int i = 0; i < NX; ++i) summ[(sum_eta(NX) + i) * C + c] = st.eta[i];
#pragma unroll
    for (int i = 0; i < NXP; ++i) summ[(sum_J(NX) + i) * C + c] = st.Jm[i];
    summ[sum_c0(NX) * C + c] = st.c0;
  }
}

// ---------------------------------------------------------------------------
// gradient: plain forward from the boundary state (storing the state before
// every event), then the adjoint backward from the boundary adjoint
// ---------------------------------------------------------------------------
template <int J>
__global__ __launch_bounds__(WAVE) void k_adjoint(DevPlan p, DevParams pr, const double* __restrict__ bstate,
                                                  const double* __restrict__ badj, double* __restrict__ rec,
                                                  double* __restrict__ gpart, double* __restrict__ llchk) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, D = Dm::D, NP = Dm::NP, NXP = Dm::NXP;
  constexpr int F = rec_fields<Dm>();
  const int seg = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t b = p.seg_series[seg];
  const int32_t nch = p.seg_nch[seg], L = p.seg_len[seg];
  const int64_t ev0 = p.seg_ev0[seg];
  const bool active = lane < nch;
  const int64_t C = p.n_chunks;
  const int64_t c = p.seg_chunk0[seg] + (active ? lane : 0);
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  const double* coef = pr.coef + b * M * 2 * NCOEF;
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  double* rb = rec + ev0 * F;

  double m[D], P[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) m[i] = (i < NX && active) ? bstate[i * C + c] : 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) P[sidx(i, j, D)] = (j < NX && active) ? bstate[(NX + sidx(i, j, NX)) * C + c] : 0.0;

  double ll = 0.0;
  for (int32_t k = 0; k < L; ++k) {
    const int64_t e = ev0 + (int64_t)k * WAVE + lane;
#pragma unroll
    for (int f = 0; f < D; ++f) rb[((int64_t)k * F + f) * WAVE + lane] = m[f];
#pragma unroll
    for (int f = 0; f < NP; ++f) rb[((int64_t)k * F + D + f) * WAVE + lane] = P[f];
    double dt;
    uint32_t info;
    const Obs o = load_event<Dm>(p, e, jit2, dt, info);
    TermQ tq[M];
    discretise<M>(tc, coef, dt, tq);
    ll += plain_step<Dm>(m, P, tq, info, o);
  }
  if (active && llchk) llchk[c] = ll;

  double mb[D], Pb[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) mb[i] = (i < NX && active) ? badj[i * C + c] : 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) Pb[sidx(i, j, D)] = (j < NX && active) ? badj[(NX + sidx(i, j, NX)) * C + c] : 0.0;
  GradAcc<M> acc;
  acc.init();
  for (int32_t k = L - 1; k >= 0; --k) {
    const int64_t e = ev0 + (int64_t)k * WAVE + lane;
#pragma unroll
    for (int f = 0; f < D; ++f) m[f] = rb[((int64_t)k * F + f) * WAVE + lane];
#pragma unroll
    for (int f = 0; f < NP; ++f) P[f] = rb[((int64_t)k * F + D + f) * WAVE + lane];
    double dt;
    uint32_t info;
    const Obs o = load_event<Dm>(p, e, jit2, dt, info);
    adjoint_step<Dm>(m, P, mb, Pb, tc, coef, dt, info, o, jit, acc);
  }
  if (active) {
    if (p.chunk_first[c]) {
      // prior of the SHO states: sigma_t^2 I in scaled coordinates
#pragma unroll
      for (int t = 0; t < M; ++t)
        acc.s[t] += 2.0 * tc[t].sigma * (Pb[sidx(2 * t, 2 * t, D)] + Pb[sidx(2 * t + 1, 2 * t + 1, D)]);
    }
#pragma unroll
    for (int t = 0; t < M; ++t) {
      gpart[(0 * M + t) * C + c] = acc.s[t];
      gpart[(1 * M + t) * C + c] = acc.w[t];
      gpart[(2 * M + t) * C + c] = acc.q[t];
    }
    gpart[(3 * M) * C + c] = acc.jit;
  }
  (void)NXP;
}

// ---------------------------------------------------------------------------
// plain sequential filter of one series (one lane): the reference launch
// ---------------------------------------------------------------------------
template <int J>
__global__ __launch_bounds__(WAVE) void k_plain(DevPlan p, DevParams pr, int64_t b, double* __restrict__ loglik) {
  using Dm = Dims<M, J>;
  constexpr int D = Dm::D, NP = Dm::NP;
  if (threadIdx.x != 0) return;
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  const double* coef = pr.coef + b * M * 2 * NCOEF;
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  double m[D], P[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) m[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NP; ++i) P[i] = 0.0;
#pragma unroll
  for (int t = 0; t < M; ++t) {
    P[sidx(2 * t, 2 * t, D)] = tc[t].sigma * tc[t].sigma;
    P[sidx(2 * t + 1, 2 * t + 1, D)] = tc[t].sigma * tc[t].sigma;
  }
  double ll = 0.0;
  const int32_t c0 = p.series_chunk0[b], nch = p.series_nch[b];
  for (int32_t q = 0; q < nch; ++q) {
    const int32_t c = c0 + q;
    const int32_t s = p.chunk_seg[c];
    const int32_t l = c - p.seg_chunk0[s];
    const int64_t ev0 = p.seg_ev0[s];
    const int32_t len = p.chunk_len[c];
    for (int32_t k = 0; k < len; ++k) {
      const int64_t e = ev0 + (int64_t)k * WAVE + l;
      double dt;
      uint32_t info;
      const Obs o = load_event<Dm>(p, e, jit2, dt, info);
      TermQ tq[M];
      discretise<M>(tc, coef, dt, tq);
      ll += plain_step<Dm>(m, P, tq, info, o);
    }
  }
  loglik[b] = ll;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int J>
void launch_summaries(const Launch& L, const DevPlan& p, const DevParams& pr, double* summ) {
  if (p.n_seg == 0) return;
  prof_begin("k_summaries", L.stream);
  hipLaunchKernelGGL(k_summaries<J>, dim3(p.n_seg), dim3(WAVE), 0, L.stream, p, pr, summ);
  prof_end("k_summaries", L.stream);
}
template <int J>
void launch_adjoint(const Launch& L, const DevPlan& p, const DevParams& pr, const double* bstate, const double* badj,
                    double* rec, double* gpart, double* llchk) {
  if (p.n_seg == 0) return;
  prof_begin("k_adjoint", L.stream);
  hipLaunchKernelGGL(k_adjoint<J>, dim3(p.n_seg), dim3(WAVE), 0, L.stream, p, pr, bstate, badj, rec, gpart, llchk);
  prof_end("k_adjoint", L.stream);
}
template <int J>
void launch_plain(const Launch& L, const DevPlan& p, const DevParams& pr, int64_t series, double* loglik) {
  prof_begin("k_plain", L.stream);
  hipLaunchKernelGGL(k_plain<J>, dim3(1), dim3(WAVE), 0, L.stream, p, pr, series, loglik);
  prof_end("k_plain", L.stream);
}

template <int J>
KernelSet make_set() {
  KernelSet k;
  k.summaries = &launch_summaries<J>;
  k.adjoint = &launch_adjoint<J>;
  k.plain = &launch_plain<J>;
  k.smooth = nullptr;
  return k;
}

}  // namespace GPSSM_NS
}  // namespace gpssm
