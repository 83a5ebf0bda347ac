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

// the series' Taylor tables of all terms, staged in LDS by the workgroup's
// single wavefront: the value tables only (term stride NCOEF), or with DUAL
// the values followed by the beta-derivatives (term stride 2 NCOEF)
template <class Dm, bool DUAL>
__device__ __forceinline__ const double* stage_coef(const DevParams& pr, int64_t b, double* lds) {
  const double* g = pr.coef + b * Dm::M * 2 * NCOEF;
  constexpr int TS = DUAL ? 2 * NCOEF : NCOEF;
  for (int i = threadIdx.x; i < Dm::M * TS; i += WAVE) {
    const int t = i / TS, j = i - t * TS;
    lds[i] = g[t * 2 * NCOEF + j];
  }
  __syncthreads();
  return lds;
}

// the raw fields of one event, loaded one step ahead of their use
struct EvRaw {
  double dt, y, r, invd;
  uint32_t info;
};
__device__ __forceinline__ EvRaw fetch_event(const DevPlan& p, int64_t e) {
  EvRaw v;
  v.dt = p.dt[e];
  v.y = p.y[e];
  v.r = p.r[e];
  v.invd = p.invd[e];
  v.info = p.info[e];
  return v;
}

// one plain filter step; returns the log-likelihood term (0 unless LL)
template <class Dm, bool LL = true>
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
  if constexpr (LL)
    return o.has ? -0.5 * (LOG_2PI + log(S) + v * viS) : 0.0;
  else
    return 0.0;
}

// ---------------------------------------------------------------------------
// chunk summaries (conditional filter), one chunk per lane
// ---------------------------------------------------------------------------
template <int J>
__global__ __launch_bounds__(WAVE) void k_summaries(DevPlan p, DevParams pr, double* __restrict__ summ) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, NXP = Dm::NXP;
  const int seg = p.seg_order ? p.seg_order[blockIdx.x] : (int)blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t b = p.seg_series[seg];
  const int32_t nch = p.seg_nch[seg], L = p.seg_len[seg];
  const int64_t ev0 = p.seg_ev0[seg];
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  __shared__ double lcoef[M * NCOEF];
  const double* coef = stage_coef<Dm, false>(pr, b, lcoef);
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  // LDS for the sensitivity block S when it is larger than at M = 3, J = 3
  // (where it stays in registers without spills) and for the information
  // accumulators (J, eta, c0), as long as four workgroups still fit in a CU
  using St0 = CondState<Dm, false, false>;
  constexpr int CB = 8 * M * NCOEF, SB = 8 * Dm::D * NX * WAVE, IB = 8 * St0::NINFO * WAVE;
  constexpr bool SL = Dm::D * NX > 54 && CB + SB <= 40960;
  constexpr bool IL = CB + (SL ? SB : 0) + IB <= 40960;
  __shared__ double lS[SL ? Dm::D * NX * WAVE : 1];
  __shared__ double lI[IL ? St0::NINFO * WAVE : 1];
  CondState<Dm, SL, IL> st;
  st.Sl = LaneLds{lS + lane};
  st.Il = LaneLds{lI + lane};
  st.init();
  EvRaw nxt = fetch_event(p, ev0 + lane);
  for (int32_t k = 0; k < L; ++k) {
    const EvRaw cur = nxt;
    if (k + 1 < L) nxt = fetch_event(p, ev0 + (int64_t)(k + 1) * WAVE + lane);
    const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2);
    TermQ tq[M];
    discretise<M>(tc, coef, cur.dt, tq);
    st.step(tq, cur.info, o);
  }
  if (lane < nch) {
    const int64_t c = p.seg_chunk0[seg] + lane;
    const int64_t C = p.n_chunks;
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int k = 0; k < NX; ++k) summ[(sum_A(NX) + i * NX + k) * C + c] = st.S(i * NX + k);
#pragma unroll
    for (int i = 0; i < NX; ++i) summ[(sum_b(NX) + i) * C + c] = st.mu[i];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int k = i; k < NX; ++k) summ[(sum_C(NX) + sidx(i, k, NX)) * C + c] = st.P[sidx(i, k, Dm::D)];
#pragma unroll
    for (int i = 0; i < NX; ++i) summ[(sum_eta(NX) + i) * C + c] = st.eta(i);
#pragma unroll
    for (int i = 0; i < NXP; ++i) summ[(sum_J(NX) + i) * C + c] = st.Jm(i);
    summ[sum_c0(NX) * C + c] = st.c0();
  }
}

// ---------------------------------------------------------------------------
// gradient: plain forward from the boundary state (storing the state before
// every event), then the adjoint backward from the boundary adjoint
// ---------------------------------------------------------------------------
template <int J>
__global__ __launch_bounds__(WAVE) void k_adjoint(DevPlan p, DevParams pr, const double* __restrict__ bstate,
                                                  const double* __restrict__ badj, double* __restrict__ rec,
                                                  double* __restrict__ gpart) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, D = Dm::D, NP = Dm::NP, NXP = Dm::NXP;
  constexpr int F = rec_fields<Dm>();
  const int seg = p.seg_order ? p.seg_order[blockIdx.x] : (int)blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t b = p.seg_series[seg];
  const int32_t nch = p.seg_nch[seg], L = p.seg_len[seg];
  const int64_t ev0 = p.seg_ev0[seg];
  const bool active = lane < nch;
  const int64_t C = p.n_chunks;
  const int64_t c = p.seg_chunk0[seg] + (active ? lane : 0);
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  __shared__ double lcoef[M * 2 * NCOEF];
  const double* coef = stage_coef<Dm, true>(pr, b, lcoef);
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

  EvRaw nxt = fetch_event(p, ev0 + lane);
  for (int32_t k = 0; k < L; ++k) {
    const EvRaw cur = nxt;
    if (k + 1 < L) nxt = fetch_event(p, ev0 + (int64_t)(k + 1) * WAVE + lane);
#pragma unroll
    for (int f = 0; f < D; ++f) rb[((int64_t)k * F + f) * WAVE + lane] = m[f];
#pragma unroll
    for (int f = 0; f < NP; ++f) rb[((int64_t)k * F + D + f) * WAVE + lane] = P[f];
    const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2);
    TermQ tq[M];
    discretise<M, DiscGrad, 2 * NCOEF>(tc, coef, cur.dt, tq);
    plain_step<Dm, false>(m, P, tq, cur.info, o);
  }

  double mb[D], Pb[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) mb[i] = (i < NX && active) ? badj[i * C + c] : 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) Pb[sidx(i, j, D)] = (j < NX && active) ? badj[(NX + sidx(i, j, NX)) * C + c] : 0.0;
  __shared__ double lacc[(3 * M + 1) * WAVE];
  const GradAcc<M> acc{lacc + lane};
  acc.init();
  nxt = fetch_event(p, ev0 + (int64_t)(L - 1) * WAVE + lane);
  for (int32_t k = L - 1; k >= 0; --k) {
    const EvRaw cur = nxt;
    if (k > 0) nxt = fetch_event(p, ev0 + (int64_t)(k - 1) * WAVE + lane);
#pragma unroll
    for (int f = 0; f < D; ++f) m[f] = rb[((int64_t)k * F + f) * WAVE + lane];
#pragma unroll
    for (int f = 0; f < NP; ++f) P[f] = rb[((int64_t)k * F + D + f) * WAVE + lane];
    const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2);
    adjoint_step<Dm>(m, P, mb, Pb, tc, coef, cur.dt, cur.info, o, jit, acc);
  }
  if (active && p.chunk_first[c]) {
    // prior of the SHO states: sigma_t^2 I in scaled coordinates
#pragma unroll
    for (int t = 0; t < M; ++t)
      acc.s(t) += 2.0 * tc[t].sigma * (Pb[sidx(2 * t, 2 * t, D)] + Pb[sidx(2 * t + 1, 2 * t + 1, D)]);
  }
  // sum over the segment's lanes (one series), one partial per segment
  const int64_t S = p.n_seg;
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const double a0 = wave_sum(active ? acc.s(t) : 0.0);
    const double a1 = wave_sum(active ? acc.w(t) : 0.0);
    const double a2 = wave_sum(active ? acc.q(t) : 0.0);
    if (lane == 0) {
      gpart[(0 * M + t) * S + seg] = a0;
      gpart[(1 * M + t) * S + seg] = a1;
      gpart[(2 * M + t) * S + seg] = a2;
    }
  }
  const double aj = wave_sum(active ? acc.jit() : 0.0);
  if (lane == 0) gpart[(3 * M) * S + seg] = aj;
  (void)NXP;
  (void)C;
}

// ---------------------------------------------------------------------------
// plain sequential filter of one series (one lane): the reference launch
// ---------------------------------------------------------------------------
template <int J>
__global__ __launch_bounds__(WAVE) void k_plain(DevPlan p, DevParams pr, int64_t b, double* __restrict__ loglik) {
  using Dm = Dims<M, J>;
  constexpr int D = Dm::D, NP = Dm::NP;
  __shared__ double lcoef[M * NCOEF];
  const double* coef = stage_coef<Dm, false>(pr, b, lcoef);
  if (threadIdx.x != 0) return;
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
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
// smoother: forward pass storing the filtered state after each event's
// update (before its integrator is closed), then the RTS sweep backward from
// the smoothed state at the chunk's end, with the exposure-averaged
// posterior at every measurement and the latent posterior at the test times
// that fall in the chunk (Algorithm 1)
// ---------------------------------------------------------------------------
template <class Dm>
__device__ __forceinline__ void latent_out(const double* m, const double* P, double& mean, double& var) {
  double mu = 0.0, v = 0.0;
#pragma unroll
  for (int t = 0; t < Dm::M; ++t) {
    mu += m[2 * t];
#pragma unroll
    for (int u = 0; u < Dm::M; ++u) v += P[sidx(2 * t, 2 * u, Dm::D)];
  }
  mean = mu;
  var = v;
}

// posterior of the latent process at a test time between a filtered state
// (prev, already closed) and the smoothed next event: predict over a, then one
// RTS step back from the next event over b (open: integrators open over both)
template <class Dm>
__device__ __forceinline__ void interp_test(const double* pm, const double* pP, const TermConst* tc, const double* coef,
                                            double a, double b, uint32_t open, const double* ms, const double* Ps,
                                            double& mean, double& var, bool& ok) {
  constexpr int D = Dm::D, NP = Dm::NP;
  if (b == 0.0) {
    latent_out<Dm>(ms, Ps, mean, var);
    return;
  }
  double m[D], P[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) m[i] = pm[i];
#pragma unroll
  for (int i = 0; i < NP; ++i) P[i] = pP[i];
  TermQ tq[Dm::M];
  discretise<Dm::M>(tc, coef, a, tq);
  predict_mean<Dm>(m, tq, open);
  predict_cov<Dm>(P, tq, open);
  discretise<Dm::M>(tc, coef, b, tq);
  ok = rts_step<Dm>(m, P, tq, open, 0u, ms, Ps) && ok;
  latent_out<Dm>(m, P, mean, var);
}

template <int J>
__global__ __launch_bounds__(WAVE) void k_smooth(DevPlan p, DevParams pr, const double* __restrict__ bstate,
                                                 const double* __restrict__ bsmooth, double* __restrict__ rec,
                                                 DevTests ts, double* __restrict__ mean_test,
                                                 double* __restrict__ var_test, double* __restrict__ mean_data,
                                                 double* __restrict__ var_data) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, D = Dm::D, NP = Dm::NP;
  constexpr int F = rec_fields<Dm>();
  const int seg = p.seg_order ? p.seg_order[blockIdx.x] : (int)blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t b = p.seg_series[seg];
  const int32_t nch = p.seg_nch[seg], L = p.seg_len[seg];
  const int64_t ev0 = p.seg_ev0[seg];
  const bool active = lane < nch;
  const int64_t C = p.n_chunks;
  const int64_t c = p.seg_chunk0[seg] + (active ? lane : 0);
  const int32_t len = active ? p.chunk_len[c] : 0;
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  __shared__ double lcoef[M * NCOEF];
  const double* coef = stage_coef<Dm, false>(pr, b, lcoef);
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  double* rb = rec + ev0 * F;
  auto ev = [&](int32_t k) { return ev0 + (int64_t)k * WAVE + lane; };

  // forward: store the state after each event's update, before closing
  double m[D], P[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) m[i] = (i < NX && active) ? bstate[i * C + c] : 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) P[sidx(i, j, D)] = (j < NX && active) ? bstate[(NX + sidx(i, j, NX)) * C + c] : 0.0;
  for (int32_t k = 0; k < len; ++k) {
    const EvRaw cur = fetch_event(p, ev(k));
    const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2);
    TermQ tq[M];
    discretise<M>(tc, coef, cur.dt, tq);
    const uint32_t open = ev_open(cur.info);
    predict_mean<Dm>(m, tq, open);
    predict_cov<Dm>(P, tq, open);
    double u[D];
    obs_gain<Dm>(P, o, u);
    const double S = obs_dot<Dm>(u, o) + o.R;
    const double iS = 1.0 / S;
    const double viS = (o.y - obs_dot<Dm>(m, o)) * iS;
#pragma unroll
    for (int i = 0; i < D; ++i) m[i] = fma(u[i], viS, m[i]);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double ui = u[i] * iS;
#pragma unroll
      for (int j = i; j < D; ++j) P[sidx(i, j, D)] = fma(-ui, u[j], P[sidx(i, j, D)]);
    }
#pragma unroll
    for (int f = 0; f < D; ++f) rb[((int64_t)k * F + f) * WAVE + lane] = m[f];
#pragma unroll
    for (int f = 0; f < NP; ++f) rb[((int64_t)k * F + D + f) * WAVE + lane] = P[f];
    close_slot<Dm>(m, P, cur.info);
  }

  // backward
  bool ok = true;
  double ms[D], Ps[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) ms[i] = (i < NX && active) ? bsmooth[i * C + c] : 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) Ps[sidx(i, j, D)] = (j < NX && active) ? bsmooth[(NX + sidx(i, j, NX)) * C + c] : 0.0;
  const int64_t tlo = active ? ts.chunk_t0[c] : 0;
  int64_t tp = active ? ts.chunk_t0[c + 1] - 1 : -1;
  const bool last_chunk = active && (c + 1 == (int64_t)p.series_chunk0[b] + p.series_nch[b]);
  double t_next = 0.0;
  uint32_t open_next = 0u;
  double dt_next = 0.0;
  for (int32_t k = len - 1; k >= 0; --k) {
    const EvRaw cur = fetch_event(p, ev(k));
    const double tk = p.t[ev(k)];
#pragma unroll
    for (int f = 0; f < D; ++f) m[f] = rb[((int64_t)k * F + f) * WAVE + lane];
#pragma unroll
    for (int f = 0; f < NP; ++f) P[f] = rb[((int64_t)k * F + D + f) * WAVE + lane];
    // the filtered state after this event, closed
    double mc[D], Pc[NP];
#pragma unroll
    for (int i = 0; i < D; ++i) mc[i] = m[i];
#pragma unroll
    for (int i = 0; i < NP; ++i) Pc[i] = P[i];
    close_slot<Dm>(mc, Pc, cur.info);
    // test times after this event
    while (tp >= tlo && ts.t[tp] > tk) {
      const double tq = ts.t[tp];
      double mean, var;
      if (k == len - 1) {
        // after the last event of the series: prediction from the final state
        double mm[D], PP[NP];
#pragma unroll
        for (int i = 0; i < D; ++i) mm[i] = mc[i];
#pragma unroll
        for (int i = 0; i < NP; ++i) PP[i] = Pc[i];
        TermQ tqq[M];
        discretise<M>(tc, coef, tq - tk, tqq);
        predict_mean<Dm>(mm, tqq, 0u);
        predict_cov<Dm>(PP, tqq, 0u);
        latent_out<Dm>(mm, PP, mean, var);
      } else {
        interp_test<Dm>(mc, Pc, tc, coef, tq - tk, t_next - tq, open_next, ms, Ps, mean, var, ok);
      }
      const int64_t o = ts.out_index[tp];
      mean_test[o] = mean;
      var_test[o] = var;
      --tp;
    }
    (void)last_chunk;
    // RTS step back from the next state (the boundary after the last event)
    {
      TermQ tq[M];
      discretise<M>(tc, coef, (k == len - 1) ? 0.0 : dt_next, tq);
      const uint32_t zmask = (ev_kind(cur.info) == EV_END) ? (1u << ev_slot(cur.info)) : 0u;
      ok = rts_step<Dm>(m, P, tq, (k == len - 1) ? 0u : open_next, zmask, ms, Ps) && ok;
    }
    // posterior at the measurement
    const uint32_t kind = ev_kind(cur.info);
    if (kind == EV_END || kind == EV_INSTANT) {
      const int64_t n = p.meas[ev(k)];
      double mean = 0.0, var = 0.0;
      if (kind == EV_END) {
        const uint32_t j = ev_slot(cur.info);
#pragma unroll
        for (int jj = 0; jj < J; ++jj)
          if ((uint32_t)jj == j) {
            mean = m[NX + jj] * cur.invd;
            var = P[sidx(NX + jj, NX + jj, D)] * cur.invd * cur.invd;
          }
      } else {
        latent_out<Dm>(m, P, mean, var);
      }
      if (mean_data) mean_data[n] = ok ? mean : __builtin_nan("");
      if (var_data) var_data[n] = ok ? var : __builtin_nan("");
    }
#pragma unroll
    for (int i = 0; i < D; ++i) ms[i] = m[i];
#pragma unroll
    for (int i = 0; i < NP; ++i) Ps[i] = P[i];
    t_next = tk;
    open_next = ev_open(cur.info);
    dt_next = cur.dt;
  }
  // test times before the chunk's first event: from the boundary state (or,
  // before the series' first event, from the prior at the test time)
  if (active && tp >= tlo) {
    const bool first = p.chunk_first[c];
    double pm[D], pP[NP];
#pragma unroll
    for (int i = 0; i < D; ++i) pm[i] = (i < NX && !first) ? bstate[i * C + c] : 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) pP[sidx(i, j, D)] = (j < NX && !first) ? bstate[(NX + sidx(i, j, NX)) * C + c] : 0.0;
    if (first) {
#pragma unroll
      for (int t = 0; t < M; ++t) {
        pP[sidx(2 * t, 2 * t, D)] = tc[t].sigma * tc[t].sigma;
        pP[sidx(2 * t + 1, 2 * t + 1, D)] = tc[t].sigma * tc[t].sigma;
      }
    }
    const double tprev = ts.chunk_tprev[c];
    while (tp >= tlo) {
      const double tq = ts.t[tp];
      double mean, var;
      interp_test<Dm>(pm, pP, tc, coef, first ? 0.0 : tq - tprev, t_next - tq, open_next, ms, Ps, mean, var, ok);
      const int64_t o = ts.out_index[tp];
      mean_test[o] = mean;
      var_test[o] = var;
      --tp;
    }
  }
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
                    double* rec, double* gpart) {
  if (p.n_seg == 0) return;
  prof_begin("k_adjoint", L.stream);
  hipLaunchKernelGGL(k_adjoint<J>, dim3(p.n_seg), dim3(WAVE), 0, L.stream, p, pr, bstate, badj, rec, gpart);
  prof_end("k_adjoint", L.stream);
}
template <int J>
void launch_plain(const Launch& L, const DevPlan& p, const DevParams& pr, int64_t series, double* loglik) {
  prof_begin("k_plain", L.stream);
  hipLaunchKernelGGL(k_plain<J>, dim3(1), dim3(WAVE), 0, L.stream, p, pr, series, loglik);
  prof_end("k_plain", L.stream);
}

template <int J>
void launch_smooth(const Launch& L, const DevPlan& p, const DevParams& pr, const double* bstate, const double* bsmooth,
                   double* rec, const DevTests& tests, double* mean_test, double* var_test, double* mean_data,
                   double* var_data) {
  if (p.n_seg == 0) return;
  prof_begin("k_smooth", L.stream);
  hipLaunchKernelGGL(k_smooth<J>, dim3(p.n_seg), dim3(WAVE), 0, L.stream, p, pr, bstate, bsmooth, rec, tests,
                     mean_test, var_test, mean_data, var_data);
  prof_end("k_smooth", L.stream);
}

template <int J>
KernelSet make_set() {
  KernelSet k;
  k.summaries = &launch_summaries<J>;
  k.adjoint = &launch_adjoint<J>;
  k.plain = &launch_plain<J>;
  k.smooth = &launch_smooth<J>;
  return k;
}

}  // namespace GPSSM_NS
}  // namespace gpssm
