// Kernels for one number of SHO terms (GPSSM_M, set by the including file)
// and every slot count J = 1..MAX_SLOTS.  The template argument FT selects
// the optional features compiled in: bit 0 real exponential terms, bit 1
// instrument tables; without them their branches fold away and the register
// allocation of the plain model is untouched.
//
// Work mapping: one wavefront per work wave (up to 64 chunks of one series of
// similar length, one chunk per lane, found through the plan's wv_chunk).
// All lanes of a wavefront share the series, so its hyperparameters and
// Taylor tables are wavefront-uniform; events are stored interleaved so each
// step of the wavefront reads 64 consecutive values.  Lanes whose chunk is
// shorter than the wave's longest read padding events (zero step, no
// measurement), which leave the state unchanged.
#pragma once

#include "../../include/gp_ssm.h"
#include "kernels.h"
#include "plan.h"
#include "sqrt_filter.h"

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
__device__ __forceinline__ Obs load_event(const DevPlan& p, int64_t e, double jit2, double& dt, uint32_t& info,
                                          const double* itab) {
  dt = p.dt[e];
  info = p.info[e];
  return make_obs<Dm>(info, p.y[e], p.r[e], p.invd[e], jit2, itab);
}

// the series' row of the instrument table, copied to LDS (made visible by
// the barrier of stage_coef, which follows); null without instruments
__device__ __forceinline__ const double* stage_inst(const DevParams& pr, int64_t b, double* ltab) {
  if (pr.ni == 0) return nullptr;
  if (threadIdx.x < ITAB_W) ltab[threadIdx.x] = pr.itab[b * ITAB_W + threadIdx.x];
  return ltab;
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
template <int J, int FT>
__global__ __launch_bounds__(WAVE) void k_summaries(DevPlan p, DevParams pr, double* __restrict__ summ) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, NXP = Dm::NXP;
  const int w = p.wv_order ? p.wv_order[blockIdx.x] : (int)blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t b = p.wv_series[w];
  const int32_t nch = p.wv_nch[w], L = p.wv_len[w];
  const int64_t ev0 = p.wv_ev0[w];
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  __shared__ double lcoef[M * NCOEF];
  __shared__ double ltab[(FT & 2) ? ITAB_W : 1];
  const double* itab = (FT & 2) ? stage_inst(pr, b, ltab) : nullptr;
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
  if (lane < nch && p.chunk_first[p.wv_chunk[(int64_t)w * WAVE + lane]]) {
    // a series' first chunk starts from the prior itself rather than from a
    // known state: its summary is then the plain filter's state and
    // log-likelihood (A = 0, J = 0, eta = 0).  Conditioning on the series'
    // first state would make the scan combine the wide prior with the
    // chunk's information about that state, (I + P0 J)^-1, which for dense,
    // nearly noise-free data has J ~ 1/R and loses every digit.
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double s2 = tc[t].sigma * tc[t].sigma;
      st.P[sidx(2 * t, 2 * t, Dm::D)] = s2;
      st.P[sidx(2 * t + 1, 2 * t + 1, Dm::D)] = s2 * second_prior<(FT & 1) != 0>(tc[t]);
    }
#pragma unroll
    for (int i = 0; i < Dm::D * NX; ++i) st.S(i) = 0.0;
  }
  EvRaw nxt = fetch_event(p, ev0 + lane);
  for (int32_t k = 0; k < L; ++k) {
    const EvRaw cur = nxt;
    if (k + 1 < L) nxt = fetch_event(p, ev0 + (int64_t)(k + 1) * WAVE + lane);
    const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2, itab);
    TermQ tq[M];
    discretise<M, DiscFull, NCOEF, (FT & 1) != 0>(tc, coef, cur.dt, tq);
    st.step(tq, cur.info, o);
  }
  if (lane < nch) {
    const int64_t c = p.wv_chunk[(int64_t)w * WAVE + lane];
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
// one work wave per workgroup: entry rs.first + blockIdx.x of the launch
// order; the per-event states of the wave live in the workgroup's record slot
template <int J, int FT>
__global__ __launch_bounds__(WAVE) void k_adjoint(DevPlan p, DevParams pr, const double* __restrict__ bstate,
                                                  const double* __restrict__ badj, RecSlots rs,
                                                  double* __restrict__ gpart) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, D = Dm::D, NP = Dm::NP;
  constexpr int F = rec_fields<Dm>();
  const int lane = threadIdx.x;
  const int64_t C = p.n_chunks;
  __shared__ double lcoef[M * 2 * NCOEF];
  __shared__ double lacc[(3 * M + 1) * WAVE];
  __shared__ double ltab[(FT & 2) ? ITAB_W : 1];
  __shared__ double linst[(FT & 2) ? 2 * MAX_INST * WAVE : 1];
  // with four open exposures the step's registers spill; the beta-derivatives
  // then wait in LDS (9 KB at M = 3)
  constexpr bool DBL = J >= 4;
  __shared__ double ldb[DBL ? 6 * M * WAVE : 1];
  {
    const int32_t qi = rs.first + (int32_t)blockIdx.x;
    const int w = p.wv_order ? p.wv_order[qi] : qi;
    const int64_t b = p.wv_series[w];
    const int32_t nch = p.wv_nch[w], L = p.wv_len[w];
    const int64_t ev0 = p.wv_ev0[w];
    double* const rb = rs.records(ev0, F);
    const bool active = lane < nch;
    const int64_t c = p.wv_chunk[(int64_t)w * WAVE + (active ? lane : 0)];
    TermConst tc[M];
    load_terms<Dm>(pr, b, tc);
    const double* itab = (FT & 2) ? stage_inst(pr, b, ltab) : nullptr;
    const double* coef = stage_coef<Dm, true>(pr, b, lcoef);
    const double jit = pr.jit[b];
    const double jit2 = jit * jit;

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
      // the records come back after the rest of the wave's forward sweep has
      // gone through the caches: streaming (non-temporal) stores here and
      // loads in the backward sweep
#pragma unroll
      for (int f = 0; f < D; ++f) __builtin_nontemporal_store(m[f], &rb[((int64_t)k * F + f) * WAVE + lane]);
#pragma unroll
      for (int f = 0; f < NP; ++f) __builtin_nontemporal_store(P[f], &rb[((int64_t)k * F + D + f) * WAVE + lane]);
      const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2, itab);
      TermQ tq[M];
      discretise<M, DiscGrad, 2 * NCOEF, (FT & 1) != 0>(tc, coef, cur.dt, tq);
      plain_step<Dm, false>(m, P, tq, cur.info, o);
    }

    double mb[D], Pb[NP];
#pragma unroll
    for (int i = 0; i < D; ++i) mb[i] = (i < NX && active) ? badj[i * C + c] : 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) Pb[sidx(i, j, D)] = (j < NX && active) ? badj[(NX + sidx(i, j, NX)) * C + c] : 0.0;
    const GradAcc<M> acc{lacc + lane, itab ? linst + lane : nullptr, itab};
    acc.init();
    nxt = fetch_event(p, ev0 + (int64_t)(L - 1) * WAVE + lane);
    for (int32_t k = L - 1; k >= 0; --k) {
      const EvRaw cur = nxt;
      if (k > 0) nxt = fetch_event(p, ev0 + (int64_t)(k - 1) * WAVE + lane);
#pragma unroll
      for (int f = 0; f < D; ++f) m[f] = __builtin_nontemporal_load(&rb[((int64_t)k * F + f) * WAVE + lane]);
#pragma unroll
      for (int f = 0; f < NP; ++f) P[f] = __builtin_nontemporal_load(&rb[((int64_t)k * F + D + f) * WAVE + lane]);
      const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2, itab);
      adjoint_step<Dm, DBL, (FT & 1) != 0>(m, P, mb, Pb, tc, coef, cur.dt, cur.info, o, jit, acc, LaneLds{ldb + lane});
    }
    if (active && p.chunk_first[c]) {
      // prior of the SHO states: sigma_t^2 I in scaled coordinates
#pragma unroll
      for (int t = 0; t < M; ++t)
        acc.s(t) += 2.0 * tc[t].sigma * (Pb[sidx(2 * t, 2 * t, D)] + second_prior<(FT & 1) != 0>(tc[t]) * Pb[sidx(2 * t + 1, 2 * t + 1, D)]);
    }
    // sum over the wave's lanes (one series), one partial per work wave
    const int64_t S = p.n_wv;
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double a0 = wave_sum(active ? acc.s(t) : 0.0);
      const double a1 = wave_sum(active ? acc.w(t) : 0.0);
      const double a2 = wave_sum(active ? acc.q(t) : 0.0);
      if (lane == 0) {
        gpart[(0 * M + t) * S + w] = a0;
        gpart[(1 * M + t) * S + w] = a1;
        gpart[(2 * M + t) * S + w] = a2;
      }
    }
    const double aj = wave_sum(active ? acc.jit() : 0.0);
    if (lane == 0) gpart[(3 * M) * S + w] = aj;
    for (int i = 0; i < pr.ni; ++i) {
      const double ga = wave_sum(active ? acc.amp(i) : 0.0);
      const double go = wave_sum(active ? acc.off(i) : 0.0);
      if (lane == 0) {
        gpart[(3 * M + 1 + i) * S + w] = ga;
        gpart[(3 * M + 1 + pr.ni + i) * S + w] = go;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// plain sequential filter of one series (one lane): the reference launch
// ---------------------------------------------------------------------------
template <int J, int FT>
__global__ __launch_bounds__(WAVE) void k_plain(DevPlan p, DevParams pr, int64_t b, double* __restrict__ loglik) {
  using Dm = Dims<M, J>;
  constexpr int D = Dm::D, NP = Dm::NP;
  __shared__ double lcoef[M * NCOEF];
  __shared__ double ltab[(FT & 2) ? ITAB_W : 1];
  const double* itab = (FT & 2) ? stage_inst(pr, b, ltab) : nullptr;
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
    P[sidx(2 * t + 1, 2 * t + 1, D)] = tc[t].sigma * tc[t].sigma * second_prior<(FT & 1) != 0>(tc[t]);
  }
  double ll = 0.0;
  const int32_t c0 = p.series_chunk0[b], nch = p.series_nch[b];
  for (int32_t q = 0; q < nch; ++q) {
    const int32_t c = c0 + q;
    const int32_t l = p.chunk_lane[c];
    const int64_t ev0 = p.wv_ev0[p.chunk_wv[c]];
    const int32_t len = p.chunk_len[c];
    for (int32_t k = 0; k < len; ++k) {
      const int64_t e = ev0 + (int64_t)k * WAVE + l;
      double dt;
      uint32_t info;
      const Obs o = load_event<Dm>(p, e, jit2, dt, info, itab);
      TermQ tq[M];
      discretise<M, DiscFull, NCOEF, (FT & 1) != 0>(tc, coef, dt, tq);
      ll += plain_step<Dm>(m, P, tq, info, o);
    }
  }
  loglik[b] = pr.bad[b] ? __builtin_nan("") : ll + inst_loglik(pr, b);
}

// ---------------------------------------------------------------------------
// square-root (Cholesky-factor) filter of whole series, SQ_GROUP lanes per
// series (one row of the factor each; see sqrt_filter.h), series taken in the
// order given (longest first), four to a wavefront
// ---------------------------------------------------------------------------
// writes the log-likelihood and status of each series as the scan's
// finishing kernel does
template <int J, int FT>
__global__ __launch_bounds__(WAVE) void k_sqrt(DevPlan p, DevParams pr, const int32_t* __restrict__ order,
                                               const CallArgs* __restrict__ args) {
  using Dm = Dims<M, J>;
  constexpr int D = Dm::D, NC = D + 3 * M;
  const int q = threadIdx.x & (SQ_GROUP - 1);
  const int64_t i = (int64_t)blockIdx.x * (WAVE / SQ_GROUP) + threadIdx.x / SQ_GROUP;
  const bool live = i < p.n_series;  // uniform over the group
  const int64_t b = live ? (order ? order[i] : i) : 0;
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  const double* coef = pr.coef + b * M * 2 * NCOEF;  // value tables at term stride 2 NCOEF
  const double* itab = ((FT & 2) && pr.ni > 0) ? pr.itab + b * ITAB_W : nullptr;
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  // this lane's row of the factor (then the noise columns) and mean entry,
  // from the stationary prior
  double row[NC], mq = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) row[c] = 0.0;
#pragma unroll
  for (int t = 0; t < M; ++t) {
    row[2 * t] = (q == 2 * t) ? tc[t].sigma : row[2 * t];
    row[2 * t + 1] = (q == 2 * t + 1) ? tc[t].sigma * second_prior<(FT & 1) != 0>(tc[t]) : row[2 * t + 1];
  }
  // lane t < M discretises term t at every event (the others repeat term 0)
  // and the group shares the results
  const int tl = q < M ? q : 0;
  const TermConst tmine = pr.tc[b * M + tl];
  const double* cmine = coef + tl * 2 * NCOEF;
  double ll = 0.0;
  const int32_t c0 = live ? p.series_chunk0[b] : 0, nch = live ? p.series_nch[b] : 0;
  for (int32_t k0 = 0; k0 < nch; ++k0) {
    const int32_t c = c0 + k0;
    const int32_t l = p.chunk_lane[c];
    const int64_t ev0 = p.wv_ev0[p.chunk_wv[c]];
    const int32_t len = p.chunk_len[c];
    for (int32_t k = 0; k < len; ++k) {
      double dt;
      uint32_t info;
      const Obs o = load_event<Dm>(p, ev0 + (int64_t)k * WAVE + l, jit2, dt, info, itab);
      TermQ mine, tq[M];
      discretise<1, DiscFull, 2 * NCOEF, (FT & 1) != 0>(&tmine, cmine, dt, &mine);
#pragma unroll
      for (int t = 0; t < M; ++t) tq[t] = grp_get_term(mine, t);
      sqrt_predict_row<Dm, 1>(row, &mq, q, tq, ev_open(info));
      ll += sqrt_update_row<Dm, 1>(row, &mq, q, info, o);
    }
  }
  if (!live || q != 0) return;
  ll += inst_loglik(pr, b);
  const bool pbad = pr.bad[b] != 0, good = isfinite(ll);
  double* const loglik = args->loglik;
  int32_t* const status = args->status;
  if (loglik) loglik[b] = (good && !pbad) ? ll : __builtin_nan("");
  if (status) status[b] = pbad ? GP_SSM_EPARAM : (good ? 0 : GP_SSM_ENUMERIC);
}

// ---------------------------------------------------------------------------
// time-split square-root filter: per chunk, the filter conditioned on the
// chunk's first SHO state x0 in factor form (SQ_GROUP lanes per chunk, four
// chunks to a wavefront), then per series a tree of pairwise combinations of
// the chunk summaries (one lane per pair, one launch per level)
// ---------------------------------------------------------------------------
// Chunk summary (offsets sq_*): the chunk's end state is x0-affine with
// mean A x0 + b and covariance U U^T; its measurements have density
// exp(-c0 - |R x0 - rho|^2 / 2 - eps^2 / 2), where [[R, rho], [0, eps]] is
// the triangular factor (Z^T) of the rows (u_k / sqrt S_k, v_k / sqrt S_k):
// u_k the x0-sensitivity of measurement k's innovation, v_k its value at
// x0 = 0, S_k its variance.  Kept as a factor of these rows rather than as
// information sums, the density involves no difference of terms of order
// v^2 / S, which nearly noise-free data make huge.  A series' first chunk
// starts from the prior instead (A = 0, R = 0): its summary is the filter's
// state and likelihood.
// (two wavefronts per SIMD up to three terms, which hides part of each
// event's latency chain: 8-17% faster at three terms despite about 220
// bytes of spills per lane; at four terms the spills would double)
template <int J, int FT>
__global__ __launch_bounds__(WAVE, M <= 3 ? 2 : 1) void k_sqrt_summ(DevPlan p, DevParams pr, double* __restrict__ out) {
  using Dm = Dims<M, J>;
  constexpr int D = Dm::D, NX = Dm::NX, NC = D + 3 * M, NE = 1 + NX, NPZ = (NX + 1) * (NX + 2) / 2;
  const int q = threadIdx.x & (SQ_GROUP - 1);
  const int64_t c = (int64_t)blockIdx.x * (WAVE / SQ_GROUP) + threadIdx.x / SQ_GROUP;
  const bool live = c < p.n_chunks;  // uniform over the group
  const int64_t cc = live ? c : 0;
  const int64_t b = p.chunk_series[cc];
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  const double* itab = ((FT & 2) && pr.ni > 0) ? pr.itab + b * ITAB_W : nullptr;
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  const int tl = q < M ? q : 0;
  const TermConst tmine = pr.tc[b * M + tl];
  const double* cmine = pr.coef + (b * M + tl) * 2 * NCOEF;
  // row q of the factor U and of [b | S] (the mean b + S x0)
  double row[NC], ext[NE];
#pragma unroll
  for (int k = 0; k < NC; ++k) row[k] = 0.0;
#pragma unroll
  for (int e = 0; e < NE; ++e) ext[e] = 0.0;
  if (p.chunk_first[cc]) {
#pragma unroll
    for (int t = 0; t < M; ++t) {
      row[2 * t] = (q == 2 * t) ? tc[t].sigma : row[2 * t];
      row[2 * t + 1] = (q == 2 * t + 1) ? tc[t].sigma * second_prior<(FT & 1) != 0>(tc[t]) : row[2 * t + 1];
    }
  } else {
#pragma unroll
    for (int k = 0; k < NX; ++k) ext[1 + k] = (q == k) ? 1.0 : 0.0;
  }
  double Z[NPZ], c0 = 0.0;
#pragma unroll
  for (int k = 0; k < NPZ; ++k) Z[k] = 0.0;
  const int32_t l = p.chunk_lane[cc];
  const int64_t ev0 = p.wv_ev0[p.chunk_wv[cc]];
  const int32_t len = live ? p.chunk_len[cc] : 0;
  for (int32_t k = 0; k < len; ++k) {
    double dt;
    uint32_t info;
    const Obs o = load_event<Dm>(p, ev0 + (int64_t)k * WAVE + l, jit2, dt, info, itab);
    TermQ mine, tq[M];
    discretise<1, DiscFull, 2 * NCOEF, (FT & 1) != 0>(&tmine, cmine, dt, &mine);
#pragma unroll
    for (int t = 0; t < M; ++t) tq[t] = grp_get_term(mine, t);
    sqrt_predict_row<Dm, NE>(row, ext, q, tq, ev_open(info));
    double wz[NE], rs;
    (void)sqrt_update_row<Dm, NE>(row, ext, q, info, o, wz, &rs);
    // log sqrt(2 pi S) (taken from sqrt S itself: the innovation at x0 = 0,
    // whose square goes to the factor, can be many times sqrt S); nothing
    // without a measurement
    if (o.has) c0 += 0.5 * LOG_2PI + log(rs);
    // the row (u / sqrt S, v / sqrt S), u = S^T h, appended to the factor by
    // rotations (wz = (v, u) / sqrt S); nothing to append without a
    // measurement (the branch is uniform over the group)
    if (!o.has) continue;
    double n[NX + 1];
#pragma unroll
    for (int e = 0; e < NX; ++e) n[e] = wz[1 + e];
    n[NX] = wz[0];
#pragma unroll
    for (int r = 0; r <= NX; ++r) {
      double cs, sn, rr;
      plane_rotation(Z[lidx(r, r)], n[r], cs, sn, rr);
      Z[lidx(r, r)] = rr;
#pragma unroll
      for (int i = r + 1; i <= NX; ++i) {
        const double z = Z[lidx(i, r)];
        Z[lidx(i, r)] = fma(cs, z, sn * n[i]);
        n[i] = fma(-sn, z, cs * n[i]);
      }
    }
  }
  if (!live) return;
  const int64_t C = p.n_chunks;
  if (q < NX) {
#pragma unroll
    for (int k = 0; k < NX; ++k) out[(sq_A(NX) + q * NX + k) * C + c] = ext[1 + k];
    out[(sq_b(NX) + q) * C + c] = ext[0];
#pragma unroll
    for (int k = 0; k < NX; ++k)
      if (k <= q) out[(sq_U(NX) + q * (q + 1) / 2 + k) * C + c] = row[k];
  }
  if (q == 0) {
#pragma unroll
    for (int k = 0; k < NPZ; ++k) out[(sq_Z(NX) + k) * C + c] = Z[k];
    out[sq_c0(NX) * C + c] = c0;
  }
}

// the first NP rows of X (NR x NC) brought to lower-triangular form in place
// by Householder reflections from the right (each scaled by the exponent of
// its pivot row's largest entry), applied to every row: on return X[i][k] for
// k <= i < NP is the factor of the first NP rows, and the rows below carry the
// same orthogonal transformation
template <int NR, int NC, int NP>
__device__ __forceinline__ void sq_tria(double (&X)[NR][NC]) {
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double mx = 0.0;
#pragma unroll
    for (int k = i; k < NC; ++k) mx = fmax(mx, fabs(X[i][k]));
    if (!(mx > 0.0)) continue;
    int e;
    (void)frexp(mx, &e);
    double v[NC], n2 = 0.0;
#pragma unroll
    for (int k = i; k < NC; ++k) {
      v[k] = ldexp(X[i][k], -e);
      n2 = fma(v[k], v[k], n2);
    }
    const double nrm = sqrt(n2);
    const double alpha = v[i] >= 0.0 ? -nrm : nrm;
    const double vv = 2.0 * nrm * (nrm + fabs(v[i]));
    v[i] -= alpha;
    const double beta = 2.0 / vv;
#pragma unroll
    for (int r = i + 1; r < NR; ++r) {
      double w = 0.0;
#pragma unroll
      for (int k = i; k < NC; ++k) w = fma(X[r][k], v[k], w);
      w *= beta;
#pragma unroll
      for (int k = i; k < NC; ++k) X[r][k] = fma(-w, v[k], X[r][k]);
    }
    X[i][i] = ldexp(alpha, e);
#pragma unroll
    for (int k = i + 1; k < NC; ++k) X[i][k] = 0.0;
  }
}

// a chunk summary of the time-split square-root filter in registers
template <int N>
struct SqElem {
  double A[N][N], b[N], U[N][N], Z[N + 1][N + 1], c0;
};
template <int N>
__device__ __forceinline__ void sq_load(const double* __restrict__ sm, int64_t C, int64_t c, SqElem<N>& e) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    e.b[i] = sm[(int64_t)(sq_b(N) + i) * C + c];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      e.A[i][k] = sm[(int64_t)(sq_A(N) + i * N + k) * C + c];
      e.U[i][k] = k <= i ? sm[(int64_t)(sq_U(N) + lidx(i, k)) * C + c] : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i <= N; ++i)
#pragma unroll
    for (int k = 0; k <= N; ++k) e.Z[i][k] = k <= i ? sm[(int64_t)(sq_Z(N) + lidx(i, k)) * C + c] : 0.0;
  e.c0 = sm[(int64_t)sq_c0(N) * C + c];
}
template <int N>
__device__ __forceinline__ void sq_store(double* __restrict__ sm, int64_t C, int64_t c, const SqElem<N>& e) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    sm[(int64_t)(sq_b(N) + i) * C + c] = e.b[i];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      sm[(int64_t)(sq_A(N) + i * N + k) * C + c] = e.A[i][k];
      if (k <= i) sm[(int64_t)(sq_U(N) + lidx(i, k)) * C + c] = e.U[i][k];
    }
  }
#pragma unroll
  for (int i = 0; i <= N; ++i)
#pragma unroll
    for (int k = 0; k <= i; ++k) sm[(int64_t)(sq_Z(N) + lidx(i, k)) * C + c] = e.Z[i][k];
  sm[(int64_t)sq_c0(N) * C + c] = e.c0;
}

// the summary of two consecutive stretches (e1 then e2) of a series: e2's
// density is a pseudo-measurement rho2 = R2 x1 + e of e1's end state x1 =
// A1 x0 + b1 + U1 w.  In array form [[I, W], [0, U1]] with W = R2 U1 becomes
// [[Xi, 0], [Kb, U1']]; with G = Xi^-1 [R2 A1 | R2 b1 - rho2], the combined
// density gains the rows (G_A, -G_b) and eps2 in its factor (a triangularised
// stack) and log det Xi in c0; x1 given e2's data is (A1 - Kb G_A) x0 +
// b1 - Kb G_b with factor U1', moved on by e2: A = A2 (A1 - Kb G_A),
// b = A2 (b1 - Kb G_b) + b2, U = tria[A2 U1' | U2]
template <int N>
__device__ __forceinline__ void sq_combine(const SqElem<N>& e1, const SqElem<N>& e2, SqElem<N>& e) {
  double X2[2 * N][2 * N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double w = 0.0;
#pragma unroll
      for (int r = i; r < N; ++r) w = fma(e2.Z[r][i], e1.U[r][k], w);
      X2[i][k] = i == k ? 1.0 : 0.0;
      X2[i][N + k] = w;
      X2[N + i][k] = 0.0;
      X2[N + i][N + k] = e1.U[i][k];
    }
  sq_tria<2 * N, 2 * N, N>(X2);
  // G = Xi^-1 [R2 A1 | R2 b1 - rho2]
  double G[N][N + 1], logdet = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int k = 0; k <= N; ++k) {
      double a = k < N ? 0.0 : -e2.Z[N][i];
#pragma unroll
      for (int r = i; r < N; ++r) a = fma(e2.Z[r][i], k < N ? e1.A[r][k] : e1.b[r], a);
#pragma unroll
      for (int j = 0; j < i; ++j) a = fma(-X2[i][j], G[j][k], a);
      G[i][k] = a / X2[i][i];
    }
    logdet += log(fabs(X2[i][i]));
  }
  // the density's factor: tria[Z1 | rows (G_A, -G_b) as columns | eps2 e_N]
  double Y[N + 1][2 * N + 2];
#pragma unroll
  for (int r = 0; r <= N; ++r) {
#pragma unroll
    for (int k = 0; k <= N; ++k) Y[r][k] = e1.Z[r][k];
#pragma unroll
    for (int i = 0; i < N; ++i) Y[r][N + 1 + i] = r < N ? G[i][r] : -G[i][N];
    Y[r][2 * N + 1] = r == N ? e2.Z[N][N] : 0.0;
  }
  sq_tria<N + 1, 2 * N + 2, N + 1>(Y);
#pragma unroll
  for (int r = 0; r <= N; ++r)
#pragma unroll
    for (int k = 0; k <= N; ++k) e.Z[r][k] = k <= r ? Y[r][k] : 0.0;
  e.c0 = e1.c0 + e2.c0 + logdet;
  // the end state
  double T[N][N + 1];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k <= N; ++k) {
      double a = k < N ? e1.A[i][k] : e1.b[i];
#pragma unroll
      for (int j = 0; j < N; ++j) a = fma(-X2[N + i][j], G[j][k], a);
      T[i][k] = a;
    }
  double X[N][2 * N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int k = 0; k <= N; ++k) {
      double a = k < N ? 0.0 : e2.b[i];
#pragma unroll
      for (int r = 0; r < N; ++r) a = fma(e2.A[i][r], T[r][k], a);
      if (k < N)
        e.A[i][k] = a;
      else
        e.b[i] = a;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a = 0.0;
#pragma unroll
      for (int r = 0; r < N; ++r) a = fma(e2.A[i][r], X2[N + r][N + k], a);
      X[i][k] = a;
      X[i][N + k] = e2.U[i][k];
    }
  }
  sq_tria<N, 2 * N, N>(X);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) e.U[i][k] = k <= i ? X[i][k] : 0.0;
}

// one level of the tree over each series' summaries: with the series'
// summaries at positions chunk0 + j, j < cnt (cnt = its chunks halved `level`
// times, rounded up), position chunk0 + j of `out` gets the combination of
// j's pair (2j, 2j + 1), or 2j alone when it has no partner
template <int J, int FT>
__global__ __launch_bounds__(WAVE) void k_sqrt_combine(DevPlan p, const double* __restrict__ in,
                                                       double* __restrict__ out, int32_t level) {
  constexpr int N = 2 * M;
  const int64_t c = (int64_t)blockIdx.x * WAVE + threadIdx.x;
  if (c >= p.n_chunks) return;
  const int64_t b = p.chunk_series[c];
  const int64_t c0 = p.series_chunk0[b];
  const int32_t nch = p.series_nch[b];
  const int64_t j = c - c0;
  const int64_t cnt = ((int64_t)nch + (int64_t(1) << level) - 1) >> level;
  if (2 * j >= cnt) return;
  const int64_t C = p.n_chunks;
  SqElem<N> e1;
  sq_load<N>(in, C, c0 + 2 * j, e1);
  if (2 * j + 1 < cnt) {
    SqElem<N> e2, e;
    sq_load<N>(in, C, c0 + 2 * j + 1, e2);
    sq_combine<N>(e1, e2, e);
    sq_store<N>(out, C, c0 + j, e);
  } else {
    sq_store<N>(out, C, c0 + j, e1);
  }
}

// each series' log-likelihood from its single remaining summary (which
// starts from the prior, so that its density does not depend on a state):
// -c0 - eps^2 / 2
template <int J, int FT>
__global__ __launch_bounds__(WAVE) void k_sqrt_total(DevPlan p, DevParams pr, const double* __restrict__ sm,
                                                     const CallArgs* __restrict__ args) {
  constexpr int N = 2 * M;
  const int64_t b = (int64_t)blockIdx.x * WAVE + threadIdx.x;
  if (b >= p.n_series) return;
  double ll = 0.0;
  if (p.series_nch[b] > 0) {
    const int64_t C = p.n_chunks, c = p.series_chunk0[b];
    const double eps = sm[(int64_t)(sq_Z(N) + lidx(N, N)) * C + c];
    ll = -sm[(int64_t)sq_c0(N) * C + c] - 0.5 * eps * eps;
  }
  ll += inst_loglik(pr, b);
  const bool pbad = pr.bad[b] != 0, good = isfinite(ll);
  double* const loglik = args->loglik;
  int32_t* const status = args->status;
  if (loglik) loglik[b] = (good && !pbad) ? ll : __builtin_nan("");
  if (status) status[b] = pbad ? GP_SSM_EPARAM : (good ? 0 : GP_SSM_ENUMERIC);
}

// ---------------------------------------------------------------------------
// smoother (Sec. 3.2.2, Algorithm 1): a forward pass storing each event's
// predicted state, then the backward sweep of the adjoint pair (lambda,
// Lambda) from its value at the chunk's end, with the exposure-averaged
// posterior at every measurement and the latent posterior at the test times
// that fall in the chunk
// ---------------------------------------------------------------------------

// latent posterior at a test time between two events: the forward moments
// (m0, P0) after the earlier event predicted over a, the adjoint pair of the
// later event (before its update) carried back over b; open: the integrators
// open over the whole step.  With tmean/tvar (a row of M entries) also each
// term's own process (Appendix C, component-wise predictive means and
// variances: h = e_{x_m}).
template <class Dm, bool X>
__device__ __forceinline__ void bf_test(const double* m0, const double* P0, const TermConst* tc, const double* coef,
                                        double a, double b, uint32_t open, const double* lam0, const double* Lam0,
                                        double& mean, double& var, double* tmean, double* tvar) {
  constexpr int M = Dm::M, D = Dm::D, NP = Dm::NP;
  double m[D], P[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) m[i] = m0[i];
#pragma unroll
  for (int i = 0; i < NP; ++i) P[i] = P0[i];
  TermQ tq[M];
  discretise<M, DiscFull, NCOEF, X>(tc, coef, a, tq);
  predict_mean<Dm>(m, tq, open);
  predict_cov<Dm>(P, tq, open);
  double l[D], L[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) l[i] = lam0[i];
#pragma unroll
  for (int i = 0; i < NP; ++i) L[i] = Lam0[i];
  discretise<M, DiscFull, NCOEF, X>(tc, coef, b, tq);
  bf_predict<Dm>(l, L, tq, open);
  // h = sum of the SHO x components
  double u[D], hm = 0.0, hu = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) v += P[sidx(i, 2 * t, D)];
    u[i] = v;
  }
#pragma unroll
  for (int t = 0; t < M; ++t) {
    hm += m[2 * t];
    hu += u[2 * t];
  }
  bf_posterior<Dm>(hm, hu, u, l, L, mean, var);
  if (tmean) {
#pragma unroll
    for (int t = 0; t < M; ++t) {
      double ut[D];
#pragma unroll
      for (int i = 0; i < D; ++i) ut[i] = P[sidx(i, 2 * t, D)];
      bf_posterior<Dm>(m[2 * t], ut[2 * t], ut, l, L, tmean[t], tvar[t]);
    }
  }
}

// adds NaN (poison) or 0 to test time o's per-term outputs, if wanted
__device__ __forceinline__ void poison_terms(const DevTests& ts, int64_t o, double poison) {
  if (!ts.term_mean) return;
#pragma unroll
  for (int t = 0; t < M; ++t) {
    ts.term_mean[o * M + t] += poison;
    ts.term_var[o * M + t] += poison;
  }
}

template <int J, int FT>
__device__ __forceinline__ void smooth_wave(const DevPlan& p, const DevParams& pr, const double* __restrict__ bstate,
                                            const double* __restrict__ bsmooth, double* __restrict__ rb, int w,
                                            double* lcoef, double* ltab, const DevTests& ts, double* __restrict__ mean_test,
                                            double* __restrict__ var_test, double* __restrict__ mean_data,
                                            double* __restrict__ var_data) {
  using Dm = Dims<M, J>;
  constexpr int NX = Dm::NX, D = Dm::D, NP = Dm::NP;
  constexpr int F = rec_fields<Dm>();
  const int lane = threadIdx.x;
  const int64_t b = p.wv_series[w];
  const int32_t nch = p.wv_nch[w];
  const int64_t ev0 = p.wv_ev0[w];
  const bool active = lane < nch;
  const int64_t C = p.n_chunks;
  const int64_t c = p.wv_chunk[(int64_t)w * WAVE + (active ? lane : 0)];
  const int32_t len = active ? p.chunk_len[c] : 0;
  TermConst tc[M];
  load_terms<Dm>(pr, b, tc);
  const double* itab = (FT & 2) ? stage_inst(pr, b, ltab) : nullptr;
  const double* coef = stage_coef<Dm, false>(pr, b, lcoef);
  const double jit = pr.jit[b];
  const double jit2 = jit * jit;
  // a series whose hyperparameters failed validation gets NaN outputs
  const double poison = pr.bad[b] ? __builtin_nan("") : 0.0;
  auto ev = [&](int32_t k) { return ev0 + (int64_t)k * WAVE + lane; };
  auto load_rec = [&](int32_t k, double* m, double* P) {
#pragma unroll
    for (int f = 0; f < D; ++f) m[f] = rb[((int64_t)k * F + f) * WAVE + lane];
#pragma unroll
    for (int f = 0; f < NP; ++f) P[f] = rb[((int64_t)k * F + D + f) * WAVE + lane];
  };
  // the update of one event applied to its predicted moments, then its close
  auto update_close = [&](const EvRaw& e, double* m, double* P) {
    const Obs o = make_obs<Dm>(e.info, e.y, e.r, e.invd, jit2, itab);
    double u[D];
    obs_gain<Dm>(P, o, u);
    const double iS = 1.0 / (obs_dot<Dm>(u, o) + o.R);
    const double viS = (o.y - obs_dot<Dm>(m, o)) * iS;
#pragma unroll
    for (int i = 0; i < D; ++i) m[i] = fma(u[i], viS, m[i]);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double ui = u[i] * iS;
#pragma unroll
      for (int j = i; j < D; ++j) P[sidx(i, j, D)] = fma(-ui, u[j], P[sidx(i, j, D)]);
    }
    close_slot<Dm>(m, P, e.info);
  };

  // forward: store the predicted moments of each event
  double m[D], P[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) m[i] = (i < NX && active) ? bstate[i * C + c] : 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) P[sidx(i, j, D)] = (j < NX && active) ? bstate[(NX + sidx(i, j, NX)) * C + c] : 0.0;
  for (int32_t k = 0; k < len; ++k) {
    const EvRaw cur = fetch_event(p, ev(k));
    TermQ tq[M];
    discretise<M, DiscFull, NCOEF, (FT & 1) != 0>(tc, coef, cur.dt, tq);
    const uint32_t open = ev_open(cur.info);
    predict_mean<Dm>(m, tq, open);
    predict_cov<Dm>(P, tq, open);
    // ordinary stores: a smoothed series' records (tens of MB) can stay in
    // the last-level cache until the backward sweep reads them
#pragma unroll
    for (int f = 0; f < D; ++f) rb[((int64_t)k * F + f) * WAVE + lane] = m[f];
#pragma unroll
    for (int f = 0; f < NP; ++f) rb[((int64_t)k * F + D + f) * WAVE + lane] = P[f];
    update_close(cur, m, P);
  }

  const int64_t tlo = active ? ts.chunk_t0[c] : 0;
  int64_t tp = active ? ts.chunk_t0[c + 1] - 1 : -1;
  // test times after the chunk's last event (only at the end of a series):
  // prediction from the final filtered state, which holds all the data
  if (len > 0) {
    const double tl = p.t[ev(len - 1)];
    while (tp >= tlo && ts.t[tp] > tl) {
      double mm[D], PP[NP];
#pragma unroll
      for (int i = 0; i < D; ++i) mm[i] = m[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) PP[i] = P[i];
      TermQ tqq[M];
      discretise<M, DiscFull, NCOEF, (FT & 1) != 0>(tc, coef, ts.t[tp] - tl, tqq);
      predict_mean<Dm>(mm, tqq, 0u);
      predict_cov<Dm>(PP, tqq, 0u);
      double mean = 0.0, var = 0.0;
#pragma unroll
      for (int t = 0; t < M; ++t) {
        mean += mm[2 * t];
#pragma unroll
        for (int u = 0; u < M; ++u) var += PP[sidx(2 * t, 2 * u, D)];
      }
      const int64_t o = ts.out_index[tp];
      mean_test[o] = mean + poison;
      var_test[o] = var + poison;
      if (ts.term_mean) {
#pragma unroll
        for (int t = 0; t < M; ++t) {
          ts.term_mean[o * M + t] = mm[2 * t] + poison;
          ts.term_var[o * M + t] = PP[sidx(2 * t, 2 * t, D)] + poison;
        }
      }
      --tp;
    }
  }

  // backward: the adjoint pair after the chunk's last event (zero at the end
  // of a series), carried back through every event
  double lam[D], Lam[NP];
#pragma unroll
  for (int i = 0; i < D; ++i) lam[i] = (i < NX && active) ? bsmooth[i * C + c] : 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) Lam[sidx(i, j, D)] = (j < NX && active) ? bsmooth[(NX + sidx(i, j, NX)) * C + c] : 0.0;
  for (int32_t k = len - 1; k >= 0; --k) {
    const EvRaw cur = fetch_event(p, ev(k));
    const double tk = p.t[ev(k)];
    bf_close<Dm>(lam, Lam, cur.info);
    {
      double mp[D], Pp[NP];
      load_rec(k, mp, Pp);
      const Obs o = make_obs<Dm>(cur.info, cur.y, cur.r, cur.invd, jit2, itab);
      double u[D];
      obs_gain<Dm>(Pp, o, u);
      const double hu = obs_dot<Dm>(u, o), hm = obs_dot<Dm>(mp, o);
      double ed[2];
      bf_update<Dm>(lam, Lam, u, o, hu + o.R, o.y - hm, ed);
      // posterior at the measurement (the exposure average, or the latent
      // process for an instantaneous one; with instruments, times the
      // amplitude plus the offset): the same h as the update, in the
      // disturbance form of bf_update
      if (o.has) {
        double mean = fma(-o.R, ed[0], o.y);
        double var = o.R * fma(-o.R, ed[1], 1.0);
        if (itab) {
          const uint32_t ii = ev_inst(cur.info);
          const double a = itab[ITAB_AMP + ii];
          mean = fma(a, mean, itab[ITAB_OFF + ii]);
          var *= a * a;
        }
        const int64_t n = p.meas[ev(k)];
        if (mean_data) mean_data[n] = mean + poison;
        if (var_data) var_data[n] = var + poison;
      }
    }
    // test times between the previous event (or the chunk's start) and this one
    if (k > 0) {
      const double tprev = p.t[ev(k - 1)];
      if (tp >= tlo && ts.t[tp] > tprev) {
        double mf[D], Pf[NP];
        load_rec(k - 1, mf, Pf);
        update_close(fetch_event(p, ev(k - 1)), mf, Pf);
        while (tp >= tlo && ts.t[tp] > tprev) {
          const double tq = ts.t[tp];
          double mean, var;
          const int64_t o = ts.out_index[tp];
          bf_test<Dm, (FT & 1) != 0>(mf, Pf, tc, coef, tq - tprev, tk - tq, ev_open(cur.info), lam, Lam, mean, var,
                      ts.term_mean ? ts.term_mean + o * M : nullptr, ts.term_var ? ts.term_var + o * M : nullptr);
          poison_terms(ts, o, poison);
          mean_test[o] = mean + poison;
          var_test[o] = var + poison;
          --tp;
        }
      }
    } else if (tp >= tlo) {
      // before the chunk's first event: from the boundary state, or from the
      // prior before the series' first event
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
          pP[sidx(2 * t + 1, 2 * t + 1, D)] = tc[t].sigma * tc[t].sigma * second_prior<(FT & 1) != 0>(tc[t]);
        }
      }
      const double tprev = ts.chunk_tprev[c];
      while (tp >= tlo) {
        const double tq = ts.t[tp];
        double mean, var;
        const int64_t o = ts.out_index[tp];
        bf_test<Dm, (FT & 1) != 0>(pm, pP, tc, coef, first ? 0.0 : tq - tprev, tk - tq, ev_open(cur.info), lam, Lam, mean, var,
                    ts.term_mean ? ts.term_mean + o * M : nullptr, ts.term_var ? ts.term_var + o * M : nullptr);
        poison_terms(ts, o, poison);
        mean_test[o] = mean + poison;
        var_test[o] = var + poison;
        --tp;
      }
    }
    // back through this event's predict
    TermQ tq[M];
    discretise<M, DiscFull, NCOEF, (FT & 1) != 0>(tc, coef, cur.dt, tq);
    bf_predict<Dm>(lam, Lam, tq, ev_open(cur.info));
  }
}

template <int J, int FT>
__global__ __launch_bounds__(WAVE) void k_smooth(DevPlan p, DevParams pr, const double* __restrict__ bstate,
                                                 const double* __restrict__ bsmooth, RecSlots rs, DevTests ts,
                                                 double* __restrict__ mean_test, double* __restrict__ var_test,
                                                 double* __restrict__ mean_data, double* __restrict__ var_data) {
  __shared__ double lcoef[M * NCOEF];
  __shared__ double ltab[(FT & 2) ? ITAB_W : 1];
  const int32_t qi = rs.first + (int32_t)blockIdx.x;
  const int w = p.wv_order ? p.wv_order[qi] : qi;
  double* const rb = rs.records(p.wv_ev0[w], rec_fields<Dims<M, J>>());
  smooth_wave<J, FT>(p, pr, bstate, bsmooth, rb, w, lcoef, ltab, ts, mean_test, var_test, mean_data, var_data);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int J, int FT>
void launch_summaries(const Launch& L, const DevPlan& p, const DevParams& pr, double* summ) {
  if (p.n_wv == 0) return;
  prof_begin("k_summaries", L.stream);
  hipLaunchKernelGGL((k_summaries<J, FT>), dim3(p.n_wv), dim3(WAVE), 0, L.stream, p, pr, summ);
  prof_end("k_summaries", L.stream);
}
template <int J, int FT>
void launch_adjoint(const Launch& L, const DevPlan& p, const DevParams& pr, const double* bstate, const double* badj,
                    const RecSlots& rec, double* gpart) {
  // rounds of at most rec.grid work waves in launch order, one record slot
  // per workgroup of a round
  for (int32_t first = 0; first < p.n_wv; first += rec.grid) {
    RecSlots r = rec;
    r.first = first;
    prof_begin("k_adjoint", L.stream);
    hipLaunchKernelGGL((k_adjoint<J, FT>), dim3(std::min(rec.grid, p.n_wv - first)), dim3(WAVE), 0, L.stream, p, pr,
                       bstate, badj, r, gpart);
    prof_end("k_adjoint", L.stream);
  }
}
template <int J, int FT>
void launch_plain(const Launch& L, const DevPlan& p, const DevParams& pr, int64_t series, double* loglik) {
  prof_begin("k_plain", L.stream);
  hipLaunchKernelGGL((k_plain<J, FT>), dim3(1), dim3(WAVE), 0, L.stream, p, pr, series, loglik);
  prof_end("k_plain", L.stream);
}

template <int J, int FT>
void launch_sqrt(const Launch& L, const DevPlan& p, const DevParams& pr, const int32_t* order, const CallArgs* args) {
  if (p.n_series == 0) return;
  prof_begin("k_sqrt", L.stream);
  constexpr int per_wave = WAVE / SQ_GROUP;
  hipLaunchKernelGGL((k_sqrt<J, FT>), dim3((unsigned)((p.n_series + per_wave - 1) / per_wave)), dim3(WAVE), 0,
                     L.stream, p, pr, order, args);
  prof_end("k_sqrt", L.stream);
}

template <int J, int FT>
void launch_sqrt_split(const Launch& L, const DevPlan& p, const DevParams& pr, double* summ, double* tmp,
                       int32_t levels, const CallArgs* args) {
  if (p.n_series == 0) return;
  constexpr int per_wave = WAVE / SQ_GROUP;
  double* cur = summ;
  if (p.n_chunks > 0) {
    prof_begin("k_sqrt_summ", L.stream);
    hipLaunchKernelGGL((k_sqrt_summ<J, FT>), dim3((unsigned)((p.n_chunks + per_wave - 1) / per_wave)), dim3(WAVE), 0,
                       L.stream, p, pr, summ);
    prof_end("k_sqrt_summ", L.stream);
    // the tree over each series' summaries, one level per launch
    double* nxt = tmp;
    for (int32_t lv = 0; lv < levels; ++lv) {
      prof_begin("k_sqrt_combine", L.stream);
      hipLaunchKernelGGL((k_sqrt_combine<J, FT>), dim3((unsigned)((p.n_chunks + WAVE - 1) / WAVE)), dim3(WAVE), 0,
                         L.stream, p, cur, nxt, lv);
      prof_end("k_sqrt_combine", L.stream);
      std::swap(cur, nxt);
    }
  }
  prof_begin("k_sqrt_total", L.stream);
  hipLaunchKernelGGL((k_sqrt_total<J, FT>), dim3((unsigned)((p.n_series + WAVE - 1) / WAVE)), dim3(WAVE), 0, L.stream,
                     p, pr, cur, args);
  prof_end("k_sqrt_total", L.stream);
}

template <int J, int FT>
void launch_smooth(const Launch& L, const DevPlan& p, const DevParams& pr, const double* bstate, const double* bsmooth,
                   const RecSlots& rec, const DevTests& tests, double* mean_test, double* var_test, double* mean_data,
                   double* var_data) {
  for (int32_t first = 0; first < p.n_wv; first += rec.grid) {
    RecSlots r = rec;
    r.first = first;
    prof_begin("k_smooth", L.stream);
    hipLaunchKernelGGL((k_smooth<J, FT>), dim3(std::min(rec.grid, p.n_wv - first)), dim3(WAVE), 0, L.stream, p, pr,
                       bstate, bsmooth, r, tests, mean_test, var_test, mean_data, var_data);
    prof_end("k_smooth", L.stream);
  }
}

template <class K>
int occupancy(K kernel) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, WAVE, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}
template <int J, int FT>
int adjoint_occupancy() {
  static const int n = occupancy(k_adjoint<J, FT>);
  return n;
}
template <int J, int FT>
int smooth_occupancy() {
  static const int n = occupancy(k_smooth<J, FT>);
  return n;
}

template <int J, int FT>
KernelSet make_set() {
  KernelSet k;
  k.summaries = &launch_summaries<J, FT>;
  k.adjoint = &launch_adjoint<J, FT>;
  k.plain = &launch_plain<J, FT>;
  k.sqrt = &launch_sqrt<J, FT>;
  k.sqrt_split = &launch_sqrt_split<J, FT>;
  k.smooth = &launch_smooth<J, FT>;
  k.adjoint_occupancy = &adjoint_occupancy<J, FT>;
  k.smooth_occupancy = &smooth_occupancy<J, FT>;
  return k;
}

}  // namespace GPSSM_NS
}  // namespace gpssm
