// Square-root (Cholesky-factor) form of the sequential filter: the steps of
// one event (the kernel, one series per lane, is k_sqrt in kernels_impl.h).
//
// The covariance of the augmented state is carried as a lower-triangular
// factor L with P = L L^T, so that every covariance the filter forms is
// positive semidefinite by construction: the factor-form remedy that
// Sec. 3.2.3 and Sec. 5 name for the loss of accuracy of the covariance form
// on nearly noise-free data.  Mean, factor and the step's terms stay in
// registers (the factor packed by rows, lidx).
//
// Time update.  With the augmented transition A (Sec. 2.4: the blocks Phi_m
// and the integrated rows fbar_m added into the open integrators), A L is
// lower triangular except for one entry above the diagonal in each term's
// 2x2 block; a plane rotation of that block's two columns restores the
// triangle (rotating columns leaves (A L)(A L)^T unchanged).  The process
// noise of term m over the step is G_m Q3_m G_m^T, with Q3_m the covariance
// of (x_m, x_m', the integral of x_m) and G_m placing the integral in every
// open integrator; each column of G_m chol(Q3_m) enters as a rank-one update
// of the factor by rotations.
//
// Measurement update.  With h the observation row and R the noise variance,
// the array [[sqrt R, h^T L], [0, L]] is brought to the lower-triangular form
// [[sqrt S, 0], [k, L+]] by plane rotations of its first column against the
// others, last to first (which keeps L+ triangular): S is the innovation
// variance, k = P h / sqrt S, and L+ a factor of the updated covariance.
//
// An exposure end then zeroes its integrator's row of L and of the mean, as
// the covariance form does.
#pragma once

#include "gp_ssm_filter.h"

namespace gpssm {

// position of entry (i, j), j <= i, of a row-packed lower triangle
__host__ __device__ constexpr int lidx(int i, int j) { return i * (i + 1) / 2 + j; }

// the plane rotation taking (a, b) to (r, 0): c = a / r, s = b / r; the
// identity when both vanish.  The pair is first scaled by the power of two of
// the larger entry (exactly), so that the squares neither underflow nor
// overflow: a pivot pair scaled down by a long step's transition (e^(-alpha
// dt) of 1e-153 squares to the subnormal range) would otherwise give (c, s)
// off the unit circle, and the rotation would distort every other row of the
// two columns it mixes.
__device__ __forceinline__ void plane_rotation(double a, double b, double& c, double& s, double& r) {
  const double mx = fmax(fabs(a), fabs(b));
  if (mx > 0.0) {
    int e;
    (void)frexp(mx, &e);
    const double as = ldexp(a, -e), bs = ldexp(b, -e);
    const double rs = sqrt(fma(as, as, bs * bs));
    const double ir = 1.0 / rs;
    c = as * ir;
    s = bs * ir;
    r = ldexp(rs, e);
  } else {
    c = 1.0;
    s = 0.0;
    r = 0.0;
  }
}

// rank-one update L L^T + n n^T of the factor; n is zero above row k0 (a
// constant once the callers' loops are unrolled)
template <int D>
__device__ __forceinline__ void factor_update(double* L, double* n, int k0) {
#pragma unroll
  for (int r = k0; r < D; ++r) {
    double c, s, rr;
    plane_rotation(L[lidx(r, r)], n[r], c, s, rr);
    L[lidx(r, r)] = rr;
#pragma unroll
    for (int i = r + 1; i < D; ++i) {
      const double l = L[lidx(i, r)];
      L[lidx(i, r)] = fma(c, l, s * n[i]);
      n[i] = fma(-s, l, c * n[i]);
    }
  }
}

// time update of (m, L) over one step (tq: the terms' step quantities, open:
// the integrators open during the step)
template <class Dm>
__device__ __forceinline__ void sqrt_predict(double* m, double* L, const TermQ* tq, uint32_t open) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D;
  predict_mean<Dm>(m, tq, open);
  double oj[J];
#pragma unroll
  for (int j = 0; j < J; ++j) oj[j] = ((open >> j) & 1u) ? 1.0 : 0.0;
  // integrator rows: + fbar . (x rows of L), read before the transition
#pragma unroll
  for (int c = 0; c < NX; ++c) {
    double fx = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
      if (2 * t >= c) fx = fma(tq[t].f0, L[lidx(2 * t, c)], fx);
      if (2 * t + 1 >= c) fx = fma(tq[t].f1, L[lidx(2 * t + 1, c)], fx);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) L[lidx(NX + j, c)] = fma(oj[j], fx, L[lidx(NX + j, c)]);
  }
  // x rows: Phi_t applied to rows (2t, 2t+1); the entry (2t, 2t+1) it
  // creates above the diagonal is kept in sup[t]
  double sup[M];
#pragma unroll
  for (int t = 0; t < M; ++t) {
#pragma unroll
    for (int c = 0; c <= 2 * t; ++c) {
      const double x0 = L[lidx(2 * t, c)], x1 = L[lidx(2 * t + 1, c)];
      L[lidx(2 * t, c)] = fma(tq[t].a00, x0, tq[t].a01 * x1);
      L[lidx(2 * t + 1, c)] = fma(-tq[t].a01, x0, tq[t].a11 * x1);
    }
    const double x1 = L[lidx(2 * t + 1, 2 * t + 1)];
    sup[t] = tq[t].a01 * x1;
    L[lidx(2 * t + 1, 2 * t + 1)] = tq[t].a11 * x1;
  }
  // rotate columns (2t, 2t+1) to clear sup[t]; rows 2t and below
#pragma unroll
  for (int t = 0; t < M; ++t) {
    double c, s, r;
    plane_rotation(L[lidx(2 * t, 2 * t)], sup[t], c, s, r);
    L[lidx(2 * t, 2 * t)] = r;
#pragma unroll
    for (int i = 2 * t + 1; i < D; ++i) {
      const double l0 = L[lidx(i, 2 * t)], l1 = L[lidx(i, 2 * t + 1)];
      L[lidx(i, 2 * t)] = fma(c, l0, s * l1);
      L[lidx(i, 2 * t + 1)] = fma(-s, l0, c * l1);
    }
  }
  // process noise: per term the Cholesky factor of Q3 (order x, x', integral;
  // a pivot that rounding leaves at or below zero gives a zero column, as for
  // a real term's absent second state), its columns added one by one
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const TermQ& q = tq[t];
    const double l00 = sqrt(fmax(q.q00, 0.0));
    const double i00 = l00 > 0.0 ? 1.0 / l00 : 0.0;
    const double l10 = q.q01 * i00, l20 = q.c0 * i00;
    const double l11 = sqrt(fmax(fma(-l10, l10, q.q11), 0.0));
    const double i11 = l11 > 0.0 ? 1.0 / l11 : 0.0;
    const double l21 = fma(-l20, l10, q.c1) * i11;
    const double l22 = sqrt(fmax(q.zz - fma(l20, l20, l21 * l21), 0.0));
    double n[D];
    // column 0: (l00, l10, l20)
#pragma unroll
    for (int i = 0; i < D; ++i) n[i] = 0.0;
    n[2 * t] = l00;
    n[2 * t + 1] = l10;
#pragma unroll
    for (int j = 0; j < J; ++j) n[NX + j] = oj[j] * l20;
    factor_update<D>(L, n, 2 * t);
    // column 1: (0, l11, l21)
#pragma unroll
    for (int i = 0; i < D; ++i) n[i] = 0.0;
    n[2 * t + 1] = l11;
#pragma unroll
    for (int j = 0; j < J; ++j) n[NX + j] = oj[j] * l21;
    factor_update<D>(L, n, 2 * t + 1);
    // column 2: (0, 0, l22), integrators only
#pragma unroll
    for (int i = 0; i < D; ++i) n[i] = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) n[NX + j] = oj[j] * l22;
    factor_update<D>(L, n, NX);
  }
}

// measurement update (when the event carries one) and the exposure's reset;
// returns the log-likelihood term
template <class Dm>
__device__ __forceinline__ double sqrt_update(double* m, double* L, uint32_t info, const Obs& o) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D;
  double ll = 0.0;
  if (o.has) {
    // h^T L, column by column
    double a[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < J; ++j)
        if (NX + j >= k) acc = fma(o.a[j], L[lidx(NX + j, k)], acc);
      double xs = 0.0;
#pragma unroll
      for (int t = 0; t < M; ++t)
        if (2 * t >= k) xs += L[lidx(2 * t, k)];
      a[k] = fma(o.b, xs, acc);
    }
    double r0 = sqrt(o.R);
    double g[D];
#pragma unroll
    for (int i = 0; i < D; ++i) g[i] = 0.0;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
      double c, s, r;
      plane_rotation(r0, a[k], c, s, r);
      r0 = r;
#pragma unroll
      for (int i = k; i < D; ++i) {
        const double l = L[lidx(i, k)];
        L[lidx(i, k)] = fma(-s, g[i], c * l);
        g[i] = fma(c, g[i], s * l);
      }
    }
    const double w = (o.y - obs_dot<Dm>(m, o)) / r0;
#pragma unroll
    for (int i = 0; i < D; ++i) m[i] = fma(g[i], w, m[i]);
    ll = -0.5 * (LOG_2PI + 2.0 * log(r0) + w * w);
  }
  const bool end = ev_kind(info) == EV_END;
  const uint32_t slot = ev_slot(info);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const bool z = end && (uint32_t)j == slot;
    m[NX + j] = z ? 0.0 : m[NX + j];
#pragma unroll
    for (int c = 0; c <= NX + j; ++c) L[lidx(NX + j, c)] = z ? 0.0 : L[lidx(NX + j, c)];
  }
  return ll;
}

}  // namespace gpssm
