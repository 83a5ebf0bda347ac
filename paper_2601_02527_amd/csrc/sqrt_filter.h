// Square-root (Cholesky-factor) form of the sequential filter: the steps of
// one event, spread over a group of SQ_GROUP lanes per series (the kernel is
// k_sqrt in kernels_impl.h).
//
// The covariance of the augmented state is carried as a lower-triangular
// factor L with P = L L^T, so that every covariance the filter forms is
// positive semidefinite by construction: the factor-form remedy that
// Sec. 3.2.3 and Sec. 5 name for the loss of accuracy of the covariance form
// on nearly noise-free data.
//
// Lane q of a group holds row q of L and entry q of the mean (rows q >= D are
// zero and stay so).  Operations on columns (rotations, reflections from the
// right) are then local to each lane once their parameters are known; the
// transition, which mixes rows, needs the partner row of each term block and
// one sum over the term rows.
//
// Time update.  With the augmented transition A (Sec. 2.4: the blocks Phi_m
// and the integrated rows fbar_m added into the open integrators) and the
// process noise of term m over the step, G_m Q3_m G_m^T (Q3_m the covariance
// of (x_m, x_m', the integral of x_m), G_m placing the integral in every open
// integrator), the new factor is the triangular part of the rows [A L | N],
// N the columns G_m chol(Q3_m): Householder reflections from the right, one
// per pivot row, each built from the pivot row (broadcast from its lane) and
// applied by every lane to its own row.
//
// Measurement update.  With h the observation row and R the noise variance,
// the array [[sqrt R, h^T L], [0, L]] is brought to the lower-triangular form
// [[sqrt S, 0], [k, L+]] by plane rotations of its first column against the
// others, last to first (which keeps L+ triangular): S is the innovation
// variance, k = P h / sqrt S, and L+ a factor of the updated covariance.  The
// rotations depend only on sqrt R and h^T L, which every lane of the group
// holds, so each lane computes them itself.
//
// An exposure end then zeroes its integrator's row of L and of the mean, as
// the covariance form does.
//
// Reflections and rotations scale their vector by the power of two of its
// largest entry (exactly) before squaring: entries scaled down by a long
// step's transition (e^(-alpha dt) of 1e-153 for a term with omega0 860/d over
// a day) square into the subnormal range, and a reflection or rotation formed
// from such squares is no longer orthogonal and distorts every other row.
#pragma once

#include "gp_ssm_filter.h"
#include "plan.h"

namespace gpssm {

constexpr int SQ_GROUP = 16;  // lanes per series (at least the largest state dimension)
static_assert(SQ_GROUP >= 2 * MAX_TERMS + MAX_SLOTS, "one lane per state row");
static_assert(SQ_GROUP == 16, "a group is one DPP row");

// Exchanges within a group, which is one 16-lane DPP row: both 32-bit halves
// of a double moved by a DPP pattern (0xB1: quad_perm 1,0,3,2, the lane at
// xor distance 1; 0x4E: quad_perm 2,3,0,1, distance 2; 0x141: each half row
// mirrored; 0x140: the row mirrored; 0x150 + i: lane i of the row broadcast)
template <int CTRL>
__device__ __forceinline__ double row_dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// v of the partner row (2t <-> 2t+1)
__device__ __forceinline__ double grp_partner(double v) { return row_dpp<0xB1>(v); }
// sum of v over the group, on every lane
__device__ __forceinline__ double grp_sum(double v) {
  v += row_dpp<0xB1>(v);
  v += row_dpp<0x4E>(v);
  v += row_dpp<0x141>(v);
  return v + row_dpp<0x140>(v);
}
// v of lane i of the group; i must be a constant once the caller's loops are
// unrolled (the switch then folds to one case)
__device__ __forceinline__ double grp_get(double v, int i) {
  switch (i) {
    case 0: return row_dpp<0x150>(v);
    case 1: return row_dpp<0x151>(v);
    case 2: return row_dpp<0x152>(v);
    case 3: return row_dpp<0x153>(v);
    case 4: return row_dpp<0x154>(v);
    case 5: return row_dpp<0x155>(v);
    case 6: return row_dpp<0x156>(v);
    case 7: return row_dpp<0x157>(v);
    case 8: return row_dpp<0x158>(v);
    case 9: return row_dpp<0x159>(v);
    case 10: return row_dpp<0x15A>(v);
    case 11: return row_dpp<0x15B>(v);
    case 12: return row_dpp<0x15C>(v);
    case 13: return row_dpp<0x15D>(v);
    case 14: return row_dpp<0x15E>(v);
    default: return row_dpp<0x15F>(v);
  }
}

// fields of a chunk summary of the time-split square-root filter (N the SHO
// state size; per chunk, field f at f * n_chunks + chunk): A (N x N, row
// major), b (N), U (lower triangle by rows), Z ((N + 1) x (N + 1) lower
// triangle by rows), c0
__host__ __device__ constexpr int sq_A(int) { return 0; }
__host__ __device__ constexpr int sq_b(int N) { return N * N; }
__host__ __device__ constexpr int sq_U(int N) { return N * N + N; }
__host__ __device__ constexpr int sq_Z(int N) { return N * N + N + N * (N + 1) / 2; }
__host__ __device__ constexpr int sq_c0(int N) { return sq_Z(N) + (N + 1) * (N + 2) / 2; }
__host__ __device__ constexpr int sq_fields(int N) { return sq_c0(N) + 1; }
// position of entry (i, j), j <= i, of a lower triangle packed by rows
__host__ __device__ constexpr int lidx(int i, int j) { return i * (i + 1) / 2 + j; }

// the step quantities of lane i's term
__device__ __forceinline__ TermQ grp_get_term(const TermQ& u, int i) {
  TermQ r;
  r.a00 = grp_get(u.a00, i);
  r.a01 = grp_get(u.a01, i);
  r.a11 = grp_get(u.a11, i);
  r.f0 = grp_get(u.f0, i);
  r.f1 = grp_get(u.f1, i);
  r.q00 = grp_get(u.q00, i);
  r.q01 = grp_get(u.q01, i);
  r.q11 = grp_get(u.q11, i);
  r.c0 = grp_get(u.c0, i);
  r.c1 = grp_get(u.c1, i);
  r.zz = grp_get(u.zz, i);
  return r;
}

// the plane rotation taking (a, b) to (r, 0): c = a / r, s = b / r; the
// identity when both vanish (scaled as stated above)
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

// whether the reflection of pivot row i involves column c of [A L | N] (the
// noise columns D + 3t, D + 3t + 1, D + 3t + 2 belong to term t)
template <int NX, int D>
__device__ __forceinline__ constexpr bool sq_involved(int i, int c) {
  return c == i || (c == i + 1 && i < NX && (i & 1) == 0) || (c >= D && (i >= NX || (c - D) / 3 <= i / 2));
}

// time update of this lane's row (row[0..D) of L, then the 3M noise columns,
// rebuilt here) and of its NE entries ext that the transition maps like the
// mean (ext[0] the mean entry; the conditional filter's sensitivity row
// follows); q: the lane's row, tq: the terms' step quantities, open: the
// integrators open during the step
template <class Dm, int NE>
__device__ __forceinline__ void sqrt_predict_row(double* row, double* ext, int q, const TermQ* tq, uint32_t open) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D, NC = D + 3 * M;
  // the integrators' increment fbar . (old x rows | old x entries of ext),
  // summed over the group (lanes outside the x rows contribute zero)
  double sum[D + NE];
  {
    double f = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
      f = (q == 2 * t) ? tq[t].f0 : f;
      f = (q == 2 * t + 1) ? tq[t].f1 : f;
    }
#pragma unroll
    for (int c = 0; c < D; ++c) sum[c] = f * row[c];
#pragma unroll
    for (int e = 0; e < NE; ++e) sum[D + e] = f * ext[e];
#pragma unroll
    for (int c = 0; c < D + NE; ++c) sum[c] = grp_sum(sum[c]);
  }
  // x rows: Phi_t applied to the rows (2t, 2t+1), partners at xor distance 1:
  // row 2t' = a00 row 2t + a01 row 2t+1, row 2t+1' = -a01 row 2t + a11 row 2t+1
  {
    double as = 1.0, ap = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
      as = (q == 2 * t) ? tq[t].a00 : ((q == 2 * t + 1) ? tq[t].a11 : as);
      ap = (q == 2 * t) ? tq[t].a01 : ((q == 2 * t + 1) ? -tq[t].a01 : ap);
    }
    const bool xrow = q < NX;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double pc = grp_partner(row[c]);
      row[c] = xrow ? fma(as, row[c], ap * pc) : row[c];
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double pe = grp_partner(ext[e]);
      ext[e] = xrow ? fma(as, ext[e], ap * pe) : ext[e];
    }
  }
  // open integrator rows: + the increment
  double oq = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) oq = (q == NX + j && ((open >> j) & 1u)) ? 1.0 : oq;
#pragma unroll
  for (int c = 0; c < D; ++c) row[c] = fma(oq, sum[c], row[c]);
#pragma unroll
  for (int e = 0; e < NE; ++e) ext[e] = fma(oq, sum[D + e], ext[e]);
  // noise columns: this row of G_m chol(Q3_m) for every term (a pivot that
  // rounding leaves at or below zero gives a zero column, as for a real term's
  // absent second state)
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const TermQ& u = tq[t];
    const double l00 = sqrt(fmax(u.q00, 0.0));
    const double i00 = l00 > 0.0 ? 1.0 / l00 : 0.0;
    const double l10 = u.q01 * i00, l20 = u.c0 * i00;
    const double l11 = sqrt(fmax(fma(-l10, l10, u.q11), 0.0));
    const double i11 = l11 > 0.0 ? 1.0 / l11 : 0.0;
    const double l21 = fma(-l20, l10, u.c1) * i11;
    const double l22 = sqrt(fmax(u.zz - fma(l20, l20, l21 * l21), 0.0));
    const double e0 = (q == 2 * t) ? 1.0 : 0.0, e1 = (q == 2 * t + 1) ? 1.0 : 0.0;
    row[D + 3 * t] = fma(e0, l00, fma(e1, l10, oq * l20));
    row[D + 3 * t + 1] = fma(e1, l11, oq * l21);
    row[D + 3 * t + 2] = oq * l22;
  }
  // triangularise [A L | N]: for pivot row i, the reflection that takes its
  // entries in the columns it involves to (alpha, 0, ...), applied by every
  // lane to its row.  Row i is nonzero beyond column i only in column i + 1
  // when that holds its term block's entry above the diagonal, and in the
  // noise columns of the terms whose rows it has met (terms up to its own for
  // a term row, every term for an integrator row): the other columns keep
  // their zeros in the rows above and below and are left out.
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double v[NC];
#pragma unroll
    for (int c = i; c < NC; ++c)
      if (sq_involved<NX, D>(i, c)) v[c] = grp_get(row[c], i);
    double mx = 0.0;
#pragma unroll
    for (int c = i; c < NC; ++c)
      if (sq_involved<NX, D>(i, c)) mx = fmax(mx, fabs(v[c]));
    if (mx > 0.0) {
      int e;
      (void)frexp(mx, &e);
      double n2 = 0.0;
#pragma unroll
      for (int c = i; c < NC; ++c)
        if (sq_involved<NX, D>(i, c)) {
          v[c] = ldexp(v[c], -e);
          n2 = fma(v[c], v[c], n2);
        }
      const double nrm = sqrt(n2);
      const double alpha = v[i] >= 0.0 ? -nrm : nrm;
      // v - alpha e_i, whose squared norm is 2 nrm (nrm + |v_i|)
      const double vv = 2.0 * nrm * (nrm + fabs(v[i]));
      v[i] -= alpha;
      const double beta = 2.0 / vv;
      double w = 0.0;
#pragma unroll
      for (int c = i; c < NC; ++c)
        if (sq_involved<NX, D>(i, c)) w = fma(row[c], v[c], w);
      w *= beta;
#pragma unroll
      for (int c = i; c < NC; ++c)
        if (sq_involved<NX, D>(i, c)) row[c] = fma(-w, v[c], row[c]);
      if (q == i) {
        row[i] = ldexp(alpha, e);
#pragma unroll
        for (int c = i + 1; c < NC; ++c) row[c] = 0.0;
      }
    }
  }
}

// measurement update (when the event carries one) and the exposure's reset of
// this lane's row and its entries ext (ext[0] the mean entry; the others, a
// sensitivity row of the mean, are updated like it with the measurement
// taken as zero); returns the log-likelihood term and, in wz (NE entries, when
// given), h^T ext / sqrt S with the innovation in place of h^T ext[0], and in
// *rs sqrt S, all the same on every lane of the group (wz zero and *rs one
// when there is no measurement)
template <class Dm, int NE>
__device__ __forceinline__ double sqrt_update_row(double* row, double* ext, int q, uint32_t info, const Obs& o,
                                                  double* wz = nullptr, double* rs = nullptr) {
  constexpr int M = Dm::M, NX = Dm::NX, D = Dm::D;
  const uint32_t kind = ev_kind(info);
  const int z = NX + (int)ev_slot(info);  // the closing integrator's row
  double ll = 0.0;
  if (wz) {
#pragma unroll
    for (int e = 0; e < NE; ++e) wz[e] = 0.0;
  }
  if (rs) *rs = 1.0;
  if (o.has) {
    // h^T L and h^T ext: the slot's row over its exposure length at an end,
    // the sum of the terms' first rows at an instantaneous measurement
    double a[D + NE];
    if (kind == EV_END) {
      // the slot's lane, selected among the integrator rows
      const uint32_t slot = ev_slot(info);
      double invd = 0.0;
#pragma unroll
      for (int j = 0; j < Dm::J; ++j) invd += o.a[j];  // one nonzero entry, the slot's
#pragma unroll
      for (int k = 0; k < D + NE; ++k) {
        const double x = k < D ? row[k] : ext[k - D];
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < Dm::J; ++j) {
          const double vj = grp_get(x, NX + j);
          v = (slot == (uint32_t)j) ? vj : v;
        }
        a[k] = v * invd;
      }
    } else {
      double wq = 0.0;
#pragma unroll
      for (int t = 0; t < M; ++t) wq = (q == 2 * t) ? 1.0 : wq;
#pragma unroll
      for (int k = 0; k < D + NE; ++k) a[k] = grp_sum(wq * (k < D ? row[k] : ext[k - D]));
    }
    double r0 = sqrt(o.R), g = 0.0;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
      double c, s, r;
      plane_rotation(r0, a[k], c, s, r);
      r0 = r;
      const double l = row[k];
      row[k] = fma(-s, g, c * l);
      g = fma(c, g, s * l);
    }
    const double w = (o.y - a[D]) / r0;
    ext[0] = fma(g, w, ext[0]);
#pragma unroll
    for (int e = 1; e < NE; ++e) ext[e] = fma(-g, a[D + e] / r0, ext[e]);
    if (rs) *rs = r0;
    if (wz) {
      wz[0] = w;
#pragma unroll
      for (int e = 1; e < NE; ++e) wz[e] = a[D + e] / r0;
    }
    ll = -0.5 * (LOG_2PI + 2.0 * log(r0) + w * w);
  }
  if (kind == EV_END && q == z) {
#pragma unroll
    for (int c = 0; c < D; ++c) row[c] = 0.0;
#pragma unroll
    for (int e = 0; e < NE; ++e) ext[e] = 0.0;
  }
  return ll;
}

}  // namespace gpssm
