// Chunk-level pieces of the augmented filter:
//
//  * the conditional filter of one chunk: the filter run with the state at
//    the chunk's start boundary treated as known (x_b), which makes the mean
//    affine in x_b (m = S x_b + mu) while the covariance does not depend on
//    it.  Its result is the chunk summary (A, b, C, eta, J, c0):
//      x_end | x_b, y_chunk ~ N(A x_b + b, C)
//      log p(y_chunk | x_b) = -c0/2 + eta^T x_b - x_b^T J x_b / 2,
//    the five-tuple of the parallel filter (Sec. 3.2.4, following SG21)
//    extended by the likelihood constant.  Chunks start and end where every
//    exposure is closed, so x_b and x_end are the SHO states only.
//  * the combination of a filtered boundary state with a summary (next
//    boundary state and the chunk's likelihood contribution), the backward
//    recursion of the future likelihood (eta~, J~), and from it the gradient
//    of the future likelihood with respect to the boundary moments.
//  * the smoother's backward sweep in adjoint (Bryson-Frazier) form.
//  * the reverse-mode adjoint of one plain filter step, accumulating the
//    gradient with respect to (sigma, omega0, Q) of every term and jitter.
#pragma once

#include "gp_ssm_math.h"

namespace gpssm {

// ---------------------------------------------------------------------------
// conditional filter of a chunk
// ---------------------------------------------------------------------------
// A lane's slots of an LDS array laid out field-major across the wavefront:
// element f at base[f * 64].
struct LaneLds {
  double* base;
  GPD double& operator[](int f) const { return base[f * 64]; }
};

// SL: the sensitivity block S lives in LDS (a LaneLds view set by the
// caller before init) instead of registers.  IL: likewise the information
// accumulators (J, eta, c0), which change once per event.
template <class Dm, bool SL = false, bool IL = false>
struct CondState {
  static constexpr int D = Dm::D, NX = Dm::NX, NP = Dm::NP, NXP = Dm::NXP;
  static constexpr int NINFO = NXP + NX + 1;  // fields of the information accumulators
  double P[NP];
  double mu[D];
  double Sr[SL ? 1 : D * NX];  // d mean / d x_b, row-major
  LaneLds Sl;
  double Ir[IL ? 1 : NINFO];  // J (packed), eta, c0
  LaneLds Il;

  GPD double& S(int i) {
    if constexpr (SL)
      return Sl[i];
    else
      return Sr[i];
  }
  GPD double& info(int i) {
    if constexpr (IL)
      return Il[i];
    else
      return Ir[i];
  }
  GPD double& Jm(int i) { return info(i); }
  GPD double& eta(int i) { return info(NXP + i); }
  GPD double& c0() { return info(NXP + NX); }

  GPD void init() {
#pragma unroll
    for (int i = 0; i < NP; ++i) P[i] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) mu[i] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int c = 0; c < NX; ++c) S(i * NX + c) = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < NINFO; ++i) info(i) = 0.0;
  }

  // one event: predict over the step that ends at it, then its observation.
  // S is processed one column at a time in two passes (predict and project;
  // then the rank-one update and the slot close), so that only one column is
  // live at once.
  GPD void step(const TermQ* tq, uint32_t info, const Obs& o) {
    constexpr int M = Dm::M, J = Dm::J;
    const uint32_t open = ev_open(info);
    predict_mean<Dm>(mu, tq, open);
    predict_cov<Dm>(P, tq, open);
    double u[D];
    obs_gain<Dm>(P, o, u);
    const double S_ = obs_dot<Dm>(u, o) + o.R;
    const double iS = 1.0 / S_;
    const double r = o.y - obs_dot<Dm>(mu, o);
    double a[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      double col[D];
#pragma unroll
      for (int i = 0; i < D; ++i) col[i] = S(i * NX + c);
      double fx = 0.0;
#pragma unroll
      for (int t = 0; t < M; ++t) fx = fma(tq[t].f0, col[2 * t], fma(tq[t].f1, col[2 * t + 1], fx));
#pragma unroll
      for (int t = 0; t < M; ++t) {
        const double x0 = col[2 * t], x1 = col[2 * t + 1];
        col[2 * t] = fma(tq[t].a00, x0, tq[t].a01 * x1);
        col[2 * t + 1] = fma(-tq[t].a01, x0, tq[t].a11 * x1);
      }
#pragma unroll
      for (int j = 0; j < J; ++j) col[NX + j] += ((open >> j) & 1u) ? fx : 0.0;
      a[c] = obs_dot<Dm>(col, o);
#pragma unroll
      for (int i = 0; i < D; ++i) S(i * NX + c) = col[i];
    }
    if constexpr (SL) table_fence();
    const double riS = r * iS;
#pragma unroll
    for (int i = 0; i < D; ++i) mu[i] = fma(u[i], riS, mu[i]);
    const bool end = ev_kind(info) == EV_END;
    const uint32_t slot = ev_slot(info);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double ui = u[i] * iS;
      // integrator rows of the slot closed by this event end at zero
      const bool z = (i >= NX) && end && (uint32_t)(i - NX) == slot;
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        const double v = fma(-ui, a[c], S(i * NX + c));
        S(i * NX + c) = z ? 0.0 : v;
      }
#pragma unroll
      for (int j = i; j < D; ++j) P[sidx(i, j, D)] = fma(-ui, u[j], P[sidx(i, j, D)]);
    }
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const double ac = a[c] * iS;
      eta(c) = fma(ac, r, eta(c));
#pragma unroll
      for (int d = c; d < NX; ++d) Jm(sidx(c, d, NX)) = fma(ac, a[d], Jm(sidx(c, d, NX)));
    }
    if (o.has) c0() += LOG_2PI + log(S_) + r * riS;
    close_slot<Dm>(mu, P, info);
  }
};

// number of doubles in a chunk summary for NX SHO states
GPD constexpr int summary_size(int NX) { return NX * NX + NX + NX * (NX + 1) / 2 + NX + NX * (NX + 1) / 2 + 1; }
// field offsets: A (NX*NX, row-major), b (NX), C (packed), eta (NX), J (packed), c0
GPD constexpr int sum_A(int) { return 0; }
GPD constexpr int sum_b(int NX) { return NX * NX; }
GPD constexpr int sum_C(int NX) { return NX * NX + NX; }
GPD constexpr int sum_eta(int NX) { return NX * NX + NX + NX * (NX + 1) / 2; }
GPD constexpr int sum_J(int NX) { return NX * NX + 2 * NX + NX * (NX + 1) / 2; }
GPD constexpr int sum_c0(int NX) { return NX * NX + 2 * NX + NX * (NX + 1); }

// ---------------------------------------------------------------------------
// small dense linear algebra (N <= 8), static indexing only
// ---------------------------------------------------------------------------
// Solves A X = B in place (A: N x N row-major, B: N x R row-major) by
// Gaussian elimination with partial pivoting.  Returns log|det A| and sets
// ok = false on a zero pivot.
template <int N, int R>
GPD double lu_solve(double* A, double* B, bool& ok) {
  double logdet = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    // pivot search
    int p = k;
    double best = fabs(A[k * N + k]);
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const double v = fabs(A[i * N + k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    // swap rows k and p (select-based, static indices)
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const bool sw = (i == p);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const double a = A[k * N + c], b = A[i * N + c];
        A[k * N + c] = sw ? b : a;
        A[i * N + c] = sw ? a : b;
      }
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const double a = B[k * R + c], b = B[i * R + c];
        B[k * R + c] = sw ? b : a;
        B[i * R + c] = sw ? a : b;
      }
    }
    const double piv = A[k * N + k];
    ok = ok && (piv != 0.0);
    logdet += log(fabs(piv));
    const double ip = 1.0 / piv;
    A[k * N + k] = ip;  // kept as its reciprocal for the back substitution
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const double f = A[i * N + k] * ip;
#pragma unroll
      for (int c = k + 1; c < N; ++c) A[i * N + c] = fma(-f, A[k * N + c], A[i * N + c]);
#pragma unroll
      for (int c = 0; c < R; ++c) B[i * R + c] = fma(-f, B[k * R + c], B[i * R + c]);
    }
  }
  // back substitution
#pragma unroll
  for (int k = N - 1; k >= 0; --k) {
    const double ip = A[k * N + k];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double v = B[k * R + c];
#pragma unroll
      for (int j = k + 1; j < N; ++j) v = fma(-A[k * N + j], B[j * R + c], v);
      B[k * R + c] = v * ip;
    }
  }
  return logdet;
}

template <int N>
GPD void unpack(const double* p, double* F) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) F[i * N + j] = p[sidx(i, j, N)];
}

// ---------------------------------------------------------------------------
// combination of a filtered boundary state (m, P) with a chunk summary
// ---------------------------------------------------------------------------
// in: m[N], P packed; summary s (read through an accessor); out: next (m, P)
// packed and the chunk's log-likelihood contribution.
template <int N, class Get>
GPD double combine_forward(const double* m, const double* Pp, Get s, double* mn, double* Pn, bool& ok) {
  double P[N * N], Jf[N * N];
  unpack<N>(Pp, P);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Jf[i * N + j] = s(sum_J(N) + sidx(i, j, N));
  // r = eta - J m
  double r[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double v = s(sum_eta(N) + i);
#pragma unroll
    for (int j = 0; j < N; ++j) v = fma(-Jf[i * N + j], m[j], v);
    r[i] = v;
  }
  // (I + P J) [W | w] = [P | P r]
  double A[N * N], B[N * (N + 1)];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(P[i * N + k], Jf[k * N + j], v);
      A[i * N + j] = v;
      B[i * (N + 1) + j] = P[i * N + j];
    }
    double pr = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) pr = fma(P[i * N + k], r[k], pr);
    B[i * (N + 1) + N] = pr;
  }
  const double logdet = lu_solve<N, N + 1>(A, B, ok);
  // likelihood contribution
  double etm = 0.0, mJm = 0.0, rw = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    etm = fma(s(sum_eta(N) + i), m[i], etm);
    double Jmi = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) Jmi = fma(Jf[i * N + j], m[j], Jmi);
    mJm = fma(m[i], Jmi, mJm);
    rw = fma(r[i], B[i * (N + 1) + N], rw);
  }
  const double ll = -0.5 * s(sum_c0(N)) + etm - 0.5 * mJm - 0.5 * logdet + 0.5 * rw;
  // posterior of x_b, then the chunk's transition
  double mt[N], W[N * N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    mt[i] = m[i] + B[i * (N + 1) + N];
#pragma unroll
    for (int j = 0; j < N; ++j) W[i * N + j] = 0.5 * (B[i * (N + 1) + j] + B[j * (N + 1) + i]);
  }
  double AW[N * N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double v = s(sum_b(N) + i);
#pragma unroll
    for (int k = 0; k < N; ++k) v = fma(s(sum_A(N) + i * N + k), mt[k], v);
    mn[i] = v;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double w = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) w = fma(s(sum_A(N) + i * N + k), W[k * N + j], w);
      AW[i * N + j] = w;
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double v = s(sum_C(N) + sidx(i, j, N));
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(AW[i * N + k], s(sum_A(N) + j * N + k), v);
      Pn[sidx(i, j, N)] = v;
    }
  return ll;
}

// future likelihood at this chunk's start from the one at its end:
//   J~ = J + A^T (I + J~' C)^-1 J~' A,  eta~ = eta + A^T (I + J~' C)^-1 (eta~' - J~' b)
template <int N, class Get>
GPD void future_step(Get s, const double* Jn, const double* en, double* Jo, double* eo, bool& ok) {
  double Jf[N * N], C[N * N];
  unpack<N>(Jn, Jf);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) C[i * N + j] = s(sum_C(N) + sidx(i, j, N));
  double A[N * N], B[N * (N + 1)];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(Jf[i * N + k], C[k * N + j], v);
      A[i * N + j] = v;
      double w = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) w = fma(Jf[i * N + k], s(sum_A(N) + k * N + j), w);
      B[i * (N + 1) + j] = w;
    }
    double w = en[i];
#pragma unroll
    for (int k = 0; k < N; ++k) w = fma(-Jf[i * N + k], s(sum_b(N) + k), w);
    B[i * (N + 1) + N] = w;
  }
  lu_solve<N, N + 1>(A, B, ok);
  // A_c^T Y
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double e = s(sum_eta(N) + i);
#pragma unroll
    for (int k = 0; k < N; ++k) e = fma(s(sum_A(N) + k * N + i), B[k * (N + 1) + N], e);
    eo[i] = e;
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        a = fma(s(sum_A(N) + k * N + i), B[k * (N + 1) + j], a);
        b = fma(s(sum_A(N) + k * N + j), B[k * (N + 1) + i], b);
      }
      Jo[sidx(i, j, N)] = s(sum_J(N) + sidx(i, j, N)) + 0.5 * (a + b);
    }
}

// A chunk summary (or a composition of consecutive ones) in registers.
template <int N>
struct Elem {
  static constexpr int NP = N * (N + 1) / 2;
  double A[N * N], b[N], C[NP], eta[N], J[NP];

  GPD void identity() {
#pragma unroll
    for (int i = 0; i < N * N; ++i) A[i] = (i % (N + 1) == 0) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = eta[i] = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) C[i] = J[i] = 0.0;
  }
  template <class Get>
  GPD void load(Get g) {
#pragma unroll
    for (int i = 0; i < N * N; ++i) A[i] = g(sum_A(N) + i);
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = g(sum_b(N) + i);
#pragma unroll
    for (int i = 0; i < NP; ++i) C[i] = g(sum_C(N) + i);
#pragma unroll
    for (int i = 0; i < N; ++i) eta[i] = g(sum_eta(N) + i);
#pragma unroll
    for (int i = 0; i < NP; ++i) J[i] = g(sum_J(N) + i);
  }
  template <class Put>
  GPD void store(Put p) const {
#pragma unroll
    for (int i = 0; i < N * N; ++i) p(sum_A(N) + i, A[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) p(sum_b(N) + i, b[i]);
#pragma unroll
    for (int i = 0; i < NP; ++i) p(sum_C(N) + i, C[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) p(sum_eta(N) + i, eta[i]);
#pragma unroll
    for (int i = 0; i < NP; ++i) p(sum_J(N) + i, J[i]);
  }
  // accessor in the summary field numbering (c0 reads as 0)
  GPD double get(int f) const {
    if (f < sum_b(N)) return A[f];
    if (f < sum_C(N)) return b[f - sum_b(N)];
    if (f < sum_eta(N)) return C[f - sum_C(N)];
    if (f < sum_J(N)) return eta[f - sum_eta(N)];
    if (f < sum_c0(N)) return J[f - sum_J(N)];
    return 0.0;
  }
};

// A lane's element in an LDS exchange area laid out [field][lane] (ST lanes
// per field) in the summary field numbering, with the same indexing as
// Elem<N>.
template <int N, int ST = 64>
struct ElemLds {
  struct Field {
    const double* p;
    GPD double operator[](int i) const { return p[i * ST]; }
  };
  Field A, b, C, eta, J;
  GPD explicit ElemLds(const double* base)
      : A{base + sum_A(N) * ST}, b{base + sum_b(N) * ST}, C{base + sum_C(N) * ST}, eta{base + sum_eta(N) * ST},
        J{base + sum_J(N) * ST} {}
};

// Associative composition of two consecutive summaries (i earlier, j
// later), the filtering operator of the parallel Kalman filter (SG21):
//   X = (I + C_i J_j)^-1
//   A = A_j X A_i,  b = A_j X (b_i + C_i eta_j) + b_j,  C = A_j X C_i A_j^T + C_j
//   eta = A_i^T X^T (eta_j - J_j b_i) + eta_i,  J = A_i^T J_j X A_i + J_i
// X is never formed: one LU solve gives [X A_i | X (b_i + C_i eta_j) | X C_i]
// (an explicit inverse loses accuracy the smoothed moments need), and
// X^T v = v - J_j (X C_i) v follows from X^T = (I + J_j C_i)^-1.
// The inputs are Elem<N> in registers or ElemLds<N> views, read where they
// are used, so that only the solve and the result occupy registers; the
// result o may alias neither input.  The fences between the stages keep the
// compiler from hoisting every operand read to the top.
template <int N, class EI, class EJ>
GPD void compose(const EI& ei, const EJ& ej, Elem<N>& o, bool& ok) {
  constexpr int R = 2 * N + 1;
  double B[N * R];
  {
    double Mx[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        double v = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) v = fma(ei.C[sidx(r, k, N)], ej.J[sidx(k, c, N)], v);
        Mx[r * N + c] = v;
        B[r * R + c] = ei.A[r * N + c];
        B[r * R + N + 1 + c] = ei.C[sidx(r, c, N)];
      }
      double v = ei.b[r];
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(ei.C[sidx(r, k, N)], ej.eta[k], v);
      B[r * R + N] = v;
    }
    lu_solve<N, R>(Mx, B, ok);
  }
  table_fence();
  // A = A_j XA, b = A_j Xb + b_j, C = A_j XC A_j^T + C_j
  {
    double AjXC[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      double bb = ej.b[r];
#pragma unroll
      for (int k = 0; k < N; ++k) bb = fma(ej.A[r * N + k], B[k * R + N], bb);
      o.b[r] = bb;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        double a = 0.0, x = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          a = fma(ej.A[r * N + k], B[k * R + c], a);
          x = fma(ej.A[r * N + k], B[k * R + N + 1 + c], x);
        }
        o.A[r * N + c] = a;
        AjXC[r * N + c] = x;
      }
    }
    table_fence();
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = r; c < N; ++c) {
        double v = ej.C[sidx(r, c, N)], w = v;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          v = fma(AjXC[r * N + k], ej.A[c * N + k], v);
          w = fma(AjXC[c * N + k], ej.A[r * N + k], w);
        }
        o.C[sidx(r, c, N)] = 0.5 * (v + w);
      }
  }
  table_fence();
  // eta = A_i^T X^T v + eta_i with v = eta_j - J_j b_i
  {
    double vv[N], t1[N], xtv[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      double v = ej.eta[r];
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(-ej.J[sidx(r, k, N)], ei.b[k], v);
      vv[r] = v;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(B[r * R + N + 1 + k], vv[k], v);
      t1[r] = v;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      double v = vv[r];
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(-ej.J[sidx(r, k, N)], t1[k], v);
      xtv[r] = v;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      double v = ei.eta[r];
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(ei.A[k * N + r], xtv[k], v);
      o.eta[r] = v;
    }
  }
  table_fence();
  // J = A_i^T (J_j XA) + J_i
  {
    double JXA[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) v = fma(ej.J[sidx(r, k, N)], B[k * R + c], v);
        JXA[r * N + c] = v;
      }
    table_fence();
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = r; c < N; ++c) {
        double v = 0.0, w = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          v = fma(ei.A[k * N + r], JXA[k * N + c], v);
          w = fma(ei.A[k * N + c], JXA[k * N + r], w);
        }
        o.J[sidx(r, c, N)] = ei.J[sidx(r, c, N)] + 0.5 * (v + w);
      }
  }
}

// gradient of the future log-likelihood with respect to the moments (m, P)
// of the boundary state, given the future information (J~, eta~):
//   B = (I + J~ P)^-1, mbar = B (eta~ - J~ m), Pbar = (mbar mbar^T - B J~)/2.
// Lam (optional) receives the symmetric B J~, which with mbar is the pair
// (lambda, Lambda) of the smoother's backward sweep: the smoothed boundary
// moments are m + P mbar and P - P Lambda P.
template <int N>
GPD void boundary_adjoint(const double* m, const double* Pp, const double* Jp, const double* et, double* mbar,
                          double* Pbar, double* Lam, bool& ok) {
  double P[N * N], Jf[N * N], A[N * N], B[N * (N + 1)];
  unpack<N>(Pp, P);
  unpack<N>(Jp, Jf);
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) v = fma(Jf[i * N + k], P[k * N + j], v);
      A[i * N + j] = v;
      B[i * (N + 1) + j] = Jf[i * N + j];
    }
    double r = et[i];
#pragma unroll
    for (int k = 0; k < N; ++k) r = fma(-Jf[i * N + k], m[k], r);
    B[i * (N + 1) + N] = r;
  }
  lu_solve<N, N + 1>(A, B, ok);
#pragma unroll
  for (int i = 0; i < N; ++i) mbar[i] = B[i * (N + 1) + N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      const double bj = 0.5 * (B[i * (N + 1) + j] + B[j * (N + 1) + i]);
      Pbar[sidx(i, j, N)] = 0.5 * (mbar[i] * mbar[j] - bj);
      if (Lam) Lam[sidx(i, j, N)] = bj;
    }
}

// ---------------------------------------------------------------------------
// smoother backward sweep in adjoint form (modified Bryson-Frazier)
// ---------------------------------------------------------------------------
// At any point of the forward filter with moments (m, P), the data after it
// enter the smoothed moments through a pair (lambda, Lambda):
//   m^ = m + P lambda,   P^ = P - P Lambda P
// (lambda = B (eta~ - J~ m), Lambda = B J~ with B = (I + J~ P)^-1 in terms of
// the future information).  The pair runs backward through the forward
// operations without any matrix inverse:
//   predict m <- A m, P <- A P A^T + Q:   lambda <- A^T lambda, Lambda <- A^T Lambda A
//   update with gain K = u / S (u = P h, S = h.u + R, innovation v):
//     lambda <- lambda + h (v - u.lambda) / S
//     Lambda <- (I - K h^T)^T Lambda (I - K h^T) + h h^T / S
//   closing integrator j (z_j <- 0):      row and column j of both cleared.
// This is the same posterior as the RTS recursion of Sec. 3.2.2; it avoids
// inverting the predicted covariance, which is nearly singular when two
// exposures start almost together (their integrators are nearly equal).

// lambda <- A^T lambda, Lambda <- A^T Lambda A for the augmented transition
// A = [[Phi, 0], [o fbar^T, I]] (o: the integrators open over the step)
template <class Dm>
GPD void bf_predict(double* lam, double* Lam, const TermQ* tq, uint32_t open) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D;
  double fb[NX];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    fb[2 * t] = tq[t].f0;
    fb[2 * t + 1] = tq[t].f1;
  }
  double oj[J > 0 ? J : 1];
#pragma unroll
  for (int j = 0; j < J; ++j) oj[j] = ((open >> j) & 1u) ? 1.0 : 0.0;
  // lambda
  double lz = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) lz = fma(oj[j], lam[NX + j], lz);
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const double l0 = lam[2 * t], l1 = lam[2 * t + 1];
    lam[2 * t] = fma(tq[t].a00, l0, fma(-tq[t].a01, l1, fb[2 * t] * lz));
    lam[2 * t + 1] = fma(tq[t].a01, l0, fma(tq[t].a11, l1, fb[2 * t + 1] * lz));
  }
  // Lambda: g = Lxz o, h = Lzz o, s = o^T Lzz o (from the old blocks)
  double g[NX], h[J > 0 ? J : 1];
#pragma unroll
  for (int a = 0; a < NX; ++a) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) v = fma(oj[j], Lam[sidx(a, NX + j, D)], v);
    g[a] = v;
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < J; ++i) v = fma(oj[i], Lam[sidx(NX + j, NX + i, D)], v);
    h[j] = v;
    s = fma(oj[j], v, s);
  }
  // SHO/integrator block: Phi^T Lxz + fbar h^T
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double y0 = Lam[sidx(2 * t, NX + j, D)], y1 = Lam[sidx(2 * t + 1, NX + j, D)];
      Lam[sidx(2 * t, NX + j, D)] = fma(tq[t].a00, y0, fma(-tq[t].a01, y1, fb[2 * t] * h[j]));
      Lam[sidx(2 * t + 1, NX + j, D)] = fma(tq[t].a01, y0, fma(tq[t].a11, y1, fb[2 * t + 1] * h[j]));
    }
  // g' = Phi^T g
  double gp[NX];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    gp[2 * t] = fma(tq[t].a00, g[2 * t], -tq[t].a01 * g[2 * t + 1]);
    gp[2 * t + 1] = fma(tq[t].a01, g[2 * t], tq[t].a11 * g[2 * t + 1]);
  }
  // SHO block: Phi^T Lxx Phi + g' fbar^T + fbar g'^T + s fbar fbar^T
#pragma unroll
  for (int t = 0; t < M; ++t)
#pragma unroll
    for (int u = t; u < M; ++u) {
      const double b00 = Lam[sidx(2 * t, 2 * u, D)], b01 = Lam[sidx(2 * t, 2 * u + 1, D)];
      const double b10 = Lam[sidx(2 * t + 1, 2 * u, D)], b11 = Lam[sidx(2 * t + 1, 2 * u + 1, D)];
      // Y = Phi_t^T B
      const double y00 = fma(tq[t].a00, b00, -tq[t].a01 * b10);
      const double y01 = fma(tq[t].a00, b01, -tq[t].a01 * b11);
      const double y10 = fma(tq[t].a01, b00, tq[t].a11 * b10);
      const double y11 = fma(tq[t].a01, b01, tq[t].a11 * b11);
      // Z = Y Phi_u
      const double z00 = fma(y00, tq[u].a00, -y01 * tq[u].a01);
      const double z01 = fma(y00, tq[u].a01, y01 * tq[u].a11);
      const double z10 = fma(y10, tq[u].a00, -y11 * tq[u].a01);
      const double z11 = fma(y10, tq[u].a01, y11 * tq[u].a11);
      const int r0 = 2 * t, r1 = 2 * t + 1, c0 = 2 * u, c1 = 2 * u + 1;
      auto add = [&](int r, int c, double z) {
        return z + gp[r] * fb[c] + fb[r] * gp[c] + s * fb[r] * fb[c];
      };
      Lam[sidx(r0, c0, D)] = add(r0, c0, z00);
      Lam[sidx(r0, c1, D)] = add(r0, c1, z01);
      if (t != u) Lam[sidx(r1, c0, D)] = add(r1, c0, z10);
      Lam[sidx(r1, c1, D)] = add(r1, c1, z11);
    }
}

// back through a measurement update (u = P h of the predicted covariance,
// S = h.u + R, v = y - h.m of the predicted mean); no-op without a
// measurement.  With ed, also the two numbers that give the posterior of the
// measured quantity h.x in disturbance form: ed[0] = (v - u.lam)/S and
// ed[1] = 1/S + u.Lam.u/S^2 from the pair after the update, so that
//   mean = y - R ed[0],   var = R (1 - R ed[1]).
// Unlike h.m + u.lam and h.P h - u.Lam.u (the pair before the update, with
// the predicted moments) these keep their relative accuracy when the
// posterior variance is far below the predicted one (nearly noise-free
// data, where the smoothed variance is of order R).
template <class Dm>
GPD void bf_update(double* lam, double* Lam, const double* u, const Obs& o, double S, double v, double* ed = nullptr) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D;
  if (!o.has) return;
  double hv[D];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    hv[2 * t] = o.b;
    hv[2 * t + 1] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < J; ++j) hv[NX + j] = o.a[j];
  const double iS = 1.0 / S;
  double ul = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) ul = fma(u[i], lam[i], ul);
  const double c1 = (v - ul) * iS;
  if (ed) ed[0] = c1;
#pragma unroll
  for (int i = 0; i < D; ++i) lam[i] = fma(hv[i], c1, lam[i]);
  // w = Lambda u / S, c = u^T Lambda u / S^2 + 1 / S
  double w[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) a = fma(Lam[sidx(i, k, D)], u[k], a);
    w[i] = a * iS;
  }
  double uw = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) uw = fma(u[i], w[i], uw);
  const double c = (uw + 1.0) * iS;
  if (ed) ed[1] = c;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      double& L = Lam[sidx(i, j, D)];
      L = fma(c * hv[i], hv[j], fma(-hv[i], w[j], fma(-w[i], hv[j], L)));
    }
}

// back through the closing of an exposure's integrator
template <class Dm>
GPD void bf_close(double* lam, double* Lam, uint32_t info) {
  constexpr int J = Dm::J, NX = Dm::NX, D = Dm::D;
  const bool end = ev_kind(info) == EV_END;
  const uint32_t slot = ev_slot(info);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const bool z = end && (uint32_t)j == slot;
    lam[NX + j] = z ? 0.0 : lam[NX + j];
#pragma unroll
    for (int i = 0; i < D; ++i) Lam[sidx(i, NX + j, D)] = z ? 0.0 : Lam[sidx(i, NX + j, D)];
  }
}

// posterior of h.x at a point with forward moments (m, P) and adjoint pair
// (lambda, Lambda), given u = P h:  mean h.m + u.lambda, variance h.u - u^T Lambda u
template <class Dm>
GPD void bf_posterior(double hm, double hu, const double* u, const double* lam, const double* Lam, double& mean,
                      double& var) {
  constexpr int D = Dm::D;
  double ul = 0.0, uLu = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    ul = fma(u[i], lam[i], ul);
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) a = fma(Lam[sidx(i, k, D)], u[k], a);
    uLu = fma(u[i], a, uLu);
  }
  mean = hm + ul;
  var = hu - uLu;
}

// ---------------------------------------------------------------------------
// reverse-mode adjoint of one plain filter step
// ---------------------------------------------------------------------------
// Gradient accumulators per term: (sigma, omega0, Q); plus jitter.
template <int M>
struct GradAcc {
  // this lane's slots of an LDS array laid out [field][lane] (fields s_t, w_t,
  // q_t, jit): the accumulators are touched a few times per event, and keeping
  // them out of the register file across the backward sweep leaves room for
  // the step itself
  double* base;
  // with instruments: the lane's slots of [amplitude 0..7, offset 0..7][lane],
  // and the series' row of the instrument table
  double* ib = nullptr;
  const double* itab = nullptr;
  GPD double& s(int t) const { return base[(0 * M + t) * 64]; }
  GPD double& w(int t) const { return base[(1 * M + t) * 64]; }
  GPD double& q(int t) const { return base[(2 * M + t) * 64]; }
  GPD double& jit() const { return base[(3 * M) * 64]; }
  GPD double& amp(int i) const { return ib[i * 64]; }
  GPD double& off(int i) const { return ib[(MAX_INST + i) * 64]; }
  GPD void init() const {
#pragma unroll
    for (int f = 0; f < 3 * M + 1; ++f) base[f * 64] = 0.0;
    if (ib) {
#pragma unroll
      for (int f = 0; f < 2 * MAX_INST; ++f) ib[f * 64] = 0.0;
    }
  }
};

// Back-propagates the adjoint weights of one term's step quantities to
// (sigma, omega0, Q).  W: abar00, abar01, abar11, fbar0, fbar1, qbar00,
// qbar01, qbar11, cbar0, cbar1, zzbar (weights of the TermQ fields, with the
// transition's (1,0) entry -a01 folded into abar01).  The base-function
// values are read back from the step quantities; db holds their
// beta-derivatives (g, g', G1, int g^2, int g'^2, int G1^2).
GPD void term_backprop(const TermConst& t, const TermQ& q, const double* db, double dt, const double* W, double& gs,
                       double& gw, double& gq) {
  const double beta = t.beta, qh = t.qhat, iw = t.inv_w0, w0 = t.w0;
  const double iq = t.inv_qhat;
  const double g = q.a01, gp = q.a11, G1 = q.f1 * w0, Igg = q.q00 * iq, Ipp = q.q11 * iq, IGG = q.zz * w0 * w0 * iq;
  double bg = 0, bgp = 0, bG1 = 0, bIgg = 0, bIpp = 0, bIGG = 0, bbeta = 0, bqh = 0, biw = 0;
  // transition
  bgp += W[0];
  bg += 2.0 * beta * W[0];
  bbeta += 2.0 * g * W[0];
  bg += W[1];
  bgp += W[2];
  // integrated row
  bg += W[3] * iw;
  bG1 += 2.0 * beta * W[3] * iw;
  bbeta += 2.0 * G1 * W[3] * iw;
  biw += W[3] * (g + 2.0 * beta * G1);
  bG1 += W[4] * iw;
  biw += W[4] * G1;
  // process noise
  bIgg += qh * W[5];
  bqh += W[5] * Igg;
  bg += qh * g * W[6];
  bqh += W[6] * 0.5 * g * g;
  bIpp += qh * W[7];
  bqh += W[7] * Ipp;
  // cross noise
  bG1 += qh * G1 * iw * W[8];
  bqh += W[8] * 0.5 * G1 * G1 * iw;
  biw += W[8] * 0.5 * qh * G1 * G1;
  bG1 += qh * g * iw * W[9];
  bg += qh * G1 * iw * W[9];
  bIgg -= qh * iw * W[9];
  bqh += W[9] * (G1 * g - Igg) * iw;
  biw += W[9] * qh * (G1 * g - Igg);
  // integrator noise
  bIGG += qh * iw * iw * W[10];
  bqh += W[10] * IGG * iw * iw;
  biw += 2.0 * W[10] * qh * IGG * iw;
  // base functions -> (x, beta): d/dx from the ODE, d/dbeta from the duals
  const double bx = bg * gp + bgp * (-g - 2.0 * beta * gp) + bG1 * g + bIgg * g * g + bIpp * gp * gp + bIGG * G1 * G1;
  bbeta += bg * db[0] + bgp * db[1] + bG1 * db[2] + bIgg * db[3] + bIpp * db[4] + bIGG * db[5];
  // (x, beta, qhat, 1/omega0) -> (sigma, omega0, Q);  x = omega0 dt, beta = 1/2Q, qhat = 2 sigma^2/Q
  // 1/Q = 2 beta, so qhat/Q = 2 beta qhat and 2 qhat/sigma = 8 beta sigma
  gw += bx * dt - biw * iw * iw;
  gq += -bbeta * 2.0 * beta * beta - bqh * qh * (2.0 * beta);
  gs += bqh * 8.0 * beta * t.sigma;
}

// Accuracy policies of the discretisation.  DiscFull: series to degree KSER
// below x max(1, beta) = XSER, about 1e-15 relative everywhere (likelihood,
// smoother).  DiscGrad: degree KSER_G below XSER_G, about 1e-11 on the step
// quantities and 1e-9 on their beta-derivatives, for the passes that only
// feed the gradient (checked against the full policy over Q in [0.3, 50]).
struct DiscFull {
  static constexpr int K = KSER;
  GPD static bool series(double x, const TermConst& t) { return x <= t.xser; }
};
struct DiscGrad {
  static constexpr int K = KSER_G;
  GPD static bool series(double x, const TermConst& t) { return x <= t.xser_g; }
};

// discretisation of all terms over one step (values only); the tables of
// term t start at coef + t * TS
template <int M, class Acc = DiscFull, int TS = NCOEF, bool X = true>
GPD void discretise(const TermConst* tc, const double* coef, double dt, TermQ* tq) {
#pragma unroll
  for (int t = 0; t < M; ++t) {
    if (is_real<X>(tc[t])) {  // wavefront-uniform: the term's kind
      tq[t] = real_step(tc[t], dt);
      continue;
    }
    const double x = tc[t].w0 * dt;
    Base<double> b;
    if (Acc::series(x, tc[t]))
      series_eval<Acc::K>(coef + t * TS, x, tc[t], b);
    else
      closed_eval(x, tc[t], b);
    tq[t] = term_step(tc[t], b);
  }
}

// with the beta-derivatives of the base functions (db[t*6 + f], a register
// array or a LaneLds view); the tables of term t (values, then
// beta-derivatives) start at coef + t * 2 NCOEF
template <int M, class Acc = DiscFull, bool X = true, class DB>
GPD void discretise_dual(const TermConst* tc, const double* coef, double dt, DB&& db, TermQ* tq) {
#pragma unroll
  for (int t = 0; t < M; ++t) {
    if (is_real<X>(tc[t])) {  // no beta: real_backprop differentiates the step itself
      tq[t] = real_step(tc[t], dt);
#pragma unroll
      for (int f = 0; f < 6; ++f) db[t * 6 + f] = 0.0;
      continue;
    }
    const double x = tc[t].w0 * dt;
    Base<Dual> bd;
    if (Acc::series(x, tc[t]))
      series_eval<Acc::K>(coef + t * 2 * NCOEF, x, tc[t], bd);
    else
      closed_eval(x, tc[t], bd);
    Base<double> b;
    b.g = bd.g.v;
    b.gp = bd.gp.v;
    b.G1 = bd.G1.v;
    b.Igg = bd.Igg.v;
    b.Ipp = bd.Ipp.v;
    b.IGG = bd.IGG.v;
    db[t * 6 + 0] = bd.g.d;
    db[t * 6 + 1] = bd.gp.d;
    db[t * 6 + 2] = bd.G1.d;
    db[t * 6 + 3] = bd.Igg.d;
    db[t * 6 + 4] = bd.Ipp.d;
    db[t * 6 + 5] = bd.IGG.d;
    tq[t] = term_step(tc[t], b);
  }
}

// Adjoint of one plain step (predict over dt, observe, close the slot).
// m, P: the filtered state before the step.  mb, Pb: on entry the adjoint
// with respect to the state after the step, on exit with respect to (m, P).
// The predicted moments are not formed: the gain u = (A P A^T + Q) h is
// computed as A (P (A^T h)) + Q h, and (A P) one column at a time.
// DBL: the beta-derivatives of the base functions, needed only at the end of
// the step, wait in the lane's LDS slots dbl instead of registers.
template <class Dm, bool DBL = false, bool X = true>
GPD void adjoint_step(const double* m, const double* P, double* mb, double* Pb, const TermConst* tc, const double* coef,
                      double dt, uint32_t info, const Obs& o, double jit, const GradAcc<Dm::M>& acc,
                      LaneLds dbl = LaneLds{nullptr}) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D;
  const uint32_t open = ev_open(info);
  double dbr[DBL ? 1 : 6 * M];
  TermQ tq[M];
  if constexpr (DBL)
    discretise_dual<M, DiscGrad, X>(tc, coef, dt, dbl, tq);
  else
    discretise_dual<M, DiscGrad, X>(tc, coef, dt, dbr, tq);
  double oj[J > 0 ? J : 1];
#pragma unroll
  for (int j = 0; j < J; ++j) oj[j] = ((open >> j) & 1u) ? 1.0 : 0.0;
  // h, the sum of h over open integrators, and A^T h
  double h[D];
#pragma unroll
  for (int i = 0; i < D; ++i) h[i] = (i >= NX) ? o.a[i - NX] : ((i % 2 == 0) ? o.b : 0.0);
  double hz = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) hz = fma(oj[j], h[NX + j], hz);
  double ht[D];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    ht[2 * t] = fma(tq[t].a00, h[2 * t], fma(-tq[t].a01, h[2 * t + 1], tq[t].f0 * hz));
    ht[2 * t + 1] = fma(tq[t].a01, h[2 * t], fma(tq[t].a11, h[2 * t + 1], tq[t].f1 * hz));
  }
#pragma unroll
  for (int j = 0; j < J; ++j) ht[NX + j] = h[NX + j];
  // y = P ht, u = A y + Q h
  double u[D];
  {
    double y[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double acc2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) acc2 = fma(P[sidx(i, k, D)], ht[k], acc2);
      y[i] = acc2;
    }
    double fy = 0.0, ch = 0.0, zz = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
      fy = fma(tq[t].f0, y[2 * t], fma(tq[t].f1, y[2 * t + 1], fy));
      ch = fma(tq[t].c0, h[2 * t], fma(tq[t].c1, h[2 * t + 1], ch));
      zz += tq[t].zz;
    }
#pragma unroll
    for (int t = 0; t < M; ++t) {
      u[2 * t] = fma(tq[t].a00, y[2 * t], tq[t].a01 * y[2 * t + 1]) + fma(tq[t].q00, h[2 * t], tq[t].q01 * h[2 * t + 1]) +
                 tq[t].c0 * hz;
      u[2 * t + 1] = fma(-tq[t].a01, y[2 * t], tq[t].a11 * y[2 * t + 1]) +
                     fma(tq[t].q01, h[2 * t], tq[t].q11 * h[2 * t + 1]) + tq[t].c1 * hz;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) u[NX + j] = y[NX + j] + oj[j] * (fy + ch + zz * hz);
  }
  double hm = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) hm = fma(ht[i], m[i], hm);
  double S = o.R;
#pragma unroll
  for (int i = 0; i < D; ++i) S = fma(h[i], u[i], S);
  const double v = o.y - hm;

  // closing the slot: the zeroed entries are constants
  close_slot<Dm>(mb, Pb, info);

  // update:  m+ = m- + u v/S,  P+ = P- - u u^T/S,  l = -(log 2 pi S + v^2/S)/2
  {
    const double hs = o.has ? 1.0 : 0.0;
    const double iS = 1.0 / S;
    double um = 0.0, uPu = 0.0, Pu[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      um = fma(u[i], mb[i], um);
      double acc2 = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) acc2 = fma(Pb[sidx(i, j, D)], u[j], acc2);
      Pu[i] = acc2;
      uPu = fma(u[i], acc2, uPu);
    }
    const double Sbar = hs * ((-0.5 + 0.5 * v * v * iS) * iS + (uPu - um * v) * iS * iS);
    const double vbar = hs * (um - v) * iS;
    double ub[D];
#pragma unroll
    for (int i = 0; i < D; ++i) ub[i] = hs * (mb[i] * v - 2.0 * Pu[i]) * iS + h[i] * Sbar;
    double jw = 2.0 * jit;  // dR/djitter
    if (acc.ib) {
      // instrument i: the filter sees y' = (y - c)/a and R' = R/a^2, so
      // dl/da = -(vbar y' + 2 Sbar R')/a, dl/dc = -vbar/a and dR'/djitter =
      // 2 jitter/a^2 (the -log a per measurement is added per series).
      // Events without a measurement add zeros (to instrument 0).
      const uint32_t ii = ev_inst(info);
      const double ia = acc.itab[ITAB_INVA + ii];
      acc.amp(ii) -= fma(vbar, o.y, 2.0 * Sbar * o.R) * ia;
      acc.off(ii) -= vbar * ia;
      jw *= ia * ia;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) mb[i] = fma(-h[i], vbar, mb[i]);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) Pb[sidx(i, j, D)] += 0.5 * (ub[i] * h[j] + h[i] * ub[j]);
    acc.jit() = fma(jw, Sbar, acc.jit());
  }

  // predict: weights of the step quantities.  Abar = mb- m^T + 2 Pb- (A P).
  double fb[NX];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    fb[2 * t] = tq[t].f0;
    fb[2 * t + 1] = tq[t].f1;
  }
  double W[M][11];
  double fw[M][2];
#pragma unroll
  for (int t = 0; t < M; ++t) fw[t][0] = fw[t][1] = 0.0;
#pragma unroll
  for (int bcol = 0; bcol < NX; ++bcol) {
    // column bcol of A P
    double T[D];
    double wv = 0.0;  // (Pxx fbar)[bcol]
#pragma unroll
    for (int c = 0; c < NX; ++c) wv = fma(P[sidx(bcol, c, D)], fb[c], wv);
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double p0 = P[sidx(2 * t, bcol, D)], p1 = P[sidx(2 * t + 1, bcol, D)];
      T[2 * t] = fma(tq[t].a00, p0, tq[t].a01 * p1);
      T[2 * t + 1] = fma(-tq[t].a01, p0, tq[t].a11 * p1);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) T[NX + j] = fma(oj[j], wv, P[sidx(NX + j, bcol, D)]);
    const int tb = bcol / 2, cb = bcol % 2;
    // rows of the same term's transition block
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      double g2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) g2 = fma(Pb[sidx(2 * tb + r, k, D)], T[k], g2);
      W[tb][r * 2 + cb] = fma(mb[2 * tb + r], m[bcol], 2.0 * g2);  // Abar[r][cb], fixed up below
    }
    // integrator rows (integrated transition row)
#pragma unroll
    for (int j = 0; j < J; ++j) {
      double g2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) g2 = fma(Pb[sidx(NX + j, k, D)], T[k], g2);
      fw[tb][cb] += oj[j] * fma(mb[NX + j], m[bcol], 2.0 * g2);
    }
  }
#pragma unroll
  for (int t = 0; t < M; ++t) {
    // W[t][0..3] hold Abar00, Abar01, Abar10, Abar11
    const double a00 = W[t][0], a01 = W[t][1], a10 = W[t][2], a11 = W[t][3];
    double w[11];
    w[0] = a00;
    w[1] = a01 - a10;
    w[2] = a11;
    w[3] = fw[t][0];
    w[4] = fw[t][1];
    w[5] = Pb[sidx(2 * t, 2 * t, D)];
    w[6] = 2.0 * Pb[sidx(2 * t, 2 * t + 1, D)];
    w[7] = Pb[sidx(2 * t + 1, 2 * t + 1, D)];
    double c0 = 0.0, c1 = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      c0 = fma(oj[j], 2.0 * Pb[sidx(2 * t, NX + j, D)], c0);
      c1 = fma(oj[j], 2.0 * Pb[sidx(2 * t + 1, NX + j, D)], c1);
    }
    w[8] = c0;
    w[9] = c1;
    double zz = 0.0;
#pragma unroll
    for (int i = 0; i < J; ++i)
#pragma unroll
      for (int j = 0; j < J; ++j) zz = fma(oj[i] * oj[j], Pb[sidx(NX + i, NX + j, D)], zz);
    w[10] = zz;
    double d6[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if constexpr (DBL)
        d6[f] = dbl[6 * t + f];
      else
        d6[f] = dbr[6 * t + f];
    }
    if (is_real<X>(tc[t]))
      real_backprop(tc[t], dt, w, acc.s(t), acc.w(t));
    else
      term_backprop(tc[t], tq[t], d6, dt, w, acc.s(t), acc.w(t), acc.q(t));
  }

  // adjoint to the state before the predict
  {
    double zsum = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) zsum = fma(oj[j], mb[NX + j], zsum);
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double b0 = mb[2 * t], b1 = mb[2 * t + 1];
      mb[2 * t] = fma(tq[t].a00, b0, fma(-tq[t].a01, b1, fb[2 * t] * zsum));
      mb[2 * t + 1] = fma(tq[t].a01, b0, fma(tq[t].a11, b1, fb[2 * t + 1] * zsum));
    }
  }
  {
    double p[NX];
#pragma unroll
    for (int a = 0; a < NX; ++a) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < J; ++j) s = fma(oj[j], Pb[sidx(a, NX + j, D)], s);
      p[a] = s;
    }
    double sz = 0.0, cz[J > 0 ? J : 1];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < J; ++i) s = fma(oj[i], Pb[sidx(NX + i, NX + j, D)], s);
      cz[j] = s;
      sz = fma(oj[j], s, sz);
    }
    // SHO/integrator block: Phi^T Pbar[x, z_j] + fbar^T cz_j
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
      for (int t = 0; t < M; ++t) {
        const double y0 = Pb[sidx(2 * t, NX + j, D)], y1 = Pb[sidx(2 * t + 1, NX + j, D)];
        Pb[sidx(2 * t, NX + j, D)] = fma(tq[t].a00, y0, fma(-tq[t].a01, y1, fb[2 * t] * cz[j]));
        Pb[sidx(2 * t + 1, NX + j, D)] = fma(tq[t].a01, y0, fma(tq[t].a11, y1, fb[2 * t + 1] * cz[j]));
      }
    }
    // q = Phi^T p
    double q[NX];
#pragma unroll
    for (int t = 0; t < M; ++t) {
      q[2 * t] = fma(tq[t].a00, p[2 * t], -tq[t].a01 * p[2 * t + 1]);
      q[2 * t + 1] = fma(tq[t].a01, p[2 * t], tq[t].a11 * p[2 * t + 1]);
    }
    // SHO block: Phi_t^T B Phi_u + q fbar^T + fbar q^T + sz fbar fbar^T
#pragma unroll
    for (int t = 0; t < M; ++t) {
#pragma unroll
      for (int uu = t; uu < M; ++uu) {
        const double b00 = Pb[sidx(2 * t, 2 * uu, D)], b01 = Pb[sidx(2 * t, 2 * uu + 1, D)];
        const double b10 = Pb[sidx(2 * t + 1, 2 * uu, D)], b11 = Pb[sidx(2 * t + 1, 2 * uu + 1, D)];
        const double y00 = fma(tq[t].a00, b00, -tq[t].a01 * b10);
        const double y01 = fma(tq[t].a00, b01, -tq[t].a01 * b11);
        const double y10 = fma(tq[t].a01, b00, tq[t].a11 * b10);
        const double y11 = fma(tq[t].a01, b01, tq[t].a11 * b11);
        const double z00 = fma(y00, tq[uu].a00, -y01 * tq[uu].a01);
        const double z01 = fma(y00, tq[uu].a01, y01 * tq[uu].a11);
        const double z10 = fma(y10, tq[uu].a00, -y11 * tq[uu].a01);
        const double z11 = fma(y10, tq[uu].a01, y11 * tq[uu].a11);
        const int a0 = 2 * t, a1 = 2 * t + 1, c0i = 2 * uu, c1i = 2 * uu + 1;
        auto extra = [&](int a, int c) { return fma(q[a], fb[c], fma(fb[a], q[c], sz * fb[a] * fb[c])); };
        Pb[sidx(a0, c0i, D)] = z00 + extra(a0, c0i);
        Pb[sidx(a0, c1i, D)] = z01 + extra(a0, c1i);
        Pb[sidx(a1, c1i, D)] = z11 + extra(a1, c1i);
        if (t != uu) Pb[sidx(a1, c0i, D)] = z10 + extra(a1, c0i);
      }
    }
  }
}

// sum over the 64 lanes of a wavefront (fixed order: identical on every lane)
__device__ __forceinline__ double wave_sum(double v) {
#ifdef __HIP_DEVICE_COMPILE__
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
#endif
  return v;
}

}  // namespace gpssm
