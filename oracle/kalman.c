/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, sequential CPU implementation of the augmented state-space
 * model for exposure-integrated (and overlapping) measurements of a
 * sum-of-SHO Gaussian process.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Arithmetic: long double (x87 80-bit, 64-bit significand) throughout; the
 * log-likelihood is returned as a double-double (hi, lo) pair so that finite
 * differences taken on it keep their precision.
 *
 * Paper followed ("Scalable Gaussian Processes for Integrated and Overlapping
 * Measurements via Augmented State-Space Models"):
 *   - SHO model F, L, Qc, Pinf ............ Appendix B (worked SHO example)
 *   - transition exp(F dt) and process noise as the integral of
 *     exp(Fs) L Qc L^T exp(F^T s) over the step ....... Sec. 2.2 (solution of
 *     the SDE, process-noise integral); for the augmented model the same
 *     integral of the augmented matrices, Sec. 3.2 (augmented SDE, augmented
 *     transition and augmented process noise)
 *   - sums of terms as block-diagonal models ........ Appendix C.1
 *   - the real (exponential) term, the celerite term
 *     with b = d = 0, as a one-state model .......... Appendix A
 *   - one integrator per instrument label ........... Sec. 3.2.3
 *   - per-measurement amplitude and offset of the
 *     instrument in the observation model (measured
 *     a_n times the exposure average plus c_n) ...... Sec. 2.2 (observation
 *                                                     matrix), Sec. 3.2.3
 *   - reset at exposure starts, update at ends ...... Sec. 3.2.1
 *   - log-likelihood from innovations ............... Sec. 2.4
 *   - the same filter in square-root (Cholesky-
 *     factor) form .................................. Sec. 3.2.3 and Sec. 5
 *                                                     (named as the remedy
 *                                                     for the filter's loss
 *                                                     of accuracy)
 *   - integrated RTS smoother ....................... Sec. 3.2.2
 *   - prediction at arbitrary times ................. Sec. 2.5, Algorithm 1
 *   - component-wise prediction (H^m applied to the
 *     smoothed state) ............................... Appendix C, component-
 *                                                     wise predictive means
 *
 * How the discretisation is computed (a method of this file, not the
 * paper's closed forms): per SHO term, in time scaled by omega0 and state
 * (x, xdot/omega0, omega0*z), the Taylor series of exp(F h) and of the
 * process-noise integral (whose integrand's n-th derivative obeys
 * T_{n+1} = F T_n + T_n F^T) for a short step h, composed to the full step
 * by the semigroup property  A(2h) = A(h)^2,  Q(2h) = A(h) Q(h) A(h)^T + Q(h).
 *
 * Readings of the paper taken here (the same list is kept in the design
 * notes): events at equal times are ordered end < instantaneous < start;
 * a zero-length exposure is an instantaneous measurement with H = sum of the
 * terms' x components; jitter adds in quadrature to each measurement error;
 * the filter starts at the first event with P0 = blkdiag(Pinf, I); several
 * integrators receive the sum over terms of the integrated transition rows;
 * Algorithm 1 is used with the smoother gain transposed in the covariance
 * lines, the interpolation gain built from the predicted state at the test
 * time and the next event's transition, and the retrodiction restricted to
 * the latent (non-integrator) block.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

#define OR_MAXM 4
#define OR_MAXJ 8
#define OR_MAXD (2 * OR_MAXM + OR_MAXJ)

enum { OR_OK = 0, OR_EINVAL = -1, OR_EDATA = -2, OR_EPARAM = -3, OR_EOVERLAP = -4, OR_ENUMERIC = -5, OR_ENOMEM = -7 };
enum { EV_END = 0, EV_INSTANT = 1, EV_START = 2 };

static const ld TWO_PI = 6.283185307179586476925286766559L;

/* ------------------------------------------------------------------ */
/* One SHO term, one integrator: 3x3 transition and process noise.      */
/* ------------------------------------------------------------------ */

static void mul3(const ld a[3][3], const ld b[3][3], ld c[3][3]) {
  ld t[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      ld s = 0;
      for (int k = 0; k < 3; ++k) s += a[i][k] * b[k][j];
      t[i][j] = s;
    }
  memcpy(c, t, sizeof(t));
}

enum { TERM_SHO = 0, TERM_REAL = 1 };

/* Transition and process noise of the augmented single-term model
 * (x, xdot, z) over a step dt, in unscaled coordinates.  A real term
 * k = sigma^2 exp(-w0 |tau|) is the one-state model dx = -w0 x dt + noise with
 * its integrator; its second state (the "xdot" slot) is unused and stays 0. */
static void term_discretise(ld w0, ld quality, ld sigma, ld dt, int kind, ld phi[3][3], ld q[3][3]) {
  const int real = kind == TERM_REAL;
  /* scaled feedback matrix (time s = w0 t): SHO d/ds (x, y, u) = (y, -x - y/Q, x)
   * with noise on y; real term d/ds (x, y, u) = (-x, 0, x) with noise on x */
  const ld F_sho[3][3] = {{0, 1, 0}, {-1, real ? 0 : -1 / quality, 0}, {1, 0, 0}};
  const ld F_real[3][3] = {{-1, 0, 0}, {0, 0, 0}, {1, 0, 0}};
  ld F[3][3];
  memcpy(F, real ? F_real : F_sho, sizeof(F));
  const ld nrm = real ? 1 : 1 + 1 / quality; /* infinity norm of F */
  ld h = w0 * dt;
  int nsq = 0;
  while (h * nrm > 0.25L) {
    h *= 0.5L;
    ++nsq;
  }
  /* exp(F h) */
  ld P[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  ld term[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int n = 1; n <= 40; ++n) {
    ld t2[3][3];
    mul3(term, F, t2);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        term[i][j] = t2[i][j] * h / n;
        P[i][j] += term[i][j];
      }
  }
  /* integral_0^h exp(Fs) B exp(F^T s) ds with B = e_y e_y^T (SHO) or
   * e_x e_x^T (real term), unit noise */
  ld T[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if (real)
    T[0][0] = 1;
  else
    T[1][1] = 1;
  ld coef = h;
  ld Qs[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Qs[i][j] = T[i][j] * coef;
  for (int n = 0; n < 40; ++n) {
    ld FT[3][3], TFt[3][3], Tn[3][3];
    mul3(F, T, FT);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        ld s = 0;
        for (int k = 0; k < 3; ++k) s += T[i][k] * F[j][k];
        TFt[i][j] = s;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Tn[i][j] = FT[i][j] + TFt[i][j];
    memcpy(T, Tn, sizeof(T));
    coef *= h / (n + 2);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Qs[i][j] += T[i][j] * coef;
  }
  /* compose to the full step */
  for (int k = 0; k < nsq; ++k) {
    ld PQ[3][3], PQPt[3][3];
    mul3(P, Qs, PQ);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        ld s = 0;
        for (int l = 0; l < 3; ++l) s += PQ[i][l] * P[j][l];
        PQPt[i][j] = s;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Qs[i][j] += PQPt[i][j];
    mul3(P, P, P);
  }
  /* scaled noise density 2 sigma^2 / Q (SHO) or 2 sigma^2 (real term);
   * unscale (x, xdot, z) = T (x, y, u), T = diag(1, w0, 1/w0) (SHO) or
   * diag(1, 1, 1/w0) (real term) */
  const ld qhat = real ? 2 * sigma * sigma : 2 * sigma * sigma / quality;
  const ld Tsc[3] = {1, real ? 1 : w0, 1 / w0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      phi[i][j] = Tsc[i] * P[i][j] / Tsc[j];
      q[i][j] = Tsc[i] * Tsc[j] * Qs[i][j] * qhat;
    }
}

int oracle_term_discretise(double omega0, double quality, double sigma, double dt, double* phi9, double* q9) {
  if (!(omega0 > 0) || !(quality > 0) || !(sigma > 0) || !(dt >= 0)) return OR_EPARAM;
  ld phi[3][3], q[3][3];
  term_discretise(omega0, quality, sigma, dt, TERM_SHO, phi, q);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      phi9[3 * i + j] = (double)phi[i][j];
      q9[3 * i + j] = (double)q[i][j];
    }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Model description and the assembled augmented matrices               */
/* ------------------------------------------------------------------ */

typedef struct {
  int M, J, D;
  ld sigma[OR_MAXM], w0[OR_MAXM], qual[OR_MAXM];
  int kind[OR_MAXM];
} model_t;

/* Augmented transition A and noise Qa over dt: terms stacked block-diagonally,
 * every integrator row holds the sum over terms of the integrated transition
 * rows, x_m/z cross noise is each term's integrated cross block, and every
 * z_i/z_j entry is the sum over terms of the integrated-integrated block. */
static void assemble(const model_t* md, ld dt, ld A[OR_MAXD][OR_MAXD], ld Qa[OR_MAXD][OR_MAXD]) {
  const int D = md->D, M = md->M, J = md->J;
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      A[i][j] = (i == j) ? 1 : 0;
      Qa[i][j] = 0;
    }
  ld q22 = 0;
  for (int m = 0; m < M; ++m) {
    ld phi[3][3], q[3][3];
    term_discretise(md->w0[m], md->qual[m], md->sigma[m], dt, md->kind[m], phi, q);
    const int a = 2 * m;
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        A[a + r][a + c] = phi[r][c];
        Qa[a + r][a + c] = q[r][c];
      }
    for (int j = 0; j < J; ++j) {
      const int z = 2 * M + j;
      A[z][a] = phi[2][0];
      A[z][a + 1] = phi[2][1];
      Qa[a][z] = Qa[z][a] = q[0][2];
      Qa[a + 1][z] = Qa[z][a + 1] = q[1][2];
    }
    q22 += q[2][2];
  }
  for (int i = 0; i < J; ++i)
    for (int j = 0; j < J; ++j) Qa[2 * M + i][2 * M + j] = q22;
}

/* P <- A P A^T + Qa ; m <- A m */
static void predict(int D, ld A[OR_MAXD][OR_MAXD], ld Qa[OR_MAXD][OR_MAXD], ld* m, ld P[OR_MAXD][OR_MAXD]) {
  ld t[OR_MAXD][OR_MAXD], mn[OR_MAXD];
  for (int i = 0; i < D; ++i) {
    ld s = 0;
    for (int k = 0; k < D; ++k) s += A[i][k] * m[k];
    mn[i] = s;
  }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      ld s = 0;
      for (int k = 0; k < D; ++k) s += A[i][k] * P[k][j];
      t[i][j] = s;
    }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      ld s = 0;
      for (int k = 0; k < D; ++k) s += t[i][k] * A[j][k];
      P[i][j] = s + Qa[i][j];
    }
  for (int i = 0; i < D; ++i) m[i] = mn[i];
}

/* ------------------------------------------------------------------ */
/* Events                                                               */
/* ------------------------------------------------------------------ */

typedef struct {
  ld t;
  int32_t kind, slot;
  int64_t n;
} ev_t;

static int ev_cmp(const void* a, const void* b) {
  const ev_t* x = (const ev_t*)a;
  const ev_t* y = (const ev_t*)b;
  if (x->t < y->t) return -1;
  if (x->t > y->t) return 1;
  if (x->kind != y->kind) return x->kind < y->kind ? -1 : 1;
  if (x->n != y->n) return x->n < y->n ? -1 : 1;
  return 0;
}

/* Instrument labels so that no label self-overlaps: exposures in start order
 * take the lowest label whose previous exposure has ended (end <= start). */
int oracle_greedy_slots(int64_t n, const double* ts, const double* te, int32_t* slot, int32_t* n_slots) {
  ld last_end[OR_MAXJ];
  int used = 0;
  int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  if (!ord) return OR_ENOMEM;
  for (int64_t i = 0; i < n; ++i) ord[i] = i;
  /* insertion-stable order by start time (inputs are normally already sorted) */
  for (int64_t i = 1; i < n; ++i) {
    int64_t v = ord[i], k = i - 1;
    while (k >= 0 && ts[ord[k]] > ts[v]) {
      ord[k + 1] = ord[k];
      --k;
    }
    ord[k + 1] = v;
  }
  for (int64_t r = 0; r < n; ++r) {
    int64_t i = ord[r];
    if (!(te[i] > ts[i])) {
      slot[i] = -1;
      continue;
    }
    int s = -1;
    for (int j = 0; j < used; ++j)
      if (last_end[j] <= ts[i]) {
        s = j;
        break;
      }
    if (s < 0) {
      if (used >= OR_MAXJ) {
        free(ord);
        return OR_EOVERLAP;
      }
      s = used++;
    }
    last_end[s] = te[i];
    slot[i] = s;
  }
  free(ord);
  *n_slots = used;
  return OR_OK;
}

static int build_events(int64_t n, const double* ts, const double* te, const int32_t* slot, ev_t** out, int64_t* n_ev) {
  int64_t k = 0;
  ev_t* ev = (ev_t*)malloc(sizeof(ev_t) * (2 * n > 0 ? 2 * n : 1));
  if (!ev) return OR_ENOMEM;
  for (int64_t i = 0; i < n; ++i) {
    if (te[i] > ts[i]) {
      ev[k].t = ts[i];
      ev[k].kind = EV_START;
      ev[k].slot = slot[i];
      ev[k].n = i;
      ++k;
      ev[k].t = te[i];
      ev[k].kind = EV_END;
      ev[k].slot = slot[i];
      ev[k].n = i;
      ++k;
    } else {
      ev[k].t = ts[i];
      ev[k].kind = EV_INSTANT;
      ev[k].slot = -1;
      ev[k].n = i;
      ++k;
    }
  }
  qsort(ev, (size_t)k, sizeof(ev_t), ev_cmp);
  *out = ev;
  *n_ev = k;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Filter                                                               */
/* ------------------------------------------------------------------ */

typedef struct {
  ld m[OR_MAXD];
  ld P[OR_MAXD][OR_MAXD];
} state_t;

static int check_inputs(int64_t n, const double* ts, const double* te, const double* y, const double* yerr, int32_t M,
                        const double* sigma, const double* omega0, const double* quality, const int32_t* kind,
                        double jitter) {
  if (n < 1 || M < 1 || M > OR_MAXM) return OR_EINVAL;
  for (int m = 0; m < M; ++m) {
    const int real = kind && kind[m] == TERM_REAL;
    if (kind && kind[m] != TERM_SHO && kind[m] != TERM_REAL) return OR_EINVAL;
    if (!(sigma[m] > 0) || !(omega0[m] > 0) || !isfinite(sigma[m]) || !isfinite(omega0[m])) return OR_EPARAM;
    if (!real && (!(quality[m] > 0) || !isfinite(quality[m]))) return OR_EPARAM;
  }
  if (!(jitter >= 0) || !isfinite(jitter)) return OR_EPARAM;
  for (int64_t i = 0; i < n; ++i) {
    if (!isfinite(ts[i]) || !isfinite(te[i]) || !isfinite(y[i]) || !isfinite(yerr[i])) return OR_EDATA;
    if (te[i] < ts[i] || yerr[i] < 0) return OR_EDATA;
  }
  return OR_OK;
}

/* Runs the integrated Kalman filter.  When pred/filt are non-NULL the
 * predicted and filtered moments of every event are stored there. */
static int run_filter(const model_t* md, int64_t n_ev, const ev_t* ev, const double* ts, const double* te, const double* y,
                      const double* yerr, const double* amp, const double* off, ld jitter, ld* loglik, state_t* pred,
                      state_t* filt) {
  const int D = md->D, M = md->M;
  state_t s;
  memset(&s, 0, sizeof(s));
  for (int m = 0; m < M; ++m) {
    s.P[2 * m][2 * m] = md->sigma[m] * md->sigma[m];
    s.P[2 * m + 1][2 * m + 1] = md->kind[m] == TERM_REAL ? 0 : md->sigma[m] * md->sigma[m] * md->w0[m] * md->w0[m];
  }
  for (int j = 0; j < md->J; ++j) s.P[2 * M + j][2 * M + j] = 1;
  ld L = 0;
  ld A[OR_MAXD][OR_MAXD], Qa[OR_MAXD][OR_MAXD];
  for (int64_t k = 0; k < n_ev; ++k) {
    const ld dt = (k == 0) ? 0 : ev[k].t - ev[k - 1].t;
    assemble(md, dt, A, Qa);
    predict(D, A, Qa, s.m, s.P);
    if (pred) pred[k] = s;
    const int64_t i = ev[k].n;
    if (ev[k].kind == EV_START) {
      const int z = 2 * M + ev[k].slot;
      s.m[z] = 0;
      for (int a = 0; a < D; ++a) s.P[z][a] = s.P[a][z] = 0;
    } else {
      ld h[OR_MAXD];
      const ld an = amp ? (ld)amp[i] : 1;
      for (int a = 0; a < D; ++a) h[a] = 0;
      if (ev[k].kind == EV_END) {
        h[2 * M + ev[k].slot] = an / ((ld)te[i] - (ld)ts[i]);
      } else {
        for (int m = 0; m < M; ++m) h[2 * m] = an;
      }
      ld u[OR_MAXD], hm = 0, S = (ld)yerr[i] * yerr[i] + jitter * jitter;
      for (int a = 0; a < D; ++a) {
        ld t = 0;
        for (int b = 0; b < D; ++b) t += s.P[a][b] * h[b];
        u[a] = t;
        hm += h[a] * s.m[a];
      }
      for (int a = 0; a < D; ++a) S += h[a] * u[a];
      if (!(S > 0)) return OR_ENUMERIC;
      const ld v = (ld)y[i] - (off ? (ld)off[i] : 0) - hm;
      for (int a = 0; a < D; ++a) s.m[a] += u[a] * v / S;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) s.P[a][b] -= u[a] * u[b] / S;
      L += -0.5L * (logl(TWO_PI * S) + v * v / S);
    }
    if (filt) filt[k] = s;
  }
  *loglik = L;
  return isfinite(L) ? OR_OK : OR_ENUMERIC;
}

static int setup(int64_t n, const double* ts, const double* te, const double* y, const double* yerr, const int32_t* slot_in,
                 int32_t M, const double* sigma, const double* omega0, const double* quality, const int32_t* kind,
                 const double* amp, const double* off, double jitter, model_t* md, ev_t** ev, int64_t* n_ev,
                 int32_t** slot_out) {
  int rc = check_inputs(n, ts, te, y, yerr, M, sigma, omega0, quality, kind, jitter);
  if (rc) return rc;
  for (int64_t i = 0; i < n; ++i) {
    if (amp && (!(amp[i] > 0) || !isfinite(amp[i]))) return OR_EPARAM;
    if (off && !isfinite(off[i])) return OR_EPARAM;
  }
  int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * n);
  if (!slot) return OR_ENOMEM;
  int32_t J = 0;
  if (slot_in) {
    for (int64_t i = 0; i < n; ++i) {
      slot[i] = (te[i] > ts[i]) ? slot_in[i] : -1;
      if (te[i] > ts[i] && (slot_in[i] < 0 || slot_in[i] >= OR_MAXJ)) {
        free(slot);
        return OR_EINVAL;
      }
      if (slot[i] + 1 > J) J = slot[i] + 1;
    }
  } else {
    rc = oracle_greedy_slots(n, ts, te, slot, &J);
    if (rc) {
      free(slot);
      return rc;
    }
  }
  md->M = M;
  md->J = J;
  md->D = 2 * M + J;
  for (int m = 0; m < M; ++m) {
    md->sigma[m] = sigma[m];
    md->w0[m] = omega0[m];
    md->qual[m] = quality[m];
    md->kind[m] = kind ? kind[m] : TERM_SHO;
  }
  rc = build_events(n, ts, te, slot, ev, n_ev);
  if (rc) {
    free(slot);
    return rc;
  }
  /* a user-supplied labelling must not self-overlap */
  if (slot_in) {
    int open[OR_MAXJ] = {0};
    for (int64_t k = 0; k < *n_ev; ++k) {
      const ev_t* e = &(*ev)[k];
      if (e->kind == EV_START) {
        if (open[e->slot]) {
          free(slot);
          free(*ev);
          return OR_EOVERLAP;
        }
        open[e->slot] = 1;
      } else if (e->kind == EV_END) {
        open[e->slot] = 0;
      }
    }
  }
  *slot_out = slot;
  return OR_OK;
}

int oracle_loglik(int64_t n, const double* ts, const double* te, const double* y, const double* yerr, const int32_t* slot_in,
                  int32_t M, const double* sigma, const double* omega0, const double* quality, const int32_t* kind,
                  const double* amp, const double* off, double jitter, int32_t extra_slots,
                  double* out_hilo) {
  model_t md;
  ev_t* ev = NULL;
  int64_t n_ev = 0;
  int32_t* slot = NULL;
  int rc = setup(n, ts, te, y, yerr, slot_in, M, sigma, omega0, quality, kind, amp, off, jitter, &md, &ev, &n_ev, &slot);
  if (rc) return rc;
  if (extra_slots > 0) {
    md.J += extra_slots;
    md.D += extra_slots;
  }
  if (md.D > OR_MAXD) {
    free(ev);
    free(slot);
    return OR_EOVERLAP;
  }
  ld L = 0;
  rc = run_filter(&md, n_ev, ev, ts, te, y, yerr, amp, off, jitter, &L, NULL, NULL);
  out_hilo[0] = (double)L;
  out_hilo[1] = (double)(L - (ld)out_hilo[0]);
  free(ev);
  free(slot);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Square-root (Cholesky-factor) filter                                 */
/* ------------------------------------------------------------------ */
/* The same filter with the covariance carried as a factor, P = L L^T (the
 * square-root form the paper names as the remedy for the filter's loss of
 * accuracy, Sec. 3.2.3 and Sec. 5): the time update takes L- as the
 * triangular factor of [A L, G] (G G^T = Qa), by Householder reflections of
 * its transpose; the measurement update rotates the array
 *     [ sqrt(R)  h^T L- ]        [ sqrt(S)  0  ]
 *     [   0        L-   ]  -->   [   kb     L+ ]
 * by Givens rotations (kb = P- h / sqrt(S)), so that no covariance is formed
 * by subtraction.  The log-likelihood terms are those of Sec. 2.4. */

/* G with G G^T = Q for a symmetric positive semi-definite Q: Cholesky with
 * pivots at or below a rounding threshold taken as zero (their column then
 * zero: such a Q is singular, e.g. identical rows of open integrators). */
static void psd_factor(int D, ld Q[OR_MAXD][OR_MAXD], ld G[OR_MAXD][OR_MAXD]) {
  ld scale = 0;
  for (int i = 0; i < D; ++i) scale = fmaxl(scale, fabsl(Q[i][i]));
  const ld tiny = scale * 1e-30L;
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) G[i][j] = 0;
  for (int k = 0; k < D; ++k) {
    ld d = Q[k][k];
    for (int j = 0; j < k; ++j) d -= G[k][j] * G[k][j];
    if (d <= tiny) continue; /* column k stays zero */
    const ld g = sqrtl(d);
    G[k][k] = g;
    for (int i = k + 1; i < D; ++i) {
      ld v = Q[i][k];
      for (int j = 0; j < k; ++j) v -= G[i][j] * G[k][j];
      G[i][k] = v / g;
    }
  }
}

/* L <- lower-triangular factor of B B^T with B = [A L, G] (D x 2D):
 * Householder QR of B^T, L = R^T. */
static void sqrt_time_update(int D, ld A[OR_MAXD][OR_MAXD], ld G[OR_MAXD][OR_MAXD], ld L[OR_MAXD][OR_MAXD]) {
  ld W[2 * OR_MAXD][OR_MAXD]; /* W = B^T */
  const int n = 2 * D;
  for (int c = 0; c < D; ++c)
    for (int r = 0; r < D; ++r) {
      ld s = 0;
      for (int k = 0; k < D; ++k) s += A[r][k] * L[k][c];
      W[c][r] = s;       /* (A L)^T */
      W[D + c][r] = G[r][c];
    }
  for (int k = 0; k < D; ++k) {
    ld nrm = 0;
    for (int i = k; i < n; ++i) nrm += W[i][k] * W[i][k];
    nrm = sqrtl(nrm);
    if (nrm == 0) continue;
    const ld alpha = W[k][k] > 0 ? -nrm : nrm;
    ld v[2 * OR_MAXD];
    for (int i = 0; i < n; ++i) v[i] = 0;
    v[k] = W[k][k] - alpha;
    for (int i = k + 1; i < n; ++i) v[i] = W[i][k];
    ld vv = 0;
    for (int i = k; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0) continue;
    for (int c = k; c < D; ++c) {
      ld dot = 0;
      for (int i = k; i < n; ++i) dot += v[i] * W[i][c];
      const ld f = 2 * dot / vv;
      for (int i = k; i < n; ++i) W[i][c] -= f * v[i];
    }
  }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) L[i][j] = (j <= i) ? W[j][i] : 0;
}

static int run_filter_sqrt(const model_t* md, int64_t n_ev, const ev_t* ev, const double* ts, const double* te,
                           const double* y, const double* yerr, const double* amp, const double* off, ld jitter,
                           ld* loglik) {
  const int D = md->D, M = md->M;
  ld m[OR_MAXD], L[OR_MAXD][OR_MAXD];
  for (int i = 0; i < D; ++i) {
    m[i] = 0;
    for (int j = 0; j < D; ++j) L[i][j] = 0;
  }
  for (int k = 0; k < M; ++k) {
    L[2 * k][2 * k] = md->sigma[k];
    L[2 * k + 1][2 * k + 1] = md->kind[k] == TERM_REAL ? 0 : md->sigma[k] * md->w0[k];
  }
  for (int j = 0; j < md->J; ++j) L[2 * M + j][2 * M + j] = 1;
  ld total = 0;
  ld A[OR_MAXD][OR_MAXD], Qa[OR_MAXD][OR_MAXD], G[OR_MAXD][OR_MAXD];
  for (int64_t k = 0; k < n_ev; ++k) {
    const ld dt = (k == 0) ? 0 : ev[k].t - ev[k - 1].t;
    assemble(md, dt, A, Qa);
    psd_factor(D, Qa, G);
    {
      ld mn[OR_MAXD];
      for (int i = 0; i < D; ++i) {
        ld s = 0;
        for (int c = 0; c < D; ++c) s += A[i][c] * m[c];
        mn[i] = s;
      }
      for (int i = 0; i < D; ++i) m[i] = mn[i];
    }
    sqrt_time_update(D, A, G, L);
    const int64_t i = ev[k].n;
    if (ev[k].kind == EV_START) {
      const int z = 2 * M + ev[k].slot;
      m[z] = 0;
      for (int a = 0; a < D; ++a) L[z][a] = 0;
      continue;
    }
    ld h[OR_MAXD];
    const ld an = amp ? (ld)amp[i] : 1;
    for (int a = 0; a < D; ++a) h[a] = 0;
    if (ev[k].kind == EV_END)
      h[2 * M + ev[k].slot] = an / ((ld)te[i] - (ld)ts[i]);
    else
      for (int t = 0; t < M; ++t) h[2 * t] = an;
    /* the array: column 0 = (sqrt R, 0...), columns 1..D = (h^T L; L) */
    ld X[OR_MAXD + 1][OR_MAXD + 1];
    for (int r = 0; r <= D; ++r)
      for (int c = 0; c <= D; ++c) X[r][c] = 0;
    X[0][0] = sqrtl((ld)yerr[i] * yerr[i] + jitter * jitter);
    for (int c = 0; c < D; ++c) {
      ld f = 0;
      for (int r = 0; r < D; ++r) f += h[r] * L[r][c];
      X[0][c + 1] = f;
      for (int r = 0; r < D; ++r) X[r + 1][c + 1] = L[r][c];
    }
    for (int c = D; c >= 1; --c) {
      const ld a = X[0][0], b = X[0][c];
      if (b == 0) continue;
      const ld rr = hypotl(a, b);
      const ld cs = a / rr, sn = b / rr;
      for (int r = 0; r <= D; ++r) {
        const ld x0 = X[r][0], x1 = X[r][c];
        X[r][0] = cs * x0 + sn * x1;
        X[r][c] = -sn * x0 + cs * x1;
      }
    }
    const ld sS = X[0][0];
    if (!(sS > 0)) return OR_ENUMERIC;
    ld hm = 0;
    for (int a = 0; a < D; ++a) hm += h[a] * m[a];
    const ld v = (ld)y[i] - (off ? (ld)off[i] : 0) - hm;
    const ld e = v / sS;
    for (int a = 0; a < D; ++a) m[a] += X[a + 1][0] * e;
    for (int r = 0; r < D; ++r)
      for (int c = 0; c < D; ++c) L[r][c] = X[r + 1][c + 1];
    total += -0.5L * (logl(TWO_PI) + 2 * logl(sS) + e * e);
  }
  *loglik = total;
  return isfinite(total) ? OR_OK : OR_ENUMERIC;
}

int oracle_loglik_sqrt(int64_t n, const double* ts, const double* te, const double* y, const double* yerr,
                       const int32_t* slot_in, int32_t M, const double* sigma, const double* omega0,
                       const double* quality, const int32_t* kind, const double* amp, const double* off,
                       double jitter, double* out_hilo) {
  model_t md;
  ev_t* ev = NULL;
  int64_t n_ev = 0;
  int32_t* slot = NULL;
  int rc = setup(n, ts, te, y, yerr, slot_in, M, sigma, omega0, quality, kind, amp, off, jitter, &md, &ev, &n_ev, &slot);
  if (rc) return rc;
  ld L = 0;
  rc = run_filter_sqrt(&md, n_ev, ev, ts, te, y, yerr, amp, off, jitter, &L);
  out_hilo[0] = (double)L;
  out_hilo[1] = (double)(L - (ld)out_hilo[0]);
  free(ev);
  free(slot);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Smoother and prediction                                              */
/* ------------------------------------------------------------------ */

/* X = C Pm^{-1} restricted to the indices where Pm has a non-zero diagonal
 * (an exactly-zero row is a deterministic zero component after a reset
 * followed by a zero-length step); other columns of X are zero. */
static int right_solve(int D, ld C[OR_MAXD][OR_MAXD], ld Pm[OR_MAXD][OR_MAXD], ld X[OR_MAXD][OR_MAXD]) {
  int idx[OR_MAXD], na = 0;
  for (int i = 0; i < D; ++i)
    if (Pm[i][i] != 0) idx[na++] = i;
  /* augmented [Pa | C^T] Gauss-Jordan with partial pivoting */
  ld a[OR_MAXD][2 * OR_MAXD];
  for (int r = 0; r < na; ++r) {
    for (int c = 0; c < na; ++c) a[r][c] = Pm[idx[r]][idx[c]];
    for (int c = 0; c < D; ++c) a[r][na + c] = C[c][idx[r]];
  }
  for (int col = 0; col < na; ++col) {
    int piv = col;
    for (int r = col + 1; r < na; ++r)
      if (fabsl(a[r][col]) > fabsl(a[piv][col])) piv = r;
    if (a[piv][col] == 0) return OR_ENUMERIC;
    if (piv != col)
      for (int c = 0; c < na + D; ++c) {
        ld t = a[piv][c];
        a[piv][c] = a[col][c];
        a[col][c] = t;
      }
    const ld inv = 1 / a[col][col];
    for (int c = 0; c < na + D; ++c) a[col][c] *= inv;
    for (int r = 0; r < na; ++r) {
      if (r == col) continue;
      const ld f = a[r][col];
      if (f == 0) continue;
      for (int c = 0; c < na + D; ++c) a[r][c] -= f * a[col][c];
    }
  }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) X[i][j] = 0;
  for (int r = 0; r < na; ++r)
    for (int c = 0; c < D; ++c) X[c][idx[r]] = a[r][na + c];
  return OR_OK;
}

/* smoothed = base + G (next_s - next_p), cov = Pbase + G (Pnext_s - Pnext_p) G^T */
static void rts_combine(int D, ld G[OR_MAXD][OR_MAXD], const state_t* base, const state_t* next_s, const state_t* next_p,
                        state_t* out) {
  ld dm[OR_MAXD], dP[OR_MAXD][OR_MAXD], t[OR_MAXD][OR_MAXD];
  for (int a = 0; a < D; ++a) dm[a] = next_s->m[a] - next_p->m[a];
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) dP[a][b] = next_s->P[a][b] - next_p->P[a][b];
  for (int a = 0; a < D; ++a) {
    ld s = base->m[a];
    for (int b = 0; b < D; ++b) s += G[a][b] * dm[b];
    out->m[a] = s;
  }
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      ld s = 0;
      for (int c = 0; c < D; ++c) s += G[a][c] * dP[c][b];
      t[a][b] = s;
    }
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      ld s = base->P[a][b];
      for (int c = 0; c < D; ++c) s += t[a][c] * G[b][c];
      out->P[a][b] = s;
    }
}

/* G = Pbase Feff^T Pm^{-1} */
static int rts_gain(int D, const ld Pbase[OR_MAXD][OR_MAXD], ld Feff[OR_MAXD][OR_MAXD], ld Pm[OR_MAXD][OR_MAXD],
                    ld G[OR_MAXD][OR_MAXD]) {
  ld C[OR_MAXD][OR_MAXD];
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      ld s = 0;
      for (int c = 0; c < D; ++c) s += Pbase[a][c] * Feff[b][c];
      C[a][b] = s;
    }
  return right_solve(D, C, Pm, G);
}

static void latent(const model_t* md, const state_t* s, double* mean, double* var) {
  ld mu = 0, v = 0;
  for (int m = 0; m < md->M; ++m) {
    mu += s->m[2 * m];
    for (int l = 0; l < md->M; ++l) v += s->P[2 * m][2 * l];
  }
  *mean = (double)mu;
  *var = (double)v;
}

/* posterior of each term's own process x_m (the component-wise prediction:
 * the latent observation vector restricted to one term), row q of the
 * [n_test][M] outputs */
static void latent_terms(const model_t* md, const state_t* s, int64_t q, double* term_mean, double* term_var) {
  if (!term_mean || !term_var) return;
  for (int m = 0; m < md->M; ++m) {
    term_mean[q * md->M + m] = (double)s->m[2 * m];
    term_var[q * md->M + m] = (double)s->P[2 * m][2 * m];
  }
}

int oracle_smooth(int64_t n, const double* ts, const double* te, const double* y, const double* yerr, const int32_t* slot_in,
                  int32_t M, const double* sigma, const double* omega0, const double* quality, const int32_t* kind,
                  const double* amp, const double* off, double jitter, int64_t n_test,
                  const double* t_test, double* mean_test, double* var_test, double* mean_data, double* var_data,
                  double* term_mean, double* term_var, double* out_hilo) {
  model_t md;
  ev_t* ev = NULL;
  int64_t K = 0;
  int32_t* slot = NULL;
  int rc = setup(n, ts, te, y, yerr, slot_in, M, sigma, omega0, quality, kind, amp, off, jitter, &md, &ev, &K, &slot);
  if (rc) return rc;
  const int D = md.D;
  state_t* pred = (state_t*)malloc(sizeof(state_t) * K);
  state_t* filt = (state_t*)malloc(sizeof(state_t) * K);
  state_t* smo = (state_t*)malloc(sizeof(state_t) * K);
  if (!pred || !filt || !smo) {
    rc = OR_ENOMEM;
    goto done;
  }
  ld L = 0;
  rc = run_filter(&md, K, ev, ts, te, y, yerr, amp, off, jitter, &L, pred, filt);
  if (out_hilo) {
    out_hilo[0] = (double)L;
    out_hilo[1] = (double)(L - (ld)out_hilo[0]);
  }
  if (rc) goto done;

  /* backward pass: smoothed moments of every event; at an exposure start the
   * smoothed quantity is the pre-reset state */
  ld A[OR_MAXD][OR_MAXD], Qa[OR_MAXD][OR_MAXD], Feff[OR_MAXD][OR_MAXD], G[OR_MAXD][OR_MAXD];
  smo[K - 1] = filt[K - 1];
  for (int64_t k = K - 2; k >= 0; --k) {
    assemble(&md, ev[k + 1].t - ev[k].t, A, Qa);
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) Feff[a][b] = A[a][b];
    const state_t* base = &filt[k];
    if (ev[k].kind == EV_START) {
      const int z = 2 * md.M + ev[k].slot;
      for (int a = 0; a < D; ++a) Feff[a][z] = 0;
      base = &pred[k];
    }
    rc = rts_gain(D, base->P, Feff, pred[k + 1].P, G);
    if (rc) goto done;
    rts_combine(D, G, base, &smo[k + 1], &pred[k + 1], &smo[k]);
  }

  /* outputs at the data (exposure-averaged, from end events) */
  if (mean_data && var_data) {
    for (int64_t k = 0; k < K; ++k) {
      const int64_t i = ev[k].n;
      /* the measured quantity without noise: amplitude times the exposure
       * average (or the latent value) plus the offset */
      const ld an = amp ? (ld)amp[i] : 1, cn = off ? (ld)off[i] : 0;
      if (ev[k].kind == EV_END) {
        const int z = 2 * md.M + ev[k].slot;
        const ld dl = (ld)te[i] - (ld)ts[i];
        mean_data[i] = (double)(an * smo[k].m[z] / dl + cn);
        var_data[i] = (double)(an * an * smo[k].P[z][z] / (dl * dl));
      } else if (ev[k].kind == EV_INSTANT) {
        double mu, va;
        latent(&md, &smo[k], &mu, &va);
        mean_data[i] = (double)(an * (ld)mu + cn);
        var_data[i] = (double)(an * an * (ld)va);
      }
    }
  }

  /* predictions of the latent process at arbitrary times */
  for (int64_t q = 0; q < n_test; ++q) {
    const ld tq = t_test[q];
    if (tq < ev[0].t) {
      /* retrodiction from the prior, latent block only */
      const int Dx = 2 * md.M;
      ld Ax[OR_MAXD][OR_MAXD], Pinf[OR_MAXD][OR_MAXD], Gx[OR_MAXD][OR_MAXD];
      assemble(&md, ev[0].t - tq, A, Qa);
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          Ax[a][b] = (a < Dx && b < Dx) ? A[a][b] : 0;
          Pinf[a][b] = 0;
        }
      for (int m = 0; m < md.M; ++m) {
        Pinf[2 * m][2 * m] = md.sigma[m] * md.sigma[m];
        Pinf[2 * m + 1][2 * m + 1] = md.kind[m] == TERM_REAL ? 0 : md.sigma[m] * md.sigma[m] * md.w0[m] * md.w0[m];
      }
      rc = rts_gain(D, Pinf, Ax, Pinf, Gx);
      if (rc) goto done;
      state_t base, nxs, nxp, out;
      memset(&base, 0, sizeof(base));
      memset(&nxs, 0, sizeof(nxs));
      memset(&nxp, 0, sizeof(nxp));
      for (int a = 0; a < Dx; ++a) {
        nxs.m[a] = smo[0].m[a];
        for (int b = 0; b < Dx; ++b) {
          base.P[a][b] = Pinf[a][b];
          nxs.P[a][b] = smo[0].P[a][b];
          nxp.P[a][b] = Pinf[a][b];
        }
      }
      rts_combine(D, Gx, &base, &nxs, &nxp, &out);
      latent(&md, &out, &mean_test[q], &var_test[q]);
      latent_terms(&md, &out, q, term_mean, term_var);
      continue;
    }
    if (tq > ev[K - 1].t) {
      state_t out = filt[K - 1];
      assemble(&md, tq - ev[K - 1].t, A, Qa);
      predict(D, A, Qa, out.m, out.P);
      latent(&md, &out, &mean_test[q], &var_test[q]);
      latent_terms(&md, &out, q, term_mean, term_var);
      continue;
    }
    /* first event with t >= tq */
    int64_t lo = 0, hi = K - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (ev[mid].t >= tq)
        hi = mid;
      else
        lo = mid + 1;
    }
    if (ev[lo].t == tq) {
      latent(&md, &smo[lo], &mean_test[q], &var_test[q]);
      latent_terms(&md, &smo[lo], q, term_mean, term_var);
      continue;
    }
    const int64_t nx = lo, pv = lo - 1; /* ev[pv].t < tq < ev[nx].t */
    state_t star = filt[pv];
    assemble(&md, tq - ev[pv].t, A, Qa);
    predict(D, A, Qa, star.m, star.P);
    state_t nxp = star;
    assemble(&md, ev[nx].t - tq, A, Qa);
    predict(D, A, Qa, nxp.m, nxp.P);
    rc = rts_gain(D, star.P, A, nxp.P, G);
    if (rc) goto done;
    state_t out;
    rts_combine(D, G, &star, &smo[nx], &nxp, &out);
    latent(&md, &out, &mean_test[q], &var_test[q]);
      latent_terms(&md, &out, q, term_mean, term_var);
  }
  rc = OR_OK;
done:
  free(pred);
  free(filt);
  free(smo);
  free(ev);
  free(slot);
  return rc;
}
