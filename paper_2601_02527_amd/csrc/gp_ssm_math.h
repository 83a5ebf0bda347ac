// Device math of the augmented state-space filter: discretisation of one SHO
// term over one step, and the structured predict / update / reset steps of
// the filter on the augmented state (SHO states stacked, then one integrator
// per instrument slot).
//
// Coordinates.  Each SHO term m is kept in the scaled state
// (x_m, xdot_m / omega0_m), whose stationary covariance is sigma_m^2 I
// (Appendix B, stationary covariance, after scaling the derivative by
// omega0).  Integrators z_j are unscaled (z_j = integral of sum_m x_m over the
// open exposure, Sec. 3.2).  An integrator is kept at exactly zero (mean and
// covariance) while its slot is closed: it is zeroed right after the update
// at the exposure end instead of at the next exposure start.  Because a closed
// integrator never feeds the SHO states or the other integrators, the joint
// law of the SHO states and the open integrators is the same as with the
// reset of Sec. 3.2.1, so every likelihood term is unchanged.
//
// Discretisation.  With x = omega0*dt, beta = 1/(2Q), the impulse response g
// of g'' + 2 beta g' + g = 0 (g(0) = 0, g'(0) = 1) gives every quantity of
// the augmented step (Appendix B closed forms, rewritten):
//   transition          [[g' + 2 beta g, g], [-g, g']]
//   integrated row      (g + 2 beta G1, G1) / omega0,     G1 = int g
//   process noise       qhat [[int g^2, g^2/2], [g^2/2, int g'^2]]
//   x/z cross noise     qhat (G1^2/2, G1 g - int g^2) / omega0
//   z/z noise           qhat int G1^2 / omega0^2,         qhat = 2 sigma^2/Q
// For x max(1, beta) > XSER the closed forms use
//   G1 = 1 - g' - 2 beta g,     int g'^2 = (1 - g'^2 - g^2) / (4 beta),
//   int g^2 = int g'^2 - g g' - beta g^2,
//   int G1^2 = x - g - 2 beta G1 - G1 g + int g^2 - beta G1^2,
// with g = e^{-beta x} sin(eta x)/eta, eta^2 = 1 - beta^2 continued
// analytically (cos/sin, cosh/sinh, or their series in eta^2 x^2 near
// Q = 1/2).  Below the threshold these lose digits (int G1^2 ~ x^5/20) and a
// Taylor series in x is used; its coefficients depend on beta only and are
// produced once per term by the recurrence of the linear ODE satisfied by
// (g, g', G1, g^2, g g', g'^2, G1^2, G1 g, G1 g', int g^2, int g'^2,
// int G1^2).  The beta-derivative rides along as a dual number for the
// adjoint; x-derivatives follow from the ODE.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GPD __host__ __device__ __forceinline__

namespace gpssm {

constexpr double XSER = 0.75;     // series used when x * max(1, beta) <= XSER
constexpr int NI = 4;             // series intervals on [0, xser]: [0, F0 xser], then NI - 1 equal ones
constexpr double F0 = 0.16;
constexpr int KSER = 15;          // highest power kept in each interval's expansion
constexpr int KSER_G = 12;        // gradient-only passes: degree and switch point
constexpr double XSER_G = 0.4;
constexpr int NSET = 4;           // coefficient sets: G1, int g^2, int g'^2, int G1^2
constexpr int NS = KSER + 1;      // coefficients per set (u^0 .. u^KSER)
// doubles per interval table: the coefficients, padded by 32 bytes so that
// the tables of the NI intervals start on different LDS banks (lanes in
// different intervals read them in the same instruction)
constexpr int ISTRIDE = NS * NSET + 4;
constexpr int NCOEF = NI * ISTRIDE;  // value tables of one term; the beta-derivatives follow
constexpr double LOG_2PI = 1.8378770664093454835606594728112;

// ---------------------------------------------------------------------------
// dual numbers: value and derivative with respect to beta
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
};
GPD Dual dual(double v, double d = 0.0) { return Dual{v, d}; }
GPD Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
GPD Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
GPD Dual operator-(Dual a) { return {-a.v, -a.d}; }
GPD Dual operator*(Dual a, Dual b) { return {a.v * b.v, fma(a.v, b.d, a.d * b.v)}; }
GPD Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
GPD Dual operator*(Dual a, double s) { return {s * a.v, s * a.d}; }
GPD Dual operator+(Dual a, double s) { return {a.v + s, a.d}; }
GPD Dual operator+(double s, Dual a) { return {a.v + s, a.d}; }
GPD Dual operator-(Dual a, double s) { return {a.v - s, a.d}; }
GPD Dual operator-(double s, Dual a) { return {s - a.v, -a.d}; }
GPD Dual operator/(Dual a, Dual b) {
  const double r = 1.0 / b.v;
  const double q = a.v * r;
  return {q, (a.d - q * b.d) * r};
}
GPD Dual operator/(Dual a, double s) { return {a.v / s, a.d / s}; }
GPD double val(double a) { return a; }
GPD double val(Dual a) { return a.v; }
GPD double fexp(double a) { return exp(a); }
GPD Dual fexp(Dual a) {
  const double e = exp(a.v);
  return {e, e * a.d};
}
GPD double fsqrt(double a) { return sqrt(a); }
GPD Dual fsqrt(Dual a) {
  const double s = sqrt(a.v);
  return {s, 0.5 * a.d / s};
}
GPD void fsincos(double a, double* s, double* c) {
#ifdef __HIP_DEVICE_COMPILE__
  sincos(a, s, c);
#else
  *s = sin(a);
  *c = cos(a);
#endif
}
GPD void fsincos(Dual a, Dual* s, Dual* c) {
  double sv, cv;
  fsincos(a.v, &sv, &cv);
  *s = {sv, cv * a.d};
  *c = {cv, -sv * a.d};
}
template <class T>
GPD T fconst(double v);
template <>
GPD double fconst<double>(double v) {
  return v;
}
template <>
GPD Dual fconst<Dual>(double v) {
  return Dual{v, 0.0};
}

// the six base functions of one term over one step
template <class T>
struct Base {
  T g, gp, G1, Igg, Ipp, IGG;
};

// ---------------------------------------------------------------------------
// Taylor coefficients (value and beta-derivative) of the base functions
// ---------------------------------------------------------------------------
// v' = B v for v = (g, g', G1, g^2, gg', g'^2, G1^2, G1g, G1g', Igg, Ipp, IGG)
// is linear, so the Taylor coefficients about any point xc follow
// c_{n+1} = B c_n / (n + 1) from c_0 = v(xc), and their beta-derivatives (at
// fixed xc) follow d_{n+1} = (B d_n + (dB/dbeta) c_n) / (n + 1).
GPD void ode_step(double beta, int n, double* c, double* d) {
  const double b2 = 2.0 * beta, b4 = 4.0 * beta;
  double nc[12], nd[12];
  nc[0] = c[1];
  nc[1] = -c[0] - b2 * c[1];
  nc[2] = c[0];
  nc[3] = 2.0 * c[4];
  nc[4] = c[5] - c[3] - b2 * c[4];
  nc[5] = -2.0 * c[4] - b4 * c[5];
  nc[6] = 2.0 * c[7];
  nc[7] = c[3] + c[8];
  nc[8] = c[4] - c[7] - b2 * c[8];
  nc[9] = c[3];
  nc[10] = c[5];
  nc[11] = c[6];
  nd[0] = d[1];
  nd[1] = -d[0] - b2 * d[1] - 2.0 * c[1];
  nd[2] = d[0];
  nd[3] = 2.0 * d[4];
  nd[4] = d[5] - d[3] - b2 * d[4] - 2.0 * c[4];
  nd[5] = -2.0 * d[4] - b4 * d[5] - 4.0 * c[5];
  nd[6] = 2.0 * d[7];
  nd[7] = d[3] + d[8];
  nd[8] = d[4] - d[7] - b2 * d[8] - 2.0 * c[8];
  nd[9] = d[3];
  nd[10] = d[5];
  nd[11] = d[6];
  const double inv = 1.0 / (n + 1);
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    c[i] = nc[i] * inv;
    d[i] = nd[i] * inv;
  }
}

// expansion point of series interval i: 0 for the first interval [0, b1],
// whose expansion about 0 keeps the relative accuracy of the functions that
// vanish there (int G1^2 ~ x^5/20), the midpoint of the others (width w)
GPD double interval_centre(int i, double b1, double w) { return i == 0 ? 0.0 : b1 + (i - 0.5) * w; }

// The tables of one term: coef[i * ISTRIDE + n * NSET + s], the coefficient
// of u^n (u = x - xc_i) of set s = G1, Igg, Ipp, IGG in interval i (degree-
// major, so one Horner step reads all four sets at once); dcoef likewise for
// the beta-derivatives.  g = G1' and g' = G1'' come out of the same Horner
// pass as G1.  The state at an interval centre xc > 0 is the series about 0
// summed to degree KSUM (terms below 1e-30 there).
//
// One interval's table (coef, dcoef point at interval i's slots):
GPD void series_interval_table(double beta, double xc, double* coef, double* dcoef) {
  constexpr int KSUM = 44;
  double c[12], d[12], v[12], dv[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) c[k] = d[k] = v[k] = dv[k] = 0.0;
  c[1] = 1.0;  // g'(0)
  c[5] = 1.0;  // g'(0)^2
  if (xc == 0.0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = c[k];
  } else {
    double pw = 1.0;
#pragma unroll
    for (int n = 0; n <= KSUM; ++n) {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        v[k] = fma(c[k], pw, v[k]);
        dv[k] = fma(d[k], pw, dv[k]);
      }
      pw *= xc;
      ode_step(beta, n, c, d);
    }
  }
  const int out[NSET] = {2, 9, 10, 11};
#pragma unroll
  for (int n = 0; n <= KSER; ++n) {
#pragma unroll
    for (int f = 0; f < NSET; ++f) {
      coef[n * NSET + f] = v[out[f]];
      dcoef[n * NSET + f] = dv[out[f]];
    }
    ode_step(beta, n, v, dv);
  }
#pragma unroll
  for (int k = NS * NSET; k < ISTRIDE; ++k) coef[k] = dcoef[k] = 0.0;
}
// all intervals of one term
GPD void series_coefficients(double beta, double b1, double w, double* coef, double* dcoef) {
  for (int i = 0; i < NI; ++i)
    series_interval_table(beta, interval_centre(i, b1, w), coef + i * ISTRIDE, dcoef + i * ISTRIDE);
}

// The kernels stage a series' tables in LDS once; every lane then reads the
// same address (a broadcast read) in the Horner loops below.  The tables are
// never written while a kernel evaluates them, so without a compiler fence
// their reads are hoisted out of the event loops or shared between calls and
// held in (spilled) registers; table_fence keeps each evaluation's reads at
// its own use.
typedef const double* coef_ptr;
GPD void table_fence() {
#ifdef __HIP_DEVICE_COMPILE__
  __asm__ __volatile__("" ::: "memory");
#endif
}

// Horner evaluation of the four series at u, all sets in one pass:
// G1 with G1' = g and G1''/2, and the three integrals
struct Series4 {
  double G1, g, gph, Igg, Ipp, IGG;
};
template <int K>
GPD Series4 horner4(coef_ptr e, double x) {
  Series4 r;
  double b = e[K * NSET + 0], d = 0.0, dd = 0.0;
  double i1 = e[K * NSET + 1], i2 = e[K * NSET + 2], i3 = e[K * NSET + 3];
#pragma unroll
  for (int n = K - 1; n >= 0; --n) {
    dd = fma(dd, x, d);
    d = fma(d, x, b);
    b = fma(b, x, e[n * NSET + 0]);
    i1 = fma(i1, x, e[n * NSET + 1]);
    i2 = fma(i2, x, e[n * NSET + 2]);
    i3 = fma(i3, x, e[n * NSET + 3]);
  }
  r.G1 = b;
  r.g = d;
  r.gph = dd;
  r.Igg = i1;
  r.Ipp = i2;
  r.IGG = i3;
  return r;
}

// interval of x (first interval [0, b1], then width w, 1/w = iw) and the
// offset from its expansion point; the index stays in [0, NI) whatever x is
GPD int series_interval(double x, double b1, double w, double iw, double& u) {
  const double q = (x - b1) * iw;
  int i = (x >= b1) ? 1 : 0;
#pragma unroll
  for (int k = 1; k < NI - 1; ++k) i += (q >= (double)k) ? 1 : 0;
  u = x - interval_centre(i, b1, w);
  return i;
}

// ---------------------------------------------------------------------------
// per-term constants and per-step quantities
// ---------------------------------------------------------------------------
struct TermConst {
  double w0, beta, qhat, inv_w0, sigma;
  double eta2;     // 1 - beta^2 (its sign selects the damping regime)
  double eta;      // sqrt(|eta2|)
  double inv_eta;  // 1/sqrt(|eta2|), 0 at critical damping
  double inv_4b;   // 1/(4 beta)
  double xser;     // the series is used for omega0 dt <= xser
  double inv_qhat; // 1/qhat
  double xser_g;   // switch point of the gradient-only passes
  double b1ser;    // end of the first series interval, F0 xser
  double wser;     // width of the other series intervals, (xser - b1ser) / (NI - 1)
  double inv_wser; // 1 / wser
};

GPD TermConst make_term(double sigma, double w0, double quality) {
  TermConst t;
  t.w0 = w0;
  t.beta = 0.5 / quality;
  t.qhat = 2.0 * sigma * sigma / quality;
  t.inv_w0 = 1.0 / w0;
  t.sigma = sigma;
  t.eta2 = 1.0 - t.beta * t.beta;
  t.eta = sqrt(fabs(t.eta2));
  t.inv_eta = (t.eta2 != 0.0) ? 1.0 / t.eta : 0.0;
  t.inv_4b = 0.25 / t.beta;
  t.xser = XSER / fmax(1.0, t.beta);
  t.inv_qhat = 1.0 / t.qhat;
  t.xser_g = XSER_G / fmax(1.0, t.beta);
  t.b1ser = F0 * t.xser;
  t.wser = (t.xser - t.b1ser) / (NI - 1);
  t.inv_wser = 1.0 / t.wser;
  return t;
}

// A real (exponential) term, k(tau) = sigma^2 exp(-c |tau|) (the real
// celerite term of Appendix A: b = d = 0), rides in an SHO term's two
// states: the first is the process (an Ornstein-Uhlenbeck process with rate
// c, kept in omega0), the second stays at exactly zero (no transition into
// it, no noise, no prior variance).  It is marked by a negative series switch
// point (its steps never take the SHO series); the other fields are those of
// an SHO term with Q = 1, so the tables built for it are valid and unused.
GPD TermConst make_real_term(double sigma, double c) {
  TermConst t = make_term(sigma, c, 1.0);  // qhat = 2 sigma^2, inv_w0 = 1/c
  t.xser = -1.0;
  t.xser_g = -1.0;
  return t;
}
// X: real terms may occur (kernels built without them take X = false, and
// the test folds away)
template <bool X = true>
GPD bool is_real(const TermConst& t) {
  return X && t.xser < 0.0;
}
// stationary variance of the term's second state over sigma^2
template <bool X = true>
GPD double second_prior(const TermConst& t) {
  return is_real<X>(t) ? 0.0 : 1.0;
}

// x - 2 (1 - e^-x) + (1 - e^-2x)/2 (the integrated process's variance over
// 2 sigma^2 / c^2), by its series below x = 0.5, where the closed form
// cancels: sum over n >= 3 of (-1)^(n+1) (2^(n-1) - 2) x^n / n!
GPD double real_gfun(double x, double em1, double e1) {
  if (x >= 0.5) return x - em1 * (3.0 - e1) * 0.5;
  double term = x * x * x / 6.0, s = 0.0, p2 = 4.0;  // x^n/n! and 2^(n-1) at n = 3
#pragma unroll
  for (int n = 3; n <= 22; ++n) {
    s += ((n & 1) ? 1.0 : -1.0) * (p2 - 2.0) * term;
    term *= x / (n + 1);
    p2 *= 2.0;
  }
  return s;
}

// x e^-x - (1 - e^-x), by its series below x = 0.5: sum over n >= 2 of
// (-1)^(n-1) (n - 1) x^n / n!
GPD double real_hfun(double x, double em1, double e1) {
  if (x >= 0.5) return x * e1 - em1;
  double term = x * x * 0.5, s = 0.0;
#pragma unroll
  for (int n = 2; n <= 21; ++n) {
    s += ((n & 1) ? 1.0 : -1.0) * (n - 1) * term;
    term *= x / (n + 1);
  }
  return s;
}

// the series at x truncated after degree K (coef: the term's tables, value
// part then beta-derivative)
template <int K = KSER>
GPD void series_eval(const double* coef, double x, const TermConst& t, Base<double>& o) {
  table_fence();
  double u;
  const int i = series_interval(x, t.b1ser, t.wser, t.inv_wser, u);
  const Series4 v = horner4<K>(coef + i * ISTRIDE, u);
  o.G1 = v.G1;
  o.g = v.g;
  o.gp = 2.0 * v.gph;
  o.Igg = v.Igg;
  o.Ipp = v.Ipp;
  o.IGG = v.IGG;
}
template <int K = KSER>
GPD void series_eval(const double* coef, double x, const TermConst& t, Base<Dual>& o) {
  table_fence();
  double u;
  const int i = series_interval(x, t.b1ser, t.wser, t.inv_wser, u);
  const Series4 v = horner4<K>(coef + i * ISTRIDE, u);
  const Series4 d = horner4<K>(coef + NCOEF + i * ISTRIDE, u);
  o.G1 = {v.G1, d.G1};
  o.g = {v.g, d.g};
  o.gp = {2.0 * v.gph, 2.0 * d.gph};
  o.Igg = {v.Igg, d.Igg};
  o.Ipp = {v.Ipp, d.Ipp};
  o.IGG = {v.IGG, d.IGG};
}

// cos(u) - sin(u)/u and its hyperbolic counterpart cosh(u) - sinh(u)/u
// (ru = 1/u), without cancellation for small u (series below 0.1)
GPD double cos_minus_sinc(double u, double ru, double s, double c) {
  if (fabs(u) < 0.1) {
    const double u2 = u * u;
    return u2 * (-1.0 / 3.0 + u2 * (1.0 / 30.0 + u2 * (-1.0 / 840.0 + u2 * (1.0 / 45360.0))));
  }
  return fma(-s, ru, c);
}
GPD double cosh_minus_sinhc(double u, double ru, double sh, double ch) {
  if (fabs(u) < 0.1) {
    const double u2 = u * u;
    return u2 * (1.0 / 3.0 + u2 * (1.0 / 30.0 + u2 * (1.0 / 840.0 + u2 * (1.0 / 45360.0))));
  }
  return fma(-sh, ru, ch);
}

// e^{-beta x} cos(eta x) and e^{-beta x} sin(eta x)/eta (eta^2 = 1 - beta^2,
// hyperbolic when negative, the limit at eta = 0) with their beta-derivatives.
// The regime is a property of the term (uniform over a wavefront); the
// eta-derivatives use d eta/d beta = -beta/eta and the cancellation-free
// combinations above.
GPD void damped_cs(double x, const TermConst& t, Dual& eC, Dual& eS) {
  const double beta = t.beta;
  const double e = exp(-beta * x);
  const double de = -x * e;  // d e / d beta
  double C, S, dC, dS;       // C(x; beta), S(x; beta) and their beta-derivatives
  if (t.eta2 > 0.0) {
    const double eta = t.eta, u = eta * x;
    double sn, cs;
    fsincos(u, &sn, &cs);
    C = cs;
    S = sn * t.inv_eta;
    // dC/d(eta^2) = -x S / 2 ; dS/d(eta^2) = x^2 (cos u - sin u/u) / (2 u^2) * ... written as below
    const double dC_deta2 = -0.5 * x * S;
    // x^3/u^2 = x/eta^2; x > 0 on the closed-form branch
    const double ru = t.inv_eta / x;
    const double dS_deta2 = 0.5 * x * cos_minus_sinc(u, ru, sn, cs) * (t.inv_eta * t.inv_eta);
    dC = -2.0 * beta * dC_deta2;
    dS = -2.0 * beta * dS_deta2;
  } else if (t.eta2 < 0.0) {
    const double k = t.eta, u = k * x;
    double sh, ch;
    if (u > 0.5) {
      // e^{-beta x} cosh/sinh through exponentials (no overflow), then divide e back out below
      const double ep = exp(u - beta * x), em = exp(-u - beta * x);
      const double eCv = 0.5 * (ep + em), eSv = 0.5 * (ep - em) * t.inv_eta;
      // derivatives: d/dbeta of e^{-bx} cosh(kx) with k^2 = beta^2 - 1, dk/dbeta = beta/k
      const double dk = beta * t.inv_eta;
      const double deC = -x * eCv + x * dk * (eSv * k);
      // S = sinh(u)/k:  dS/dk = (x cosh u - sinh(u)/k)/k
      const double dSdk = (x * (eCv) - eSv) * t.inv_eta;  // times e already included
      const double deS = -x * eSv + dk * dSdk;
      eC = Dual{eCv, deC};
      eS = Dual{eSv, deS};
      return;
    }
    const double a = expm1(u), bm = expm1(-u);
    sh = 0.5 * (a - bm);
    ch = 1.0 + 0.5 * (a + bm);
    C = ch;
    S = sh * t.inv_eta;
    // with kappa = k^2 = beta^2 - 1: dC/dkappa = x S/2, dS/dkappa = x^3 (cosh u - sinh u/u)/(2 u^2)
    const double dC_dk2 = 0.5 * x * S;
    const double ru = t.inv_eta / x;
    const double dS_dk2 = 0.5 * x * cosh_minus_sinhc(u, ru, sh, ch) * (t.inv_eta * t.inv_eta);
    dC = 2.0 * beta * dC_dk2;
    dS = 2.0 * beta * dS_dk2;
  } else {
    // critical damping: C = 1, S = x, dC/d(eta^2) = -x^2/2, dS/d(eta^2) = -x^3/6
    C = 1.0;
    S = x;
    dC = -2.0 * beta * (-0.5 * x * x);
    dS = -2.0 * beta * (-(1.0 / 6.0) * x * x * x);
  }
  eC = Dual{e * C, fma(de, C, e * dC)};
  eS = Dual{e * S, fma(de, S, e * dS)};
}

// closed forms with the beta-derivative
GPD void closed_eval(double x, const TermConst& t, Base<Dual>& o) {
  const Dual beta{t.beta, 1.0};
  Dual eC, eS;
  damped_cs(x, t, eC, eS);
  const Dual g = eS;
  const Dual gp = eC - beta * eS;
  const Dual G1 = 1.0 - gp - 2.0 * beta * g;
  const Dual ipn = 1.0 - gp * gp - g * g;  // Ipp = ipn / (4 beta)
  const double ipv = ipn.v * t.inv_4b;
  const Dual Ipp{ipv, (ipn.d - 4.0 * ipv) * t.inv_4b};
  const Dual Igg = Ipp - g * gp - beta * g * g;
  const Dual IGG = (x - g) - 2.0 * beta * G1 - G1 * g + Igg - beta * G1 * G1;
  o.g = g;
  o.gp = gp;
  o.G1 = G1;
  o.Igg = Igg;
  o.Ipp = Ipp;
  o.IGG = IGG;
}

// value-only closed forms.  The damping regime is a property of the term, so
// this branch is uniform over a wavefront that shares hyperparameters.
GPD void closed_eval(double x, const TermConst& t, Base<double>& o) {
  const double beta = t.beta;
  double eC, eS;
  if (t.eta2 > 0.0) {
    double sn, cs;
    fsincos(t.eta * x, &sn, &cs);
    const double e = exp(-beta * x);
    eC = e * cs;
    eS = e * sn * t.inv_eta;
  } else if (t.eta2 < 0.0) {
    const double r = t.eta * x, bx = beta * x;
    if (r > 0.5) {
      const double ep = exp(r - bx), em = exp(-r - bx);
      eC = 0.5 * (ep + em);
      eS = 0.5 * (ep - em) * t.inv_eta;
    } else {  // sinh without cancellation near critical damping
      const double e = exp(-bx);
      const double a = expm1(r), b = expm1(-r);
      eC = e * (1.0 + 0.5 * (a + b));
      eS = e * 0.5 * (a - b) * t.inv_eta;
    }
  } else {
    const double e = exp(-beta * x);
    eC = e;
    eS = e * x;
  }
  const double g = eS;
  const double gp = fma(-beta, eS, eC);
  const double G1 = (1.0 - gp) - 2.0 * beta * g;
  const double Ipp = (1.0 - gp * gp - g * g) * t.inv_4b;
  const double Igg = Ipp - g * gp - beta * g * g;
  const double IGG = (x - g) - 2.0 * beta * G1 - G1 * g + Igg - beta * G1 * G1;
  o.g = g;
  o.gp = gp;
  o.G1 = G1;
  o.Igg = Igg;
  o.Ipp = Ipp;
  o.IGG = IGG;
}

// one term over one step, scaled SHO coordinates, unscaled integrator
struct TermQ {
  double a00, a01, a11;  // transition [[a00, a01], [-a01, a11]]
  double f0, f1;         // integrated transition row
  double q00, q01, q11;  // process noise
  double c0, c1;         // SHO/integrator cross noise
  double zz;             // integrator/integrator noise
};


GPD TermQ term_step(const TermConst& t, const Base<double>& b) {
  TermQ q;
  const double beta = t.beta;
  q.a00 = b.gp + 2.0 * beta * b.g;
  q.a01 = b.g;
  q.a11 = b.gp;
  q.f0 = (b.g + 2.0 * beta * b.G1) * t.inv_w0;
  q.f1 = b.G1 * t.inv_w0;
  q.q00 = t.qhat * b.Igg;
  q.q01 = t.qhat * 0.5 * b.g * b.g;
  q.q11 = t.qhat * b.Ipp;
  q.c0 = t.qhat * 0.5 * b.G1 * b.G1 * t.inv_w0;
  q.c1 = t.qhat * (b.G1 * b.g - b.Igg) * t.inv_w0;
  q.zz = t.qhat * b.IGG * t.inv_w0 * t.inv_w0;
  return q;
}

// one step of a real term (state (x, 0) and an integrator): transition e^-x,
// integrated row (1 - e^-x)/c, noise sigma^2 (1 - e^-2x), cross noise
// sigma^2 (1 - e^-x)^2 / c, integrator noise 2 sigma^2 g(x) / c^2, x = c dt
GPD TermQ real_step(const TermConst& t, double dt) {
  const double x = t.w0 * dt;
  const double em1 = -expm1(-x), e1 = 1.0 - em1;
  const double s2 = 0.5 * t.qhat;  // sigma^2
  TermQ q;
  q.a00 = e1;
  q.a01 = 0.0;
  q.a11 = 0.0;
  q.f0 = em1 * t.inv_w0;
  q.f1 = 0.0;
  q.q00 = s2 * em1 * (1.0 + e1);
  q.q01 = 0.0;
  q.q11 = 0.0;
  q.c0 = s2 * em1 * em1 * t.inv_w0;
  q.c1 = 0.0;
  q.zz = 2.0 * s2 * real_gfun(x, em1, e1) * t.inv_w0 * t.inv_w0;
  return q;
}

// Gradient of one real-term step: W holds the weights of the step's fields
// (see term_backprop); the fields depend on sigma (noise, cross noise and
// integrator noise are proportional to sigma^2) and on c through x = c dt.
GPD void real_backprop(const TermConst& t, double dt, const double* W, double& gs, double& gw) {
  const double c = t.w0, ic = t.inv_w0, x = c * dt;
  const double em1 = -expm1(-x), e1 = 1.0 - em1;
  const double s2 = 0.5 * t.qhat;
  const double g = real_gfun(x, em1, e1);
  // d/dc of each field
  const double da00 = -dt * e1;
  const double df0 = real_hfun(x, em1, e1) * ic * ic;
  const double dq00 = 2.0 * s2 * dt * e1 * e1;
  const double dc0 = s2 * em1 * (2.0 * x * e1 - em1) * ic * ic;
  const double dzz = 2.0 * s2 * (x * em1 * em1 - 2.0 * g) * ic * ic * ic;
  gw += W[0] * da00 + W[3] * df0 + W[5] * dq00 + W[8] * dc0 + W[10] * dzz;
  // d/dsigma: the noise fields over sigma, twice
  const double q00 = s2 * em1 * (1.0 + e1), c0 = s2 * em1 * em1 * ic, zz = 2.0 * s2 * g * ic * ic;
  gs += 2.0 * (W[5] * q00 + W[8] * c0 + W[10] * zz) / t.sigma;
}

// ---------------------------------------------------------------------------
// packed symmetric storage (upper triangle, row major)
// ---------------------------------------------------------------------------
GPD constexpr int sidx(int i, int j, int D) {
  return (i <= j) ? (i * D - (i * (i - 1)) / 2 + (j - i)) : (j * D - (j * (j - 1)) / 2 + (i - j));
}

template <int M_, int J_>
struct Dims {
  static constexpr int M = M_;
  static constexpr int J = J_;
  static constexpr int NX = 2 * M_;
  static constexpr int D = 2 * M_ + J_;
  static constexpr int NP = D * (D + 1) / 2;
  static constexpr int NXP = NX * (NX + 1) / 2;
};

// event encoding (32 bits): kind in bits 0-1, slot in bits 2-4, the set of
// slots open during the step that ends at this event in bits 8-15, the
// instrument of a measurement in bits 16-18
enum : uint32_t { EV_END = 0u, EV_INSTANT = 1u, EV_START = 2u, EV_PAD = 3u };
constexpr int MAX_INST = 8;
constexpr uint32_t EV_INST_SHIFT = 16u;
// a series' row of the instrument table: per instrument 1/amplitude, offset,
// amplitude and log(amplitude), each block MAX_INST wide
enum : int { ITAB_INVA = 0, ITAB_OFF = MAX_INST, ITAB_AMP = 2 * MAX_INST, ITAB_LOGA = 3 * MAX_INST, ITAB_W = 4 * MAX_INST };
GPD uint32_t ev_kind(uint32_t info) { return info & 3u; }
GPD uint32_t ev_slot(uint32_t info) { return (info >> 2) & 7u; }
GPD uint32_t ev_open(uint32_t info) { return (info >> 8) & 0xffu; }
GPD uint32_t ev_inst(uint32_t info) { return (info >> EV_INST_SHIFT) & 7u; }

// ---------------------------------------------------------------------------
// predict: m <- A m, P <- A P A^T + Q on the augmented state
// ---------------------------------------------------------------------------
template <class Dm>
GPD void predict_mean(double* m, const TermQ* tq, uint32_t open) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX;
  double fx = 0.0;
#pragma unroll
  for (int t = 0; t < M; ++t) fx = fma(tq[t].f0, m[2 * t], fma(tq[t].f1, m[2 * t + 1], fx));
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const double x0 = m[2 * t], x1 = m[2 * t + 1];
    m[2 * t] = fma(tq[t].a00, x0, tq[t].a01 * x1);
    m[2 * t + 1] = fma(-tq[t].a01, x0, tq[t].a11 * x1);
  }
#pragma unroll
  for (int j = 0; j < J; ++j) m[NX + j] += ((open >> j) & 1u) ? fx : 0.0;
}

template <class Dm>
GPD void predict_cov(double* P, const TermQ* tq, uint32_t open) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D;
  // fbar = (f0_1, f1_1, f0_2, ...)
  double fb[NX];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    fb[2 * t] = tq[t].f0;
    fb[2 * t + 1] = tq[t].f1;
  }
  // w = Pxx fbar, s = fbar.w, v_j = fbar . Pxz[:, j]
  double w[NX];
#pragma unroll
  for (int a = 0; a < NX; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < NX; ++c) acc = fma(P[sidx(a, c, D)], fb[c], acc);
    w[a] = acc;
  }
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < NX; ++a) s = fma(fb[a], w[a], s);
  double v[J > 0 ? J : 1];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < NX; ++a) acc = fma(fb[a], P[sidx(a, NX + j, D)], acc);
    v[j] = acc;
  }
  double zz = 0.0;
#pragma unroll
  for (int t = 0; t < M; ++t) zz += tq[t].zz;
  // integrator block
#pragma unroll
  for (int i = 0; i < J; ++i) {
    const double oi = ((open >> i) & 1u) ? 1.0 : 0.0;
#pragma unroll
    for (int j = i; j < J; ++j) {
      const double oj = ((open >> j) & 1u) ? 1.0 : 0.0;
      double& p = P[sidx(NX + i, NX + j, D)];
      p = p + oi * v[j] + oj * v[i] + oi * oj * (s + zz);
    }
  }
  // SHO/integrator block: Phi (Pxz[:, j] + o_j w) + o_j c
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const double oj = ((open >> j) & 1u) ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const double y0 = fma(oj, w[2 * t], P[sidx(2 * t, NX + j, D)]);
      const double y1 = fma(oj, w[2 * t + 1], P[sidx(2 * t + 1, NX + j, D)]);
      P[sidx(2 * t, NX + j, D)] = fma(tq[t].a00, y0, fma(tq[t].a01, y1, oj * tq[t].c0));
      P[sidx(2 * t + 1, NX + j, D)] = fma(-tq[t].a01, y0, fma(tq[t].a11, y1, oj * tq[t].c1));
    }
  }
  // SHO block: Phi_t B Phi_u^T (+ Q on the diagonal blocks)
#pragma unroll
  for (int t = 0; t < M; ++t) {
#pragma unroll
    for (int u = t; u < M; ++u) {
      const double b00 = P[sidx(2 * t, 2 * u, D)], b01 = P[sidx(2 * t, 2 * u + 1, D)];
      const double b10 = P[sidx(2 * t + 1, 2 * u, D)], b11 = P[sidx(2 * t + 1, 2 * u + 1, D)];
      // Y = Phi_t B
      const double y00 = fma(tq[t].a00, b00, tq[t].a01 * b10);
      const double y01 = fma(tq[t].a00, b01, tq[t].a01 * b11);
      const double y10 = fma(-tq[t].a01, b00, tq[t].a11 * b10);
      const double y11 = fma(-tq[t].a01, b01, tq[t].a11 * b11);
      // Z = Y Phi_u^T
      const double z00 = fma(y00, tq[u].a00, y01 * tq[u].a01);
      const double z01 = fma(-y00, tq[u].a01, y01 * tq[u].a11);
      const double z11 = fma(-y10, tq[u].a01, y11 * tq[u].a11);
      if (t == u) {
        P[sidx(2 * t, 2 * t, D)] = z00 + tq[t].q00;
        P[sidx(2 * t, 2 * t + 1, D)] = z01 + tq[t].q01;
        P[sidx(2 * t + 1, 2 * t + 1, D)] = z11 + tq[t].q11;
      } else {
        const double z10 = fma(y10, tq[u].a00, y11 * tq[u].a01);
        P[sidx(2 * t, 2 * u, D)] = z00;
        P[sidx(2 * t, 2 * u + 1, D)] = z01;
        P[sidx(2 * t + 1, 2 * u, D)] = z10;
        P[sidx(2 * t + 1, 2 * u + 1, D)] = z11;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// observation of one event.  h = e_{z_slot}/delta at an exposure end,
// h = sum_m e_{x_m} at an instantaneous measurement, none at a start.
// With instruments, a measurement of instrument i reads a_i h.x + c_i plus
// noise of variance R (Sec. 2.2's observation matrix scaled per instrument
// label of Sec. 3.2.3); the filter takes it as the equivalent measurement
// (y - c_i)/a_i of h.x with variance R/a_i^2, whose density differs by the
// constant factor 1/a_i (added to the log-likelihood once per series).
// ---------------------------------------------------------------------------
struct Obs {
  double a[8];  // weight of each integrator in h (a_j = 1/delta for the slot)
  double b;     // weight of every SHO x component (instantaneous)
  double y, R;  // measurement and its noise variance (R = 1 for no measurement)
  bool has;     // a measurement is made at this event
};

// itab: the series' row of the instrument table, or null without instruments
template <class Dm>
GPD Obs make_obs(uint32_t info, double y, double r, double invd, double jit2, const double* itab = nullptr) {
  Obs o;
  const uint32_t kind = ev_kind(info), slot = ev_slot(info);
  const bool end = (kind == EV_END), inst = (kind == EV_INSTANT);
#pragma unroll
  for (int j = 0; j < 8; ++j) o.a[j] = (end && (uint32_t)j == slot) ? invd : 0.0;
  o.b = inst ? 1.0 : 0.0;
  o.has = end || inst;
  double yy = y, rr = r + jit2;
  if (itab) {
    const uint32_t i = ev_inst(info);
    const double ia = itab[ITAB_INVA + i];
    yy = (y - itab[ITAB_OFF + i]) * ia;
    rr = rr * (ia * ia);
  }
  o.y = o.has ? yy : 0.0;
  o.R = o.has ? rr : 1.0;
  return o;
}

// u = P h
template <class Dm>
GPD void obs_gain(const double* P, const Obs& o, double* u) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX, D = Dm::D;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) acc = fma(o.a[j], P[sidx(i, NX + j, D)], acc);
    double xs = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) xs += P[sidx(i, 2 * t, D)];
    u[i] = fma(o.b, xs, acc);
  }
}

// h . vec for a D-vector
template <class Dm>
GPD double obs_dot(const double* vec, const Obs& o) {
  constexpr int M = Dm::M, J = Dm::J, NX = Dm::NX;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) acc = fma(o.a[j], vec[NX + j], acc);
  double xs = 0.0;
#pragma unroll
  for (int t = 0; t < M; ++t) xs += vec[2 * t];
  return fma(o.b, xs, acc);
}

// zero the integrator closed by an exposure end
template <class Dm>
GPD void close_slot(double* m, double* P, uint32_t info) {
  constexpr int J = Dm::J, NX = Dm::NX, D = Dm::D;
  const bool end = ev_kind(info) == EV_END;
  const uint32_t slot = ev_slot(info);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const bool z = end && (uint32_t)j == slot;
    m[NX + j] = z ? 0.0 : m[NX + j];
#pragma unroll
    for (int i = 0; i < D; ++i) P[sidx(i, NX + j, D)] = z ? 0.0 : P[sidx(i, NX + j, D)];
  }
}

}  // namespace gpssm
