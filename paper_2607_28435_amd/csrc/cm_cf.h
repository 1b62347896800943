// Characteristic functions of the log-price (Eq. characteristic_function) and the damped
// transform psi (Eq. psi), evaluated on device in FP64 or FP32.
//
// The integrand is split as psi(v) = h(v) * exp(i v m_f) with the forward log-price
// m_f = ln S0 + (r - q) T. The factor exp(i v m_f) is exponential in the grid index and is
// applied exactly (rank-1 train / reduced phase); h is smooth and non-oscillating:
//   h(v) = exp(-r T + (alpha + 1) m_f + Lc(u)) / ((alpha + i v)(alpha + 1 + i v)),
//   u = v - i (alpha + 1),  Lc(u) = ln phi(u) - i u m_f  (the centred log cf).
#pragma once

#include "cm_internal.h"

template <typename R> struct cx { R x, y; };

template <typename R> struct rm;
template <> struct rm<double> {
  __device__ __forceinline__ static double ex(double a) { return exp(a); }
  __device__ __forceinline__ static double lg(double a) { return log(a); }
  __device__ __forceinline__ static double sq(double a) { return sqrt(a); }
  __device__ __forceinline__ static double hy(double a, double b) { return hypot(a, b); }
  __device__ __forceinline__ static double at2(double a, double b) { return atan2(a, b); }
  __device__ __forceinline__ static void sc(double a, double *s, double *c) { sincos(a, s, c); }
};
template <> struct rm<float> {
  __device__ __forceinline__ static float ex(float a) { return expf(a); }
  __device__ __forceinline__ static float lg(float a) { return logf(a); }
  __device__ __forceinline__ static float sq(float a) { return sqrtf(a); }
  __device__ __forceinline__ static float hy(float a, float b) { return hypotf(a, b); }
  __device__ __forceinline__ static float at2(float a, float b) { return atan2f(a, b); }
  __device__ __forceinline__ static void sc(float a, float *s, float *c) { sincosf(a, s, c); }
};

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { cx<R> z; z.x = a; z.y = b; return z; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return mk(s * a.x, s * a.y); }
template <typename R> __device__ __forceinline__ cx<R> operator/(cx<R> a, cx<R> b) {
  // scaled division (Smith) to avoid overflow in |b|^2
  if (fabs(b.x) >= fabs(b.y)) {
    R rr = b.y / b.x, den = b.x + b.y * rr;
    return mk((a.x + a.y * rr) / den, (a.y - a.x * rr) / den);
  }
  R rr = b.x / b.y, den = b.y + b.x * rr;
  return mk((a.x * rr + a.y) / den, (a.y * rr - a.x) / den);
}
template <typename R> __device__ __forceinline__ cx<R> cexp(cx<R> z) {
  R e = rm<R>::ex(z.x), s, c;
  rm<R>::sc(z.y, &s, &c);
  return mk(e * c, e * s);
}
template <typename R> __device__ __forceinline__ cx<R> clog(cx<R> z) {
  return mk(rm<R>::lg(rm<R>::hy(z.x, z.y)), rm<R>::at2(z.y, z.x));
}
// principal square root
template <typename R> __device__ __forceinline__ cx<R> csqrt(cx<R> z) {
  R r = rm<R>::hy(z.x, z.y);
  if (r == R(0)) return mk(R(0), R(0));
  if (z.x >= R(0)) {
    R t = rm<R>::sq(R(0.5) * (r + z.x));
    return mk(t, z.y / (R(2) * t));
  }
  R t = rm<R>::sq(R(0.5) * (r - z.x));
  return mk(fabs(z.y) / (R(2) * t), copysign(t, z.y));
}

// Model constants prepared once per problem (host or device).
template <typename R> struct CfModel {
  int model;
  R T, alpha;
  R pref;        // -r T + (alpha + 1) m_f  (log prefactor of h)
  R a0, a1, a2, a3, a4;  // model parameters (see cm_problem.p)
  R kJ;          // Merton: E[e^J] - 1
  R omT;         // Variance Gamma: omega T, omega = ln(1 - theta nu - sigma^2 nu / 2) / nu
};

template <typename R>
__device__ __forceinline__ CfModel<R> make_model(const cm_problem &pr) {
  CfModel<R> m;
  m.model = pr.model;
  m.T = (R)pr.T;
  m.alpha = (R)pr.alpha;
  const double mf = log(pr.S0) + (pr.r - pr.q) * pr.T;
  m.pref = (R)(-pr.r * pr.T + (pr.alpha + 1.0) * mf);
  m.a0 = (R)pr.p[0]; m.a1 = (R)pr.p[1]; m.a2 = (R)pr.p[2]; m.a3 = (R)pr.p[3]; m.a4 = (R)pr.p[4];
  m.kJ = (R)(pr.model == CM_MERTON ? exp(pr.p[2] + 0.5 * pr.p[3] * pr.p[3]) - 1.0 : 0.0);
  m.omT = (R)(pr.model == CM_VG
                  ? log(1.0 - pr.p[2] * pr.p[1] - 0.5 * pr.p[0] * pr.p[0] * pr.p[1]) / pr.p[1] * pr.T
                  : 0.0);
  return m;
}

// Lc(u) = ln phi(u) - i u m_f.
template <typename R>
__device__ __forceinline__ cx<R> logcf_centered(const CfModel<R> &m, cx<R> u) {
  const cx<R> iu = mk(-u.y, u.x);
  const cx<R> u2 = u * u;
  if (m.model == CM_BS) {
    const R s2T = m.a0 * m.a0 * m.T;
    return (R(-0.5) * s2T) * (u2 + iu);
  }
  if (m.model == CM_MERTON) {
    const R s2T = m.a0 * m.a0 * m.T;
    const R lam = m.a1, muJ = m.a2, dJ = m.a3;
    cx<R> jump = cexp(mk(-u.y * muJ, u.x * muJ) - (R(0.5) * dJ * dJ) * u2) - mk(R(1), R(0));
    return (R(-0.5) * s2T) * (u2 + iu) - (lam * m.kJ * m.T) * iu + (lam * m.T) * jump;
  }
  if (m.model == CM_VG) {
    // gamma time change: E[e^{G (i u theta - sigma^2 u^2 / 2)}] with G of mean T and
    // variance nu T; the base has a positive real part wherever the damping moment exists,
    // so the principal logarithm is continuous along the integration line
    const R sig = m.a0, nu = m.a1, th = m.a2;
    const cx<R> base = mk(R(1), R(0)) - (th * nu) * iu + (R(0.5) * sig * sig * nu) * u2;
    return m.omT * iu - (m.T / nu) * clog(base);
  }
  // Heston, Albrecher et al. (2007) form
  const R kappa = m.a0, theta = m.a1, sv = m.a2, rho = m.a3, v0 = m.a4;
  const R sv2 = sv * sv;
  const cx<R> b = mk(kappa, R(0)) - (rho * sv) * iu;
  const cx<R> d = csqrt(b * b + sv2 * (iu + u2));
  const cx<R> bm = b - d;
  const cx<R> g = bm / (b + d);
  const cx<R> e = cexp((-m.T) * d);
  const cx<R> one = mk(R(1), R(0));
  const cx<R> ge1 = one - g * e;
  const cx<R> C = (kappa * theta / sv2) * (m.T * bm - R(2) * clog(ge1 / (one - g)));
  const cx<R> D = (R(1) / sv2) * (bm * (one - e) / ge1);
  return C + v0 * D;
}

// h(v) = psi(v) exp(-i v m_f)
template <typename R>
__device__ __forceinline__ cx<R> h_centered(const CfModel<R> &m, R v) {
  const cx<R> u = mk(v, -(m.alpha + R(1)));
  const cx<R> L = logcf_centered(m, u);
  const cx<R> num = cexp(mk(L.x + m.pref, L.y));
  const cx<R> den = mk(m.alpha, v) * mk(m.alpha + R(1), v);
  return num / den;
}

// Time at which E[S_T^omega] explodes under Heston (Andersen & Piterbarg 2007); the damping
// condition of Eq. damping_moment_condition needs T < T*(alpha + 1).
__host__ __device__ inline double heston_explosion_time(double kappa, double sv, double rho, double om) {
  const double k = rho * sv * om - kappa;
  const double D = k * k - sv * sv * om * (om - 1.0);
  if (D >= 0.0) {
    if (k < 0.0) return INFINITY;
    const double sD = sqrt(D);
    return (k > sD) ? log((k + sD) / (k - sD)) / sD : INFINITY;
  }
  const double sD = sqrt(-D);
  return 2.0 / sD * ((k < 0.0 ? M_PI : 0.0) + atan(sD / k));
}

// Per-instance validation shared by every entry point. Returns a cm_status.
__host__ __device__ inline int check_problem(const cm_problem &pr) {
  if (pr.n < 1 || pr.n > CM_MAX_N) return CM_E_INVALID;
  if (pr.model < CM_BS || pr.model > CM_VG) return CM_E_INVALID;
  if (pr.quad != CM_QUAD_RECT2 && pr.quad != CM_QUAD_SIMPSON1) return CM_E_INVALID;
  if (!(pr.S0 > 0.0) || !(pr.T > 0.0) || !(pr.eta > 0.0)) return CM_E_INVALID;
  if (!(pr.alpha == pr.alpha) || pr.alpha == 0.0 || pr.alpha == -1.0) return CM_E_INVALID;
  if (pr.model == CM_BS && !(pr.p[0] > 0.0)) return CM_E_INVALID;
  if (pr.model == CM_MERTON && (!(pr.p[0] > 0.0) || pr.p[1] < 0.0 || pr.p[3] < 0.0)) return CM_E_INVALID;
  if (pr.model == CM_HESTON) {
    if (!(pr.p[0] > 0.0) || !(pr.p[1] > 0.0) || !(pr.p[2] > 0.0) || !(pr.p[3] >= -1.0 && pr.p[3] <= 1.0) ||
        !(pr.p[4] >= 0.0))
      return CM_E_INVALID;
    if (pr.T >= heston_explosion_time(pr.p[0], pr.p[2], pr.p[3], pr.alpha + 1.0)) return CM_E_MOMENT;
  }
  if (pr.model == CM_VG) {
    const double sig = pr.p[0], nu = pr.p[1], th = pr.p[2];
    if (!(sig > 0.0) || !(nu > 0.0) || !(th == th) || !(1.0 - th * nu - 0.5 * sig * sig * nu > 0.0))
      return CM_E_INVALID;
    // E[S_T^w] is finite iff the gamma moment generating function exists at the exponent
    const double w = pr.alpha + 1.0;
    if (!(1.0 - w * th * nu - 0.5 * sig * sig * nu * w * w > 0.0)) return CM_E_MOMENT;
  }
  return CM_OK;
}

// Default-aware lowest log-strike: NaN selects ln(S0) - pi/eta.
__host__ __device__ inline bool k0_is_default(const cm_problem &pr) { return !(pr.k0 == pr.k0); }
__host__ __device__ inline double k0_of(const cm_problem &pr) {
  return k0_is_default(pr) ? log(pr.S0) - M_PI / pr.eta : pr.k0;
}
