// cm_fft_price: dense Carr–Madan baseline (Section 2.1, Eqs. x, dft, discretization_dft).
//
// Mixed-radix Stockham FFT (decimation in time, autosorting). Pass p with radix R_p and
// stride p_len = R_1 ... R_{p-1} maps work item i in [0, M/R_p), k = i mod p_len, as
//   u[r] = x[i + r M/R_p] * exp(-2 pi i r k / (R_p p_len)),  u <- DFT_{R_p}(u),
//   y[(i - k) R_p + k + r p_len] = u[r].
// Inside a workgroup each R_p-point DFT is itself a Stockham FFT in LDS with register radix
// 16 for CM_C64 and 8 for CM_C128 (smaller radices for the remaining bits): a thread reads its butterflies' points into registers,
// the workgroup synchronises, and the thread writes the transformed points back, so one
// LDS buffer suffices. LDS indices carry one pad slot per 32 against bank conflicts.
//   - Pass 1 (p_len = 1, one work item per 1024-thread workgroup, radix 2^14 for CM_C64 and
//     2^13 for CM_C128) generates x on the fly, so it reads nothing from HBM. x is set to
//     exactly zero where |psi| has decayed below a per-problem cutoff far under the storage
//     precision (found once per problem by k_fft_support), which skips the characteristic
//     function outside the integrand's numerical support.
//   - Later passes handle 16 consecutive work items per workgroup, so every global load
//     and store moves 16 consecutive elements.
//   - The last pass multiplies by the readout scalars and stores prices; in FP64 each price
//     takes its log-strike from the error-free grid sum (1e-15 NRMSE on the paper grid up
//     to n = 30).
// Characteristic functions run in the storage precision (FP32 for CM_C64); every phase that
// grows with j or u is reduced exactly in FP64 first.
#include <array>
#include <utility>
#include <type_traits>

#include "cm_cf.h"
#include "cm_tt.h"

namespace {

constexpr int NT = 1024;       // threads per FFT workgroup
constexpr int LOG_COLS = 4;
constexpr int FFT_COLS = 1 << LOG_COLS;   // work items per workgroup after the first pass
constexpr size_t DENSE_PROB_BYTES = 512;  // workspace slot per problem
constexpr int MAX_CHUNK = 32768;

template <typename T> struct fr;
template <> struct fr<float2> {
  using R = float;
  __device__ __forceinline__ static float2 mk(double a, double b) { return make_float2((float)a, (float)b); }
  __device__ __forceinline__ static float2 mul(float2 a, float2 b) { return fmulc(a, b); }
  __device__ __forceinline__ static float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
  __device__ __forceinline__ static float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
  // exp(-2 pi i f), f a turn fraction
  __device__ __forceinline__ static float2 cis_neg(double f) {
    float s, c;
    sincospif((float)(-2.0 * f), &s, &c);
    return make_float2(c, s);
  }
  // e^{-alpha k} / (s pi) for the readout: FP64 exponent split, FP32 mantissa
  __device__ __forceinline__ static double escale(double z) {   // 2^z
    const double zi = floor(z);
    return ldexp((double)exp2f((float)(z - zi)), (int)zi);
  }
};
template <> struct fr<double2> {
  using R = double;
  __device__ __forceinline__ static double2 mk(double a, double b) { return cmk(a, b); }
  __device__ __forceinline__ static double2 mul(double2 a, double2 b) { return cmul(a, b); }
  __device__ __forceinline__ static double2 add(double2 a, double2 b) { return cadd(a, b); }
  __device__ __forceinline__ static double2 sub(double2 a, double2 b) { return csub(a, b); }
  __device__ __forceinline__ static double2 cis_neg(double f) {
    double s, c;
    sincospi(-2.0 * f, &s, &c);
    return cmk(c, s);
  }
  __device__ __forceinline__ static double escale(double z) { return exp2(z); }
};

// cos(2 pi m / 16) for any integer m
__host__ __device__ constexpr double cos16(int m) {
  m &= 15;
  if (m > 8) m = 16 - m;
  return m == 0 ? 1.0 : m == 1 ? 0.92387953251128676 : m == 2 ? 0.70710678118654752 : m == 3 ? 0.38268343236508977
       : m == 4 ? 0.0 : m == 5 ? -0.38268343236508977 : m == 6 ? -0.70710678118654752 : m == 7 ? -0.92387953251128676
       : -1.0;
}

struct FftPlan {
  int n, npass;
  int logr[4];     // radix bits per pass
  int chunk;       // instances per launch group
};

__host__ inline int first_radix_bits(int dtype) { return dtype == CM_C64 ? 14 : 13; }
__host__ inline int later_radix_bits(int dtype) { return dtype == CM_C64 ? 10 : 9; }

__host__ inline FftPlan make_plan(int n, int dtype, int batch) {
  FftPlan p;
  p.n = n;
  int rem = n, np = 0;
  const int f = first_radix_bits(dtype), g = later_radix_bits(dtype);
  int b0 = rem < f ? rem : f;
  p.logr[np++] = b0;
  rem -= b0;
  while (rem > 0) {
    int b = rem < g ? rem : g;
    p.logr[np++] = b;
    rem -= b;
  }
  p.npass = np;
  int ch = 1;
  if (n < 22) ch = 1 << (22 - n);
  if (ch > MAX_CHUNK) ch = MAX_CHUNK;
  p.chunk = batch < ch ? batch : ch;
  if (p.chunk < 1) p.chunk = 1;
  return p;
}

__host__ inline size_t al256f(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ inline size_t fft_ws_bytes(const FftPlan &p, int dtype, bool gather, int batch) {
  const size_t es = dtype == CM_C64 ? 8 : 16;
  const size_t M = (size_t)1 << p.n;
  size_t o = al256f(DENSE_PROB_BYTES * (size_t)batch);   // per-problem constants
  o += al256f(es * M * p.chunk);                       // buffer A
  if (p.npass >= 3) o += al256f(es * M * p.chunk);     // buffer B
  if (gather) o += al256f(es / 2 * M * p.chunk);       // full prices before gathering
  return o;
}

// one pad slot per 16 elements: stride-16 accesses of 8- and 16-byte elements spread over
// all banks
__host__ __device__ inline int pidx(int x) { return x + (x >> 4); }
__host__ __device__ inline int col_stride(int logL) { return pidx(1 << logL) + 1; }
__host__ inline size_t lds_bytes(int logL, int ncol, size_t es) { return es * (size_t)col_stride(logL) * ncol; }

// u <- w u for the constant twiddle w = exp(-2 pi i m / 16)
template <typename T, int m>
__device__ __forceinline__ T tw16(T u) {
  if constexpr (m == 0) return u;
  else if constexpr (m == 4) return fr<T>::mk(u.y, -u.x);    // -i u
  else {
    using R = typename fr<T>::R;
    const R c = (R)cos16(m), s = (R)cos16((m + 12) & 15);   // sin(2 pi m/16) = cos(2 pi (m-4)/16)
    // (c - i s)(x + i y) = (c x + s y) + i (c y - s x)
    T r;
    r.x = c * u.x + s * u.y;
    r.y = c * u.y - s * u.x;
    return r;
  }
}

template <typename T, int R, int S, int G, int Q>
__device__ __forceinline__ void bfly(T *u) {
  constexpr int m = Q * (8 / S);
  const T t = tw16<T, m>(u[G + Q + S]);
  u[G + Q + S] = fr<T>::sub(u[G + Q], t);
  u[G + Q] = fr<T>::add(u[G + Q], t);
}

template <typename T, int R, int S, int G, int Q>
__device__ __forceinline__ void bfly_q(T *u) {
  if constexpr (Q < S) {
    bfly<T, R, S, G, Q>(u);
    bfly_q<T, R, S, G, Q + 1>(u);
  }
}
template <typename T, int R, int S, int G>
__device__ __forceinline__ void bfly_g(T *u) {
  if constexpr (G < R) {
    bfly_q<T, R, S, G, 0>(u);
    bfly_g<T, R, S, G + 2 * S>(u);
  }
}
template <typename T, int R, int S>
__device__ __forceinline__ void bfly_s(T *u) {
  if constexpr (S < R) {
    bfly_g<T, R, S, 0>(u);
    bfly_s<T, R, 2 * S>(u);
  }
}

__host__ __device__ constexpr int brev_c(int i, int R) {
  int rb = 0;
  for (int b = 1; b < R; b <<= 1, i >>= 1) rb = (rb << 1) | (i & 1);
  return rb;
}

// In-register DFT of R points with the minus sign, R in {2, 4, 8, 16}.
template <typename T, int R>
__device__ __forceinline__ void dft_reg(T *v) {
  T u[R];
#pragma unroll
  for (int i = 0; i < R; ++i) u[brev_c(i, R)] = v[i];
  bfly_s<T, R, 1>(u);
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = u[i];
}

template <typename T> struct price_t;
template <> struct price_t<float2> { using type = float; };
template <> struct price_t<double2> { using type = double; };

// One Stockham stage of radix R over 2^logc columns of L = 2^logL points, current
// sub-transform length Ls. Butterfly g -> column col = g mod 2^logc (fastest, so that global
// loads and stores of neighbouring lanes touch neighbouring work items), i = g / 2^logc,
// k = i mod Ls: reads element i + r L/R, twiddles by exp(-2 pi i r k / (Ls R)), transforms,
// writes element (i - k) R + k + r Ls. Elements come from LDS (column stride Lp, padded
// indices) or, in the first stage, from src(col, i, L/R, v); they go to LDS or, in the last
// stage, to dst(col, (i - k) R + k, Ls, v). Needs L 2^logc <= pts_per_thread<T> NT.
template <typename T> constexpr int pts_per_thread = sizeof(T) == 8 ? 16 : 8;

template <typename T, int R, bool FROM_LDS, bool TO_LDS, class Src, class Dst>
__device__ __forceinline__ void fft_stage(T *a, int logL, int logc, int Lp, int Ls, const Src &src, const Dst &dst) {
  constexpr int PT = pts_per_thread<T>;
  constexpr int NB = PT / R;  // butterflies per thread (at most)
  constexpr int LOGR = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
  const int logLR = logL - LOGR;
  const int nbut = 1 << (logLR + logc);
  const int cmask = (1 << logc) - 1;
  T v[PT];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int g = threadIdx.x + t * NT;
    if (g < nbut) {
      const int col = g & cmask, i = g >> logc;
      if constexpr (FROM_LDS) {
        const T *c = a + col * Lp;
#pragma unroll
        for (int r = 0; r < R; ++r) v[t * R + r] = c[pidx(i + (r << logLR))];
      } else {
        src.template load<R>(col, i, 1 << logLR, v + t * R);
      }
    }
  }
  if constexpr (FROM_LDS && TO_LDS) __syncthreads();
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int g = threadIdx.x + t * NT;
    if (g < nbut) {
      const int col = g & cmask, i = g >> logc;
      const int k = i & (Ls - 1);
      if (k) {
        const T w = fr<T>::cis_neg(ldexp((double)k, -LOGR) / (double)Ls);
        T wr = w;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[t * R + r] = fr<T>::mul(v[t * R + r], wr);
          if (r + 1 < R) wr = fr<T>::mul(wr, w);
        }
      }
      dft_reg<T, R>(v + t * R);
      const int base = (i - k) * R + k;
      if constexpr (TO_LDS) {
        T *c = a + col * Lp;
#pragma unroll
        for (int r = 0; r < R; ++r) c[pidx(base + r * Ls)] = v[t * R + r];
      } else {
        dst.template store<R>(col, base, Ls, v + t * R);
      }
    }
  }
  if constexpr (TO_LDS) __syncthreads();
}

// DFT of 2^logc columns of 2^LOGL points, inputs from src (or from LDS if GEN_LDS: the
// caller has already written them there), outputs to dst, LDS in between. Register radix
// 16 for CM_C64 and 8 for CM_C128; the remaining bits go last. The stage sequence is fixed
// at compile time.
template <typename T, int LOGL, int LOGLS, bool GEN_LDS, class Src, class Dst>
__device__ __forceinline__ void fft_block(T *a, int logc, int Lp, const Src &src, const Dst &dst) {
  constexpr int RB = pts_per_thread<T> >= 16 ? 4 : 3;
  constexpr int rem = LOGL - LOGLS;
  if constexpr (rem > 0) {
    constexpr int b = rem >= RB ? RB : rem;
    constexpr bool first = LOGLS == 0, last = b == rem;
    fft_stage<T, (1 << b), (!first || GEN_LDS), !last>(a, LOGL, logc, Lp, 1 << LOGLS, src, dst);
    fft_block<T, LOGL, LOGLS + b, GEN_LDS>(a, logc, Lp, src, dst);
  }
}

}  // namespace

// Per-problem constants of the integrand and readout.
struct DenseConst {
  double eta, v0;
  int64_t jmid;            // index of v = 0: 2^(n-1) for the symmetric rule, else 0
  double th_hi, th_lo;     // theta / (2 pi) as double-double, theta = eta (m_f - k0)
  double2 g0;              // exp(i v0 m_f)
  double k0, nalog2e, lsf; // log2 of the readout scale e^{-alpha k_u} / (s pi) is nalog2e k_u + lsf
  double dz, zorg;         // its step per unit of u and its value at u = us (single-precision outputs)
  int64_t us;              // k_u = k0 + lambda (u - us): the default grid is centred on ln S0
  int n;
  double2 ro;              // exp(-i v0 k0)
  int simpson;
  int alt;                 // readout alternates sign with u (symmetric rule)
};

// Everything a dense FFT workgroup needs about its problem, computed once per problem.
template <typename T> struct DenseProb {
  DenseConst c;
  CfModel<typename fr<T>::R> m;
  int64_t jlo, jhi;        // x_j may be non-zero only for jlo <= j < jhi
  int32_t bad;             // the problem failed its checks: prices are NaN
};
static_assert(sizeof(DenseProb<double2>) <= DENSE_PROB_BYTES, "DenseProb too large");
static_assert(sizeof(DenseProb<float2>) <= DENSE_PROB_BYTES, "DenseProb too large");

__device__ inline DenseConst dense_const(const cm_problem &pr) {
  DenseConst c;
  const int n = pr.n;
  c.eta = pr.eta;
  c.simpson = pr.quad == CM_QUAD_SIMPSON1;
  c.v0 = c.simpson ? 0.0 : -ldexp(pr.eta, n - 1);
  c.jmid = c.simpson ? 0 : ((int64_t)1 << (n - 1));
  const double rq = (pr.r - pr.q) * pr.T;
  double p, e;
  if (k0_is_default(pr)) {
    two_prod(pr.eta, rq, p, e);
    // theta/(2 pi) = eta rq / (2 pi) + 1/2
    double ch = p * CM_INV2PI_HI;
    double cl = fma(p, CM_INV2PI_HI, -ch) + p * CM_INV2PI_LO + e * CM_INV2PI_HI;
    // (ch + 0.5) may round; keep its rounding error in th_lo
    double s, err;
    two_sum(ch, 0.5, s, err);
    c.th_hi = s; c.th_lo = cl + err;
  } else {
    drift_angle(pr.eta, log(pr.S0), pr.k0, rq, p, e);
    c.th_hi = p * CM_INV2PI_HI;
    c.th_lo = fma(p, CM_INV2PI_HI, -c.th_hi) + p * CM_INV2PI_LO + e * CM_INV2PI_HI;
  }
  if (c.simpson) c.g0 = cmk(1.0, 0.0);
  else {
    double f = prod_cycles_frac(c.v0, log(pr.S0), 0) + prod_cycles_frac(c.v0, rq, 0);
    c.g0 = turn(f - floor(f));
  }
  // the default k0 = ln S0 - pi/eta is ln S0 - lambda M/2 exactly: strikes from ln S0 and an
  // exact integer offset
  const double k0 = k0_is_default(pr) ? log(pr.S0) : pr.k0;
  c.us = k0_is_default(pr) ? ((int64_t)1 << (n - 1)) : 0;
  const double sfac = c.simpson ? 1.0 / M_PI : 0.5 / M_PI;
  c.k0 = k0;
  c.n = n;
  c.nalog2e = -pr.alpha * M_LOG2E;
  c.dz = c.nalog2e * (2.0 * M_PI / (ldexp(1.0, n) * pr.eta));
  c.lsf = log2(sfac);
  c.zorg = fma(c.nalog2e, k0, c.lsf);
  c.alt = !c.simpson;
  if (c.simpson) c.ro = cmk(1.0, 0.0);
  else {
    // -v0 k0 = eta 2^(n-1) k0; with the default k0 = ln S0 - pi/eta the pi part is a whole
    // number of turns for n >= 2
    double f;
    if (k0_is_default(pr)) {
      f = prod_cycles_frac(pr.eta, log(pr.S0), n - 1);
      if (n == 1) { f += 0.5; f -= floor(f); }
    } else {
      f = prod_cycles_frac(pr.eta, pr.k0, n - 1);
    }
    c.ro = turn(f);
  }
  return c;
}

// x_j for the dense path, in storage precision (zero outside the support)
template <typename T>
__device__ __forceinline__ T integrand_at(const DenseProb<T> &d, int64_t j) {
  using R = typename fr<T>::R;
  if (j < d.jlo || j >= d.jhi) return fr<T>::mk(0.0, 0.0);
  const DenseConst &c = d.c;
  // v_j = v0 + j eta formed from the exact offset j - jmid: adding v0 to j eta would cancel
  // to an absolute error of |v0| ulp near v = 0 on large symmetric grids
  const double v = (double)(j - c.jmid) * c.eta;
  const cx<R> h = h_centered<R>(d.m, (R)v);
  // exp(i j theta): fraction of j * (th_hi + th_lo)
  double p, e;
  two_prod((double)j, c.th_hi, p, e);
  double f = frac2(p, e + (double)j * c.th_lo);
  double w;
  if (c.simpson) w = c.eta / 3.0 * ((j & 1) ? 4.0 : (j == 0 ? 1.0 : 2.0));
  else w = c.eta;
  const T ph = fr<T>::cis_neg(-f);   // exp(+2 pi i f)
  T hv = fr<T>::mk((double)h.x, (double)h.y);
  T g = fr<T>::mk(c.g0.x * w, c.g0.y * w);
  return fr<T>::mul(fr<T>::mul(hv, ph), g);
}

// C(k_u) = Re[e^{-alpha k_u}/(s pi) ro (+-1)^u y_u]; the scale is 2^z with the
// exponent kept in FP64.
// z, the log2 of the scale, is passed in: the last pass forms it from the accurate log-strike
// (strike_log), for every output in FP64 and for the first of each R in FP32.
__device__ __forceinline__ float price_at(const DenseConst &c, int64_t u, double z, float2 y, bool bad) {
  if (bad) return NAN;
  const double zi = floor(z);
  float rx = (float)c.ro.x, ry = (float)c.ro.y;
  if (c.alt && (u & 1)) { rx = -rx; ry = -ry; }
  const float re = rx * y.x - ry * y.y;
  return ldexpf(re * exp2f((float)(z - zi)), (int)zi);
}
__device__ __forceinline__ double price_at(const DenseConst &c, int64_t u, double z, double2 y, bool bad) {
  if (bad) return NAN;
  double2 ro = c.ro;
  if (c.alt && (u & 1)) ro = cmk(-ro.x, -ro.y);
  return exp2(z) * (ro.x * y.x - ro.y * y.y);
}

// Sources and sinks of a pass. Work item of column col is item0 + col; a pass with radix R
// and stride plen reads x[item + e M/R] (element e of the item's DFT) and writes
// y[(item - k) R + k + q plen] (output q), k = item mod plen.
struct NoSrc {
  template <int R, typename T> __device__ __forceinline__ void load(int, int, int, T *) const {}
};

template <typename T> struct BufSrc {     // later passes: read the previous pass, apply its twiddle
  const T *src;
  int64_t item0, T_items, plen;
  int twl_bits;                          // log2(R plen)
  template <int R> __device__ __forceinline__ void load(int col, int e0, int de, T *v) const {
    const int64_t item = item0 + col;
    const int64_t k = item & (plen - 1);
    const int64_t mask = ((int64_t)1 << twl_bits) - 1;
    T w = fr<T>::cis_neg(ldexp((double)(((int64_t)e0 * k) & mask), -twl_bits));
    const T ws = fr<T>::cis_neg(ldexp((double)(((int64_t)de * k) & mask), -twl_bits));
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = fr<T>::mul(src[item + (int64_t)(e0 + r * de) * T_items], w);
      if (r + 1 < R) w = fr<T>::mul(w, ws);
    }
  }
};

template <typename T> struct BufDst {     // intermediate passes
  T *dst;
  int64_t item0, plen;
  int logR;
  template <int R> __device__ __forceinline__ void store(int col, int q0, int dq, const T *v) const {
    const int64_t item = item0 + col;
    const int64_t k = item & (plen - 1);
    T *o = dst + ((item - k) << logR) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) o[(int64_t)(q0 + r * dq) * plen] = v[r];
  }
};

template <typename T> struct PriceDst {   // last pass: readout scalars, prices
  typename price_t<T>::type *prices;
  const DenseConst *c;
  int64_t item0, plen;
  int logR, bad;
  template <int R> __device__ __forceinline__ void store(int col, int q0, int dq, const T *v) const {
    const int64_t item = item0 + col;
    const int64_t k = item & (plen - 1);
    const int64_t b = ((item - k) << logR) + k;
    const int64_t u0 = b + (int64_t)q0 * plen, du = (int64_t)dq * plen;
    if constexpr (std::is_same<T, double2>::value) {
      // every output from its accurate log-strike: the outputs of one call lie up to M apart,
      // where steps of a rounded lambda would be off by the whole strike range times ulp(1)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t u = u0 + r * du;
        const double z = fma(c->nalog2e, strike_log(c->k0, c->eta, c->n, (double)(u - c->us)), c->lsf);
        prices[u] = price_at(*c, u, z, v[r], bad != 0);
      }
    } else {
      // single-precision prices: the scale's exponent as z_org + dz (u - us) in FP64, one FMA per
      // call and steps for its outputs (the FP64 error of a rounded lambda, at most the strike
      // range times ulp(1), stays far below the FP32 rounding of the price)
      const double z0 = fma(c->dz, (double)(u0 - c->us), c->zorg);
      const double dz = c->dz * (double)du;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t u = u0 + r * du;
        prices[u] = price_at(*c, u, fma((double)r, dz, z0), v[r], bad != 0);
      }
    }
  }
};

// Per problem: constants, and the numerical support of x. One wavefront per problem
// evaluates |h| at v = +-2^{q/4 - 4}, q < 256, finds the first q from which five consecutive
// points lie below thr |h(0)|, and keeps indices with |v| < 2 v_q. A problem that fails
// its checks keeps the whole range and is marked bad.
template <typename T>
__global__ __launch_bounds__(64) void k_fft_prepare(const cm_problem *__restrict__ prob, int batch, int n, double thr,
                                                    DenseProb<T> *__restrict__ out, int32_t *__restrict__ status) {
  const int b = blockIdx.x;
  if (b >= batch) return;
  const cm_problem pr = prob[b];
  int code = check_problem(pr);
  if (code == CM_OK && pr.n != n) code = CM_E_INVALID;
  const int64_t M = (int64_t)1 << n;
  int64_t jlo = 0, jhi = M;
  if (code == CM_OK) {
    const CfModel<double> m = make_model<double>(pr);
    const cx<double> h0 = h_centered<double>(m, 0.0);
    const double lim = thr * sqrt(h0.x * h0.x + h0.y * h0.y);
    uint64_t below[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int q = w * 64 + (int)threadIdx.x;
      const double v = exp2(0.25 * q - 4.0);
      const cx<double> hp = h_centered<double>(m, v), hm = h_centered<double>(m, -v);
      const double a = fmax(sqrt(hp.x * hp.x + hp.y * hp.y), sqrt(hm.x * hm.x + hm.y * hm.y));
      below[w] = __ballot(a < lim);
    }
    int qcut = -1;
    for (int q = 0; q + 4 < 256 && qcut < 0; ++q) {
      bool all = true;
      for (int t = 0; t < 5; ++t) all = all && ((below[(q + t) >> 6] >> ((q + t) & 63)) & 1);
      if (all) qcut = q;
    }
    if (qcut >= 0) {
      const double half = 2.0 * exp2(0.25 * qcut - 4.0) / pr.eta;
      if (pr.quad == CM_QUAD_SIMPSON1) {
        jhi = (int64_t)fmin((double)M, ceil(half) + 1.0);
      } else {
        const double c0 = (double)(M / 2);
        jlo = (int64_t)fmax(0.0, floor(c0 - half) - 1.0);
        jhi = (int64_t)fmin((double)M, ceil(c0 + half) + 1.0);
      }
    }
  }
  if (threadIdx.x == 0) {
    DenseProb<T> d;
    d.c = dense_const(pr);
    d.m = make_model<typename fr<T>::R>(pr);
    d.jlo = jlo;
    d.jhi = jhi;
    d.bad = code != CM_OK;
    out[b] = d;
    if (status) status[b] = code;
  }
}

// Pass 1, from stage S + 1 on. With the support of x starting at 0, the work item's inputs
// e >= E are zero. If E <= L / R^S (R the register radix), each of the first S stages sees at
// most one non-zero input per butterfly, its first, which no twiddle touches; the radix-R
// DFT of such a vector is that input repeated. So after S stages the array is
// y[m] = x_e with e = m >> (S log2 R) for m < R^S E, and zero beyond. It is written directly
// (one evaluation of x per e) and the transform continues with the remaining stages.
template <typename T, int LOGR, int S, class Dst>
__device__ __forceinline__ void first_pass_from(T *a, const DenseProb<T> &d, int64_t item, int64_t T_items, int64_t E,
                                                const Dst &dst) {
  constexpr int RB = pts_per_thread<T> >= 16 ? 4 : 3;
  constexpr int SB = S * RB;
  if constexpr (S == 0) {
    for (int e = threadIdx.x; e < (1 << LOGR); e += NT) a[pidx(e)] = integrand_at<T>(d, item + (int64_t)e * T_items);
  } else {
    const T zero = fr<T>::mk(0.0, 0.0);
    for (int e = threadIdx.x; e < E; e += NT) a[pidx(e << SB)] = integrand_at<T>(d, item + (int64_t)e * T_items);
    __syncthreads();
    for (int m = threadIdx.x; m < (1 << LOGR); m += NT) {
      const int e = m >> SB;
      if (e >= E) a[pidx(m)] = zero;
      else if (m & ((1 << SB) - 1)) a[pidx(m)] = a[pidx(e << SB)];
    }
  }
  __syncthreads();
  fft_block<T, LOGR, SB, true>(a, 0, 0, NoSrc{}, dst);
}

template <typename T, int LOGR, class Dst>
__device__ __forceinline__ void first_pass(T *a, const DenseProb<T> &d, int64_t item, int64_t T_items, const Dst &dst) {
  constexpr int RB = pts_per_thread<T> >= 16 ? 4 : 3;
  constexpr int MAXS = (LOGR - 1) / RB;   // keep at least one stage
  int S = 0;
  int64_t E = 0;
  if (d.jlo == 0) {
    E = (d.jhi + T_items - 1) / T_items;
    while (S < MAXS && E <= ((int64_t)1 << (LOGR - (S + 1) * RB))) ++S;
  }
  if constexpr (MAXS >= 3) {
    if (S == 3) { first_pass_from<T, LOGR, 3>(a, d, item, T_items, E, dst); return; }
  }
  if constexpr (MAXS >= 2) {
    if (S == 2) { first_pass_from<T, LOGR, 2>(a, d, item, T_items, E, dst); return; }
  }
  if constexpr (MAXS >= 1) {
    if (S == 1) { first_pass_from<T, LOGR, 1>(a, d, item, T_items, E, dst); return; }
  }
  first_pass_from<T, LOGR, 0>(a, d, item, T_items, E, dst);
}

// Pass 1: one work item (blockIdx.x) per workgroup; x is generated into LDS (only lanes
// inside the support evaluate the characteristic function), then transformed.
template <typename T, int LOGR>
__global__ __launch_bounds__(NT) void k_fft_first(const DenseProb<T> *__restrict__ dprob, int inst0, int n,
                                                  T *__restrict__ out, typename price_t<T>::type *__restrict__ prices,
                                                  int single) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *a = (T *)lds_raw;
  const int64_t M = (int64_t)1 << n;
  const DenseProb<T> *d = dprob + inst0 + blockIdx.y;
  const int64_t item = blockIdx.x, T_items = M >> LOGR;
  if (single) {
    PriceDst<T> dst{prices + (int64_t)blockIdx.y * M, &d->c, item, 1, LOGR, d->bad};
    first_pass<T, LOGR>(a, *d, item, T_items, dst);
  } else {
    BufDst<T> dst{out + (int64_t)blockIdx.y * M, item, 1, LOGR};
    first_pass<T, LOGR>(a, *d, item, T_items, dst);
  }
}

// Later passes: FFT_COLS consecutive work items per workgroup, loaded straight into the
// first stage's registers.
template <typename T, int LOGR>
__global__ __launch_bounds__(NT) void k_fft_next(const DenseProb<T> *__restrict__ dprob, int inst0, int n,
                                                 int64_t plen, const T *__restrict__ in, T *__restrict__ out,
                                                 typename price_t<T>::type *__restrict__ prices, int last) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *a = (T *)lds_raw;
  const int64_t M = (int64_t)1 << n;
  const int64_t item0 = (int64_t)blockIdx.x * FFT_COLS;
  const int twl_bits = LOGR + (int)__builtin_ctzll(plen);
  BufSrc<T> src{in + (int64_t)blockIdx.y * M, item0, M >> LOGR, plen, twl_bits};
  const int Lp = col_stride(LOGR);
  if (last) {
    const DenseProb<T> *d = dprob + inst0 + blockIdx.y;
    PriceDst<T> dst{prices + (int64_t)blockIdx.y * M, &d->c, item0, plen, LOGR, d->bad};
    fft_block<T, LOGR, 0, false>(a, LOG_COLS, Lp, src, dst);
  } else {
    BufDst<T> dst{out + (int64_t)blockIdx.y * M, item0, plen, LOGR};
    fft_block<T, LOGR, 0, false>(a, LOG_COLS, Lp, src, dst);
  }
}

// Host-side tables of the instantiations, indexed by radix bits.
template <typename T, int... B>
static constexpr std::array<decltype(&k_fft_first<T, 1>), sizeof...(B)> first_table(std::integer_sequence<int, B...>) {
  return {&k_fft_first<T, B + 1>...};
}
template <typename T, int... B>
static constexpr std::array<decltype(&k_fft_next<T, 1>), sizeof...(B)> next_table(std::integer_sequence<int, B...>) {
  return {&k_fft_next<T, B + 1>...};
}

template <typename P>
__global__ void k_gather(const P *__restrict__ full, int64_t M, const int64_t *__restrict__ idx, int nk, int inst0,
                         int cnt, P *__restrict__ out, int32_t *__restrict__ status) {
  const int64_t total = (int64_t)cnt * nk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / nk), s = (int)(e % nk);
    const int64_t u = idx[(int64_t)(inst0 + b) * nk + s];
    P v;
    if (u < 0 || u >= M) {
      v = (P)NAN;
      set_status(status, inst0 + b, CM_E_INVALID);
    } else v = full[(int64_t)b * M + u];
    out[(int64_t)(inst0 + b) * nk + s] = v;
  }
}

extern "C" size_t cm_fft_ws_bytes(int batch, int n, int dtype, int gather) {
  if (n < 1 || n > 30 || batch < 1) return 0;
  FftPlan p = make_plan(n, dtype, batch);
  return fft_ws_bytes(p, dtype, gather != 0, batch);
}

// The plan for a workspace of ws_bytes: the default launch group, widened to the largest
// instance count (at most the batch and MAX_CHUNK) whose pass buffers still fit.
__host__ inline FftPlan plan_for_ws(int n, int dtype, int batch, bool gather, size_t ws_bytes) {
  FftPlan p = make_plan(n, dtype, batch);
  while (p.chunk < batch && p.chunk < MAX_CHUNK) {
    FftPlan q = p;
    q.chunk = p.chunk + 1;
    if (fft_ws_bytes(q, dtype, gather, batch) > ws_bytes) break;
    p = q;
  }
  return p;
}

template <typename T>
static cm_status fft_run(const cm_problem *prob, int batch, int n, const int64_t *strike_idx, int nk, void *prices,
                         int32_t *status, void *ws, size_t ws_bytes, hipStream_t s) {
  using P = typename price_t<T>::type;
  const int dtype = sizeof(T) == 8 ? CM_C64 : CM_C128;
  const bool gather = strike_idx != nullptr;
  FftPlan p = plan_for_ws(n, dtype, batch, gather, ws_bytes);
  const int64_t M = (int64_t)1 << n;
  char *w = (char *)ws;
  DenseProb<T> *dp = (DenseProb<T> *)w;
  w += al256f(DENSE_PROB_BYTES * (size_t)batch);
  T *bufA = (T *)w;
  w += al256f(sizeof(T) * M * p.chunk);
  T *bufB = bufA;
  if (p.npass >= 3) { bufB = (T *)w; w += al256f(sizeof(T) * M * p.chunk); }
  P *full = gather ? (P *)w : nullptr;
  // cut-off of |psi| relative to |psi(0)|, far below the storage precision
  const double thr = dtype == CM_C64 ? 1e-16 : 1e-32;
  hipLaunchKernelGGL(k_fft_prepare<T>, dim3(batch), dim3(64), 0, s, prob, batch, n, thr, dp, status);
  CM_LAUNCH_CHECK();
  constexpr int FB = sizeof(T) == 8 ? 14 : 13, NB = sizeof(T) == 8 ? 10 : 9;
  static constexpr auto kfirst = first_table<T>(std::make_integer_sequence<int, FB>{});
  static constexpr auto knext = next_table<T>(std::make_integer_sequence<int, NB>{});
  const int lr0 = p.logr[0];
  if (lr0 < 1 || lr0 > FB) return CM_E_UNSUPPORTED;
  for (int ps = 1; ps < p.npass; ++ps)
    if (p.logr[ps] < 1 || p.logr[ps] > NB) return CM_E_UNSUPPORTED;
  const size_t lds0 = lds_bytes(lr0, 1, sizeof(T));
  CM_HIP_CHECK(cm_allow_lds(kfirst[lr0 - 1], lds0));
  for (int ps = 1; ps < p.npass; ++ps)
    CM_HIP_CHECK(cm_allow_lds(knext[p.logr[ps] - 1], lds_bytes(p.logr[ps], FFT_COLS, sizeof(T))));
  for (int inst0 = 0; inst0 < batch; inst0 += p.chunk) {
    const int cnt = (batch - inst0) < p.chunk ? (batch - inst0) : p.chunk;
    P *dstp = gather ? full : (P *)prices + (int64_t)inst0 * M;
    hipLaunchKernelGGL(kfirst[lr0 - 1], dim3((unsigned)(M >> lr0), cnt), dim3(NT), lds0, s, dp, inst0, n, bufA, dstp,
                       p.npass == 1 ? 1 : 0);
    CM_LAUNCH_CHECK();
    int64_t plen = (int64_t)1 << lr0;
    const T *in = bufA;
    for (int ps = 1; ps < p.npass; ++ps) {
      const int lr = p.logr[ps];
      const bool last = ps == p.npass - 1;
      T *outb = (in == bufA) ? bufB : bufA;
      hipLaunchKernelGGL(knext[lr - 1], dim3((unsigned)((M >> lr) / FFT_COLS), cnt), dim3(NT),
                         lds_bytes(lr, FFT_COLS, sizeof(T)), s, dp, inst0, n, plen, in, outb, dstp, last ? 1 : 0);
      CM_LAUNCH_CHECK();
      in = outb;
      plen <<= lr;
    }
    if (gather) {
      hipLaunchKernelGGL(k_gather<P>, dim3(256), dim3(256), 0, s, full, M, strike_idx, nk, inst0, cnt, (P *)prices,
                         status);
      CM_LAUNCH_CHECK();
    }
  }
  return CM_OK;
}

extern "C" cm_status cm_fft_price(const cm_problem *prob, int batch, int n, int dtype, const int64_t *strike_idx,
                                  int nk, void *prices, int32_t *status, void *ws, size_t ws_bytes, void *stream) {
  if (!prob || !prices || batch < 0 || n < 1) return CM_E_INVALID;
  if (n > 30) return CM_E_UNSUPPORTED;
  if (dtype != CM_C64 && dtype != CM_C128) return CM_E_INVALID;
  if (strike_idx && nk < 1) return CM_E_INVALID;
  if (batch == 0) return CM_OK;
  if (batch > 65535) return CM_E_UNSUPPORTED;
  const size_t need = cm_fft_ws_bytes(batch, n, dtype, strike_idx != nullptr);
  if (!ws || ws_bytes < need) return CM_E_INVALID;
  // later passes need at least FFT_COLS work items
  {
    FftPlan p = make_plan(n, dtype, batch);
    for (int ps = 1; ps < p.npass; ++ps)
      if (((int64_t)1 << (n - p.logr[ps])) < FFT_COLS) return CM_E_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dtype == CM_C64) return fft_run<float2>(prob, batch, n, strike_idx, nk, prices, status, ws, ws_bytes, s);
  return fft_run<double2>(prob, batch, n, strike_idx, nk, prices, status, ws, ws_bytes, s);
}
