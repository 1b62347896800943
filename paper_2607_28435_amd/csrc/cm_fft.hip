// cm_fft_price: dense Carr–Madan baseline (Section 2.1, Eqs. x, dft, discretization_dft).
//
// Mixed-radix Stockham FFT (decimation in time, autosorting). Pass p with radix R_p and
// stride p_len = R_1 ... R_{p-1} maps work item i in [0, M/R_p), k = i mod p_len, as
//   u[r] = x[i + r M/R_p] * exp(-2 pi i r k / (R_p p_len)),  u <- DFT_{R_p}(u),
//   y[(i - k) R_p + k + r p_len] = u[r].
// Each work item's R_p-point DFT runs in LDS (bit-reversed load, in-place radix-2 stages).
//   - Pass 1 (p_len = 1, one work item per workgroup, radix up to 2^14 for CM_C64 /
//     2^13 for CM_C128) generates x on the fly from the characteristic function, so it
//     reads nothing from HBM.
//   - Later passes handle 16 consecutive work items per workgroup, so every global load
//     and store moves 16 consecutive elements.
//   - The last pass multiplies by the readout scalars and stores prices.
// Characteristic functions run in the storage precision (FP32 for CM_C64); every phase that
// grows with j or u is reduced exactly in FP64 first.
#include "cm_cf.h"
#include "cm_tt.h"

namespace {

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
};

constexpr int FFT_COLS = 16;

struct FftPlan {
  int n, npass;
  int logr[4];     // radix bits per pass
  int chunk;       // instances per launch group
  int tw_log;      // twiddle table length 2^tw_log (largest radix)
};

__host__ __device__ inline int first_radix_bits(int dtype) { return dtype == CM_C64 ? 14 : 13; }
__host__ __device__ inline int later_radix_bits(int dtype) { return dtype == CM_C64 ? 10 : 9; }

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
  int tw = 0;
  for (int i = 0; i < np; ++i) tw = p.logr[i] > tw ? p.logr[i] : tw;
  p.tw_log = tw;
  int ch = 1;
  if (n < 22) ch = 1 << (22 - n);
  p.chunk = batch < ch ? batch : ch;
  if (p.chunk < 1) p.chunk = 1;
  return p;
}

__host__ inline size_t al256f(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ inline size_t fft_ws_bytes(const FftPlan &p, int dtype, bool gather) {
  const size_t es = dtype == CM_C64 ? 8 : 16;
  const size_t M = (size_t)1 << p.n;
  size_t o = al256f(es * ((size_t)1 << (p.tw_log > 1 ? p.tw_log - 1 : 1)));
  o += al256f(es * M * p.chunk);                       // buffer A
  if (p.npass >= 3) o += al256f(es * M * p.chunk);     // buffer B
  if (gather) o += al256f(es / 2 * M * p.chunk);       // full prices before gathering
  return o;
}

}  // namespace

template <typename T>
__global__ void k_twiddles(T *tw, int logR) {
  const int half = 1 << (logR - 1);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < half; t += gridDim.x * blockDim.x)
    tw[t] = fr<T>::cis_neg(ldexp((double)t, -logR));
}

// In-place radix-2 DIT stages on ncol columns of length 2^logR held in LDS (bit-reversed).
template <typename T>
__device__ __forceinline__ void lds_fft(T *a, int logR, int ncol, const T *__restrict__ tw, int tw_log) {
  const int R = 1 << logR;
  const int hb = R >> 1;
  for (int s = 1; s <= logR; ++s) {
    const int half = 1 << (s - 1);
    const int tstr = 1 << (tw_log - s);
    for (int e = threadIdx.x; e < ncol * hb; e += blockDim.x) {
      const int col = e >> (logR - 1), bf = e & (hb - 1);
      const int pos = bf & (half - 1);
      const int i0 = ((bf >> (s - 1)) << s) + pos, i1 = i0 + half;
      T *c = a + col * R;
      const T w = tw[pos * tstr];
      const T x0 = c[i0], x1 = c[i1];
      const T t = fr<T>::mul(w, x1);
      c[i0] = fr<T>::add(x0, t);
      c[i1] = fr<T>::sub(x0, t);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int brev_bits(int r, int bits) { return bits ? (int)(__brev((unsigned)r) >> (32 - bits)) : 0; }

// Per-problem constants of the integrand and readout.
struct DenseConst {
  double eta, v0;
  double th_hi, th_lo;     // theta / (2 pi) as double-double, theta = eta (m_f - k0)
  double2 g0;              // exp(i v0 m_f)
  bool simpson;
  double k0, lam, alpha, sfac;  // readout
  double2 ro;              // exp(-i v0 k0)
  bool alt;                // readout alternates sign with u (symmetric rule)
};

__device__ inline DenseConst dense_const(const cm_problem &pr) {
  DenseConst c;
  const int n = pr.n;
  c.eta = pr.eta;
  c.simpson = pr.quad == CM_QUAD_SIMPSON1;
  c.v0 = c.simpson ? 0.0 : -ldexp(pr.eta, n - 1);
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
    two_prod(pr.eta, (log(pr.S0) - pr.k0) + rq, p, e);
    c.th_hi = p * CM_INV2PI_HI;
    c.th_lo = fma(p, CM_INV2PI_HI, -c.th_hi) + p * CM_INV2PI_LO + e * CM_INV2PI_HI;
  }
  if (c.simpson) c.g0 = cmk(1.0, 0.0);
  else {
    double f = prod_cycles_frac(c.v0, log(pr.S0), 0) + prod_cycles_frac(c.v0, rq, 0);
    c.g0 = turn(f - floor(f));
  }
  c.k0 = k0_of(pr);
  c.lam = 2.0 * M_PI / (ldexp(1.0, n) * pr.eta);
  c.alpha = pr.alpha;
  c.sfac = c.simpson ? 1.0 / M_PI : 0.5 / M_PI;
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

// x_j for the dense path, in storage precision
template <typename T>
__device__ __forceinline__ T integrand_at(const DenseConst &c, const CfModel<typename fr<T>::R> &m, int64_t j) {
  using R = typename fr<T>::R;
  const double v = c.v0 + (double)j * c.eta;
  const cx<R> h = h_centered<R>(m, (R)v);
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

template <typename T>
__device__ __forceinline__ double price_at(const DenseConst &c, int64_t u, T y) {
  const double k = c.k0 + c.lam * (double)u;
  double sc = exp(-c.alpha * k) * c.sfac;
  double2 ro = c.ro;
  if (c.alt && (u & 1)) ro = cmk(-ro.x, -ro.y);
  // Re[sc * ro * y]
  return sc * (ro.x * (double)y.x - ro.y * (double)y.y);
}

template <typename T> struct price_t;
template <> struct price_t<float2> { using type = float; };
template <> struct price_t<double2> { using type = double; };

// Pass 1: one work item (i = blockIdx.x) per workgroup; generates x[i + r M/R1].
template <typename T>
__global__ __launch_bounds__(256) void k_fft_first(const cm_problem *__restrict__ prob, int inst0, int n, int logR,
                                                   const T *__restrict__ tw, int tw_log, T *__restrict__ out,
                                                   typename price_t<T>::type *__restrict__ prices, int single) {
  extern __shared__ unsigned char lds_raw[];
  T *a = (T *)lds_raw;
  const int inst = inst0 + blockIdx.y;
  const cm_problem pr = prob[inst];
  const DenseConst c = dense_const(pr);
  const CfModel<typename fr<T>::R> m = make_model<typename fr<T>::R>(pr);
  const int64_t M = (int64_t)1 << n;
  const int R = 1 << logR;
  const int64_t T_items = M >> logR;
  const int64_t i = blockIdx.x;
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    const int64_t j = i + (int64_t)r * T_items;
    a[brev_bits(r, logR)] = integrand_at<T>(c, m, j);
  }
  __syncthreads();
  lds_fft<T>(a, logR, 1, tw, tw_log);
  if (single) {
    // whole transform done (M == R): write prices
    typename price_t<T>::type *pp = prices + (int64_t)blockIdx.y * M;
    for (int r = threadIdx.x; r < R; r += blockDim.x) pp[r] = (typename price_t<T>::type)price_at<T>(c, r, a[r]);
  } else {
    T *o = out + (int64_t)blockIdx.y * M + i * R;
    for (int r = threadIdx.x; r < R; r += blockDim.x) o[r] = a[r];
  }
}

// Later passes: FFT_COLS consecutive work items per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_next(const cm_problem *__restrict__ prob, int inst0, int n, int logR,
                                                  int64_t plen, const T *__restrict__ tw, int tw_log,
                                                  const T *__restrict__ in, T *__restrict__ out,
                                                  typename price_t<T>::type *__restrict__ prices, int last) {
  extern __shared__ unsigned char lds_raw[];
  T *a = (T *)lds_raw;
  const int64_t M = (int64_t)1 << n;
  const int R = 1 << logR;
  const int64_t T_items = M >> logR;
  const int64_t i0 = (int64_t)blockIdx.x * FFT_COLS;
  const T *src = in + (int64_t)blockIdx.y * M;
  const int64_t twl = (int64_t)R * plen;   // twiddle denominator
  // load + pass twiddle; element (col, r) -> LDS a[col*R + brev(r)]
  for (int e = threadIdx.x; e < FFT_COLS * R; e += blockDim.x) {
    const int col = e % FFT_COLS, r = e / FFT_COLS;
    const int64_t i = i0 + col;
    const int64_t k = i & (plen - 1);
    T v = src[i + (int64_t)r * T_items];
    const int64_t t = ((int64_t)r * k) & (twl - 1);
    if (t) v = fr<T>::mul(v, fr<T>::cis_neg(ldexp((double)t, -(int)(__builtin_ctzll(twl)))));
    a[col * R + brev_bits(r, logR)] = v;
  }
  __syncthreads();
  lds_fft<T>(a, logR, FFT_COLS, tw, tw_log);
  if (last) {
    const cm_problem pr = prob[inst0 + blockIdx.y];
    const DenseConst c = dense_const(pr);
    typename price_t<T>::type *pp = prices + (int64_t)blockIdx.y * M;
    for (int e = threadIdx.x; e < FFT_COLS * R; e += blockDim.x) {
      const int col = e % FFT_COLS, r = e / FFT_COLS;
      const int64_t i = i0 + col;
      const int64_t k = i & (plen - 1);
      const int64_t u = (i - k) * R + k + (int64_t)r * plen;
      pp[u] = (typename price_t<T>::type)price_at<T>(c, u, a[col * R + r]);
    }
  } else {
    T *dst = out + (int64_t)blockIdx.y * M;
    for (int e = threadIdx.x; e < FFT_COLS * R; e += blockDim.x) {
      const int col = e % FFT_COLS, r = e / FFT_COLS;
      const int64_t i = i0 + col;
      const int64_t k = i & (plen - 1);
      dst[(i - k) * R + k + (int64_t)r * plen] = a[col * R + r];
    }
  }
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

__global__ void k_check_problems(const cm_problem *__restrict__ prob, int batch, int n, int32_t *__restrict__ status) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < batch; b += gridDim.x * blockDim.x) {
    int c = check_problem(prob[b]);
    if (c == CM_OK && prob[b].n != n) c = CM_E_INVALID;
    if (status) status[b] = c;
  }
}

extern "C" size_t cm_fft_ws_bytes(int batch, int n, int dtype, int gather) {
  if (n < 1 || n > 30 || batch < 1) return 0;
  FftPlan p = make_plan(n, dtype, batch);
  return fft_ws_bytes(p, dtype, gather != 0);
}

template <typename T>
static cm_status fft_run(const cm_problem *prob, int batch, int n, const int64_t *strike_idx, int nk, void *prices,
                         int32_t *status, void *ws, hipStream_t s) {
  using P = typename price_t<T>::type;
  const int dtype = sizeof(T) == 8 ? CM_C64 : CM_C128;
  FftPlan p = make_plan(n, dtype, batch);
  const bool gather = strike_idx != nullptr;
  const int64_t M = (int64_t)1 << n;
  char *w = (char *)ws;
  T *tw = (T *)w;
  w += al256f(sizeof(T) * ((size_t)1 << (p.tw_log > 1 ? p.tw_log - 1 : 1)));
  T *bufA = (T *)w;
  w += al256f(sizeof(T) * M * p.chunk);
  T *bufB = bufA;
  if (p.npass >= 3) { bufB = (T *)w; w += al256f(sizeof(T) * M * p.chunk); }
  P *full = gather ? (P *)w : nullptr;
  hipLaunchKernelGGL(k_check_problems, dim3((batch + 255) / 256), dim3(256), 0, s, prob, batch, n, status);
  hipLaunchKernelGGL(k_twiddles<T>, dim3(64), dim3(256), 0, s, tw, p.tw_log);
  CM_LAUNCH_CHECK();
  for (int inst0 = 0; inst0 < batch; inst0 += p.chunk) {
    const int cnt = (batch - inst0) < p.chunk ? (batch - inst0) : p.chunk;
    P *dstp = gather ? full : (P *)prices + (int64_t)inst0 * M;
    const int lr0 = p.logr[0];
    const size_t lds0 = sizeof(T) << lr0;
    CM_HIP_CHECK(cm_allow_lds(k_fft_first<T>, lds0));
    hipLaunchKernelGGL(k_fft_first<T>, dim3((unsigned)(M >> lr0), cnt), dim3(256), lds0, s, prob, inst0, n, lr0, tw,
                       p.tw_log, bufA, dstp, p.npass == 1 ? 1 : 0);
    CM_LAUNCH_CHECK();
    int64_t plen = (int64_t)1 << lr0;
    const T *in = bufA;
    for (int ps = 1; ps < p.npass; ++ps) {
      const int lr = p.logr[ps];
      const bool last = ps == p.npass - 1;
      T *outb = (in == bufA) ? bufB : bufA;
      const size_t lds = sizeof(T) * FFT_COLS << lr;
      CM_HIP_CHECK(cm_allow_lds(k_fft_next<T>, lds));
      hipLaunchKernelGGL(k_fft_next<T>, dim3((unsigned)((M >> lr) / FFT_COLS), cnt), dim3(256), lds, s, prob, inst0,
                         n, lr, plen, tw, p.tw_log, in, outb, dstp, last ? 1 : 0);
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
  const size_t need = cm_fft_ws_bytes(batch, n, dtype, strike_idx != nullptr);
  if (!ws || ws_bytes < need) return CM_E_INVALID;
  // later passes need at least FFT_COLS work items
  {
    FftPlan p = make_plan(n, dtype, batch);
    for (int ps = 1; ps < p.npass; ++ps)
      if (((int64_t)1 << (n - p.logr[ps])) < FFT_COLS) return CM_E_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dtype == CM_C64) return fft_run<float2>(prob, batch, n, strike_idx, nk, prices, status, ws, s);
  return fft_run<double2>(prob, batch, n, strike_idx, nk, prices, status, ws, s);
}
