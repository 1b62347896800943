// cm_readout_prices: prices from an SFFT output train (Eq. discretization_dft).
//
// Output core l carries log-strike bit 2^l (the bit reversal of Section 3.2 is absorbed
// in the index map), so y_u = Y_0[0, u_0, :] Y_1[:, u_1, :] ... Y_{n-1}[:, u_{n-1}, 0].
// A lane group of width RW (a power of two >= the bond cap) holds one strike's vector;
// each lane owns one bond component and the vector is contracted from the right, core by
// core, through LDS. The price is
//   C(k_u) = Re[ exp(-alpha k_u)/(s pi) * exp(-i v0 k_u) * sqrt(M) * y_u ],
// with exp(-i v0 k_u) = exp(-i v0 k0) (-1)^u for the symmetric rule and 1 for Simpson.
#include "cm_cf.h"
#include "cm_tt.h"

namespace {
template <typename T> struct rd;
template <> struct rd<float2> {
  using V = float2;
  __device__ __forceinline__ static float2 zero() { return make_float2(0.f, 0.f); }
  __device__ __forceinline__ static void fma_(float2 &a, float2 b, float2 c) { ffma(a, b, c); }
  __device__ __forceinline__ static double2 to(float2 v) { return cmk(v.x, v.y); }
};
template <> struct rd<double2> {
  using V = double2;
  __device__ __forceinline__ static double2 zero() { return cmk(0.0, 0.0); }
  __device__ __forceinline__ static void fma_(double2 &a, double2 b, double2 c) { cfma(a, b, c); }
  __device__ __forceinline__ static double2 to(double2 v) { return v; }
};
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_readout(TTView y, const cm_problem *__restrict__ prob,
                                                 const int64_t *__restrict__ strike_idx, int nk,
                                                 double *__restrict__ prices, int32_t *__restrict__ status, int RW) {
  extern __shared__ unsigned char lds_raw[];
  T *buf = (T *)lds_raw;  // [2][256]
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int spw = 256 / RW;
  const int sl = tid / RW, lane = tid % RW;
  const int s = blockIdx.x * spw + sl;
  const bool valid = s < nk;
  const cm_problem pr = prob[b];
  const int n = y.n[b];
  const int64_t M = (int64_t)1 << n;
  int64_t u = valid ? strike_idx[(int64_t)b * nk + s] : 0;
  const bool bad = valid && (u < 0 || u >= M || pr.n != n);
  if (bad) u = 0;
  const T *cores = (const T *)y.cores;
  const int32_t *rk = y.rk(b);
  T *cur = buf, *nxt = buf + 256;
  // start: vector over bond n (dimension 1) = [1]
  cur[tid] = (lane == 0) ? T{1, 0} : T{0, 0};
  __syncthreads();
  for (int l = n - 1; l >= 0; --l) {
    const int rl = rk[l], rr = rk[l + 1];
    const int bit = (int)((u >> l) & 1);
    typename rd<T>::V acc = rd<T>::zero();
    if (lane < rl) {
      const T *row = cores + y.coff(b, l) + ((int64_t)lane * 2 + bit) * rr;
      const T *v = cur + sl * RW;
      for (int q = 0; q < rr; ++q) rd<T>::fma_(acc, row[q], v[q]);
    }
    nxt[tid] = acc;
    __syncthreads();
    T *t = cur; cur = nxt; nxt = t;
  }
  if (valid && lane == 0) {
    const double2 yu = rd<T>::to(cur[tid]);
    double price;
    if (bad) {
      price = NAN;
      set_status(status, b, CM_E_INVALID);
    } else {
      const bool simpson = pr.quad == CM_QUAD_SIMPSON1;
      const double k0 = k0_of(pr);
      const double lam = 2.0 * M_PI / (ldexp(1.0, n) * pr.eta);
      const double k = k0 + lam * (double)u;
      const double sqM = ldexp((n & 1) ? M_SQRT2 : 1.0, n >> 1);
      const double sc = exp(-pr.alpha * k) / ((simpson ? 1.0 : 2.0) * M_PI) * sqM;
      double2 ro = cmk(1.0, 0.0);
      if (!simpson) {
        double f;
        if (k0_is_default(pr)) {
          f = prod_cycles_frac(pr.eta, log(pr.S0), n - 1);
          if (n == 1) { f += 0.5; f -= floor(f); }
        } else {
          f = prod_cycles_frac(pr.eta, pr.k0, n - 1);
        }
        ro = turn(f);
        if (u & 1) ro = cmk(-ro.x, -ro.y);
      }
      price = sc * (ro.x * yu.x - ro.y * yu.y);
    }
    prices[(int64_t)b * nk + s] = price;
  }
}

extern "C" cm_status cm_readout_prices(const cm_tt_batch *y, const cm_problem *prob, const int64_t *strike_idx,
                                       int nk, double *prices, int32_t *status, void *stream) {
  if (!y || !prob || !strike_idx || !prices || nk < 0) return CM_E_INVALID;
  if (y->d_out != 2 || y->d_in != 1 || y->batch < 0) return CM_E_INVALID;
  if (y->dtype != CM_C64 && y->dtype != CM_C128) return CM_E_INVALID;
  if (y->cap_rank < 1 || y->cap_rank > 256) return CM_E_INVALID;
  if (y->batch == 0 || nk == 0) return CM_OK;
  if (y->batch > 65535) return CM_E_UNSUPPORTED;
  int RW = 1;
  while (RW < y->cap_rank) RW <<= 1;
  if (RW > 256) return CM_E_UNSUPPORTED;
  const int spw = 256 / RW;
  dim3 grid((unsigned)((nk + spw - 1) / spw), (unsigned)y->batch);
  hipStream_t s = (hipStream_t)stream;
  TTView v = tt_view(y);
  if (y->dtype == CM_C64)
    hipLaunchKernelGGL(k_readout<float2>, grid, dim3(256), 2 * 256 * sizeof(float2), s, v, prob, strike_idx, nk,
                       prices, status, RW);
  else
    hipLaunchKernelGGL(k_readout<double2>, grid, dim3(256), 2 * 256 * sizeof(double2), s, v, prob, strike_idx, nk,
                       prices, status, RW);
  CM_LAUNCH_CHECK();
  return CM_OK;
}
