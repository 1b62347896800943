// cm_readout_prices: prices from an SFFT output train (Eq. discretization_dft).
//
// Output core l carries log-strike bit 2^l (the bit reversal of Section 3.2 is absorbed
// in the index map), so y_u = Y_0[0, u_0, :] Y_1[:, u_1, :] ... Y_{n-1}[:, u_{n-1}, 0].
// k_readout: one lane per strike. The instance's cores are staged once per workgroup into
// LDS (when they fit), and each lane contracts its strike's vector from the right, core by
// core, in registers sized by a compile-time bound on the instance's largest bond; loops
// stop at the actual bond dimensions, which are uniform over the workgroup.
// k_readout_groups (bonds above that bound): a lane group of width RW (a power of two >=
// the bond cap) holds one strike's vector, one bond component per lane, through LDS.
// The price is
//   C(k_u) = Re[ exp(-alpha k_u)/(s pi) * exp(-i v0 k_u) * sqrt(M) * y_u ],
// with exp(-i v0 k_u) = exp(-i v0 k0) (-1)^u for the symmetric rule and 1 for Simpson.
// The observable mode (the measurement read-out of Section 2.2 with exact probabilities)
// drops the phase: C(k_u) = exp(-alpha k_u)/(s pi) * sqrt(M) * |y_u|.
#include <climits>

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

// Per-instance readout scalars.
struct ReadConst {
  double k0, eta, alpha, sfac;   // sfac = sqrt(M) / (s pi)
  int64_t us;                    // k_u = k0 + lambda (u - us): the default grid is centred on ln S0
  int n;
  double2 ro;                    // exp(-i v0 k0)
  bool alt;                      // sign alternates with u (symmetric rule)
};

__device__ __forceinline__ ReadConst read_const(const cm_problem &pr, int n) {
  ReadConst c;
  const bool simpson = pr.quad == CM_QUAD_SIMPSON1;
  // the default k0 = ln S0 - pi/eta is k0 = ln S0 - lambda M/2 exactly, so index u sits at
  // ln S0 + lambda (u - M/2) with an exact integer offset
  c.k0 = k0_is_default(pr) ? log(pr.S0) : pr.k0;
  c.us = k0_is_default(pr) ? ((int64_t)1 << (n - 1)) : 0;
  c.eta = pr.eta;
  c.n = n;
  c.alpha = pr.alpha;
  c.sfac = ldexp((n & 1) ? M_SQRT2 : 1.0, n >> 1) / ((simpson ? 1.0 : 2.0) * M_PI);
  c.alt = !simpson;
  c.ro = cmk(1.0, 0.0);
  if (!simpson) {
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

__device__ __forceinline__ double read_price(const ReadConst &c, int64_t u, double2 yu, int absval) {
  const double k = strike_log(c.k0, c.eta, c.n, (double)(u - c.us));
  if (absval) return exp(-c.alpha * k) * c.sfac * hypot(yu.x, yu.y);
  double2 ro = c.ro;
  if (c.alt && (u & 1)) ro = cmk(-ro.x, -ro.y);
  return exp(-c.alpha * k) * c.sfac * (ro.x * yu.x - ro.y * yu.y);
}

constexpr int RD_WG = 256;
constexpr int RD_SPT = 16;                // strikes per lane
// core staging arena and prefix tree: 48 KB for complex64 (three workgroups per CU, as many
// as the registers allow), 64 KB for complex128 (two)
template <typename T> constexpr int rd_lds();
template <> constexpr int rd_lds<float2>() { return 48 * 1024; }
template <> constexpr int rd_lds<double2>() { return 64 * 1024; }
// Prefix tree for strikes that share their high bits (a contiguous block of a workgroup's
// 4096 strikes spans at most two values of u >> 12): y_u = Lo[u mod 32] . MR[u >> 12][(u >> 5)
// mod 128], where Lo holds the 32 row vectors of cores 0..4, R[h] the right vectors of cores
// 12..n-1 for high part h, and MR[h][m] = cores 5..11 at bits m applied to R[h]. Each strike
// then costs r_5 multiply-adds instead of a contraction through all n cores.
constexpr int TB_LO = 5, TB_H = 12, TB_K = 2;
constexpr int TB_MID = 1 << (TB_H - TB_LO);

// Contracts one strike: v <- Y_l[:, bit_l, :] v from l = n-1 down to 0; returns y_u.
// Core l starts at base + off(l) and holds [rk[l]][2][rk[l+1]] values.
template <typename T, int RM, class Off>
__device__ __forceinline__ T contract_strike(const T *base, const Off &off, const int32_t *rk, int n, int64_t u) {
  T v[RM], w[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) v[a] = T{0, 0};
  v[0] = T{1, 0};
  for (int l = n - 1; l >= 0; --l) {
    const int ra = rk[l], rb = rk[l + 1];
    const T *C = base + off(l) + (int)((u >> l) & 1) * rb;
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      if (a < ra) {
        typename rd<T>::V acc = rd<T>::zero();
        const T *row = C + a * 2 * rb;
#pragma unroll
        for (int q = 0; q < RM; ++q)
          if (q < rb) rd<T>::fma_(acc, row[q], v[q]);
        w[a] = acc;
      }
    }
#pragma unroll
    for (int a = 0; a < RM; ++a) v[a] = w[a];
  }
  return v[0];
}

// v <- Y_l[:, bit_l(u), :] v for l = l_hi down to l_lo; v is indexed by bond l_hi + 1 on
// entry and by bond l_lo on exit (entries past the bond dimension are left undefined).
template <typename T, int RM, class Off>
__device__ __forceinline__ void contract_right(const T *base, const Off &off, const int32_t *rk, int l_hi, int l_lo,
                                               int64_t u, T *v) {
  T w[RM];
  for (int l = l_hi; l >= l_lo; --l) {
    const int ra = rk[l], rb = rk[l + 1];
    const T *C = base + off(l) + (int)((u >> l) & 1) * rb;
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      if (a < ra) {
        typename rd<T>::V acc = rd<T>::zero();
        const T *row = C + a * 2 * rb;
#pragma unroll
        for (int q = 0; q < RM; ++q)
          if (q < rb) rd<T>::fma_(acc, row[q], v[q]);
        w[a] = acc;
      }
    }
#pragma unroll
    for (int a = 0; a < RM; ++a) v[a] = w[a];
  }
}

// Row vector v <- v Y_l[:, bit_l(u), :] for l = l_lo up to l_hi; v is indexed by bond l_lo on
// entry and by bond l_hi + 1 on exit.
template <typename T, int RM, class Off>
__device__ __forceinline__ void contract_left(const T *base, const Off &off, const int32_t *rk, int l_lo, int l_hi,
                                              int64_t u, T *v) {
  T w[RM];
  for (int l = l_lo; l <= l_hi; ++l) {
    const int ra = rk[l], rb = rk[l + 1];
    const T *C = base + off(l) + (int)((u >> l) & 1) * rb;
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      if (c < rb) {
        typename rd<T>::V acc = rd<T>::zero();
#pragma unroll
        for (int a = 0; a < RM; ++a)
          if (a < ra) rd<T>::fma_(acc, C[a * 2 * rb + c], v[a]);
        w[c] = acc;
      }
    }
#pragma unroll
    for (int c = 0; c < RM; ++c) v[c] = w[c];
  }
}

struct LdsOff {
  const int32_t *o;
  __device__ __forceinline__ int64_t operator()(int l) const { return o[l]; }
};
struct GlobalOff {
  const TTView *y;
  int b;
  __device__ __forceinline__ int64_t operator()(int l) const { return y->coff(b, l); }
};

__device__ __forceinline__ int max_bond(const int32_t *rk, int n) {
  int r = 1;
  for (int l = 0; l <= n; ++l) r = rk[l] > r ? rk[l] : r;
  return r;
}

template <typename T, int RM>
__global__ __launch_bounds__(RD_WG) void k_readout(TTView y, const cm_problem *__restrict__ prob,
                                                   const int64_t *__restrict__ strike_idx, int nk,
                                                   double *__restrict__ prices, int32_t *__restrict__ status,
                                                   int rm_lo, int absval) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int32_t s_off[CM_MAX_N + 1], s_rk[CM_MAX_N + 1];
  __shared__ int64_t s_goff[CM_MAX_N];   // the cores' offsets in global memory
  __shared__ int s_ok;
  const int b = blockIdx.y;
  const int n = y.n[b];
  const int32_t *rk = y.rk(b);
  // this instantiation serves instances whose largest bond lies in (rm_lo, RM]
  const int rmax = max_bond(rk, n);
  if (rmax <= rm_lo || rmax > RM) return;
  const T *gcores = (const T *)y.cores;
  T *arena = (T *)lds_raw;
  if (threadIdx.x == 0) {
    int o = 0;
    for (int l = 0; l < n; ++l) {
      s_off[l] = o;
      s_rk[l] = rk[l];
      s_goff[l] = y.coff(b, l);
      o += rk[l] * 2 * rk[l + 1];
    }
    s_rk[n] = rk[n];
    s_off[n] = o;
    s_ok = (size_t)o * sizeof(T) <= (size_t)rd_lds<T>();
  }
  __syncthreads();
  const bool in_lds = s_ok != 0;
  if (in_lds) {
    // all cores as one flat range, four loads in flight per thread
    constexpr int U = 4;
    const int total = s_off[n];
    int l = 0;
    for (int e0 = threadIdx.x; e0 < total; e0 += RD_WG * U) {
      T v[U];
      int dst[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int e = e0 + k * RD_WG;
        dst[k] = -1;
        if (e < total) {
          while (s_off[l + 1] <= e) ++l;
          v[k] = gcores[s_goff[l] + (e - s_off[l])];
          dst[k] = e;
        }
      }
#pragma unroll
      for (int k = 0; k < U; ++k)
        if (dst[k] >= 0) arena[dst[k]] = v[k];
    }
  }
  __syncthreads();
  const cm_problem pr = prob[b];
  const ReadConst rc = read_const(pr, n);
  const int64_t M = (int64_t)1 << n;
  const int s0 = blockIdx.x * RD_WG * RD_SPT;
  // this workgroup's strikes; the range of their high parts decides the prefix tree. Each
  // lane reduces its strikes, the wave reduces by shuffles, and one lane per wave updates
  // the workgroup's range: atomics from every lane to one LDS word serialise and cost more
  // than the rest of the read-out.
  __shared__ long long s_hmin, s_hmax;
  __shared__ int s_bad;
  if (threadIdx.x == 0) { s_hmin = LLONG_MAX; s_hmax = -1; s_bad = 0; }
  __syncthreads();
  int64_t uu[RD_SPT];
  long long hlo = LLONG_MAX, hhi = -1;
  int bad = 0;
#pragma unroll
  for (int t = 0; t < RD_SPT; ++t) {
    const int s = s0 + t * RD_WG + (int)threadIdx.x;
    uu[t] = -1;
    if (s < nk) {
      const int64_t u = strike_idx[(int64_t)b * nk + s];
      uu[t] = u;
      if (u < 0 || u >= M) {
        bad = 1;
      } else {
        const long long h = (long long)(u >> TB_H);
        hlo = h < hlo ? h : hlo;
        hhi = h > hhi ? h : hhi;
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const long long a = __shfl_xor(hlo, o), c = __shfl_xor(hhi, o);
    hlo = a < hlo ? a : hlo;
    hhi = c > hhi ? c : hhi;
    bad |= __shfl_xor(bad, o);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&s_hmin, hlo);
    atomicMax(&s_hmax, hhi);
    if (bad) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  const int r5 = (n > TB_H) ? s_rk[TB_LO] : 0, r10 = (n > TB_H) ? s_rk[TB_H] : 0;
  const int tree_elems = TB_K * r10 + (32 + TB_K * TB_MID) * r5;
  const bool tree = in_lds && n > TB_H && pr.n == n && s_bad == 0 && s_hmax >= s_hmin &&
                    s_hmax - s_hmin < TB_K && (size_t)(s_off[n] + tree_elems) * sizeof(T) <= (size_t)rd_lds<T>();
  if (tree) {
    const int64_t hmin = s_hmin;
    const int nh = (int)(s_hmax - s_hmin) + 1;
    T *R = arena + s_off[n];          // [TB_K][r10]
    T *Lo = R + TB_K * r10;           // [32][r5]
    T *MR = Lo + 32 * r5;             // [TB_K][TB_MID][r5]
    const int tid = threadIdx.x;
    if (tid < nh) {
      T v[RM];
#pragma unroll
      for (int a = 0; a < RM; ++a) v[a] = T{0, 0};
      v[0] = T{1, 0};
      contract_right<T, RM>(arena, LdsOff{s_off}, s_rk, n - 1, TB_H, (hmin + tid) << TB_H, v);
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < r10) R[tid * r10 + a] = v[a];
    } else if (tid >= 64 && tid < 96) {
      T v[RM];
#pragma unroll
      for (int a = 0; a < RM; ++a) v[a] = T{0, 0};
      v[0] = T{1, 0};
      contract_left<T, RM>(arena, LdsOff{s_off}, s_rk, 0, TB_LO - 1, tid - 64, v);
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < r5) Lo[(tid - 64) * r5 + c] = v[c];
    }
    __syncthreads();
    for (int e = tid; e < TB_MID * nh; e += RD_WG) {
      const int q = e / TB_MID, m5 = e % TB_MID;
      T v[RM];
#pragma unroll
      for (int a = 0; a < RM; ++a) v[a] = (a < r10) ? R[q * r10 + a] : T{0, 0};
      contract_right<T, RM>(arena, LdsOff{s_off}, s_rk, TB_H - 1, TB_LO, ((hmin + q) << TB_H) | ((int64_t)m5 << TB_LO),
                            v);
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < r5) MR[(q * TB_MID + m5) * r5 + a] = v[a];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RD_SPT; ++t) {
      const int s = s0 + t * RD_WG + tid;
      const int64_t u = uu[t];
      if (s >= nk) break;
      const T *lo = Lo + (int)(u & 31) * r5;
      const T *mr = MR + (((int)((u >> TB_H) - hmin) * TB_MID) + (int)((u >> TB_LO) & (TB_MID - 1))) * r5;
      typename rd<T>::V acc = rd<T>::zero();
      for (int a = 0; a < r5; ++a) rd<T>::fma_(acc, lo[a], mr[a]);
      prices[(int64_t)b * nk + s] = read_price(rc, u, rd<T>::to(acc), absval);
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < RD_SPT; ++t) {
    const int s = s0 + t * RD_WG + (int)threadIdx.x;
    if (s >= nk) break;
    const int64_t u = uu[t];
    double price;
    if (u < 0 || u >= M || pr.n != n) {
      price = NAN;
      set_status(status, b, CM_E_INVALID);
    } else {
      T yu;
      if (in_lds) yu = contract_strike<T, RM>(arena, LdsOff{s_off}, s_rk, n, u);
      else yu = contract_strike<T, RM>(gcores, GlobalOff{&y, b}, s_rk, n, u);
      price = read_price(rc, u, rd<T>::to(yu), absval);
    }
    prices[(int64_t)b * nk + s] = price;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_readout_groups(TTView y, const cm_problem *__restrict__ prob,
                                                 const int64_t *__restrict__ strike_idx, int nk,
                                                 double *__restrict__ prices, int32_t *__restrict__ status, int RW,
                                                 int rm_lo, int absval) {
  extern __shared__ unsigned char lds_raw[];
  T *buf = (T *)lds_raw;  // [2][256]
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  if (max_bond(y.rk(b), y.n[b]) <= rm_lo) return;
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
      price = read_price(read_const(pr, n), u, yu, absval);
    }
    prices[(int64_t)b * nk + s] = price;
  }
}

static cm_status readout(const cm_tt_batch *y, const cm_problem *prob, const int64_t *strike_idx, int nk,
                         double *prices, int32_t *status, void *stream, int absval) {
  if (!y || !prob || !strike_idx || !prices || nk < 0) return CM_E_INVALID;
  if (y->d_out != 2 || y->d_in != 1 || y->batch < 0) return CM_E_INVALID;
  if (y->dtype != CM_C64 && y->dtype != CM_C128) return CM_E_INVALID;
  if (y->cap_rank < 1 || y->cap_rank > 256) return CM_E_INVALID;
  if (y->batch == 0 || nk == 0) return CM_OK;
  if (y->batch > 65535) return CM_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  TTView v = tt_view(y);
  const dim3 grid((unsigned)((nk + RD_WG * RD_SPT - 1) / (RD_WG * RD_SPT)), (unsigned)y->batch);
  const int cap = y->cap_rank;
  // one-lane-per-strike kernels by bound on the largest bond; the lane-group kernel takes
  // the rest
  int fast_max;
  if (y->dtype == CM_C64) {
    constexpr int L = rd_lds<float2>();
    CM_HIP_CHECK(cm_allow_lds(k_readout<float2, 8>, L));
    CM_HIP_CHECK(cm_allow_lds(k_readout<float2, 16>, L));
    CM_HIP_CHECK(cm_allow_lds(k_readout<float2, 32>, L));
    hipLaunchKernelGGL((k_readout<float2, 8>), grid, dim3(RD_WG), L, s, v, prob, strike_idx, nk, prices, status, 0,
                       absval);
    if (cap > 8)
      hipLaunchKernelGGL((k_readout<float2, 16>), grid, dim3(RD_WG), L, s, v, prob, strike_idx, nk, prices, status, 8,
                         absval);
    if (cap > 16)
      hipLaunchKernelGGL((k_readout<float2, 32>), grid, dim3(RD_WG), L, s, v, prob, strike_idx, nk, prices, status, 16,
                         absval);
    fast_max = 32;
  } else {
    constexpr int L = rd_lds<double2>();
    CM_HIP_CHECK(cm_allow_lds(k_readout<double2, 8>, L));
    CM_HIP_CHECK(cm_allow_lds(k_readout<double2, 16>, L));
    hipLaunchKernelGGL((k_readout<double2, 8>), grid, dim3(RD_WG), L, s, v, prob, strike_idx, nk, prices, status, 0,
                       absval);
    if (cap > 8)
      hipLaunchKernelGGL((k_readout<double2, 16>), grid, dim3(RD_WG), L, s, v, prob, strike_idx, nk, prices, status, 8,
                         absval);
    fast_max = 16;
  }
  CM_LAUNCH_CHECK();
  if (cap > fast_max) {
    int RW = 1;
    while (RW < cap) RW <<= 1;
    if (RW > 256) return CM_E_UNSUPPORTED;
    const int spw = 256 / RW;
    dim3 g2((unsigned)((nk + spw - 1) / spw), (unsigned)y->batch);
    if (y->dtype == CM_C64)
      hipLaunchKernelGGL(k_readout_groups<float2>, g2, dim3(256), 2 * 256 * sizeof(float2), s, v, prob, strike_idx,
                         nk, prices, status, RW, fast_max, absval);
    else
      hipLaunchKernelGGL(k_readout_groups<double2>, g2, dim3(256), 2 * 256 * sizeof(double2), s, v, prob,
                         strike_idx, nk, prices, status, RW, fast_max, absval);
  }
  CM_LAUNCH_CHECK();
  return CM_OK;
}

extern "C" cm_status cm_readout_prices(const cm_tt_batch *y, const cm_problem *prob, const int64_t *strike_idx,
                                       int nk, double *prices, int32_t *status, void *stream) {
  return readout(y, prob, strike_idx, nk, prices, status, stream, 0);
}

extern "C" cm_status cm_readout_observable(const cm_tt_batch *y, const cm_problem *prob, const int64_t *strike_idx,
                                           int nk, double *prices, int32_t *status, void *stream) {
  return readout(y, prob, strike_idx, nk, prices, status, stream, 1);
}

// ------------------------------------------------------------------ shot prices
// Observable prices from measured outcomes (Eqs. qft_probability_estimator and
// qft_observable_price): R_u of the R shots landed on outcome u, p_hat_u = R_u / R, and
//   C_hat(k_u) = exp(-alpha k_u)/(s pi) * sqrt(M) * sqrt(||y||^2 p_hat_u).
// k_shot_count: one lane per shot, a binary search of the instance's sorted strike list
// and an atomic increment of the matching count. k_shot_price: one lane per strike.
__global__ __launch_bounds__(256) void k_fill_zero_i32(int32_t *__restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_shot_count(const cm_problem *__restrict__ prob,
                                                    const int64_t *__restrict__ samples, int R,
                                                    const int64_t *__restrict__ strike_idx, int nk,
                                                    int32_t *__restrict__ counts, int32_t *__restrict__ status) {
  const int b = blockIdx.y;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= R) return;
  const int n = prob[b].n;
  const int64_t u = samples[(int64_t)b * R + s];
  if (u == -1) return;  // the sampler's mark for an instance it could not sample
  if (n < 1 || n > CM_MAX_N || u < 0 || u >= ((int64_t)1 << n)) {
    set_status(status, b, CM_E_INVALID);
    return;
  }
  const int64_t *row = strike_idx + (int64_t)b * nk;
  int lo = 0, hi = nk;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (row[mid] < u) lo = mid + 1;
    else hi = mid;
  }
  if (lo < nk && row[lo] == u) atomicAdd(counts + (int64_t)b * nk + lo, 1);
}

__global__ __launch_bounds__(256) void k_shot_price(const cm_problem *__restrict__ prob,
                                                    const double *__restrict__ norm2, int R,
                                                    const int64_t *__restrict__ strike_idx, int nk,
                                                    const int32_t *__restrict__ counts, double *__restrict__ prices,
                                                    int32_t *__restrict__ status) {
  const int b = blockIdx.y;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= nk) return;
  const cm_problem pr = prob[b];
  const int n = pr.n;
  const int64_t *row = strike_idx + (int64_t)b * nk;
  const int64_t u = row[s];
  const double nv = norm2[b];
  const bool ok = n >= 1 && n <= CM_MAX_N && u >= 0 && u < ((int64_t)1 << n) && (s == 0 || row[s - 1] < u) &&
                  isfinite(nv) && nv > 0.0;
  double price = NAN;
  if (!ok) {
    set_status(status, b, CM_E_INVALID);
  } else {
    const ReadConst rc = read_const(pr, n);
    const double k = strike_log(rc.k0, rc.eta, rc.n, (double)(u - rc.us));
    const double c = (double)counts[(int64_t)b * nk + s];
    price = exp(-rc.alpha * k) * rc.sfac * sqrt(nv * c / (double)R);
  }
  prices[(int64_t)b * nk + s] = price;
}

extern "C" cm_status cm_shot_prices(const cm_problem *prob, int batch, const double *norm2, const int64_t *samples,
                                    int R, const int64_t *strike_idx, int nk, int32_t *counts, double *prices,
                                    int32_t *status, void *stream) {
  if (!prob || !norm2 || batch < 0 || nk < 0 || R < 1) return CM_E_INVALID;
  if (batch == 0 || nk == 0) return CM_OK;
  if (!samples || !strike_idx || !counts || !prices) return CM_E_INVALID;
  if (batch > 65535) return CM_E_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int64_t total = (int64_t)batch * nk;
  const int64_t zb = (total + 255) / 256;
  hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)(zb < 65536 ? zb : 65536)), dim3(256), 0, st, counts, total);
  hipLaunchKernelGGL(k_shot_count, dim3((unsigned)((R + 255) / 256), (unsigned)batch), dim3(256), 0, st, prob,
                     samples, R, strike_idx, nk, counts, status);
  hipLaunchKernelGGL(k_shot_price, dim3((unsigned)((nk + 255) / 256), (unsigned)batch), dim3(256), 0, st, prob,
                     norm2, R, strike_idx, nk, counts, prices, status);
  CM_LAUNCH_CHECK();
  return CM_OK;
}
