// cm_sample_outcomes: measurement outcomes of the QFT register (Section 2.2, Eq.
// qft_probabilities) drawn from an SFFT output train without forming its 2^n amplitudes.
//
// Output core l carries outcome bit 2^l, so the probability mass of the outcomes whose low
// t+1 bits are (b_0, ..., b_t) is
//   q(b_0..b_t) = w E_{t+1} w^H,   w = Y_0[0,b_0,:] Y_1[:,b_1,:] ... Y_t[:,b_t,:]  (a row),
// with the right environments E_l = sum_b Y_l[:,b,:] E_{l+1} Y_l[:,b,:]^H, E_n = [1]: E_l
// is the Gram matrix of the right partial contractions, and E_0 = ||y||^2. A shot fixes
// bit 0 first. With prefix row w of mass q, let w0 = w Y_t[:,0,:] and q0 = w0 E_{t+1} w0^H;
// bit t is 1 iff U_t q >= q0 for the shot's uniform U_t, and the prefix becomes
// w Y_t[:,bit,:] with its own mass. Every decision is taken in FP64 whatever the storage
// precision of the train.
//
// k_envs: one workgroup per instance builds E_n, ..., E_0 in LDS and stores E_1..E_n and
// the FP64 cores in the workspace, zero-padded to bond dimensions rounded up to multiples
// of 4. k_sample: one lane per shot holding its prefix row in registers (sized by a
// compile-time bound on the instance's largest bond); the products run over 4 x 4 blocks
// of the padded operands, whose addresses are the same for every lane, so the operands
// arrive through scalar loads and each block's loads are issued together.
#include "cm_internal.h"

namespace {

constexpr int SMP_WG = 256;
constexpr int SMP_RS = 32;  // largest bond dimension the sampler takes

__device__ __forceinline__ int max_bond_of(const int32_t *rk, int n) {
  int r = 1;
  for (int l = 0; l <= n; ++l) r = rk[l] > r ? rk[l] : r;
  return r;
}

__host__ __device__ __forceinline__ int pad4(int r) { return (r + 3) & ~3; }

// Workspace slab of one instance (complex FP64 elements):
//   E_l, l = 1..n:   at l * RS * RS, [p4(r_l)][p4(r_l)]
//   Y_l, l = 0..n-1: at (n_max + 1) RS^2 + l * 2 RS^2, [p4(r_l)][2][p4(r_{l+1})]
// with p4 = round up to a multiple of 4 and zeros in the padding.
template <typename T>
__global__ __launch_bounds__(SMP_WG) void k_envs(TTView y, int RS, int n_max, int64_t inst_stride,
                                                 double2 *__restrict__ ws, double *__restrict__ norm2,
                                                 int32_t *__restrict__ status) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double2 *Yd = (double2 *)lds_raw;   // [r_l][2][r_{l+1}]
  double2 *Tm = Yd + 2 * RS * RS;     // [2][r_l][r_{l+1}]
  double2 *Ea = Tm + 2 * RS * RS;     // E_{l+1}
  double2 *Eb = Ea + RS * RS;         // E_l
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int n = y.n[b];
  if (n < 0 || n > n_max) {   // the slab holds n_max levels
    if (tid == 0) {
      norm2[b] = NAN;
      set_status(status, b, CM_E_INVALID);
    }
    return;
  }
  const int32_t *rk = y.rk(b);
  if (max_bond_of(rk, n) > RS) {
    if (tid == 0) {
      norm2[b] = NAN;
      set_status(status, b, CM_E_UNSUPPORTED);
    }
    return;
  }
  double2 *Eg = ws + (int64_t)b * inst_stride;
  double2 *Yg = Eg + (int64_t)(n_max + 1) * RS * RS;
  const T *cores = (const T *)y.cores;
  // E_n = [1], padded to 4 x 4
  for (int e = tid; e < 16; e += SMP_WG) Eg[(int64_t)n * RS * RS + e] = cmk(e == 0 ? 1.0 : 0.0, 0.0);
  if (tid == 0) Ea[0] = cmk(1.0, 0.0);
  __syncthreads();
  for (int l = n - 1; l >= 0; --l) {
    const int ra = rk[l], rb = rk[l + 1];
    const int pa = pad4(ra), pb = pad4(rb);
    const T *C = cores + y.coff(b, l);
    for (int e = tid; e < ra * 2 * rb; e += SMP_WG) Yd[e] = cstore<T>::ld(C, e);
    // padded FP64 copy of the core for the sampler
    double2 *Yl = Yg + (int64_t)l * 2 * RS * RS;
    for (int e = tid; e < pa * 2 * pb; e += SMP_WG) {
      const int a = e / (2 * pb), bit = (e / pb) % 2, c = e % pb;
      Yl[e] = (a < ra && c < rb) ? cstore<T>::ld(C, (a * 2 + bit) * rb + c) : cmk(0.0, 0.0);
    }
    __syncthreads();
    // Tm[bit][c][f] = sum_e Y[c][bit][e] E_{l+1}[e][f]
    for (int e = tid; e < 2 * ra * rb; e += SMP_WG) {
      const int bit = e / (ra * rb), c = (e / rb) % ra, f = e % rb;
      const double2 *row = Yd + (c * 2 + bit) * rb;
      double2 acc = cmk(0.0, 0.0);
      for (int q = 0; q < rb; ++q) cfma(acc, row[q], Ea[q * rb + f]);
      Tm[e] = acc;
    }
    __syncthreads();
    // E_l[c][d] = sum_bit sum_f Tm[bit][c][f] conj(Y[d][bit][f])
    for (int e = tid; e < ra * ra; e += SMP_WG) {
      const int c = e / ra, d = e % ra;
      double2 acc = cmk(0.0, 0.0);
      for (int bit = 0; bit < 2; ++bit) {
        const double2 *tr = Tm + (bit * ra + c) * rb;
        const double2 *yr = Yd + (d * 2 + bit) * rb;
        for (int f = 0; f < rb; ++f) ccfma(acc, yr[f], tr[f]);
      }
      Eb[e] = acc;
    }
    __syncthreads();
    if (l > 0) {
      double2 *El = Eg + (int64_t)l * RS * RS;
      for (int e = tid; e < pa * pa; e += SMP_WG) {
        const int c = e / pa, d = e % pa;
        El[e] = (c < ra && d < ra) ? Eb[c * ra + d] : cmk(0.0, 0.0);
      }
    }
    double2 *t = Ea; Ea = Eb; Eb = t;
  }
  if (tid == 0) {
    const double nv = Ea[0].x;
    norm2[b] = nv;
    if (!isfinite(nv)) set_status(status, b, CM_E_NONFINITE);
    else if (!(nv > 0.0)) set_status(status, b, CM_E_INVALID);
  }
}

// w <- v Y[:, bit, :] over 4 x 4 blocks of the padded core Y ([pa][2][pb], pa, pb <= RM).
// Entries of v past the bond are zero, and so are the padded columns of Y.
template <int RM>
__device__ __forceinline__ void row_times_core(const double2 *v, const double2 *__restrict__ Y, int pa, int pb,
                                               int bit, double2 *w) {
#pragma unroll
  for (int c = 0; c < RM; ++c) w[c] = cmk(0.0, 0.0);
#pragma unroll
  for (int c4 = 0; c4 < RM; c4 += 4) {
    if (c4 < pb) {
#pragma unroll
      for (int a4 = 0; a4 < RM; a4 += 4) {
        if (a4 < pa) {
          double2 yb[4][4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) yb[i][j] = Y[((a4 + i) * 2 + bit) * pb + c4 + j];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) cfma(w[c4 + j], v[a4 + i], yb[i][j]);
        }
      }
    }
  }
}

// w E w^H for Hermitian E (padded [p][p], p <= RM) from its upper triangle, 4 x 4 blocks.
template <int RM>
__device__ __forceinline__ double quad_form(const double2 *w, const double2 *__restrict__ E, int p) {
  double acc = 0.0;
#pragma unroll
  for (int c4 = 0; c4 < RM; c4 += 4) {
    if (c4 < p) {
      // z_i = sum_{d > c4+i} conj(E[c4+i][d]) w[d]
      double2 z[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) z[i] = cmk(0.0, 0.0);
      double diag[4];
#pragma unroll
      for (int d4 = c4; d4 < RM; d4 += 4) {
        if (d4 < p) {
          double2 eb[4][4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (d4 > c4 || j >= i) eb[i][j] = E[(c4 + i) * p + d4 + j];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (d4 == c4) diag[i] = eb[i][i].x;
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (d4 > c4 || j > i) ccfma(z[i], eb[i][j], w[d4 + j]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double2 wc = w[c4 + i];
        acc = fma(diag[i], cabs2(wc), acc);
        acc = fma(2.0, wc.x * z[i].x + wc.y * z[i].y, acc);
      }
    }
  }
  return acc;
}

template <int RM>
__global__ __launch_bounds__(SMP_WG) void k_sample(TTView y, const double2 *__restrict__ ws, int RS, int n_max,
                                                   int64_t inst_stride, const double *__restrict__ norm2,
                                                   const double *__restrict__ uni, int ustride, int R,
                                                   int64_t *__restrict__ out, int rm_lo) {
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int n = y.n[b];
  const int s = blockIdx.x * SMP_WG + tid;
  if (n < 0 || n > n_max) {   // k_envs has set CM_E_INVALID
    if (rm_lo == 0 && s < R) out[(int64_t)b * R + s] = -1;   // the always-launched bound marks it
    return;
  }
  const int32_t *rk = y.rk(b);
  // this instantiation serves instances whose largest bond lies in (rm_lo, RM]; the widest
  // one also writes -1 for instances above every bound
  const int rmax = max_bond_of(rk, n);
  if (rmax <= rm_lo) return;
  if (s >= R) return;
  const double q_all = norm2[b];
  if (rmax > RM || !(q_all > 0.0) || !isfinite(q_all)) {
    if (rmax <= RM || RM == SMP_RS) out[(int64_t)b * R + s] = -1;
    return;
  }
  // uniforms are bit-major, [batch][ustride][R]: level t of consecutive shots is contiguous
  const double *U = uni + (int64_t)b * ustride * R + s;
  const double2 *Eg = ws + (int64_t)b * inst_stride;
  const double2 *Yg = Eg + (int64_t)(n_max + 1) * RS * RS;
  double2 v[RM], w[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) v[a] = cmk(0.0, 0.0);
  v[0] = cmk(1.0, 0.0);
  double q = q_all;
  int64_t idx = 0;
  for (int t = 0; t < n; ++t) {
    const int pa = pad4(rk[t]), pb = pad4(rk[t + 1]);
    const double ut = U[(int64_t)t * R];
    const double2 *Y = Yg + (int64_t)t * 2 * RS * RS;
    const double2 *E = Eg + (int64_t)(t + 1) * RS * RS;
    row_times_core<RM>(v, Y, pa, pb, 0, w);
    const double q0 = quad_form<RM>(w, E, pb);
    const bool one = ut * q >= q0;
    q = q0;
    if (one) {
      row_times_core<RM>(v, Y, pa, pb, 1, w);
      q = quad_form<RM>(w, E, pb);
      idx |= (int64_t)1 << t;
    }
#pragma unroll
    for (int a = 0; a < RM; ++a) v[a] = w[a];
  }
  out[(int64_t)b * R + s] = idx;
}

// slot edge: the bond bound rounded up to a multiple of 4 (the padded blocks fit)
int env_rs(int cap_rank) { return pad4(cap_rank < SMP_RS ? cap_rank : SMP_RS); }

}  // namespace

// environments (n_max + 1) RS^2 plus padded FP64 cores 2 n_max RS^2 per instance
extern "C" size_t cm_sample_ws_bytes(int batch, int n_max, int cap_rank) {
  const int RS = env_rs(cap_rank);
  return (size_t)batch * (size_t)(3 * n_max + 1) * RS * RS * sizeof(double2);
}

extern "C" cm_status cm_sample_outcomes(const cm_tt_batch *y, const double *uniforms, int R, int64_t *out,
                                        double *norm2, int32_t *status, void *ws, size_t ws_bytes, void *stream) {
  if (!y || !norm2 || R < 0) return CM_E_INVALID;
  if (y->d_out != 2 || y->d_in != 1 || y->batch < 0) return CM_E_INVALID;
  if (y->dtype != CM_C64 && y->dtype != CM_C128) return CM_E_INVALID;
  if (y->cap_rank < 1 || y->cap_rank > 256 || y->n_max < 1 || y->n_max > CM_MAX_N) return CM_E_INVALID;
  if (y->batch == 0) return CM_OK;
  if (y->batch > 65535) return CM_E_UNSUPPORTED;
  if (R > 0 && (!uniforms || !out)) return CM_E_INVALID;
  const int RS = env_rs(y->cap_rank);
  const int64_t inst_stride = (int64_t)(3 * y->n_max + 1) * RS * RS;
  if (!ws || ws_bytes < cm_sample_ws_bytes(y->batch, y->n_max, y->cap_rank)) return CM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  TTView v = tt_view(y);
  double2 *slab = (double2 *)ws;
  const int nm = y->n_max;
  const size_t env_lds = (size_t)6 * RS * RS * sizeof(double2);
  if (y->dtype == CM_C64) {
    CM_HIP_CHECK(cm_allow_lds(k_envs<float2>, env_lds));
    hipLaunchKernelGGL(k_envs<float2>, dim3((unsigned)y->batch), dim3(SMP_WG), env_lds, s, v, RS, nm, inst_stride,
                       slab, norm2, status);
  } else {
    CM_HIP_CHECK(cm_allow_lds(k_envs<double2>, env_lds));
    hipLaunchKernelGGL(k_envs<double2>, dim3((unsigned)y->batch), dim3(SMP_WG), env_lds, s, v, RS, nm, inst_stride,
                       slab, norm2, status);
  }
  CM_LAUNCH_CHECK();
  if (R == 0) return CM_OK;
  const dim3 grid((unsigned)((R + SMP_WG - 1) / SMP_WG), (unsigned)y->batch);
  const int us = y->n_max;
#define CM_SAMPLE_LAUNCH(RM, LO)                                                                         \
  hipLaunchKernelGGL((k_sample<RM>), grid, dim3(SMP_WG), 0, s, v, slab, RS, nm, inst_stride, norm2, uniforms, us, R, \
                     out, LO)
  CM_SAMPLE_LAUNCH(8, 0);
  if (y->cap_rank > 8) CM_SAMPLE_LAUNCH(16, 8);
  if (y->cap_rank > 16) CM_SAMPLE_LAUNCH(32, 16);
#undef CM_SAMPLE_LAUNCH
  CM_LAUNCH_CHECK();
  return CM_OK;
}
