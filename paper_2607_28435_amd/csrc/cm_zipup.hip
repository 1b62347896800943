// cm_sfft_apply: y = Q_n x by a left-to-right zip-up (Section 3.2-3.3; cost per site
// O(chi w r (r' + w' chi)) plus an FP64 factorisation, linear in n as in Eq. complexity_TTO).
//
// Site l receives the carry C[chi][w][r] (the already-truncated left part of y, contracted
// with the open operator bond w and input bond r), forms
//   T[chi][u][w'][r'] = sum_{w, j, r} C[chi][w][r] A_l[r][j][r'] W_l[w][u][j][w'],
// and factors T as a (2 chi) x (w' r') matrix: T ~= U_k B with orthonormal U_k (the output
// core) and B the next carry. Truncation keeps the smallest k whose discarded singular
// values have squared sum <= tol^2 ||x||^2 / (n-1). With both operator and input in
// right-canonical form the right environment is close to orthonormal, so this per-step
// truncation is accurate; a following cm_tt_round makes the ranks optimal.
// The contraction runs in the storage precision (FP32 complex for CM_C64); the
// Householder QR and Jacobi SVD run in FP64.
#include "cm_tt.h"

namespace {

constexpr int ZCHI = 32;   // zip-up bond limit (Jacobi size 2*ZCHI <= 64)
constexpr int ZW = 24;     // largest operator bond supported by the workspace layout

__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline size_t zip_mat_cap(int cap) {
  const int chi = cap < ZCHI ? cap : ZCHI;
  return (size_t)2 * chi * ZW * cap;
}

__host__ __device__ inline size_t zip_slab_bytes(int cap, size_t *parts) {
  const size_t mc = zip_mat_cap(cap);
  size_t o = 0;
  parts[0] = o; o += al256(sizeof(double2) * mc);   // carry C
  parts[1] = o; o += al256(sizeof(double2) * mc);   // D (storage type, sized for FP64)
  parts[2] = o; o += al256(sizeof(double2) * mc);   // Y
  parts[3] = o; o += al256(sizeof(double2) * mc);   // X
  parts[4] = o; o += al256(sizeof(double2) * mc);   // Z
  parts[5] = o; o += al256(sizeof(double2) * mc);   // L
  parts[6] = o; o += al256(sizeof(double2) * mc);   // R
  return o;
}

template <typename T> struct acc_t;
template <> struct acc_t<float2> {
  using type = float2;
  __device__ __forceinline__ static float2 zero() { return make_float2(0.f, 0.f); }
  __device__ __forceinline__ static void fma_(float2 &a, float2 b, float2 c) { ffma(a, b, c); }
  __device__ __forceinline__ static float2 from(double2 v) { return make_float2((float)v.x, (float)v.y); }
  __device__ __forceinline__ static double2 to(float2 v) { return cmk(v.x, v.y); }
};
template <> struct acc_t<double2> {
  using type = double2;
  __device__ __forceinline__ static double2 zero() { return cmk(0.0, 0.0); }
  __device__ __forceinline__ static void fma_(double2 &a, double2 b, double2 c) { cfma(a, b, c); }
  __device__ __forceinline__ static double2 from(double2 v) { return v; }
  __device__ __forceinline__ static double2 to(double2 v) { return v; }
};

}  // namespace

template <typename T>
__global__ __launch_bounds__(CM_WG) void k_zipup(TTView w, TTView x, TTView y, double tol, int cap,
                                                 int batch, int32_t *__restrict__ status,
                                                 char *__restrict__ ws, size_t slab_bytes, int64_t mat_cap) {
  using A = acc_t<T>;
  extern __shared__ double2 dyn[];
  __shared__ la::Sh sh;
  __shared__ int code_sh;
  __shared__ double xn2_sh;
  const int tid = threadIdx.x;
  double2 *S = dyn, *J = dyn + 64 * 64;
  size_t parts[7];
  zip_slab_bytes(cap, parts);
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  double2 *C = (double2 *)(slab + parts[0]);
  T *D = (T *)(slab + parts[1]);
  double2 *Y = (double2 *)(slab + parts[2]);
  double2 *X = (double2 *)(slab + parts[3]);
  double2 *Z = (double2 *)(slab + parts[4]);
  double2 *Lm = (double2 *)(slab + parts[5]);
  double2 *Rm = (double2 *)(slab + parts[6]);
  const int chicap = cap < ZCHI ? cap : ZCHI;
  const T *Wc = (const T *)w.cores;
  const T *Xc = (const T *)x.cores;
  T *Yc = (T *)y.cores;

  for (int b = blockIdx.x; b < batch; b += gridDim.x) {
    const int n = x.n[b];
    if (tid == 0) {
      int c = CM_OK;
      if (n < 1 || n > CM_MAX_N || y.n[b] != n || w.n[n] != n) c = CM_E_INVALID;
      code_sh = c;
    }
    __syncthreads();
    if (code_sh != CM_OK) {
      if (tid == 0 && status) status[b] = code_sh;
      __syncthreads();
      continue;
    }
    const int32_t *wr = w.rk(n);
    const int32_t *xr = x.rk(b);
    // ||x|| from core 0 (x is right-canonical)
    {
      const int cnt = 2 * xr[1];
      double part = 0.0;
      for (int e = tid; e < cnt; e += CM_WG) part += cabs2(cstore<T>::ld(Xc, x.coff(b, 0) + e));
      const double s2 = la::wg_sum(part, sh.red);
      if (tid == 0) xn2_sh = s2;
      __syncthreads();
    }
    const double delta2 = (n > 1) ? tol * tol * xn2_sh / (double)(n - 1) : 0.0;
    if (tid == 0) { C[0] = cmk(1.0, 0.0); y.rk(b)[0] = 1; }
    __syncthreads();
    int chi = 1;
    for (int l = 0; l < n; ++l) {
      const int w0 = wr[l], w1 = wr[l + 1];
      const int r0 = xr[l], r1 = xr[l + 1];
      const int rows = 2 * chi, cols = w1 * r1;
      if ((int64_t)chi * w0 * 2 * r1 > mat_cap || (int64_t)rows * cols > mat_cap || w0 > ZW || w1 > ZW) {
        if (tid == 0) code_sh = CM_E_RANKCAP;
        __syncthreads();
        break;
      }
      const T *Wl = Wc + w.coff(n, l);   // [w0][2 u][2 j][w1]
      const T *Al = Xc + x.coff(b, l);   // [r0][2 j][r1]
      // D[chi][w0][j][r1] = sum_r C[chi][w0][r] A[r][j][r1]  (C row-major [chi][w0][r0])
      for (int e = tid; e < chi * w0 * 2 * r1; e += CM_WG) {
        const int rp = e % r1, j = (e / r1) & 1, ww = (e / (2 * r1)) % w0, ch = e / (2 * r1 * w0);
        typename A::type acc = A::zero();
        const double2 *crow = C + ((int64_t)ch * w0 + ww) * r0;
        for (int r = 0; r < r0; ++r) A::fma_(acc, A::from(crow[r]), Al[((int64_t)r * 2 + j) * r1 + rp]);
        D[e] = acc;
      }
      __syncthreads();
      // T[chi][u][w1][r1] = sum_{w0, j} D[chi][w0][j][r1] W[w0][u][j][w1]
      T *Yout = Yc + y.coff(b, l);
      const bool last = (l == n - 1);
      for (int e = tid; e < rows * cols; e += CM_WG) {
        const int rp = e % r1, wp = (e / r1) % w1, u = (e / cols) & 1, ch = e / (2 * cols);
        typename A::type acc = A::zero();
        for (int ww = 0; ww < w0; ++ww) {
          const T *dd = D + (((int64_t)ch * w0 + ww) * 2) * r1 + rp;
          const T *wl = Wl + (((int64_t)ww * 2 + u) * 2) * w1 + wp;
          A::fma_(acc, dd[0], wl[0]);
          A::fma_(acc, dd[r1], wl[w1]);
        }
        const double2 tv = A::to(acc);
        if (last) {
          // cols == 1: output core (chi x 2 x 1)
          cstore<T>::st(Yout, (int64_t)ch * 2 + u, tv);
        } else {
          // Y = T^H as (cols x rows), column-major ld cols
          const int row = ch * 2 + u, col = wp * r1 + rp;
          Y[col + (int64_t)cols * row] = cconj(tv);
        }
      }
      __syncthreads();
      if (last) {
        if (tid == 0) { y.rk(b)[l] = chi; y.rk(b)[l + 1] = 1; }
        __syncthreads();
        break;
      }
      // Y (cols x rows) ~= L Rk ; T ~= Rk^H L^H
      const int k = la::svd_trunc_rows(Y, cols, rows, delta2, chicap, X, Z, S, J, Lm, Rm, sh);
      merge_flags(sh, &code_sh);
      // output core l = Rk^H : (rows x k) as [chi][u][k]
      for (int e = tid; e < rows * k; e += CM_WG) {
        const int i = e % k, row = e / k;
        cstore<T>::st(Yout, (int64_t)row * k + i, cconj(Rm[i + (int64_t)k * row]));
      }
      // next carry C[k][w1][r1] = L^H  (L is cols x k, ld cols)
      for (int e = tid; e < k * cols; e += CM_WG) {
        const int col = e % cols, i = e / cols;
        C[(int64_t)i * cols + col] = cconj(Lm[col + (int64_t)cols * i]);
      }
      if (tid == 0) y.rk(b)[l + 1] = k;
      __syncthreads();
      chi = k;
    }
    if (tid == 0 && status) status[b] = code_sh;
    __syncthreads();
  }
}

extern "C" size_t cm_zip_slab_bytes(int cap) {
  size_t parts[7];
  return zip_slab_bytes(cap, parts);
}

extern "C" int cm_slots_for(int batch);

extern "C" cm_status cm_sfft_apply(const cm_tt_batch *w_by_n, const cm_tt_batch *x, double tol, int cap_rank,
                                   cm_tt_batch *y, int32_t *status, void *ws, size_t ws_bytes, void *stream) {
  if (!w_by_n || !x || !y || !(tol > 0.0) || cap_rank < 1 || cap_rank > 64) return CM_E_INVALID;
  if (x->batch < 0 || y->batch < x->batch) return CM_E_INVALID;
  if (x->batch == 0) return CM_OK;
  if (w_by_n->d_out != 2 || w_by_n->d_in != 2 || x->d_out != 2 || x->d_in != 1 || y->d_out != 2 || y->d_in != 1)
    return CM_E_INVALID;
  if (w_by_n->dtype != x->dtype || y->dtype != x->dtype) return CM_E_INVALID;
  if (x->dtype != CM_C64 && x->dtype != CM_C128) return CM_E_INVALID;
  if (w_by_n->batch <= x->n_max || x->cap_rank > cap_rank || cap_rank > y->cap_rank) return CM_E_INVALID;
  if (w_by_n->rank_max > ZW) return CM_E_UNSUPPORTED;
  const int batch = x->batch;
  const size_t need = cm_workspace_bytes(CM_OP_SFFT_APPLY, batch, x->n_max, cap_rank, x->dtype);
  if (!ws || ws_bytes < need) return CM_E_INVALID;
  const int slots = cm_slots_for(batch);
  const size_t slab = cm_zip_slab_bytes(cap_rank);
  const int64_t mc = (int64_t)zip_mat_cap(cap_rank);
  const size_t lds = sizeof(double2) * 2 * 64 * 64;
  hipStream_t s = (hipStream_t)stream;
  TTView vw = tt_view(w_by_n), vx = tt_view(x), vy = tt_view(y);
  CM_HIP_CHECK(cm_allow_lds(k_zipup<float2>, lds));
  CM_HIP_CHECK(cm_allow_lds(k_zipup<double2>, lds));
  if (x->dtype == CM_C64)
    hipLaunchKernelGGL(k_zipup<float2>, dim3(slots), dim3(CM_WG), lds, s, vw, vx, vy, tol, cap_rank, batch, status,
                       (char *)ws, slab, mc);
  else
    hipLaunchKernelGGL(k_zipup<double2>, dim3(slots), dim3(CM_WG), lds, s, vw, vx, vy, tol, cap_rank, batch, status,
                       (char *)ws, slab, mc);
  CM_LAUNCH_CHECK();
  return CM_OK;
}
