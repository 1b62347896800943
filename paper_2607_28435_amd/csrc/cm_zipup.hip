// cm_sfft_apply: y = Q_n x by a left-to-right zip-up (Section 3.2-3.3; cost per site
// O(chi w r (r' + w' chi)) for the contraction plus an FP64 factorisation, linear in n as in
// Eq. complexity_TTO).
//
// Site l receives the carry C[chi][w][r] (the already-truncated left part of y, contracted
// with the open operator bond w and input bond r), forms
//   T[(chi, u)][(w', r')] = sum_{w, j, r} C[chi][w][r] A_l[r][j][r'] W_l[w][u][j][w'],
// and factors the (2 chi) x (w' r') matrix T by Householder QR with column pivoting,
// stopping as soon as the dropped block's Frobenius norm is below tol ||x|| / sqrt(n-1).
// Q (orthonormal) is the output core, R P^T the next carry. With operator and input in
// right-canonical form the right environment is close to orthonormal, so this per-step
// truncation is accurate; the following cm_tt_round makes the ranks optimal with SVDs.
// The contraction runs in the storage precision (FP32 complex for CM_C64); the pivoted QR
// runs in FP64. Per-site matrices live in LDS when they fit (the common case), otherwise in
// the workgroup's global slab.
#include "cm_tt.h"

namespace {

constexpr int ZCHI = 32;          // zip-up bond limit
constexpr int ZW = 24;            // largest operator bond supported by the workspace layout
// LDS arena per workgroup: sized so that four 256-thread workgroups share a CU (typical sites
// fit; larger ones use the slab), which measured faster than two with a 72 KB arena.
constexpr int ZLDS = 16 * 1024;

__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// global per-workgroup slab: carry C (FP64), D (storage), and the fallback arena
__host__ __device__ inline size_t zip_mat_cap(int cap) {
  const int chi = cap < ZCHI ? cap : ZCHI;
  return (size_t)2 * chi * ZW * cap;
}
__host__ __device__ inline size_t zip_arena_bytes(int cap) {
  const int chi = cap < ZCHI ? cap : ZCHI;
  const size_t m = 2 * chi, p = (size_t)ZW * cap;
  return al256(16 * m * p) + al256(16 * m * (m < p ? m : p)) + al256(8 * p) + al256(4 * p) +
         al256(16 * (size_t)ZW * 4 * ZW) + al256(16 * (size_t)cap * 2 * cap);
}
__host__ __device__ inline size_t zip_slab_bytes(int cap, size_t *parts) {
  const size_t mc = zip_mat_cap(cap);
  size_t o = 0;
  parts[0] = o; o += al256(sizeof(double2) * mc);   // carry C
  parts[1] = o; o += al256(sizeof(double2) * mc);   // D
  parts[2] = o; o += zip_arena_bytes(cap);          // fallback arena
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

struct SiteDims {
  int chi, w0, w1, r0, r1;
};

// Arena layout for one site (byte offsets).
__host__ __device__ inline size_t site_bytes(const SiteDims &s, size_t *o) {
  const size_t m = 2 * s.chi, p = (size_t)s.w1 * s.r1;
  size_t x = 0;
  o[0] = x; x += al256(16 * m * p);                   // T (FP64)
  o[1] = x; x += al256(16 * m * (m < p ? m : p));     // Qk (FP64)
  o[2] = x; x += al256(8 * p);                        // column norms
  o[3] = x; x += al256(4 * p);                        // permutation
  o[4] = x; x += al256(16 * (size_t)s.w0 * 4 * s.w1); // operator core
  o[5] = x; x += al256(16 * (size_t)s.r0 * 2 * s.r1); // input core
  return x;
}

// One zip-up site; `arena` is LDS or global memory (the caller specialises the call so that
// LDS accesses compile to LDS instructions).
template <typename T>
__device__ __forceinline__ int zip_site(char *arena, const SiteDims &sd, const T *__restrict__ Wl,
                                        const T *__restrict__ Al, double2 *C, T *D, T *Yout, bool last,
                                        double delta2, int kcap, la::Sh &sh, int *code) {
  using A = acc_t<T>;
  const int tid = threadIdx.x;
  size_t o[6];
  site_bytes(sd, o);
  double2 *Tm = (double2 *)(arena + o[0]);
  double2 *Qk = (double2 *)(arena + o[1]);
  double *nrm = (double *)(arena + o[2]);
  int *perm = (int *)(arena + o[3]);
  T *Wc = (T *)(arena + o[4]);
  T *Ac = (T *)(arena + o[5]);
  const int chi = sd.chi, w0 = sd.w0, w1 = sd.w1, r0 = sd.r0, r1 = sd.r1;
  const int m = 2 * chi, p = w1 * r1;
  for (int e = tid; e < w0 * 4 * w1; e += CM_WG) Wc[e] = Wl[e];
  for (int e = tid; e < r0 * 2 * r1; e += CM_WG) Ac[e] = Al[e];
  __syncthreads();
  // D[chi][w0][j][r1] = sum_r C[chi][w0][r] A[r][j][r1]
  for (int e = tid; e < chi * w0 * 2 * r1; e += CM_WG) {
    const int rp = e % r1, j = (e / r1) & 1, ww = (e / (2 * r1)) % w0, ch = e / (2 * r1 * w0);
    typename A::type acc = A::zero();
    const double2 *crow = C + ((int64_t)ch * w0 + ww) * r0;
    for (int r = 0; r < r0; ++r) A::fma_(acc, A::from(crow[r]), Ac[(r * 2 + j) * r1 + rp]);
    D[e] = acc;
  }
  __syncthreads();
  // T[(ch, u)][(wp, rp)] = sum_{w0, j} D[ch][w0][j][rp] W[w0][u][j][wp]
  for (int e = tid; e < m * p; e += CM_WG) {
    const int row = e % m, col = e / m;
    const int ch = row >> 1, u = row & 1, wp = col / r1, rp = col % r1;
    typename A::type acc = A::zero();
    const T *dd = D + ((int64_t)ch * w0 * 2) * r1 + rp;
    const T *wl = Wc + (u * 2) * w1 + wp;
    for (int ww = 0; ww < w0; ++ww) {
      A::fma_(acc, dd[(ww * 2) * r1], wl[(ww * 4) * w1]);
      A::fma_(acc, dd[(ww * 2 + 1) * r1], wl[(ww * 4 + 1) * w1]);
    }
    Tm[e] = A::to(acc);
  }
  __syncthreads();
  if (last) {
    // p == 1: output core (chi x 2 x 1)
    for (int e = tid; e < m; e += CM_WG) cstore<T>::st(Yout, e, Tm[e]);
    __syncthreads();
    return 1;
  }
  // pivoted QR; B = R P^T (k x p, column-major ld k) lands in C
  const int k = la::cpqr_trunc(Tm, m, p, delta2, kcap, Qk, C, nrm, perm, sh);
  if (tid == 0) {
    if (sh.rankcap && *code == CM_OK) *code = CM_E_RANKCAP;
    if (sh.nonfinite && *code == CM_OK) *code = CM_E_NONFINITE;
  }
  // output core l = Qk as [chi][u][k]
  for (int e = tid; e < m * k; e += CM_WG) {
    const int row = e % m, i = e / m;
    cstore<T>::st(Yout, (int64_t)row * k + i, Qk[row + (int64_t)m * i]);
  }
  // carry for the next site as row-major [k][w1][r1]: transpose B through the (now free) T
  for (int e = tid; e < k * p; e += CM_WG) Tm[e] = C[e];
  __syncthreads();
  for (int e = tid; e < k * p; e += CM_WG) {
    const int i = e / p, col = e % p;
    C[e] = Tm[i + (int64_t)k * col];
  }
  __syncthreads();
  return k;
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(CM_WG) void k_zipup(TTView w, TTView x, TTView y, double tol, int cap,
                                                 int batch, int32_t *__restrict__ status,
                                                 char *__restrict__ ws, size_t slab_bytes, int64_t mat_cap) {
  extern __shared__ __align__(16) char lds_arena[];
  __shared__ la::Sh sh;
  __shared__ int code_sh;
  __shared__ double xn2_sh;
  const int tid = threadIdx.x;
  size_t parts[3];
  zip_slab_bytes(cap, parts);
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  double2 *C = (double2 *)(slab + parts[0]);
  T *D = (T *)(slab + parts[1]);
  char *garena = slab + parts[2];
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
      SiteDims sd;
      sd.chi = chi; sd.w0 = wr[l]; sd.w1 = wr[l + 1]; sd.r0 = xr[l]; sd.r1 = xr[l + 1];
      const int m = 2 * chi, p = sd.w1 * sd.r1;
      if ((int64_t)chi * sd.w0 * 2 * sd.r1 > mat_cap || (int64_t)m * p > mat_cap || sd.w0 > ZW || sd.w1 > ZW ||
          sd.r0 > cap || sd.r1 > cap) {
        if (tid == 0) code_sh = CM_E_RANKCAP;
        __syncthreads();
        break;
      }
      size_t o[6];
      const size_t need = site_bytes(sd, o);
      const bool last = (l == n - 1);
      const T *Wl = Wc + w.coff(n, l);
      const T *Al = Xc + x.coff(b, l);
      T *Yout = Yc + y.coff(b, l);
      int k;
      if (need <= (size_t)ZLDS)
        k = zip_site<T>(lds_arena, sd, Wl, Al, C, D, Yout, last, delta2, chicap, sh, &code_sh);
      else
        k = zip_site<T>(garena, sd, Wl, Al, C, D, Yout, last, delta2, chicap, sh, &code_sh);
      if (tid == 0) {
        if (last) { y.rk(b)[l] = chi; y.rk(b)[l + 1] = 1; }
        else y.rk(b)[l + 1] = k;
      }
      __syncthreads();
      if (last) break;
      chi = k;
    }
    if (tid == 0 && status) status[b] = code_sh;
    __syncthreads();
  }
}

extern "C" size_t cm_zip_slab_bytes(int cap) {
  size_t parts[3];
  return zip_slab_bytes(cap, parts);
}

extern "C" int cm_slots_for_ws(int op, int batch, int n_max, int cap_rank, int dtype, size_t ws_bytes);

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
  // one workgroup per workspace slab (cm_workspace_bytes gives the default count)
  const int slots = cm_slots_for_ws(CM_OP_SFFT_APPLY, batch, x->n_max, cap_rank, x->dtype, ws ? ws_bytes : 0);
  if (slots < 1) return CM_E_INVALID;
  const size_t slab = cm_zip_slab_bytes(cap_rank);
  const int64_t mc = (int64_t)zip_mat_cap(cap_rank);
  const size_t lds = ZLDS;
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
  y->flags = CM_TT_LEFT_ORTHO;
  return CM_OK;
}
