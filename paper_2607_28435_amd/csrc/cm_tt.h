// Tensor-train sweeps shared by the library entry points: the FP64 rounding sweep
// (QR left-to-right, truncated SVD right-to-left) and exact phase reduction helpers.
#pragma once

#include "cm_linalg.h"

// ------------------------------------------------------------------ exact phases
// 1/(2 pi) as a double-double.
#define CM_INV2PI_HI 0.15915494309189535
#define CM_INV2PI_LO (-9.839338337591243e-18)
#define CM_2PI 6.283185307179586

__host__ __device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Double-double cycles c = (hi + lo) / (2 pi); returns the fractional part of c * 2^s.
__host__ __device__ __forceinline__ double cycles_frac(double hi, double lo, int s) {
#pragma clang fp contract(off)
  double ch = hi * CM_INV2PI_HI;
  double cl = fma(hi, CM_INV2PI_HI, -ch) + hi * CM_INV2PI_LO + lo * CM_INV2PI_HI;
  double sc = ldexp(1.0, s);
  return frac2(ch * sc, cl * sc);
}

// exp(i * 2 pi * f), f a fraction of a turn
__host__ __device__ __forceinline__ double2 turn(double f) {
  double sn, cs;
  sincos(CM_2PI * f, &sn, &cs);
  return cmk(cs, sn);
}

// Angle a*b (both doubles, product formed exactly) as a fraction of a turn, times 2^s.
__host__ __device__ __forceinline__ double prod_cycles_frac(double a, double b, int s) {
  double p, e;
  two_prod(a, b, p, e);
  return cycles_frac(p, e, s);
}

// Phase angle eta (ln S0 - k0 + (r - q) T) of the first frequency step as a double-double
// (hi + lo, radians), with ln S0 - k0 + (r - q) T summed error-free: on a grid centred far from
// the money k0 is ~2^(n/2), and the rounded difference would shift every strike by up to half
// its ulp (3e-11 at n = 40), moving each price by that times its slope in k.
__host__ __device__ __forceinline__ void drift_angle(double eta, double lnS0, double k0, double rq, double &hi,
                                                     double &lo) {
#pragma clang fp contract(off)
  double a, al, b, bl;
  two_sum(lnS0, -k0, a, al);
  two_sum(a, rq, b, bl);
  two_prod(eta, b, hi, lo);
  lo = fma(eta, al + bl, lo);
}

// Log-strike of grid index u, k_u = k0 + lambda u with lambda = 2 pi / (2^n eta): the strike
// that the transform's phase exp(-2 pi i j u / 2^n) pairs with u (the grid relation
// eta lambda = 2 pi / M of Section 2.1 holds exactly there). Formed from 2 pi / eta as a
// double-double, its exact product with u and exact scaling by 2^-n, and an error-free sum
// with k0, so that k_u stays within a few ulps of itself even where k0 and lambda u are large
// and cancel (on a grid centred far from the money both are ~2^(n/2); rounding lambda first
// would cost |lambda u| ulp(1), 4e-11 at n = 40, and the damping factor alpha times that).
#define CM_2PI_LO 2.4492935982947064e-16
__host__ __device__ __forceinline__ double strike_log(double k0, double eta, int n, double u) {
#pragma clang fp contract(off)
  const double c = CM_2PI / eta;
  const double cl = (fma(-c, eta, CM_2PI) + CM_2PI_LO) / eta;   // 2 pi / eta = c + cl
  double p, e;
  two_prod(c, u, p, e);
  e = fma(cl, u, e);
  p = ldexp(p, -n);
  e = ldexp(e, -n);
  double sm, t;
  two_sum(k0, p, sm, t);
  return sm + (t + e);
}

// ------------------------------------------------------------------ rounding sweep
// Per-workgroup scratch for one rounding job (FP64 complex, global memory). `tt` holds n
// cores of core_cap elements; Y, X, Z, L, R, C hold mat_cap elements each.
struct RoundScratch {
  double2 *tt;
  int64_t core_cap;
  double2 *Y, *X, *Z, *L, *R, *C;
  double2 *S, *J;  // global fallback for the Jacobi pair (64 x 64 each)
};

// Source train for the rounding sweep: core l element (t, ph, j) is at
// off[l] + (t*d + ph)*r_{l+1} + j, stored as float2 (CM_C64) or double2 (otherwise).
struct CoreSrc {
  const void *cores;
  const int64_t *off;
  const int32_t *ranks;
  int dtype;
  __device__ __forceinline__ double2 get(int l, int64_t e) const {
    if (dtype == CM_C64) return cstore<float2>::ld((const float2 *)cores, off[l] + e);
    return ((const double2 *)cores)[off[l] + e];
  }
};

// Brings two byte ranges into the caches with one memory latency: every lane loads one dword
// of up to two 128-byte lines of each range and all four values are consumed together. The
// short dependent dot products that follow then hit the L2 instead of paying one miss per
// batch of operands (with thousands of resident workgroups the sweep's working set does not
// stay in the L2 between bonds).
__device__ __forceinline__ void touch_lines(const void *p, size_t pb, const void *q, size_t qb) {
  const char *a = (const char *)p, *b = (const char *)q;
  const int la = (int)((pb + 127) >> 7), lb = (int)((qb + 127) >> 7);
  const int i0 = threadIdx.x, i1 = threadIdx.x + CM_WG;
  float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
  if (i0 < la) v0 = *(const float *)(a + ((size_t)i0 << 7));
  if (i1 < la) v1 = *(const float *)(a + ((size_t)i1 << 7));
  if (i0 < lb) v2 = *(const float *)(b + ((size_t)i0 << 7));
  if (i1 < lb) v3 = *(const float *)(b + ((size_t)i1 << 7));
  asm volatile("" ::"v"(v0), "v"(v1), "v"(v2), "v"(v3));
}

__device__ __forceinline__ void merge_flags(const la::Sh &sh, int *code) {
  if (threadIdx.x == 0) {
    if (sh.nonfinite && *code == CM_OK) *code = CM_E_NONFINITE;
    if (sh.noconv && *code == CM_OK) *code = CM_E_NOCONV;
    if (sh.rankcap && *code == CM_OK) *code = CM_E_RANKCAP;
  }
}

// Rounds a train of n cores with physical size d from `src` into dst (storage OutT, core
// offsets dst_off, ranks dst_ranks). Phase A orthogonalises left to right with thin QR;
// phase B truncates right to left with the per-bond threshold tol*||t||/sqrt(n-1) and
// bonds <= cap (cap <= 64). Afterwards cores 1..n-1 are right-orthonormal and the norm sits
// in core 0. dst may alias src (every source core is read in phase A, before phase B
// writes). Returns the relative Frobenius error bound; *code receives a cm_status (thread 0
// writes; first error wins).
template <typename OutT>
__device__ __forceinline__ double round_train(int n, int d, const CoreSrc &src, double tol, int cap,
                              OutT *dst_cores, const int64_t *dst_off, int32_t *dst_ranks,
                              const RoundScratch &w, double2 *S, double2 *J, la::Sh &sh,
                              int *code, bool skip_a = false, double2 *lds = nullptr, int lds_elems = 0) {
  const int tid = threadIdx.x;
  __shared__ int rk[CM_MAX_N + 1];
  __shared__ double norm2_sh;
  if (tid == 0) { rk[0] = 1; norm2_sh = 0.0; w.C[0] = cmk(1.0, 0.0); }
  __syncthreads();
  // ---- phase A: carry C (kprev x r_l, ld kprev), starts as [1]. Skipped when the source
  // cores 0..n-2 are already left-orthonormal; then only the norm of the last core is needed.
  if (skip_a) {
    const int rl = src.ranks[n - 1];
    double part = 0.0;
    for (int e = tid; e < rl * d; e += CM_WG) part += cabs2(src.get(n - 1, e));
    const double nrm2 = la::wg_sum(part, sh.red);
    if (tid == 0) norm2_sh = nrm2;
    for (int l = tid; l <= n; l += CM_WG) rk[l] = src.ranks[l];
    __syncthreads();
  }
  int kprev = 1;
  for (int l = 0; l < n && !skip_a; ++l) {
    const int rl = src.ranks[l], rr = src.ranks[l + 1];
    const int rows = kprev * d;
    const int kq = rows < rr ? rows : rr;
    // the product and its Q factor go to the LDS scratch when both fit (the QR is a chain of
    // small dependent steps)
    const bool in_lds = lds != nullptr && l < n - 1 && rows * rr + rows * kq <= lds_elems;
    double2 *Yw = in_lds ? lds : w.Y;
    const int64_t base = src.off[l];
    const double2 *Cg = w.C;
    // Y[(a, ph)][j] = sum_t C[a][t] core[t][ph][j]: the core's column (ph, j) has stride d rr,
    // C's row a stride kprev
    auto yform = [&](const auto *cs) {
      for (int e = tid; e < rows * rr; e += CM_WG) {
        int i, ph;
        const int j = la::divmod_small(e, rows, i);
        const int a = la::divmod_small(i, d, ph);
        Yw[e] = la::dot_strided(cs + ph * rr + j, (int64_t)d * rr, Cg + a, (int64_t)kprev, rl);
      }
    };
    if (src.dtype == CM_C64) yform((const float2 *)src.cores + base);
    else yform((const double2 *)src.cores + base);
    __syncthreads();
    double2 *core = w.tt + (int64_t)l * w.core_cap;
    if (l == n - 1) {
      double part = 0.0;
      for (int e = tid; e < rows * rr; e += CM_WG) {
        core[e] = w.Y[e];
        part += cabs2(w.Y[e]);
      }
      const double nrm2 = la::wg_sum(part, sh.red);
      if (tid == 0) { norm2_sh = nrm2; rk[l + 1] = rr; }
      __syncthreads();
      break;
    }
    if (in_lds) {
      la::qr_thin(lds, rows, rr, lds + rows * rr, w.L, sh);
      for (int e = tid; e < rows * kq; e += CM_WG) core[e] = lds[rows * rr + e];
    } else {
      la::qr_thin(w.Y, rows, rr, w.Z, w.L, sh);
      for (int e = tid; e < rows * kq; e += CM_WG) core[e] = w.Z[e];
    }
    for (int e = tid; e < kq * rr; e += CM_WG) w.C[e] = w.L[e];
    if (tid == 0) rk[l + 1] = kq;
    __syncthreads();
    kprev = kq;
  }
  const double nrm = sqrt(norm2_sh);
  if (tid == 0 && (!(nrm == nrm) || isinf(nrm)) && *code == CM_OK) *code = CM_E_NONFINITE;
  const double delta2 = (n > 1) ? (tol * nrm) * (tol * nrm) / (double)(n - 1) : 0.0;
  // ---- phase B: carry C (kr x rpp, ld kr), starts as [1]
  double err2 = 0.0;
  int rpp = 1;
  if (tid == 0) w.C[0] = cmk(1.0, 0.0);
  __syncthreads();
  for (int l = n - 1; l >= 0; --l) {
    const int kl = rk[l], kr = rk[l + 1];
    const double2 *core = w.tt + (int64_t)l * w.core_cap;  // column-major (kl*d) x kr
    const int b = d * rpp;
    const double2 *Cg = w.C;
    // X = Y^H (b x kl, ld b) with Y[i][(ph, j)] = sum_t core[i][ph][t] C[t][j], formed in the LDS
    // scratch when it fits. Lanes run over j fastest, so the lanes of a load share one core row
    // (and neighbouring lanes' rows are adjacent in memory): a few cache lines per load instead
    // of one per lane, and X is written contiguously. The source's storage type is resolved
    // once per bond so that each element's loads are issued together.
    const bool x_lds = lds != nullptr && kl * b <= lds_elems;
    double2 *Xw = x_lds ? lds : w.X;
    // the destination is resolved per call so that the LDS case stores with LDS instructions
    auto xform_to = [&](double2 *Xd, auto rowdot) {
      for (int e = tid; e < kl * b; e += CM_WG) {
        int j, ph;
        const int row = la::divmod_small(e, rpp, j);   // row = i d + ph
        const int i = la::divmod_small(row, d, ph);
        Xd[ph * rpp + j + b * i] = cconj(rowdot(row, Cg + kr * j));
      }
    };
    auto xform = [&](auto rowdot) {
      if (x_lds) xform_to(lds, rowdot);
      else xform_to(w.X, rowdot);
    };
    if (skip_a) {
      const int64_t base = src.off[l];
      const size_t esz = src.dtype == CM_C64 ? sizeof(float2) : sizeof(double2);
      touch_lines((const char *)src.cores + esz * base, esz * (size_t)kl * d * kr, Cg, sizeof(double2) * (size_t)kr * rpp);
      // source cores are row-major [row][t]: contiguous rows
      if (src.dtype == CM_C64) {
        const float2 *cs = (const float2 *)src.cores + base;
        xform([&](int row, const double2 *cj) { return la::dot_contig(cs + row * kr, cj, kr); });
      } else {
        const double2 *cs = (const double2 *)src.cores + base;
        xform([&](int row, const double2 *cj) { return la::dot_contig(cs + row * kr, cj, kr); });
      }
    } else {
      const int64_t ld = (int64_t)kl * d;
      touch_lines(core, sizeof(double2) * (size_t)ld * kr, Cg, sizeof(double2) * (size_t)kr * rpp);
      xform([&](int row, const double2 *cj) { return la::dot_strided(core + row, ld, cj, (int64_t)1, kr); });
    }
    __syncthreads();
    OutT *out = dst_cores + dst_off[l];
    if (l == 0) {
      // kl == 1; core 0 = Y (1 x d*rpp), element (0, ph, j) at ph*rpp + j == column index
      for (int e = tid; e < b; e += CM_WG) cstore<OutT>::st(out, e, cconj(Xw[e]));
      if (tid == 0) { dst_ranks[0] = 1; dst_ranks[1] = rpp; }
      __syncthreads();
      break;
    }
    // core l = Rk (k x b, row-major, the element order of [k][d][rpp]) goes straight to the
    // output (the source core l was read in full into X above, so in-place rounding is safe)
    // and the carry L (kl x k, ld kl) straight to C (read only by the product above)
    const int k = la::svd_trunc_rows(Xw, x_lds, kl, b, delta2, cap, w.Y, w.Z, S, J, w.C, out, sh, lds, lds_elems);
    merge_flags(sh, code);
    err2 += sh.err2;
    if (tid == 0) { dst_ranks[l + 1] = rpp; }
    __syncthreads();
    rpp = k;
  }
  if (tid == 0) dst_ranks[n] = 1;
  __syncthreads();
  return sqrt(err2) / (nrm > 0 ? nrm : 1.0);
}

// round_train with the hot matrices (Y, X, Z and the Jacobi pair) in the LDS arena when the
// train's largest bond allows it, and in the global scratch otherwise (then the pivoted QR
// input and the Jacobi pair of each bond still move to the arena when they fit).
template <typename OutT>
__device__ __forceinline__ double round_train_auto(int n, int d, const CoreSrc &src, double tol, int cap,
                                                   OutT *dst_cores, const int64_t *dst_off, int32_t *dst_ranks,
                                                   const RoundScratch &wg, char *arena, size_t arena_bytes,
                                                   la::Sh &sh, int *code, bool skip_a = false) {
  __shared__ int rmax_sh;
  if (threadIdx.x == 0) {
    int r = 1;
    for (int l = 0; l <= n; ++l) r = src.ranks[l] > r ? src.ranks[l] : r;
    rmax_sh = r;
  }
  __syncthreads();
  const int64_t rmax = rmax_sh;
  const int64_t mat = rmax * d * rmax;
  const size_t need = sizeof(double2) * (size_t)(3 * mat + 3 * rmax * rmax);
  if (need <= arena_bytes && rmax <= 64) {
    RoundScratch w = wg;
    w.Y = (double2 *)arena;
    w.X = w.Y + mat;
    w.Z = w.X + mat;
    double2 *S = w.Z + mat;
    double2 *J = S + rmax * rmax;
    w.C = J + rmax * rmax;
    return round_train<OutT>(n, d, src, tol, cap, dst_cores, dst_off, dst_ranks, w, S, J, sh, code, skip_a);
  }
  // matrices in global scratch; the SVD steps still use the arena for whatever fits per bond
  return round_train<OutT>(n, d, src, tol, cap, dst_cores, dst_off, dst_ranks, wg, wg.S, wg.J, sh, code, skip_a,
                           (double2 *)arena, (int)(arena_bytes / sizeof(double2)));
}
