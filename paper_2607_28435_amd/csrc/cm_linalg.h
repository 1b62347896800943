// Workgroup-cooperative FP64 complex factorisations for the tensor-train sweeps.
//
// Every routine here is called by all CM_WG threads of a workgroup and contains
// __syncthreads(); arguments must be uniform across the workgroup. Matrices in global
// scratch are column-major (A[i + lda*j]); the Jacobi working pair (S, J) lives in LDS.
//
// The truncated SVD is QR-preconditioned one-sided Jacobi (Hestenes): Householder QR of
// the tall orientation, then Jacobi rotations on the small square factor, with the
// column pairs of one round (circle-method ordering) handled by disjoint lane groups.
#pragma once
#include <type_traits>

#include "cm_internal.h"

namespace la {

// 1/a and 1/sqrt(a) from the hardware approximations refined by two Newton steps each
// (relative error a few ulp; a > 0 finite).
__device__ __forceinline__ double rcp_nr(double a) {
  double y = __builtin_amdgcn_rcp(a);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-a, y, 1.0), y);
  return y;
}
__device__ __forceinline__ double rsq_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-0.5 * a * y, y, 0.5), y);   // y (3 - a y^2) / 2
  return y;
}

__device__ __forceinline__ int pow2floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// Cross-lane moves inside rows of 16 lanes (DPP, no LDS traffic): quad_perm [1,0,3,2] and
// [2,3,0,1], row_half_mirror and row_mirror. In an aligned group of 2, 4, 8 or 16 lanes each
// step pairs every lane with one holding the complementary partial result, so after
// log2(G) steps every lane of the group holds the same (bit-identical) reduction.
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

// Every lane has a valid source lane under these four controls, so no lane keeps an old value
// and the move needs no copy of its source in front of it.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Exchanges across rows of 16 lanes and across halves of the wave with the lane swaps
// (VALU, no LDS round trip). Swapping a value with itself leaves, at every lane, the value of
// the lower member of its pair (lane l and l ^ W) in `lo` and the upper member's in `hi`, so a
// symmetric combination of lo and hi is bit-identical on both lanes of a pair.
template <int W>
__device__ __forceinline__ void swap_pair_i(int v, int &lo, int &hi) {
  static_assert(W == 16 || W == 32, "lane swap width");
  if constexpr (W == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    lo = r[0]; hi = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    lo = r[0]; hi = r[1];
  }
}
template <int W>
__device__ __forceinline__ void swap_pair_d(double v, double &lo, double &hi) {
  int l0, h0, l1, h1;
  swap_pair_i<W>(__double2loint(v), l0, h0);
  swap_pair_i<W>(__double2hiint(v), l1, h1);
  lo = __hiloint2double(l1, l0);
  hi = __hiloint2double(h1, h0);
}

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of the wave must
// take part.
__device__ __forceinline__ double grp_sum(double v, int G) {
  if (G >= 2) v += dpp_d<DPP_XOR1>(v);
  if (G >= 4) v += dpp_d<DPP_XOR2>(v);
  if (G >= 8) v += dpp_d<DPP_HALF_MIRROR>(v);
  if (G >= 16) v += dpp_d<DPP_MIRROR>(v);
  if (G >= 32) { double a, b; swap_pair_d<16>(v, a, b); v = a + b; }
  if (G >= 64) { double a, b; swap_pair_d<32>(v, a, b); v = a + b; }
  return v;
}

// grp_sum of several values at once: every stage moves all of them before the next, so that
// their dependent chains overlap (and a run-time G costs one test per stage, not per value).
template <int N>
__device__ __forceinline__ void grp_sum_n(double (&v)[N], int G) {
  auto dpp_stage = [&](auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    double t[N];
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = dpp_d<C>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += t[i];
  };
  auto swap_stage = [&](auto wc) {
    constexpr int W = decltype(wc)::value;
    double a[N], b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) swap_pair_d<W>(v[i], a[i], b[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = a[i] + b[i];
  };
  if (G >= 2) dpp_stage(std::integral_constant<int, DPP_XOR1>{});
  if (G >= 4) dpp_stage(std::integral_constant<int, DPP_XOR2>{});
  if (G >= 8) dpp_stage(std::integral_constant<int, DPP_HALF_MIRROR>{});
  if (G >= 16) dpp_stage(std::integral_constant<int, DPP_MIRROR>{});
  if (G >= 32) swap_stage(std::integral_constant<int, 16>{});
  if (G >= 64) swap_stage(std::integral_constant<int, 32>{});
}
__device__ __forceinline__ void grp_sum2(double &x, double &y, int G) {
  double v[2] = {x, y};
  grp_sum_n(v, G);
  x = v[0]; y = v[1];
}

// Maximum over the 64 lanes of a wave; every lane must take part.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<DPP_XOR1>(v));
  v = fmax(v, dpp_d<DPP_XOR2>(v));
  v = fmax(v, dpp_d<DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp_d<DPP_MIRROR>(v));
  double a, b;
  swap_pair_d<16>(v, a, b);
  v = fmax(a, b);
  swap_pair_d<32>(v, a, b);
  return fmax(a, b);
}

// Over the 64 lanes of a wave: the largest `best` (ties to the smaller index `bi`) and the
// sum of `sum`; every lane must take part and ends with the same result.
template <int CTRL>
__device__ __forceinline__ void argmax_sum_step(double &best, int &bi, double &sum) {
  const double ob = dpp_d<CTRL>(best);
  const int oi = dpp_i<CTRL>(bi);
  sum += dpp_d<CTRL>(sum);
  if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
}
__device__ __forceinline__ void wave_argmax_sum(double &best, int &bi, double &sum) {
  argmax_sum_step<DPP_XOR1>(best, bi, sum);
  argmax_sum_step<DPP_XOR2>(best, bi, sum);
  argmax_sum_step<DPP_HALF_MIRROR>(best, bi, sum);
  argmax_sum_step<DPP_MIRROR>(best, bi, sum);
  // across rows, then halves: both members of a pair combine the same (lower, upper) values
  auto cross = [&](auto wc) {
    constexpr int W = decltype(wc)::value;
    double b0, b1, s0, s1;
    int i0, i1;
    swap_pair_d<W>(best, b0, b1);
    swap_pair_i<W>(bi, i0, i1);
    swap_pair_d<W>(sum, s0, s1);
    sum = s0 + s1;
    const bool up = b1 > b0 || (b1 == b0 && i1 < i0);
    best = up ? b1 : b0;
    bi = up ? i1 : i0;
  };
  cross(std::integral_constant<int, 16>{});
  cross(std::integral_constant<int, 32>{});
}

// Block-wide sum; `red` = LDS scratch of at least CM_WG/64 + 1 doubles. Includes syncs.
__device__ __forceinline__ double wg_sum(double v, double *red) {
  v = grp_sum(v, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < CM_WG / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Lane-group size (a power of two) for processing `ncols` independent columns with the whole
// workgroup.
__device__ __forceinline__ int group_for(int ncols) {
  int g = pow2floor(CM_WG / (ncols > 0 ? ncols : 1));
  return g > 64 ? 64 : (g < 1 ? 1 : g);
}

// q = n / d and r = n - q d for 0 <= n < 2^20 and 1 <= d <= 2^12 (the index decoding of the
// small matrices here): (float)n is exact and n times the hardware reciprocal of d (within an
// ulp) is within n / d * 2^-22 < 1/4 of n / d, so the truncated quotient is off by at most
// one, which one correction each way fixes. A third of the instructions of a general 32-bit
// division; d is loop-invariant in every use, so the reciprocal is taken once per loop.
__device__ __forceinline__ int divmod_small(int n, int d, int &r) {
  int q = (int)((float)n * __builtin_amdgcn_rcpf((float)d));
  r = n - q * d;
  if (r >= d) { ++q; r -= d; }
  if (r < 0) { --q; r += d; }
  return q;
}

// sum_{t < K} a[t] b[t] for a contiguous row a (storage S) and a contiguous FP64 column b:
// groups of four terms whose eight loads share one base pointer each (immediate offsets) and
// are issued together, two accumulators, then the remaining terms one by one. No masking
// inside the groups: a masked tail costs more selects than the arithmetic it guards.
template <typename S>
__device__ __forceinline__ double2 dot_contig(const S *__restrict__ a, const double2 *__restrict__ b, int K) {
  double2 s0 = cmk(0.0, 0.0), s1 = cmk(0.0, 0.0);
  int t = 0;
  for (; t + 4 <= K; t += 4) {
    double2 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = cstore<S>::ld(a, t + u);
      y[u] = b[t + u];
    }
    cfma(s0, x[0], y[0]);
    cfma(s1, x[1], y[1]);
    cfma(s0, x[2], y[2]);
    cfma(s1, x[3], y[3]);
  }
  for (; t < K; ++t) cfma(s0, cstore<S>::ld(a, t), b[t]);
  return cadd(s0, s1);
}

// sum_{t < K} a[t sa] b[t sb] for strided operands (a in storage S, b in FP64): the same
// groups of four terms with pointers advanced by whole strides, two accumulators, and the
// remainder one by one.
template <typename S>
__device__ __forceinline__ double2 dot_strided(const S *__restrict__ a, int64_t sa, const double2 *__restrict__ b,
                                               int64_t sb, int K) {
  double2 s0 = cmk(0.0, 0.0), s1 = cmk(0.0, 0.0);
  int t = 0;
  for (; t + 4 <= K; t += 4) {
    double2 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = cstore<S>::ld(a, u * sa);
      y[u] = b[u * sb];
    }
    a += 4 * sa;
    b += 4 * sb;
    cfma(s0, x[0], y[0]);
    cfma(s1, x[1], y[1]);
    cfma(s0, x[2], y[2]);
    cfma(s1, x[3], y[3]);
  }
  for (; t < K; ++t, a += sa, b += sb) cfma(s0, cstore<S>::ld(a, 0), b[0]);
  return cadd(s0, s1);
}

// Shared per-workgroup bookkeeping for the factorisations (lives in LDS).
struct Sh {
  double red[CM_WG / 64 + 2];
  int flag;
  int flag_big;
  int k;
  int rankcap;
  int nonfinite;
  int noconv;
  double err2;
  double sig2[64];
  int perm[64];
  double2 tau[64];
};

// In-place Householder QR of the first s columns of Y (m rows, ntot >= s columns,
// lda >= m, s <= min(m, 64)); the reflectors are also applied to columns s..ntot-1.
// R lies on and above the diagonal (real diagonal), reflector tails below it, tau[c] in
// sh.tau. Reflector H_c = I - tau_c v v^H with v = (0..0, 1, Y[c+1:, c]);
// Q = H_0 H_1 ... H_{s-1}.
__device__ __forceinline__ void qr_householder(double2 *Y, int lda, int m, int s, int ntot, Sh &sh) {
  const int tid = threadIdx.x;
  for (int c = 0; c < s; ++c) {
    double part = 0.0;
    for (int i = c + 1 + tid; i < m; i += CM_WG) part += cabs2(Y[i + (int64_t)lda * c]);
    const double xn2 = wg_sum(part, sh.red);
    // every thread forms the reflector from the same inputs with the same operations (no
    // barrier and LDS round trip to share it); beta replaces the diagonal once all have read it
    const double2 a = Y[c + (int64_t)lda * c];
    double2 tc = cmk(0.0, 0.0), sc = cmk(0.0, 0.0);
    double beta = 0.0;
    if (!(xn2 == 0.0 && a.y == 0.0)) {
      beta = -copysign(sqrt(a.x * a.x + a.y * a.y + xn2), a.x);
      tc = cmk((beta - a.x) / beta, -a.y / beta);
      sc = cdiv(cmk(1.0, 0.0), csub(a, cmk(beta, 0.0)));
    }
    if (tid == 0) sh.tau[c] = tc;
    if (tc.x == 0.0 && tc.y == 0.0) continue;  // uniform; the next column starts with barriers
    for (int i = c + 1 + tid; i < m; i += CM_WG) Y[i + (int64_t)lda * c] = cmul(Y[i + (int64_t)lda * c], sc);
    __syncthreads();
    if (tid == 0) Y[c + (int64_t)lda * c] = cmk(beta, 0.0);
    const int ncols = ntot - c - 1;
    if (ncols > 0) {
      const int G = group_for(ncols), lgG = __builtin_ctz(G), groups = CM_WG >> lgG;
      const int lane = tid & (G - 1);
      const double2 ctc = cconj(tc);
      for (int jb = 0; jb < ncols; jb += groups) {
        const int j = c + 1 + jb + (tid >> lgG);
        const bool ok = j < ntot;
        double2 w = cmk(0.0, 0.0);
        if (ok) {
          if (lane == 0) w = Y[c + (int64_t)lda * j];
          for (int i = c + 1 + lane; i < m; i += G) ccfma(w, Y[i + (int64_t)lda * c], Y[i + (int64_t)lda * j]);
        }
        grp_sum2(w.x, w.y, G);
        if (ok) {
          w = cmul(ctc, w);
          if (lane == 0) Y[c + (int64_t)lda * j] = csub(Y[c + (int64_t)lda * j], w);
          for (int i = c + 1 + lane; i < m; i += G) {
            double2 v = Y[i + (int64_t)lda * c];
            Y[i + (int64_t)lda * j] = csub(Y[i + (int64_t)lda * j], cmul(v, w));
          }
        }
      }
    }
    __syncthreads();
  }
}

// Z (m x k, ldz) <- Q Z with Q from qr_householder(Y, lda, m, s).
__device__ __forceinline__ void qr_apply_q(const double2 *Y, int lda, int m, int s, const Sh &sh, double2 *Z, int ldz, int k) {
  const int tid = threadIdx.x;
  const int G = group_for(k), lgG = __builtin_ctz(G), groups = CM_WG >> lgG, lane = tid & (G - 1);
  for (int c = s - 1; c >= 0; --c) {
    const double2 tc = sh.tau[c];
    if (tc.x == 0.0 && tc.y == 0.0) continue;
    for (int jb = 0; jb < k; jb += groups) {
      const int j = jb + (tid >> lgG);
      const bool ok = j < k;
      double2 w = cmk(0.0, 0.0);
      if (ok) {
        if (lane == 0) w = Z[c + (int64_t)ldz * j];
        for (int i = c + 1 + lane; i < m; i += G) ccfma(w, Y[i + (int64_t)lda * c], Z[i + (int64_t)ldz * j]);
      }
      grp_sum2(w.x, w.y, G);
      if (ok) {
        w = cmul(tc, w);
        if (lane == 0) Z[c + (int64_t)ldz * j] = csub(Z[c + (int64_t)ldz * j], w);
        for (int i = c + 1 + lane; i < m; i += G)
          Z[i + (int64_t)ldz * j] = csub(Z[i + (int64_t)ldz * j], cmul(Y[i + (int64_t)lda * c], w));
      }
    }
    __syncthreads();
  }
}

// Qk (m x k, ld m) = H_0 ... H_{k-1} [I_k; 0] from the reflector tails below the diagonal of T
// (ld m, read only) and sh.tau, without barriers: column j of Qk lives in the registers of a
// group of G lanes (lane g holding rows g, g + G, ..., NR of them; G the smallest power of two
// with G NR >= m, and at least group_for(k)), which applies the k reflectors from the last to
// the first, summing each inner product over the group with DPP; the 64 / G groups take the
// columns in passes. Needs m <= 64 NR.
template <int NR>
__device__ __forceinline__ void qr_form_q_reg(const double2 *T, int m, int k, const Sh &sh, double2 *Qk) {
  const int tid = threadIdx.x;
  int G = group_for(k);
  while (G * NR < m) G *= 2;
  const int lgG = __builtin_ctz(G), groups = CM_WG >> lgG, g = tid & (G - 1);
  for (int jb = 0; jb < k; jb += groups) {   // uniform
    const int j = jb + (tid >> lgG);
    const bool ok = j < k;   // uniform over each group
    double2 q[NR];
#pragma unroll
    for (int s = 0; s < NR; ++s) q[s] = cmk((ok && g + G * s == j) ? 1.0 : 0.0, 0.0);
    for (int c = k - 1; c >= 0; --c) {
      const double2 tc = sh.tau[c];
      if (tc.x == 0.0 && tc.y == 0.0) continue;   // uniform
      // v_r = T[r, c] below the diagonal, 1 on it, 0 above
      double2 v[NR];
      double2 w = cmk(0.0, 0.0);
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        const int r = g + G * s;
        v[s] = (r > c && r < m) ? T[r + (int64_t)m * c] : cmk(r == c ? 1.0 : 0.0, 0.0);
        ccfma(w, v[s], q[s]);
      }
      grp_sum2(w.x, w.y, G);
      w = cmul(tc, w);
#pragma unroll
      for (int s = 0; s < NR; ++s) q[s] = csub(q[s], cmul(v[s], w));
    }
    if (ok) {
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        const int r = g + G * s;
        if (r < m) Qk[r + (int64_t)m * j] = q[s];
      }
    }
  }
}

// Qk = H_0 ... H_{k-1} [I_k; 0] (see qr_form_q_reg); identity plus qr_apply_q beyond 256 rows.
__device__ __forceinline__ void qr_form_q(const double2 *T, int m, int k, const Sh &sh, double2 *Qk) {
  if (m <= CM_WG * 4) {
    qr_form_q_reg<4>(T, m, k, sh, Qk);
  } else {
    for (int e = threadIdx.x; e < m * k; e += CM_WG) {
      const int r = e % m, c = e / m;
      Qk[e] = cmk(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    qr_apply_q(T, m, m, k, sh, Qk, m, k);
  }
  __syncthreads();
}

// One-sided Jacobi on the s columns of S (m x s, column-major, ld m, in LDS; s <= 64),
// accumulating the rotations in J (s x s, LDS). On return the columns of S are mutually
// orthogonal, S_in J = S_out, and sh.sig2[i] / sh.perm[i] list squared column norms in
// descending order. Sets sh.noconv if the sweep limit was reached, sh.nonfinite on NaN/Inf.
__device__ __forceinline__ void jacobi_onesided(double2 *S, double2 *J, int m, int s, Sh &sh) {
  const int tid = threadIdx.x;
  for (int e = tid; e < s * s; e += CM_WG) {
    int i;
    const int j = divmod_small(e, s, i);
    J[e] = cmk(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) { sh.noconv = 0; sh.nonfinite = 0; }
  __syncthreads();
  const int N = s + (s & 1);
  const int npairs = N / 2;
  const int G = group_for(npairs), lgG = __builtin_ctz(G);
  const int lane = tid & (G - 1), pi = tid >> lgG;
  // A pair is rotated while its cosine |<s_p, s_q>| / (|s_p| |s_q|) exceeds 1e-13, far below
  // any truncation threshold used (singular values then carry relative errors of that
  // order). Columns below 1e-32 of the largest squared norm are numerically null and are left
  // alone; the product of two tiny norms is never formed, so nothing underflows.
  double amax_part = 0.0;
  if (tid < s) {
    double a = 0.0;
    for (int i = 0; i < m; ++i) a += cabs2(S[i + m * tid]);
    amax_part = a;
  }
  __syncthreads();
  {
    const double v = wave_max(amax_part);
    if ((tid & 63) == 0) sh.red[tid >> 6] = v;
  }
  __syncthreads();
  double amax = 0.0;
  for (int i = 0; i < CM_WG / 64; ++i) amax = fmax(amax, sh.red[i]);
  __syncthreads();
  const double null2 = 1e-32 * amax;
  const double tol = 1e-13;
  const double last_tol = 1e-8;   // see the end of the sweep loop
  const int max_sweeps = 30;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) { sh.flag = 0; sh.flag_big = 0; }
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      int p = -1, q = -1;
      if (pi < npairs && N > 1) {
        if (pi == 0) { p = N - 1; q = r; }
        else {
          // (r + pi) mod (N - 1) and (r - pi) mod (N - 1), both arguments in [0, 2 (N - 1))
          p = r + pi;
          if (p >= N - 1) p -= N - 1;
          q = r - pi + (N - 1);
          if (q >= N - 1) q -= N - 1;
        }
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= s) p = -1;
      }
      double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
      if (p >= 0) {
        for (int i = lane; i < m; i += G) {
          double2 xp = S[i + m * p], xq = S[i + m * q];
          a += cabs2(xp); b += cabs2(xq);
          gr += xp.x * xq.x + xp.y * xq.y;
          gi += xp.x * xq.y - xp.y * xq.x;
        }
      }
      {
        double r4[4] = {a, b, gr, gi};
        grp_sum_n(r4, G);
        a = r4[0]; b = r4[1]; gr = r4[2]; gi = r4[3];
      }
      if (p >= 0) {
        if (!(a == a) || !(b == b)) {
          if (lane == 0) sh.nonfinite = 1;
        } else if (a > null2 && b > null2) {
          const double ag2 = gr * gr + gi * gi;
          if (ag2 > (tol * tol) * a * b) {
            // reciprocal square roots and reciprocals refined by Newton steps keep the
            // dependent chain short (relative errors of a few ulp)
            const double rag = rsq_nr(ag2);   // 1 / |g|
            const double zeta = 0.5 * (b - a) * rag;
            const double z2 = 1.0 + zeta * zeta;
            const double sq = z2 * rsq_nr(z2);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(zeta) + sq);
            const double c = rsq_nr(1.0 + t * t);
            const double sn = c * t;
            const double2 e = cmk(gr * rag, gi * rag);
            const double2 se = cscale(e, sn);          // s e
            const double2 sce = cscale(cconj(e), sn);  // s conj(e)
            for (int i = lane; i < m; i += G) {
              double2 xp = S[i + m * p], xq = S[i + m * q];
              S[i + m * p] = csub(cscale(xp, c), cmul(sce, xq));
              S[i + m * q] = cadd(cmul(se, xp), cscale(xq, c));
            }
            for (int i = lane; i < s; i += G) {
              double2 vp = J[i + s * p], vq = J[i + s * q];
              J[i + s * p] = csub(cscale(vp, c), cmul(sce, vq));
              J[i + s * q] = cadd(cmul(se, vp), cscale(vq, c));
            }
            if (lane == 0) {
              sh.flag = 1;
              if (ag2 > (last_tol * last_tol) * a * b) sh.flag_big = 1;
            }
          }
        }
      }
      __syncthreads();
    }
    const int f = sh.flag, fb = sh.flag_big;
    __syncthreads();
    // A sweep whose rotations all had cosines below last_tol leaves off-diagonal cosines of
    // order its square (the cyclic sweeps converge quadratically), under the rotation
    // threshold: the next sweep would rotate nothing, so it is not run.
    if (f == 0 || fb == 0) break;
  }
  if (sweep == max_sweeps && tid == 0) sh.noconv = 1;
  // squared column norms and descending order
  if (tid < s) {
    double a = 0.0;
    for (int i = 0; i < m; ++i) a += cabs2(S[i + m * tid]);
    if (!(a == a) || isinf(a)) { sh.nonfinite = 1; a = 0.0; }
    sh.sig2[tid] = a;
  }
  __syncthreads();
  if (tid < s) {
    const double a = sh.sig2[tid];
    int pos = 0;
    for (int i = 0; i < s; ++i) {
      const double b2 = sh.sig2[i];
      pos += (b2 > a) || (b2 == a && i < tid);
    }
    sh.perm[pos] = tid;
  }
  __syncthreads();
  double v = 0.0;
  if (tid < s) v = sh.sig2[sh.perm[tid]];
  __syncthreads();
  if (tid < s) sh.sig2[tid] = v;
  __syncthreads();
}

// Chooses the kept rank from sh.sig2 (descending): the smallest k >= 1 whose discarded tail
// has squared norm <= delta2, then clipped to cap. Writes sh.k, sh.err2, sh.rankcap.
__device__ __forceinline__ void choose_rank_t0(Sh &sh, int s, double delta2, int cap) {
  if (threadIdx.x == 0) {
    int k = s;
    double tail = 0.0;
    while (k > 1 && tail + sh.sig2[k - 1] <= delta2) { tail += sh.sig2[k - 1]; --k; }
    int rc = 0;
    if (k > cap) {
      for (int i = cap; i < k; ++i) tail += sh.sig2[i];
      k = cap;
      rc = tail > delta2;
    }
    sh.k = k;
    sh.err2 = tail;
    sh.rankcap = rc;
  }
  __syncthreads();
}

// Thin QR: Y (m x p, ld m, destroyed) = Q Rr with Q (m x kq, orthonormal columns) and
// Rr (kq x p, upper trapezoidal), kq = min(m, p). Q -> Qout (ld m), Rr -> Rout (ld kq).
__device__ __forceinline__ int qr_thin(double2 *Y, int m, int p, double2 *Qout, double2 *Rout, Sh &sh) {
  const int tid = threadIdx.x;
  const int kq = m < p ? m : p;
  qr_householder(Y, m, m, kq, p, sh);
  // R (with trailing columns when p > m)
  for (int e = tid; e < kq * p; e += CM_WG) {
    int i;
    const int j = divmod_small(e, kq, i);
    Rout[e] = (i <= j) ? Y[i + (int64_t)m * j] : cmk(0.0, 0.0);
  }
  __syncthreads();
  qr_form_q(Y, m, kq, sh, Qout);
  return kq;
}

// Truncated column-pivoted Householder QR of T (m x p, column-major ld m, destroyed):
// T P = Q R. Columns are pivoted by largest remaining norm; the factorisation stops at the
// first k >= 1 with ||R_22||_F^2 <= delta2 (the exact squared Frobenius norm of what is
// dropped), or at k = cap (then sh.rankcap is set if the tail still exceeds delta2).
// Outputs: Qk (m x k, ld m) with orthonormal columns; the k x p factor B = R[:k,:] P^T is
// written to B (ld k). nrm (p doubles) and perm (p ints) are scratch. Returns k; sh.err2
// holds the dropped squared norm. p <= 1024.
// The remaining column norms nrm[c] (rows >= i at step i) are recomputed exactly from the
// updated entries after every reflection, so the pivot column's norm gives the reflector's
// beta without another reduction, wave 0 forms the tail sum together with the pivot search,
// and every thread forms the reflector itself: three barriers per step (four when columns
// are swapped).
__device__ __forceinline__ int cpqr_trunc(double2 *T, int m, int p, double delta2, int cap, double2 *Qk,
                                          double2 *B, double *nrm, int *perm, Sh &sh) {
  const int tid = threadIdx.x;
  const int kmax = m < p ? m : p;
  // column norms
  {
    const int G = group_for(p), lgG = __builtin_ctz(G), groups = CM_WG >> lgG, lane = tid & (G - 1);
    for (int cb = 0; cb < p; cb += groups) {
      const int c = cb + (tid >> lgG);
      double a = 0.0;
      if (c < p)
        for (int r = lane; r < m; r += G) a += cabs2(T[r + (int64_t)m * c]);
      a = grp_sum(a, G);
      if (c < p && lane == 0) { nrm[c] = a; perm[c] = c; }
    }
  }
  __shared__ double tail_sh;
  __shared__ int piv_sh;
  __shared__ int k_sh;
  if (tid == 0) { k_sh = 0; sh.rankcap = 0; sh.nonfinite = 0; tail_sh = 0.0; }
  __syncthreads();
  for (int i = 0; i < kmax; ++i) {
    // wave 0: tail = sum of the remaining norms, pivot = their argmax
    if (tid < 64) {
      double best = -1.0, sum = 0.0;
      int bi = i;
      for (int c = i + tid; c < p; c += 64) {
        const double v = nrm[c];
        sum += v;
        if (v > best) { best = v; bi = c; }
      }
      wave_argmax_sum(best, bi, sum);
      if (tid == 0) { piv_sh = bi; tail_sh = sum; }
    }
    __syncthreads();
    const double tail = tail_sh;
    if (!(tail == tail) || isinf(tail)) {
      if (tid == 0) sh.nonfinite = 1;
      break;
    }
    if (i >= 1 && tail <= delta2) break;
    if (i == cap) {
      if (tid == 0) sh.rankcap = 1;
      break;
    }
    const int pv = piv_sh;
    if (pv != i) {   // uniform
      for (int r = tid; r < m; r += CM_WG) {
        const double2 t = T[r + (int64_t)m * i];
        T[r + (int64_t)m * i] = T[r + (int64_t)m * pv];
        T[r + (int64_t)m * pv] = t;
      }
      if (tid == 0) {
        const double t = nrm[i]; nrm[i] = nrm[pv]; nrm[pv] = t;
        const int q = perm[i]; perm[i] = perm[pv]; perm[pv] = q;
      }
      __syncthreads();
    }
    // Householder reflector for T[i:m, i]; ||T[i:m, i]||^2 = nrm[i]. Every thread forms it
    // from the same inputs (reciprocal square root and reciprocal refined by Newton steps)
    // and scales its share of the column; beta replaces T[i, i] after the barrier.
    double2 tc = cmk(0.0, 0.0);
    double beta = 0.0;
    {
      const double2 a = T[i + (int64_t)m * i];
      const double norm2 = nrm[i];
      if (norm2 > 0.0) {
        const double rs = rsq_nr(norm2);
        const double sg = a.x >= 0.0 ? 1.0 : -1.0;
        beta = -sg * (norm2 * rs);
        const double ib = -sg * rs;   // 1 / beta
        const double2 am = cmk(a.x - beta, a.y);
        const double id = rcp_nr(cabs2(am));
        tc = cmk(1.0 - a.x * ib, -a.y * ib);
        const double2 sc = cmk(am.x * id, -am.y * id);
        for (int r = i + 1 + tid; r < m; r += CM_WG) T[r + (int64_t)m * i] = cmul(T[r + (int64_t)m * i], sc);
      }
    }
    if (tid == 0) { sh.tau[i] = tc; k_sh = i + 1; }
    __syncthreads();
    const bool refl = !(tc.x == 0.0 && tc.y == 0.0);
    if (refl && tid == 0) T[i + (int64_t)m * i] = cmk(beta, 0.0);
    // apply H^H to trailing columns; refresh their norms below row i
    const int ncols = p - i - 1;
    if (ncols > 0) {
      const int G = group_for(ncols), lgG = __builtin_ctz(G), groups = CM_WG >> lgG, lane = tid & (G - 1);
      const double2 ctc = cconj(tc);
      for (int jb = 0; jb < ncols; jb += groups) {
        const int j = i + 1 + jb + (tid >> lgG);
        const bool ok = j < p;
        double2 w = cmk(0.0, 0.0);
        if (ok && refl) {
          if (lane == 0) w = T[i + (int64_t)m * j];
          for (int r = i + 1 + lane; r < m; r += G) ccfma(w, T[r + (int64_t)m * i], T[r + (int64_t)m * j]);
        }
        grp_sum2(w.x, w.y, G);
        double a = 0.0;
        if (ok) {
          if (refl) {
            w = cmul(ctc, w);
            if (lane == 0) T[i + (int64_t)m * j] = csub(T[i + (int64_t)m * j], w);
          }
          for (int r = i + 1 + lane; r < m; r += G) {
            double2 v = T[r + (int64_t)m * j];
            if (refl) { v = csub(v, cmul(T[r + (int64_t)m * i], w)); T[r + (int64_t)m * j] = v; }
            a += cabs2(v);
          }
        }
        a = grp_sum(a, G);
        if (ok && lane == 0) nrm[j] = a;
      }
    }
    if (tid == 0 && i + 1 == kmax) tail_sh = 0.0;   // nothing remains below or beside
    __syncthreads();
  }
  const int k = k_sh;
  if (tid == 0) sh.err2 = tail_sh;
  // B = R[:k, :] P^T  (rows r < k; R[r, c] = 0 for r > c)
  for (int e = tid; e < k * p; e += CM_WG) {
    int r;
    const int c = divmod_small(e, k, r);
    B[r + (int64_t)k * perm[c]] = (r <= c) ? T[r + (int64_t)m * c] : cmk(0.0, 0.0);
  }
  // Qk = H_0 ... H_{k-1} [I_k; 0]
  __syncthreads();
  qr_form_q(T, m, k, sh, Qk);
  return k;
}

// Truncated factorisation Y ~= L * Rk of Y (a x b), given as X = Y^H (b x a, column-major,
// ld b; destroyed), where Rk (k x b) has orthonormal rows (the top-k right singular vectors)
// and L = Y Rk^H (a x k), a <= 64. Column-pivoted QR of X first drops a tail of squared norm
// <= delta2/2 and leaves X ~= Q B (Q: b x kc orthonormal, B: kc x a); one-sided Jacobi on the
// kc columns of B^H (ordered by decreasing norm by the pivoting, which speeds convergence)
// then yields its SVD, truncated with the rest of the budget. The kept rank k is the smallest
// whose total dropped squared norm is <= delta2, clipped to cap (sh.rankcap is set if that
// loses more).
//   X : the input, in the LDS scratch `lds` (x_lds) or in global memory
//   Y : scratch of at least a*b complex (receives B);  Z : scratch of at least a*b complex
//   S, J : at least a*min(a,b) and min(a,b)^2 complex
//   L (ld a, FP64) and R (row-major, k x b, stored as RT) : outputs, written straight to
//   where the caller keeps them (the sweep's carry and its output core).
//   lds, lds_elems : optional LDS scratch; the Jacobi pair moves there when it fits (the
//   factorisations are latency-bound chains of small steps).
// Returns k (uniform); sh.err2 holds the dropped squared norm.
template <typename RT>
__device__ __forceinline__ int svd_trunc_rows(double2 *X, bool x_lds, int a, int b, double delta2, int cap,
                                              double2 *Y, double2 *Z, double2 *S, double2 *J,
                                              double2 *L, RT *R, Sh &sh, double2 *lds = nullptr,
                                              int lds_elems = 0) {
  const int tid = threadIdx.x;
  // X P = Q R, truncated: Q -> Z (b x kc), B = R[:kc] P^T -> Y (kc x a, ld kc)
  int kc;
  if (x_lds) kc = cpqr_trunc(lds, b, a, 0.5 * delta2, 64, Z, Y, sh.sig2, sh.perm, sh);
  else kc = cpqr_trunc(X, b, a, 0.5 * delta2, 64, Z, Y, sh.sig2, sh.perm, sh);
  __syncthreads();
  const double err_c = sh.err2;
  const bool sj_lds = lds != nullptr && a * kc + kc * kc <= lds_elems;
  double2 *Sw = sj_lds ? lds : S;
  double2 *Jw = sj_lds ? lds + a * kc : J;
  // S = B^H (a x kc, ld a)
  for (int e = tid; e < a * kc; e += CM_WG) {
    int i;
    const int j = divmod_small(e, a, i);
    Sw[e] = cconj(Y[j + (int64_t)kc * i]);
  }
  __syncthreads();
  if (sj_lds) jacobi_onesided(lds, lds + a * kc, a, kc, sh);
  else jacobi_onesided(S, J, a, kc, sh);
  const double rest = delta2 - err_c;
  choose_rank_t0(sh, kc, rest > 0.0 ? rest : 0.0, cap);
  const int k = sh.k;
  // L = (B^H J)[:, perm[:k]];  Rk^H = Q J[:, perm[:k]]
  for (int e = tid; e < a * k; e += CM_WG) {
    int i;
    const int j = divmod_small(e, a, i);
    L[e] = Sw[i + (int64_t)a * sh.perm[j]];
  }
  for (int e = tid; e < k * b; e += CM_WG) {
    int c;
    const int i = divmod_small(e, b, c);   // lanes run along a row of Rk: Z reads are coalesced
    cstore<RT>::st(R, e, cconj(dot_strided(Z + c, (int64_t)b, Jw + (int64_t)kc * sh.perm[i], (int64_t)1, kc)));
  }
  __syncthreads();
  if (tid == 0) sh.err2 += err_c;
  __syncthreads();
  return k;
}

}  // namespace la
