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

#include "cm_internal.h"

namespace la {

__device__ __forceinline__ int pow2floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

__device__ __forceinline__ double grp_sum(double v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
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

// Lane-group size for processing `ncols` independent columns with the whole workgroup.
__device__ __forceinline__ int group_for(int ncols) {
  int g = pow2floor(CM_WG / (ncols > 0 ? ncols : 1));
  return g > 64 ? 64 : (g < 1 ? 1 : g);
}

// Shared per-workgroup bookkeeping for the factorisations (lives in LDS).
struct Sh {
  double red[CM_WG / 64 + 2];
  double2 scal;
  int flag;
  int k;
  int rankcap;
  int nonfinite;
  int noconv;
  double err2;
  double sig2[64];
  int perm[64];
  double2 tau[128];
};

// In-place Householder QR of the first s columns of Y (m rows, ntot >= s columns,
// lda >= m, s <= min(m, 128)); the reflectors are also applied to columns s..ntot-1.
// R lies on and above the diagonal (real diagonal), reflector tails below it, tau[c] in
// sh.tau. Reflector H_c = I - tau_c v v^H with v = (0..0, 1, Y[c+1:, c]);
// Q = H_0 H_1 ... H_{s-1}.
__device__ void qr_householder(double2 *Y, int lda, int m, int s, int ntot, Sh &sh) {
  const int tid = threadIdx.x;
  for (int c = 0; c < s; ++c) {
    double part = 0.0;
    for (int i = c + 1 + tid; i < m; i += CM_WG) part += cabs2(Y[i + (int64_t)lda * c]);
    const double xn2 = wg_sum(part, sh.red);
    if (tid == 0) {
      double2 a = Y[c + (int64_t)lda * c];
      if (xn2 == 0.0 && a.y == 0.0) {
        sh.tau[c] = cmk(0.0, 0.0);
        sh.scal = cmk(0.0, 0.0);
      } else {
        double beta = -copysign(sqrt(a.x * a.x + a.y * a.y + xn2), a.x);
        sh.tau[c] = cmk((beta - a.x) / beta, -a.y / beta);
        sh.scal = cdiv(cmk(1.0, 0.0), csub(a, cmk(beta, 0.0)));
        Y[c + (int64_t)lda * c] = cmk(beta, 0.0);
      }
    }
    __syncthreads();
    const double2 tc = sh.tau[c];
    if (tc.x == 0.0 && tc.y == 0.0) continue;  // uniform
    const double2 sc = sh.scal;
    for (int i = c + 1 + tid; i < m; i += CM_WG) Y[i + (int64_t)lda * c] = cmul(Y[i + (int64_t)lda * c], sc);
    __syncthreads();
    const int ncols = ntot - c - 1;
    if (ncols > 0) {
      const int G = group_for(ncols), groups = CM_WG / G;
      const int lane = tid % G;
      const double2 ctc = cconj(tc);
      for (int jb = 0; jb < ncols; jb += groups) {
        const int j = c + 1 + jb + tid / G;
        const bool ok = j < ntot;
        double2 w = cmk(0.0, 0.0);
        if (ok) {
          if (lane == 0) w = Y[c + (int64_t)lda * j];
          for (int i = c + 1 + lane; i < m; i += G) ccfma(w, Y[i + (int64_t)lda * c], Y[i + (int64_t)lda * j]);
        }
        w.x = grp_sum(w.x, G);
        w.y = grp_sum(w.y, G);
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
__device__ void qr_apply_q(const double2 *Y, int lda, int m, int s, const Sh &sh, double2 *Z, int ldz, int k) {
  const int tid = threadIdx.x;
  const int G = group_for(k), groups = CM_WG / G, lane = tid % G;
  for (int c = s - 1; c >= 0; --c) {
    const double2 tc = sh.tau[c];
    if (tc.x == 0.0 && tc.y == 0.0) continue;
    for (int jb = 0; jb < k; jb += groups) {
      const int j = jb + tid / G;
      const bool ok = j < k;
      double2 w = cmk(0.0, 0.0);
      if (ok) {
        if (lane == 0) w = Z[c + (int64_t)ldz * j];
        for (int i = c + 1 + lane; i < m; i += G) ccfma(w, Y[i + (int64_t)lda * c], Z[i + (int64_t)ldz * j]);
      }
      w.x = grp_sum(w.x, G);
      w.y = grp_sum(w.y, G);
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

// One-sided Jacobi on the columns of S (s x s, column-major, ld s, in LDS), accumulating
// the rotations in J (s x s, LDS). On return the columns of S are mutually orthogonal,
// S_in J = S_out, and sh.sig2[i] / sh.perm[i] list squared column norms in descending
// order. Sets sh.noconv if the sweep limit was reached, sh.nonfinite on NaN/Inf.
__device__ void jacobi_onesided(double2 *S, double2 *J, int s, Sh &sh) {
  const int tid = threadIdx.x;
  for (int e = tid; e < s * s; e += CM_WG) J[e] = cmk((e % s) == (e / s) ? 1.0 : 0.0, 0.0);
  if (tid == 0) { sh.noconv = 0; sh.nonfinite = 0; }
  __syncthreads();
  const int N = s + (s & 1);
  const int npairs = N / 2;
  const int G = group_for(npairs);
  const int lane = tid % G, pi = tid / G;
  const double tol = 2.3e-16 * (s > 8 ? s : 8);
  const int max_sweeps = 40;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      int p = -1, q = -1;
      if (pi < npairs && N > 1) {
        if (pi == 0) { p = N - 1; q = r; }
        else { p = (r + pi) % (N - 1); q = (r - pi + (N - 1)) % (N - 1); }
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= s) p = -1;
      }
      double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
      if (p >= 0) {
        for (int i = lane; i < s; i += G) {
          double2 xp = S[i + s * p], xq = S[i + s * q];
          a += cabs2(xp); b += cabs2(xq);
          gr += xp.x * xq.x + xp.y * xq.y;
          gi += xp.x * xq.y - xp.y * xq.x;
        }
      }
      a = grp_sum(a, G); b = grp_sum(b, G); gr = grp_sum(gr, G); gi = grp_sum(gi, G);
      if (p >= 0) {
        const double ag = sqrt(gr * gr + gi * gi);
        if (ag > tol * sqrt(a * b) && ag > 1e-300) {
          const double zeta = (b - a) / (2.0 * ag);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double sn = c * t;
          const double2 e = cmk(gr / ag, gi / ag);
          const double2 se = cscale(e, sn);          // s e
          const double2 sce = cscale(cconj(e), sn);  // s conj(e)
          for (int i = lane; i < s; i += G) {
            double2 xp = S[i + s * p], xq = S[i + s * q];
            S[i + s * p] = csub(cscale(xp, c), cmul(sce, xq));
            S[i + s * q] = cadd(cmul(se, xp), cscale(xq, c));
            double2 vp = J[i + s * p], vq = J[i + s * q];
            J[i + s * p] = csub(cscale(vp, c), cmul(sce, vq));
            J[i + s * q] = cadd(cmul(se, vp), cscale(vq, c));
          }
          if (lane == 0) sh.flag = 1;
        } else if (!(a == a) || !(b == b)) {
          if (lane == 0) sh.nonfinite = 1;
        }
      }
      __syncthreads();
    }
    const int f = sh.flag;
    __syncthreads();
    if (f == 0) break;
  }
  if (sweep == max_sweeps && tid == 0) sh.noconv = 1;
  // squared column norms and descending order
  if (tid < s) {
    double a = 0.0;
    for (int i = 0; i < s; ++i) a += cabs2(S[i + s * tid]);
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

// Truncated factorisation Y ~= L * Rk of Y (a x b, column-major in global scratch, ld a;
// destroyed), where Rk (k x b) has orthonormal rows (the top-k right singular vectors)
// and L = Y Rk^H (a x k). The kept rank k follows choose_rank_t0(delta2, cap).
//   X : global scratch of at least a*b complex (used when a < b)
//   Z : global scratch of at least max(a,b)*min(a,b) complex
//   S, J : LDS, s*s complex each, s = min(a,b) <= 64
//   L (ld a) and R (ld k) : global outputs.
// Returns k (uniform).
__device__ int svd_trunc_rows(double2 *Y, int a, int b, double delta2, int cap,
                              double2 *X, double2 *Z, double2 *S, double2 *J,
                              double2 *L, double2 *R, Sh &sh) {
  const int tid = threadIdx.x;
  if (a >= b) {
    const int s = b;
    qr_householder(Y, a, a, s, s, sh);
    for (int e = tid; e < s * s; e += CM_WG) {
      const int i = e % s, j = e / s;
      S[e] = (i <= j) ? Y[i + (int64_t)a * j] : cmk(0.0, 0.0);
    }
    __syncthreads();
    jacobi_onesided(S, J, s, sh);
    choose_rank_t0(sh, s, delta2, cap);
    const int k = sh.k;
    // Rk[i, c] = conj(J[c, perm[i]])
    for (int e = tid; e < k * b; e += CM_WG) {
      const int i = e % k, c = e / k;
      R[i + (int64_t)k * c] = cconj(J[c + s * sh.perm[i]]);
    }
    // L = Q [W_k; 0]
    for (int e = tid; e < a * k; e += CM_WG) {
      const int i = e % a, j = e / a;
      Z[e] = (i < s) ? S[i + s * sh.perm[j]] : cmk(0.0, 0.0);
    }
    __syncthreads();
    qr_apply_q(Y, a, a, s, sh, Z, a, k);
    for (int e = tid; e < a * k; e += CM_WG) L[e] = Z[e];
    __syncthreads();
    return k;
  } else {
    const int s = a;
    // X = Y^H (b x a)
    for (int e = tid; e < a * b; e += CM_WG) {
      const int i = e % b, j = e / b;   // X[i, j] = conj(Y[j, i])
      X[e] = cconj(Y[j + (int64_t)a * i]);
    }
    __syncthreads();
    qr_householder(X, b, b, s, s, sh);
    // S = R^H (a x a)
    for (int e = tid; e < s * s; e += CM_WG) {
      const int i = e % s, j = e / s;
      S[e] = (j <= i) ? cconj(X[j + (int64_t)b * i]) : cmk(0.0, 0.0);
    }
    __syncthreads();
    jacobi_onesided(S, J, s, sh);
    choose_rank_t0(sh, s, delta2, cap);
    const int k = sh.k;
    for (int e = tid; e < a * k; e += CM_WG) {
      const int i = e % a, j = e / a;
      L[e] = S[i + s * sh.perm[j]];
    }
    for (int e = tid; e < b * k; e += CM_WG) {
      const int i = e % b, j = e / b;
      Z[e] = (i < s) ? J[i + s * sh.perm[j]] : cmk(0.0, 0.0);
    }
    __syncthreads();
    qr_apply_q(X, b, b, s, sh, Z, b, k);
    for (int e = tid; e < k * b; e += CM_WG) {
      const int i = e % k, c = e / k;
      R[i + (int64_t)k * c] = cconj(Z[c + (int64_t)b * i]);
    }
    __syncthreads();
    return k;
  }
}

// Thin QR: Y (m x p, ld m, destroyed) = Q Rr with Q (m x kq, orthonormal columns) and
// Rr (kq x p, upper trapezoidal), kq = min(m, p). Q -> Qout (ld m), Rr -> Rout (ld kq).
__device__ int qr_thin(double2 *Y, int m, int p, double2 *Qout, double2 *Rout, Sh &sh) {
  const int tid = threadIdx.x;
  const int kq = m < p ? m : p;
  qr_householder(Y, m, m, kq, p, sh);
  // R (with trailing columns when p > m)
  for (int e = tid; e < kq * p; e += CM_WG) {
    const int i = e % kq, j = e / kq;
    Rout[e] = (i <= j) ? Y[i + (int64_t)m * j] : cmk(0.0, 0.0);
  }
  for (int e = tid; e < m * kq; e += CM_WG) {
    const int i = e % m, j = e / m;
    Qout[e] = cmk(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  qr_apply_q(Y, m, m, kq, sh, Qout, m, kq);
  return kq;
}

}  // namespace la
