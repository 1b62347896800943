// cm_build_qtt: quantised tensor train of the Carr–Madan integrand (Eq. x).
//
// Index j has bits j_1 (weight 2^(n-1)) ... j_n (weight 1); core l carries j_l
// (Eq. discretized_x). The integrand factors exactly as
//   x_j = w(j_n) * exp(i v0 m_f) * exp(i j theta) * h(v0 + j eta),  theta = eta (m_f - k0),
// where exp(i j theta) is the rank-1 train of Section 3.3 (one phase per bit), the
// quadrature weight depends on the last bit only (Simpson: 2eta/3, 4eta/3, with the j = 0
// weight eta/3 folded into the value at j = 0), and h (cm_cf.h) is smooth.
//
// h is represented on an adaptive dyadic partition of [0, M): an interval [c, c + 2^m) is
//   - a zero leaf if |h| stays below eps(m) on its Chebyshev nodes and check points,
//   - a polynomial leaf if the degree P-1 Chebyshev interpolant matches h at P-1 check
//     points to eps(m),
//   - exact if 2^m <= P (values at all points), otherwise it is split in two.
// eps(m) = tol |h(0)| 2^(-m/2) bounds each leaf's contribution to ||x||_2.
// Polynomials in the remaining suffix share one P-dimensional bond space (values at the
// suffix interval's Chebyshev nodes; Lagrange cores pass them down exactly), so the bond
// dimension before rounding is (#split intervals at that depth) + min(P, 2^m). The train is
// then rounded to `tol` by the shared FP64 sweep. This replaces the TT-cross of the paper
// (Section 3.3) with a deterministic construction whose cost is O(#leaves * P) evaluations
// of h plus O(n P^3) assembly, independent of the grid size 2^n.
// One wavefront per problem (see cm_round.hip).
#define CM_WG 64
#include "cm_cf.h"
#include "cm_tt.h"

namespace {

constexpr int QP = 10;          // Chebyshev nodes per polynomial leaf
constexpr int QNC = 96;         // max candidate intervals per depth
constexpr int QI = QNC / 2;     // max split intervals per depth
constexpr int QNPT = 2 * QP - 1;
constexpr int PRE_CAP = QI + QP + 1;   // bond bound before rounding (<= 64)
// LDS arena per workgroup: small on purpose (see cm_round.hip), and with the static LDS
// within a sixteenth of the CU's 160 KB so that the rounding launch keeps four one-wave
// workgroups per SIMD; the tree phase's candidate values live in the slab.
constexpr int QLDS = 7680;

struct TreeDepth {
  int n_int;                 // split intervals at this depth
  int n_cand;                // candidates = 2 * split intervals of the previous depth
  int64_t int_a[QI];         // prefixes of split intervals
  int8_t kind[QNC];          // 0 zero leaf, 1 split, 2 value leaf
  int8_t idx[QNC];           // index into int_a (kind 1)
  double2 vals[QNC][QP];     // values of value leaves at their nodes (or points)
};

struct QttSlab {
  TreeDepth *tree;    // [n+1]
  double2 *pre;       // pre-rounding train, n cores of PRE_CAP*2*PRE_CAP
  int32_t *pre_ranks; // [CM_MAX_N + 1]
  int64_t *pre_off;   // [CM_MAX_N]
  RoundScratch rs;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Slab layout (bytes) for one workgroup; also used by the host workspace query.
__host__ __device__ inline size_t qtt_slab_bytes(int n_max, int cap, size_t *parts) {
  const int capm = cap > PRE_CAP ? cap : PRE_CAP;
  const size_t core_cap = (size_t)capm * 2 * capm;
  size_t o = 0;
  parts[0] = o; o += align256(sizeof(TreeDepth) * (size_t)(n_max + 1));
  parts[1] = o; o += align256(sizeof(double2) * (size_t)PRE_CAP * 2 * PRE_CAP * n_max);
  parts[2] = o; o += align256(sizeof(int32_t) * (CM_MAX_N + 2));   // ranks, then the instance mark
  parts[3] = o; o += align256(sizeof(int64_t) * CM_MAX_N);
  parts[4] = o; o += align256(sizeof(double2) * core_cap * n_max);  // rs.tt
  parts[5] = o; o += align256(sizeof(double2) * core_cap * 6);      // rs.Y..C
  parts[6] = o; o += align256(sizeof(double2) * 2 * 64 * 64);        // global Jacobi pair
  parts[7] = o; o += align256(sizeof(double2) * QNC * QNPT);         // candidate values
  return o;
}

// Index of the slab's instance mark: the instance whose pre-rounding train the slab holds,
// or -1 (set by k_build_qtt, read by k_build_round).
constexpr int QMARK = CM_MAX_N + 1;

__device__ inline QttSlab qtt_slab_view(char *slab, int n_max, int cap) {
  size_t parts[8];
  qtt_slab_bytes(n_max, cap, parts);
  QttSlab W;
  W.tree = (TreeDepth *)(slab + parts[0]);
  W.pre = (double2 *)(slab + parts[1]);
  W.pre_ranks = (int32_t *)(slab + parts[2]);
  W.pre_off = (int64_t *)(slab + parts[3]);
  const int capm = cap > PRE_CAP ? cap : PRE_CAP;
  W.rs.core_cap = (int64_t)capm * 2 * capm;
  W.rs.tt = (double2 *)(slab + parts[4]);
  double2 *mats = (double2 *)(slab + parts[5]);
  W.rs.Y = mats; W.rs.X = mats + W.rs.core_cap; W.rs.Z = mats + 2 * W.rs.core_cap;
  W.rs.L = mats + 3 * W.rs.core_cap; W.rs.R = mats + 4 * W.rs.core_cap; W.rs.C = mats + 5 * W.rs.core_cap;
  W.rs.S = (double2 *)(slab + parts[6]);
  W.rs.J = W.rs.S + 64 * 64;
  return W;
}

__device__ __forceinline__ double node_pos(double Lm1, double c) { return Lm1 * 0.5 * (1.0 - c); }

// barycentric weight of Chebyshev points of the second kind
__device__ __forceinline__ double bary_w(int q) {
  double w = (q & 1) ? -1.0 : 1.0;
  return (q == 0 || q == QP - 1) ? 0.5 * w : w;
}

// All QP Lagrange basis values L_p(x) on the nodes t_q = Lm1 (1 - cos(pi q/(P-1)))/2, in
// barycentric form: the weights w_q / (x - t_q) and their sum are shared by the whole row. At a
// node the row is the unit vector of that node.
__device__ void lagrange_row(double x, double Lm1, const double *cq, double *out) {
  double w[QP], den = 0.0;
  int hit = -1;
  for (int q = 0; q < QP; ++q) {
    const double dx = x - node_pos(Lm1, cq[q]);
    if (hit < 0 && fabs(dx) <= 1e-13 * (Lm1 + 1.0)) hit = q;
    w[q] = bary_w(q) / dx;
    den += w[q];
  }
  const double rd = 1.0 / den;
  for (int p = 0; p < QP; ++p) out[p] = (hit >= 0) ? (p == hit ? 1.0 : 0.0) : w[p] * rd;
}

}  // namespace

// theta = eta (m_f - k0) as phase fraction of bit weight 2^s.
__device__ __forceinline__ double theta_frac(const cm_problem &pr, int s) {
  const double rq = (pr.r - pr.q) * pr.T;
  if (k0_is_default(pr)) {
    // k0 = ln S0 - pi/eta: theta = eta (r - q) T + pi
    double f = prod_cycles_frac(pr.eta, rq, s);
    if (s == 0) { f += 0.5; f -= floor(f); }
    return f;
  }
  double hi, lo;
  drift_angle(pr.eta, log(pr.S0), pr.k0, rq, hi, lo);
  return cycles_frac(hi, lo, s);
}

// exp(i v0 m_f) as phase fraction (v0 = -eta 2^(n-1) for the symmetric rule, else 0).
__device__ __forceinline__ double v0mf_frac(const cm_problem &pr) {
  if (pr.quad != CM_QUAD_RECT2) return 0.0;
  const double v0 = -ldexp(pr.eta, pr.n - 1);
  const double f1 = prod_cycles_frac(v0, log(pr.S0), 0);
  const double f2 = prod_cycles_frac(v0, (pr.r - pr.q) * pr.T, 0);
  double f = f1 + f2;
  return f - floor(f);
}

// Tree and assembly for instances base + g (workgroup g, one instance each): the
// pre-rounding train stays in slab g, marked with its instance; k_build_round then rounds it
// into x. The two phases are separate launches because the tree phase (the characteristic
// function) needs 256 VGPRs while the rounding runs at twice the occupancy without it.
template <typename OutT>
// At most 256 VGPRs (two waves per SIMD): left alone the compiler takes 256 VGPRs plus AGPRs
// and one wave per SIMD; two halve the time despite a small spill.
__global__ __launch_bounds__(CM_WG, 2) void k_build_qtt(const cm_problem *__restrict__ prob, int batch, int base,
                                                     double tol, int cap, TTView x,
                                                     int32_t *__restrict__ status,
                                                     char *__restrict__ ws, size_t slab_bytes, int n_max) {
  extern __shared__ __align__(16) char lds_arena[];
  __shared__ la::Sh sh;
  __shared__ double cq[QP], ck[QP];
  __shared__ int code_sh;
  __shared__ int8_t kind_sh[QNC];
  __shared__ double err_sh[QNC];
  const int tid = threadIdx.x;
  // candidate values (vals[QNC][QNPT]) of the tree phase: in the LDS arena when it is large
  // enough, else in the slab; the rounding phase reuses the arena for its matrices
  size_t parts[8];
  qtt_slab_bytes(n_max, cap, parts);
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  double2 *vals = (sizeof(double2) * QNC * QNPT <= (size_t)QLDS) ? (double2 *)lds_arena : (double2 *)(slab + parts[7]);
  QttSlab W = qtt_slab_view(slab, n_max, cap);
  if (tid < QP) {
    cq[tid] = cos(M_PI * tid / (QP - 1));
    ck[tid] = cos(M_PI * (tid + 0.5) / (QP - 1));
  }
  if (tid == 0) W.pre_ranks[QMARK] = -1;
  __syncthreads();
  // Leaf-test weights: the interpolant at check point k is sum_q lw[k][q] f(t_q). Nodes and
  // check points are the same affine image of fixed Chebyshev points, so the interval length
  // cancels from the normalised barycentric weights and one table serves every depth.
  __shared__ double lw[QP - 1][QP];
  if (tid < QP - 1) {
    double w[QP], den = 0.0;
    for (int q = 0; q < QP; ++q) { w[q] = bary_w(q) / (cq[q] - ck[tid]); den += w[q]; }
    const double rd = 1.0 / den;
    for (int q = 0; q < QP; ++q) lw[tid][q] = w[q] * rd;
  }
  __syncthreads();

  // exactly one instance per workgroup (the host launches one workgroup per instance of the
  // chunk); the loop form keeps `continue` for the early exits
  const int end = (base + (int)gridDim.x < batch) ? base + (int)gridDim.x : batch;
  for (int b = base + (int)blockIdx.x; b < end; b += gridDim.x) {
    const cm_problem pr = prob[b];
    if (tid == 0) {
      int c = check_problem(pr);
      if (c == CM_OK && x.n[b] != pr.n) c = CM_E_INVALID;
      if (c == CM_OK && pr.n > n_max) c = CM_E_INVALID;
      code_sh = c;
    }
    __syncthreads();
    const int n = pr.n;
    if (code_sh != CM_OK) {
      // leave a valid rank-1 zero train so later stages stay well defined
      if (code_sh != CM_E_INVALID || (x.n[b] == n && n >= 1 && n <= n_max)) {
        OutT *cores = (OutT *)x.cores;
        for (int l = 0; l < n; ++l)
          for (int e = tid; e < 2; e += CM_WG) cstore<OutT>::st(cores, x.coff(b, l) + e, cmk(0.0, 0.0));
        for (int l = tid; l <= n; l += CM_WG) x.rk(b)[l] = 1;
      }
      if (tid == 0 && status) status[b] = code_sh;
      __syncthreads();
      continue;
    }
    const CfModel<double> cm = make_model<double>(pr);
    const bool simpson = pr.quad == CM_QUAD_SIMPSON1;
    const double eta = pr.eta;
    const double v0 = simpson ? 0.0 : -ldexp(eta, n - 1);
    const int64_t jpeak = simpson ? 0 : ((int64_t)1 << (n - 1));
    const double2 hpk = [&] { cx<double> z = h_centered<double>(cm, v0 + (double)jpeak * eta); return cmk(z.x, z.y); }();
    const double hscale = sqrt(cabs2(hpk));
    const double eps_rel = tol;

    // ---------------- tree
    TreeDepth *T = W.tree;
    if (tid == 0) { T[0].n_int = 1; T[0].n_cand = 1; T[0].int_a[0] = 0; T[0].kind[0] = 1; T[0].idx[0] = 0; }
    __syncthreads();
    int depth_done = 0;
    for (int d = 1; d <= n; ++d) {
      const int I_prev = T[d - 1].n_int;
      const int NC = 2 * I_prev;
      const int m = n - d;
      const int64_t L = (int64_t)1 << m;
      const bool exact = L <= QP;
      const int npts = exact ? (int)L : QNPT;
      const double Lm1 = (double)(L - 1);
      if (NC > QNC) {
        if (tid == 0) code_sh = CM_E_NOCONV;
        __syncthreads();
        break;
      }
      if (tid == 0) T[d].n_cand = NC;
      for (int e = tid; e < NC * npts; e += CM_WG) {
        int q;
        const int ci = la::divmod_small(e, npts, q);
        const int64_t c = T[d - 1].int_a[ci >> 1] + ((int64_t)(ci & 1) << m);
        double pos;
        if (exact) pos = (double)q;
        else pos = (q < QP) ? node_pos(Lm1, cq[q]) : node_pos(Lm1, ck[q - QP]);
        // v = v0 + (c + pos) eta from the exact offset c - jpeak (jpeak eta = -v0): the
        // direct sum cancels to an absolute error of |v0| ulp near the peak on large
        // symmetric grids, which breaks the leaf tests there
        const double v = ((double)(c - jpeak) + pos) * eta;
        const cx<double> h = h_centered<double>(cm, v);
        vals[ci * QNPT + q] = cmk(h.x, h.y);
      }
      __syncthreads();
      const double eps = eps_rel * hscale * exp2(-0.5 * m);
      if (!exact) {
        // LG lanes per candidate: lane j takes the magnitudes of points j and j + LG and the
        // interpolation error at check point j; the group reduces both maxima by lane moves.
        // The loop runs whole groups (NC LG is a multiple of LG) so every swap partner is live.
        constexpr int LG = 16;
        static_assert(QNPT <= 2 * LG && QP - 1 <= LG && CM_WG % 64 == 0, "leaf-test lane groups");
        for (int e0 = 0; e0 < NC * LG; e0 += CM_WG) {
          const int e = e0 + tid, ci = e / LG, j = e % LG;
          const bool on = e < NC * LG;
          double mx2 = 0.0, er2 = 0.0;
          if (on) {
            const double2 *vc = vals + ci * QNPT;
            const double a = cabs2(vc[j]);
            mx2 = (a == a) ? a : INFINITY;
            if (j + LG < QNPT) {
              const double a2 = cabs2(vc[j + LG]);
              mx2 = fmax(mx2, (a2 == a2) ? a2 : INFINITY);
            }
            if (j < QP - 1) {
              double2 p = cmk(0.0, 0.0);
              for (int q = 0; q < QP; ++q) p = cadd(p, cscale(vc[q], lw[j][q]));
              er2 = cabs2(csub(p, vc[QP + j]));
            }
          }
          // groups of LG = 16 lanes are the rows of the DPP lane moves
          mx2 = fmax(mx2, la::dpp_d<la::DPP_XOR1>(mx2));
          er2 = fmax(er2, la::dpp_d<la::DPP_XOR1>(er2));
          mx2 = fmax(mx2, la::dpp_d<la::DPP_XOR2>(mx2));
          er2 = fmax(er2, la::dpp_d<la::DPP_XOR2>(er2));
          mx2 = fmax(mx2, la::dpp_d<la::DPP_HALF_MIRROR>(mx2));
          er2 = fmax(er2, la::dpp_d<la::DPP_HALF_MIRROR>(er2));
          mx2 = fmax(mx2, la::dpp_d<la::DPP_MIRROR>(mx2));
          er2 = fmax(er2, la::dpp_d<la::DPP_MIRROR>(er2));
          if (on && j == 0) {
            const int64_t c = T[d - 1].int_a[ci >> 1] + ((int64_t)(ci & 1) << m);
            const bool forced = simpson && c == 0;
            const double mx = sqrt(mx2), err = sqrt(er2);
            int kind;
            if (isinf(mx)) kind = -1;
            else if (mx <= eps && !forced) kind = 0;
            else kind = (err <= eps && !forced) ? 2 : 1;
            kind_sh[ci] = (int8_t)kind;
          }
        }
      } else {
        // point leaves: every candidate keeps its values (the Simpson end weight halves u = 0)
        for (int ci = tid; ci < NC; ci += CM_WG) {
          const int64_t c = T[d - 1].int_a[ci >> 1] + ((int64_t)(ci & 1) << m);
          if (simpson && c == 0) vals[ci * QNPT] = cscale(vals[ci * QNPT], 0.5);
          kind_sh[ci] = 2;
        }
      }
      __syncthreads();
      if (tid == 0) {
        int ni = 0;
        for (int ci = 0; ci < NC; ++ci) {
          int k = kind_sh[ci];
          if (k < 0) { code_sh = CM_E_NONFINITE; k = 0; }
          if (k == 1) {
            if (ni >= QI) { code_sh = CM_E_NOCONV; k = 0; }
            else { T[d].int_a[ni] = T[d - 1].int_a[ci >> 1] + ((int64_t)(ci & 1) << m); T[d].idx[ci] = (int8_t)ni; ++ni; }
          }
          T[d].kind[ci] = (int8_t)k;
        }
        T[d].n_int = ni;
      }
      __syncthreads();
      const int pv = exact ? (int)L : QP;
      for (int e = tid; e < NC * pv; e += CM_WG) {
        int q;
        const int ci = la::divmod_small(e, pv, q);
        T[d].vals[ci][q] = vals[ci * QNPT + q];
      }
      __syncthreads();
      depth_done = d;
      if (code_sh != CM_OK) break;
    }
    (void)depth_done;
    if (code_sh != CM_OK) {
      if (tid == 0 && status) status[b] = code_sh;
      OutT *cores = (OutT *)x.cores;
      for (int l = 0; l < n; ++l)
        for (int e = tid; e < 2; e += CM_WG) cstore<OutT>::st(cores, x.coff(b, l) + e, cmk(0.0, 0.0));
      for (int l = tid; l <= n; l += CM_WG) x.rk(b)[l] = 1;
      __syncthreads();
      continue;
    }

    // ---------------- assembly of the pre-rounding train (FP64)
    // active[d]: some value leaf exists at depth <= d
    __shared__ int active[CM_MAX_N + 1];
    __shared__ int rks[CM_MAX_N + 1];
    if (tid == 0) {
      int a = 0;
      for (int d = 0; d <= n; ++d) {
        if (d > 0)
          for (int ci = 0; ci < T[d].n_cand; ++ci) a |= (T[d].kind[ci] == 2);
        active[d] = a;
        const int m = n - d;
        const int pb = (m >= 5) ? QP : ((1 << m) < QP ? (1 << m) : QP);
        rks[d] = (d == 0) ? 1 : (T[d].n_int + (a ? pb : 0));
      }
      if (rks[n] < 1) rks[n] = 1;  // all-zero integrand: keep a valid (zero) train
      for (int d = 0; d <= n; ++d) W.pre_ranks[d] = rks[d] < 1 ? 1 : rks[d];
      for (int l = 0; l < n; ++l) W.pre_off[l] = (int64_t)l * PRE_CAP * 2 * PRE_CAP;
    }
    __syncthreads();
    const double vf = v0mf_frac(pr);
    for (int l = 1; l <= n; ++l) {  // core l maps bond l-1 -> bond l
      const int m = n - l;          // suffix bits after this core; bit weight 2^m
      const int rl = W.pre_ranks[l - 1], rr = W.pre_ranks[l];
      const int Il = T[l - 1].n_int;
      const int Ir = (l < n) ? T[l].n_int : 0;
      const int pbl = (m + 1 >= 5) ? QP : ((1 << (m + 1)) < QP ? (1 << (m + 1)) : QP);
      const int pbr = (m >= 5) ? QP : ((1 << m) < QP ? (1 << m) : QP);
      const bool actl = active[l - 1] && l > 1;
      const bool actr = active[l];
      const bool exl = ((int64_t)1 << (m + 1)) <= QP;
      const bool exr = ((int64_t)1 << m) <= QP;
      const double Lm1l = (double)(((int64_t)1 << (m + 1)) - 1);
      const double Lm1r = (double)(((int64_t)1 << m) - 1);
      double2 *G = W.pre + W.pre_off[l - 1];
      // rank-1 factors of this core
      const double2 ph1 = turn(theta_frac(pr, m));
      double2 wt0 = cmk(1.0, 0.0), wt1 = ph1;
      if (l == n) {
        const double w0 = simpson ? 2.0 * eta / 3.0 : eta, w1 = simpson ? 4.0 * eta / 3.0 : eta;
        wt0 = cscale(wt0, w0);
        wt1 = cscale(wt1, w1);
      }
      if (l == 1) {
        const double2 g = turn(vf);
        wt0 = cmul(wt0, g);
        wt1 = cmul(wt1, g);
      }
      // Lagrange rows of the child nodes in the parent interval: lt[beta][q][p] = L_p(x_q)
      __shared__ double lt[2][QP][QP];
      if (actl && !exl) {
        if (tid < 2 * QP) {
          const int beta = tid >= QP, q = tid - beta * QP;
          const double tq = exr ? (double)q : node_pos(Lm1r, cq[q]);
          lagrange_row(beta * ldexp(1.0, m) + tq, Lm1l, cq, lt[beta][q]);
        }
        __syncthreads();
      }
      for (int e = tid; e < rl * 2 * rr; e += CM_WG) {
        int jr;
        const int ib = la::divmod_small(e, rr, jr), i = ib >> 1, beta = ib & 1;
        double2 v = cmk(0.0, 0.0);
        if (i < Il || l == 1) {
          // split interval i (at depth l-1), child ci = 2 i + beta
          const int ci = 2 * (l == 1 ? 0 : i) + beta;
          const int k = T[l].kind[ci];
          if (k == 1) {
            if (jr == T[l].idx[ci]) v = cmk(1.0, 0.0);
          } else if (k == 2) {
            if (jr >= Ir && actr && jr - Ir < pbr) v = T[l].vals[ci][jr - Ir];
          }
        } else if (actl) {
          const int p = i - Il;
          if (jr >= Ir && actr) {
            const int q = jr - Ir;
            const double tq = exr ? (double)q : node_pos(Lm1r, cq[q]);
            const double xq = beta * ldexp(1.0, m) + tq;
            double lv;
            if (exl) lv = (fabs(xq - (double)p) < 0.5) ? 1.0 : 0.0;
            else lv = lt[beta][q][p];
            v = cmk(lv, 0.0);
          }
        }
        v = cmul(v, beta ? wt1 : wt0);
        G[e] = v;
      }
      __syncthreads();
    }

    // the rounding into x is k_build_round's
    if (tid == 0) W.pre_ranks[QMARK] = b;
    __syncthreads();
  }
}

// Rounds the pre-rounding train of slab g (if k_build_qtt marked one) into x, with cores
// 1..n-1 right-orthonormal, and writes the instance's status.
template <typename OutT>
__global__ __launch_bounds__(CM_WG, 4) void k_build_round(const cm_problem *__restrict__ prob, double tol, int cap,
                                                       TTView x, int32_t *__restrict__ status,
                                                       char *__restrict__ ws, size_t slab_bytes, int n_max) {
  extern __shared__ __align__(16) char lds_arena[];
  __shared__ la::Sh sh;
  __shared__ int code_sh;
  const int tid = threadIdx.x;
  QttSlab W = qtt_slab_view(ws + (size_t)blockIdx.x * slab_bytes, n_max, cap);
  const int b = W.pre_ranks[QMARK];
  if (b < 0) return;
  const int n = prob[b].n;
  if (tid == 0) code_sh = CM_OK;
  __syncthreads();
  CoreSrc src;
  src.cores = W.pre; src.off = W.pre_off; src.ranks = W.pre_ranks; src.dtype = CM_C128;
  const double err = round_train_auto<OutT>(n, 2, src, tol, cap, (OutT *)x.cores, x.off + (int64_t)b * CM_MAX_N,
                                            x.rk(b), W.rs, lds_arena, QLDS, sh, &code_sh);
  (void)err;
  __syncthreads();
  if (tid == 0 && status) status[b] = code_sh;
}

// ------------------------------------------------------------------ host side
extern "C" size_t cm_qtt_slab_bytes(int n_max, int cap) {
  size_t parts[8];
  return qtt_slab_bytes(n_max, cap, parts);
}

extern "C" int cm_slots_for_ws(int op, int batch, int n_max, int cap_rank, int dtype, size_t ws_bytes);

extern "C" cm_status cm_build_qtt(const cm_problem *prob, int batch, double tol, int cap_rank,
                                  cm_tt_batch *x, int32_t *status, void *ws, size_t ws_bytes,
                                  void *stream) {
  if (!prob || !x || batch < 0 || !(tol > 0.0) || cap_rank < 1 || cap_rank > 64) return CM_E_INVALID;
  if (batch == 0) return CM_OK;
  if (x->d_out != 2 || x->d_in != 1 || x->batch < batch || x->n_max < 1 || x->n_max > CM_MAX_N) return CM_E_INVALID;
  if (cap_rank > x->cap_rank) return CM_E_INVALID;
  if (x->dtype != CM_C64 && x->dtype != CM_C128) return CM_E_INVALID;
  // one workgroup per workspace slab (cm_workspace_bytes gives the default count)
  const int slots = cm_slots_for_ws(CM_OP_BUILD_QTT, batch, x->n_max, cap_rank, x->dtype, ws ? ws_bytes : 0);
  if (slots < 1) return CM_E_INVALID;
  const size_t slab = cm_qtt_slab_bytes(x->n_max, cap_rank);
  const size_t lds = QLDS;
  TTView v = tt_view(x);
  hipStream_t s = (hipStream_t)stream;
  CM_HIP_CHECK(cm_allow_lds(k_build_qtt<float2>, lds));
  CM_HIP_CHECK(cm_allow_lds(k_build_qtt<double2>, lds));
  CM_HIP_CHECK(cm_allow_lds(k_build_round<float2>, lds));
  CM_HIP_CHECK(cm_allow_lds(k_build_round<double2>, lds));
  // chunks of `slots` instances: tree and assembly (one workgroup per instance), then the
  // rounding of the chunk's trains
  for (int base = 0; base < batch; base += slots) {
    const int cnt = batch - base < slots ? batch - base : slots;
    if (x->dtype == CM_C64) {
      hipLaunchKernelGGL(k_build_qtt<float2>, dim3(cnt), dim3(CM_WG), lds, s, prob, batch, base, tol, cap_rank, v,
                         status, (char *)ws, slab, x->n_max);
      hipLaunchKernelGGL(k_build_round<float2>, dim3(cnt), dim3(CM_WG), lds, s, prob, tol, cap_rank, v, status,
                         (char *)ws, slab, x->n_max);
    } else {
      hipLaunchKernelGGL(k_build_qtt<double2>, dim3(cnt), dim3(CM_WG), lds, s, prob, batch, base, tol, cap_rank, v,
                         status, (char *)ws, slab, x->n_max);
      hipLaunchKernelGGL(k_build_round<double2>, dim3(cnt), dim3(CM_WG), lds, s, prob, tol, cap_rank, v, status,
                         (char *)ws, slab, x->n_max);
    }
    CM_LAUNCH_CHECK();
  }
  x->flags = CM_TT_RIGHT_ORTHO;
  return CM_OK;
}
