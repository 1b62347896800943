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
// runs in FP64. Sites with 2 chi <= 48 and w' r' <= 128 (the bulk of a pricing chain) keep
// T in registers for the whole factorisation, each column on a group of two, four or eight
// lanes (zip_site_pair); other sites stage their matrices in LDS when they fit, otherwise in the
// workgroup's global slab.
#include <mutex>
#include <type_traits>

#include "cm_tt.h"

namespace {

constexpr int ZCHI = 48;          // zip-up bond limit (sites above 24 take the generic path)
constexpr int ZW = 24;            // largest operator bond supported by the workspace layout
// LDS arena per workgroup. The pair-resident path holds half a column of T (up to 24 rows)
// in 96 VGPRs per lane; the kernel is bounded to 168 VGPRs (three waves per SIMD, which
// measured faster than two without spills or four with spills in the pivot loop), and the
// FP32 arena lets three 256-thread workgroups share a CU while holding the staged carry and
// D chunks of the largest sites of a 2^24-point chain, or the reflectors.
template <typename T> constexpr int zlds_bytes();
template <> constexpr int zlds_bytes<float2>() { return 40 * 1024; }
template <> constexpr int zlds_bytes<double2>() { return 64 * 1024; }

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
  __device__ __forceinline__ static float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
};
template <> struct acc_t<double2> {
  using type = double2;
  __device__ __forceinline__ static double2 zero() { return cmk(0.0, 0.0); }
  __device__ __forceinline__ static void fma_(double2 &a, double2 b, double2 c) { cfma(a, b, c); }
  __device__ __forceinline__ static double2 from(double2 v) { return v; }
  __device__ __forceinline__ static double2 to(double2 v) { return v; }
  __device__ __forceinline__ static double2 add(double2 a, double2 b) { return cadd(a, b); }
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

// ---- register-resident site ------------------------------------------------------------
// T (m x p, FP64) is held in registers for the whole pivoted QR. Column c lives on the G
// lanes G c .. G c + G - 1 (G = 8 for sites with p <= 32 and G = 4 for p <= 64, so that
// all four waves hold columns, else G = 2); at step i (j = i / G shifts done) lane g of the group holds row G (s + j) + g
// in register slot s. All lanes of a group move their slots down by one after every step i
// with i % G = G - 1, so row i always sits in slot 0 of lane i % G and every register index
// is static; rows finished before i in the same group of G sit in slot 0 of the lanes below
// and take no part (their reflector entries are zero). A dot product is lane-local plus
// log2 G DPP exchanges within the group. A pivot step needs one workgroup barrier, at which
// each wave publishes its best candidate column (its pivot key, which packs norm and index
// into one integer, the sum of its columns' norms, its entry alpha in row i and its rows from
// i on, with the Householder data it would give) and all waves then take the same global
// choice. Column
// norms are recomputed exactly from the updated entries at every step. Rows of
// B = R P^T are emitted as they are finished, straight into the carry buffer in the
// [k][w'][r'] order the next site reads. Q = H_0 ... H_{k-1} [I_k; 0] is then accumulated
// barrier-free with eight lanes per column, from the reflectors kept in LDS.
constexpr int PW = CM_WG / 64;    // waves per workgroup
constexpr int MR = 48;            // rows: m = 2 chi <= 48
constexpr int SM = MR / 2;        // register slots per lane at the largest m
// The pivot loop is compiled for G = 2 lanes per column with 8, 12, 16 and 24 slots
// (m <= 16, 24, 32, 48), G = 4 with 8 and 12 slots (p <= 64, m <= 32, 48) and G = 8 with 4
// slots (p <= 32, m <= 32); each site takes the widest G and then the fewest slots that hold
// it. Fewer slots leave the loop's addresses and scalars in registers instead of spilling
// them across the barrier, and a wider G spreads a step's column work over more waves.
constexpr int CP = CM_WG / 2;     // columns: p <= 128
struct CandInfo {
  unsigned long long key;   // pivot key (see pivot_key), 0 when the wave has no candidate
  double sum;
  double pad[2];
};
static_assert(sizeof(CandInfo) == 32, "CandInfo layout");
// LDS layout (bytes): candidate columns [2][PW][MR] (two buffers, by step parity; entry
// 2 s + g is row 2 (s + j) + g), their CandInfo and Householder data [2][PW], taus, then a
// region holding the
// carry, the operator core, the input core and chunks of D during the contraction and the
// reflectors V [k][MR] during the factorisation.
constexpr size_t PL_CAND = 0;
constexpr size_t PL_INFO = PL_CAND + 16 * 2 * PW * MR;
constexpr size_t PL_HOUSE = PL_INFO + 32 * 2 * PW;       // House [2][PW]
constexpr size_t PL_TAU = PL_HOUSE + 64 * 2 * PW;
constexpr size_t PL_REGION = (PL_TAU + 16 * ZCHI + 255) & ~(size_t)255;

template <typename T>
__device__ __forceinline__ bool pair_site_fits(const SiteDims &s, int kcap, size_t lds_bytes) {
  const int m = 2 * s.chi, p = s.w1 * s.r1;
  if (m > MR || p > CP) return false;
  // carry, operator core, input core and two 4-row chunks of D (storage precision)
  const size_t dwa = sizeof(T) * ((size_t)s.chi * s.w0 * s.r0 + (size_t)s.w0 * 4 * s.w1 + (size_t)s.r0 * 2 * s.r1 +
                                  (size_t)2 * 4 * s.w0 * 2 * s.r1);
  int kmax = m < p ? m : p;
  if (kcap < kmax) kmax = kcap;
  const size_t v = (size_t)16 * MR * kmax;
  return PL_REGION + (dwa > v ? dwa : v) <= lds_bytes;
}

// a wave-uniform copy of a value every lane already holds
__device__ __forceinline__ int uni_i(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Pivot key of column c (< 128) with squared norm n2 >= 0: the bit pattern of n2 (non-negative
// doubles order as their bits do) with the low byte replaced by 255 - c, so that the largest
// key belongs to the largest norm, ties going to the smaller column, and 0 means no candidate.
// Norms that differ only in their last eight bits (relative 2^-44) count as tied, which does
// not matter for the quality of a pivot. A NaN or infinite norm gives a key above every finite
// one; the tail sum reports it before the pivot is used.
__device__ __forceinline__ unsigned long long pivot_key(double n2, int c) {
  return ((unsigned long long)__double_as_longlong(n2) & ~0xFFull) | (unsigned long long)(255 - c);
}
__device__ __forceinline__ int key_col(unsigned long long key) { return 255 - (int)(key & 0xFF); }

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const unsigned lo = (unsigned)la::dpp_i<CTRL>((int)(unsigned)v), hi = (unsigned)la::dpp_i<CTRL>((int)(unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// Over the 64 lanes of a wave: the largest pivot key and the sum of one `sum` per aligned
// group of G lanes, returned wave-uniform. Both are already equal on the G lanes of a group, so
// only the stages across groups run: DPP inside rows of 16 lanes, then lane swaps across rows
// and across the two halves of the wave.
template <int G>
__device__ __forceinline__ void wave_keymax_sum_uni(unsigned long long &key, double &sum) {
  auto step = [&](auto ctrl, bool across) {
    constexpr int C = decltype(ctrl)::value;
    if (across) {
      const unsigned long long o = dpp_u64<C>(key);
      key = o > key ? o : key;
      sum += la::dpp_d<C>(sum);
    }
  };
  step(std::integral_constant<int, la::DPP_XOR1>{}, G <= 1);
  step(std::integral_constant<int, la::DPP_XOR2>{}, G <= 2);
  step(std::integral_constant<int, la::DPP_HALF_MIRROR>{}, G <= 4);
  step(std::integral_constant<int, la::DPP_MIRROR>{}, true);
  // across rows, then halves, by the lane swaps: both lanes of a pair combine the same
  // (lower, upper) values, so every lane ends with the same key and sum
  auto cross = [&](auto wc) {
    constexpr int W = decltype(wc)::value;
    int l0, l1, h0, h1;
    la::swap_pair_i<W>((int)(unsigned)key, l0, l1);
    la::swap_pair_i<W>((int)(unsigned)(key >> 32), h0, h1);
    const unsigned long long k0 = ((unsigned long long)(unsigned)h0 << 32) | (unsigned)l0;
    const unsigned long long k1 = ((unsigned long long)(unsigned)h1 << 32) | (unsigned)l1;
    key = k1 > k0 ? k1 : k0;
    double s0, s1;
    la::swap_pair_d<W>(sum, s0, s1);
    sum = s0 + s1;
  };
  cross(std::integral_constant<int, 16>{});
  cross(std::integral_constant<int, 32>{});
}

// Householder data of a pivot column with squared norm n2 (rows >= i) and entry alpha in row
// i: beta = -sign(Re alpha) sqrt(n2), x_i = alpha - beta (so that v = x scal has v_i = 1),
// tau = (beta - alpha) / beta and scal = 1 / (alpha - beta). The reciprocal square root and
// the reciprocal come from the hardware approximations refined by two Newton steps each
// (relative error a few ulp), which keeps the chain short.
struct House {
  double2 am, tau, scal;
  double beta, pad;
};
static_assert(sizeof(House) == 64, "House layout");
// The published reflector: the step's factor conj(tau) |scal|^2 of w_c (formed once by the
// winning lane instead of by every lane of every wave) in place of alpha - beta, which only
// the winner needs.
struct HouseRec {
  double2 wf, tau, scal;
  double beta, pad;
};
static_assert(sizeof(HouseRec) == 64, "HouseRec layout");
__device__ __forceinline__ House householder(double n2, double2 alpha) {
  House H;
  H.beta = 0.0;
  H.pad = 0.0;
  H.am = alpha;
  H.tau = cmk(0.0, 0.0);
  H.scal = cmk(0.0, 0.0);
  if (n2 > 0.0) {
    const double rs = la::rsq_nr(n2);
    const double sg = alpha.x >= 0.0 ? 1.0 : -1.0;
    H.beta = -sg * (n2 * rs);
    const double ib = -sg * rs;   // 1 / beta
    H.am.x = alpha.x - H.beta;
    const double id = la::rcp_nr(cabs2(H.am));
    H.tau = cmk(1.0 - alpha.x * ib, -alpha.y * ib);
    H.scal = cmk(H.am.x * id, -H.am.y * id);
  }
  return H;
}

template <typename T, int SMX, int G>
__device__ __forceinline__ int zip_site_pair(char *arena, const SiteDims &sd, const T *__restrict__ Wl,
                                             const T *__restrict__ Al, double2 *C, T *Yout, double delta2,
                                             int kcap, int *code) {
  using A = acc_t<T>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = uni_i(tid >> 6);   // wave index, known to the compiler as wave-uniform
  const int chi = sd.chi, w0 = sd.w0, w1 = sd.w1, r0 = sd.r0, r1 = sd.r1;
  const int m = 2 * chi, p = w1 * r1;
  static_assert(G == 2 || G == 4 || G == 8, "lanes per column");
  static_assert(G * SMX <= MR, "a column's slots fit the candidate buffer");
  const int c = tid / G, g = tid % G;   // this lane's column and its share of the rows
  const int u = g & 1, gh = g >> 1;     // its rows are 2 ch + u with ch = gh (mod G / 2)
  double2 *cand = (double2 *)(arena + PL_CAND);
  CandInfo *info = (CandInfo *)(arena + PL_INFO);
  HouseRec *hinf = (HouseRec *)(arena + PL_HOUSE);
  double2 *taus = (double2 *)(arena + PL_TAU);
  T *Cl = (T *)(arena + PL_REGION);
  T *Wc = Cl + chi * w0 * r0;
  T *Ac = Wc + w0 * 4 * w1;
  T *Dch = Ac + r0 * 2 * r1;                       // two chunks of D[4][w0][2][r1]
  double2 *V = (double2 *)(arena + PL_REGION);   // reuses the region once T is in registers
  const int dchunk = 4 * w0 * 2 * r1;
  // the whole D (rows padded with zero rows to a multiple of four, which the chunk reads below
  // cover) in the region after the staged operands, when it fits
  const int chi4 = (chi + 3) & ~3;
  const bool fullD = chi > 4 &&
                     PL_REGION + sizeof(T) * ((size_t)chi * w0 * r0 + (size_t)w0 * 4 * w1 + (size_t)r0 * 2 * r1 +
                                              (size_t)chi4 * w0 * 2 * r1) <= (size_t)zlds_bytes<T>();
  // stage the carry (in the storage precision, which the contraction uses) and the cores;
  // loads are issued in batches so that their latencies overlap
  {
    const int nc = chi * w0 * r0;
    for (int e0 = tid; e0 < nc; e0 += 4 * CM_WG) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * CM_WG;
        v[u] = e < nc ? C[e] : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * CM_WG;
        if (e < nc) Cl[e] = A::from(v[u]);
      }
    }
  }
  for (int e = tid; e < w0 * 4 * w1; e += CM_WG) Wc[e] = Wl[e];
  for (int e = tid; e < r0 * 2 * r1; e += CM_WG) Ac[e] = Al[e];
  // T[(ch, g)][(wp, rp)] = sum_{w0, j} D[ch][w0][j][rp] W[w0][g][j][wp] (row 2 ch + g, slot ch)
  // with D[ch][w0][j][r1] = sum_r C[ch][w0][r] A[r][j][r1], both in the storage precision,
  // four ch at a time; D chunks alternate between two buffers, one barrier per chunk
  const bool cok = c < p;
  // waves whose 64 / G columns all lie beyond p hold no column of T: they skip the
  // contraction's second product, the pivot search and the column updates, and only take
  // part in the barriers and the row writes
  const bool wcols = (64 / G) * wv < p;
  double2 t[SMX];
#pragma unroll
  for (int sl = 0; sl < SMX; ++sl) t[sl] = cmk(0.0, 0.0);
  {
    const int wp = cok ? c / r1 : 0, rp = cok ? c - (c / r1) * r1 : 0;
#pragma unroll
    for (int ch0 = 0; ch0 < SMX * G / 2; ch0 += 4) {
      if (ch0 < chi) {
        // D rows ch0 .. ch0 + 3: one chunk of the double buffer, or of the whole D (all chi4
        // rows, formed in one pass before the first chunk) when it fits the region
        T *Db = fullD ? Dch + ch0 * w0 * 2 * r1 : Dch + ((ch0 / 4) & 1) * dchunk;
        if (!fullD || ch0 == 0) {
          T *Dw = fullD ? Dch : Db;
          const int ne = fullD ? chi4 * w0 * 2 * r1 : dchunk;
          __syncthreads();   // staging done (first chunk) / this buffer's previous readers done
          for (int e = tid; e < ne; e += CM_WG) {
            // e = ((cc w0 + ww) 2 + j) r1 + rpp
            int pr, ww;
            const int row = la::divmod_small(e, 2 * r1, pr);
            const int cc = la::divmod_small(row, w0, ww);
            const int j = pr >= r1 ? 1 : 0, rpp = pr - j * r1;
            typename A::type acc = A::zero();
            if (ch0 + cc < chi) {
              const T *crow = Cl + ((ch0 + cc) * w0 + ww) * r0;
              for (int r = 0; r < r0; ++r) A::fma_(acc, crow[r], Ac[(r * 2 + j) * r1 + rpp]);
            }
            Dw[e] = acc;
          }
          __syncthreads();
        }
        if (wcols) {
          // this lane's rows in the chunk: ch = ch0 + gh + (G / 2) e, in slot ch / (G / 2)
          constexpr int NE = 8 / G;
          // the two input bits j accumulate separately (two dependent chains of w0 terms
          // instead of one of 2 w0), summed at the end
          typename A::type acc[2][NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) acc[0][e] = acc[1][e] = A::zero();
          for (int ww = 0; ww < w0; ++ww)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const T wvv = Wc[(ww * 4 + 2 * u + j) * w1 + wp];
              const T *dd = Db + (ww * 2 + j) * r1 + rp;
#pragma unroll
              for (int e = 0; e < NE; ++e) A::fma_(acc[j][e], dd[(gh + (G / 2) * e) * w0 * 2 * r1], wvv);
            }
#pragma unroll
          for (int e = 0; e < NE; ++e)
            if (cok && ch0 + gh + (G / 2) * e < chi) t[ch0 / (G / 2) + e] = A::to(A::add(acc[0][e], acc[1][e]));
        }
      }
    }
  }
  __syncthreads();   // the region now holds V
  bool act = cok;    // still a candidate pivot column
  double nrm;
  {
    double nz[2] = {0.0, 0.0};
#pragma unroll
    for (int sl = 0; sl < SMX; ++sl) nz[sl & 1] += cabs2(t[sl]);
    nrm = la::grp_sum(nz[0] + nz[1], G);
  }
  const int kmax = m < p ? m : p;
  const int hrows = (m + G - 1) / G;   // slots in use before any shift

  // Pivot choice for step i: publishes this wave's candidate, waits for the other waves',
  // and returns true when the factorisation stops at rank i (the same decision in every
  // wave). The loop below exits only at its end, which keeps T in registers.
  int pc = 0;
  double beta = 0.0;
  double2 scal = cmk(0.0, 0.0), wf = cmk(0.0, 0.0);
  const double2 *X = cand;
  auto select = [&](int i) -> bool {
    const int b = i & 1, j = i / G;
    unsigned long long key = act ? pivot_key(nrm, c) : 0ull;
    double sum = act ? nrm : 0.0;   // one term per group (all of its lanes hold it)
    // every lane forms the reflector its column would give from its own (exact) norm; only the
    // winner's row-i lane keeps it. Formed ahead of the pivot reduction, whose result it does
    // not need.
    const House Hs = householder(nrm, t[0]);
    if (__ballot(act) != 0) wave_keymax_sum_uni<G>(key, sum);   // else already the reduction's result
    double2 *mine = cand + (b * PW + wv) * MR;
    CandInfo *inf = info + b * PW + wv;
    if (key != 0ull && c == key_col(key)) {
      // slot 0 is row G j + g: finished (zero), row i (x_i = alpha - beta) or a later row
      const int r0w = G * j + g;
      double2 v0 = t[0];
      if (r0w < i) v0 = cmk(0.0, 0.0);
      if (r0w == i) {
        const House &H = Hs;
        v0 = H.am;
        HouseRec rec;
        rec.wf = cscale(cconj(H.tau), cabs2(H.scal));
        rec.tau = H.tau;
        rec.scal = H.scal;
        rec.beta = H.beta;
        rec.pad = 0.0;
        hinf[b * PW + wv] = rec;
        inf->key = key;   // the pad is never read
        inf->sum = sum;
      }
      mine[g] = v0;
#pragma unroll
      for (int sl = 1; sl < SMX; ++sl) mine[G * sl + g] = t[sl];
    }
    if (key == 0ull && lane == 0) {   // no candidate left in this wave
      inf->key = 0ull;
      inf->sum = sum;
    }
    __syncthreads();
    // every wave's record is loaded before any is compared, so that one LDS latency covers
    // all four, and the choice is made with selects
    unsigned long long ck[PW];
    double cs[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      ck[q] = info[b * PW + q].key;
      cs[q] = info[b * PW + q].sum;
    }
    unsigned long long gkey = 0ull;
    double tail = 0.0;
    int gw = 0;
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      tail += cs[q];
      const bool better = ck[q] > gkey;
      gkey = better ? ck[q] : gkey;
      gw = better ? q : gw;
    }
    // the winner's column and reflector are taken before the stop tests, so that every path
    // through here defines them (no copies of the previous step's values are kept for the
    // exit); with no candidate left they are stale and unused
    pc = key_col(gkey);
    X = cand + (b * PW + gw) * MR;
    const HouseRec H = hinf[b * PW + gw];
    beta = H.beta;
    scal = H.scal;
    wf = H.wf;
    if (!(tail == tail) || isinf(tail)) {
      if (tid == 0 && *code == CM_OK) *code = CM_E_NONFINITE;
      return true;
    }
    if (i >= kmax || (i >= 1 && tail <= delta2)) return true;
    if (i == kcap) {
      if (tid == 0 && *code == CM_OK) *code = CM_E_RANKCAP;
      return true;
    }
    if (tid == 0) taus[i] = H.tau;
    return false;
  };

  int i = 0;
  bool stop = select(0);
  while (!stop) {
    const int j = i / G;
    // slots holding rows >= i (and possibly one finished row); none in a wave with no
    // candidate column left, whose entries are not read again (it only writes its zeros of
    // row i of R)
    const int live = __ballot(act) != 0 ? hrows - j : 0;
    const double2 *Xg = X + g;
    // this lane's rows of the pivot column: with up to 12 slots all are loaded at once (one
    // LDS latency) and kept for the update; above that they are read per group of four
    constexpr bool XPRE = SMX <= 12;
    double2 xv[XPRE ? SMX : 1];
    if constexpr (XPRE) {
#pragma unroll
      for (int sl = 0; sl < SMX; ++sl) xv[sl] = Xg[G * sl];
    }
    auto xat = [&](int sl) -> double2 {
      if constexpr (XPRE) return xv[sl];
      else return Xg[G * sl];
    };
    // w_c = conj(tau) sum_r conj(v_r) T[r, c] with v = x scal, summed over the pair
    double2 pz[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) pz[e] = cmk(0.0, 0.0);
#pragma unroll
    for (int q4 = 0; q4 < SMX / 4; ++q4)
      if (4 * q4 < live) {
#pragma unroll
        for (int e = 0; e < 4; ++e) ccfma(pz[e], xat(4 * q4 + e), t[4 * q4 + e]);
      }
    double2 pw = cadd(cadd(pz[0], pz[1]), cadd(pz[2], pz[3]));
    la::grp_sum2(pw.x, pw.y, G);   // both parts' stages interleaved
    const double2 ws = cmul(wf, pw);   // scal w_c
    // T <- H^H T; slot 0 of lane g holds row G j + g: row i (g = i % G) or a row finished
    // before it (g < i % G), neither of which counts towards the remaining norms
    double nz[2] = {0.0, 0.0};
    const bool skip0 = g <= i % G;
#pragma unroll
    for (int q4 = 0; q4 < SMX / 4; ++q4)
      if (4 * q4 < live) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int sl = 4 * q4 + e;
          const double2 x = xat(sl);
          double2 y = t[sl];
          // y -= x ws and the remaining norm, as chained FMAs (two per component)
          y.x = fma(x.y, ws.y, fma(-x.x, ws.x, y.x));
          y.y = fma(-x.y, ws.x, fma(-x.x, ws.y, y.y));
          t[sl] = y;
          if (sl > 0 || !skip0) nz[e & 1] = fma(y.y, y.y, fma(y.x, y.x, nz[e & 1]));
        }
      }
    // row i of R: slot 0 of lane i % G, just updated (a wave with no candidate left updates
    // nothing and writes zeros)
    if (cok && g == i % G) C[(int64_t)i * p + c] = (c == pc) ? cmk(beta, 0.0) : (act ? t[0] : cmk(0.0, 0.0));
    // after the last step of a group of G, every lane moves its slots down by one (every
    // slot moves: a copy bounded by the live count would become a memmove that keeps T out
    // of registers)
    if (i % G == G - 1) {
#pragma unroll
      for (int sl = 0; sl + 1 < SMX; ++sl) t[sl] = t[sl + 1];
      t[SMX - 1] = cmk(0.0, 0.0);
    }
    nrm = la::grp_sum(nz[0] + nz[1], G);
    if (c == pc) act = false;
    // reflector i for the Q accumulation: V[i][r] = v_r (zero above row i and below row m)
    if (tid < MR) {
      double2 v = cmk(0.0, 0.0);
      if (tid == i) v = cmk(1.0, 0.0);
      else if (tid > i && tid < m) v = cmul(X[tid - G * j], scal);
      V[i * MR + tid] = v;
    }
    ++i;
    stop = select(i);
  }
  const int k = i;
  // Q = H_0 ... H_{k-1} [I_k; 0], barrier-free: column cq of Q on the eight lanes
  // 8 (cq mod 32) .. 8 (cq mod 32) + 7 (a workgroup's 32 groups of eight take columns cq,
  // cq + 32, ... up to k <= 48), lane h of the eight holding rows 8 s + h (s < SMX / 4, as
  // m <= 2 SMX); the dot products are summed with DPP. Reflector jj - 1 and its tau are
  // loaded while reflector jj is applied, so the LDS latency overlaps the arithmetic.
  {
    constexpr int QS = (G * SMX / 8 < MR / 8) ? G * SMX / 8 : MR / 8;
    const int h = tid & 7;
    for (int cq = tid >> 3; cq < k; cq += CM_WG / 8) {   // uniform over each group of eight lanes
      double2 qv[QS], vc[QS], vn[QS];
#pragma unroll
      for (int sl = 0; sl < QS; ++sl) qv[sl] = cmk(8 * sl + h == cq ? 1.0 : 0.0, 0.0);
      double2 tc = taus[k - 1], tn = cmk(0.0, 0.0);
#pragma unroll
      for (int sl = 0; sl < QS; ++sl) vc[sl] = V[(k - 1) * MR + 8 * sl + h];
      for (int jj = k - 1; jj >= 0; --jj) {
        if (jj > 0) {
          tn = taus[jj - 1];
#pragma unroll
          for (int sl = 0; sl < QS; ++sl) vn[sl] = V[(jj - 1) * MR + 8 * sl + h];
        }
        if (tc.x != 0.0 || tc.y != 0.0) {
          double2 d = cmk(0.0, 0.0);
#pragma unroll
          for (int sl = 0; sl < QS; ++sl)
            if (8 * sl + 7 >= jj && 8 * sl < m) ccfma(d, vc[sl], qv[sl]);   // V[jj][r] = 0 for r < jj, r >= m
          la::grp_sum2(d.x, d.y, 8);
          const double2 wq = cmul(tc, d);
#pragma unroll
          for (int sl = 0; sl < QS; ++sl)
            if (8 * sl + 7 >= jj && 8 * sl < m) {   // qv -= v wq, as chained FMAs
              qv[sl].x = fma(vc[sl].y, wq.y, fma(-vc[sl].x, wq.x, qv[sl].x));
              qv[sl].y = fma(-vc[sl].y, wq.x, fma(-vc[sl].x, wq.y, qv[sl].y));
            }
        }
        tc = tn;
#pragma unroll
        for (int sl = 0; sl < QS; ++sl) vc[sl] = vn[sl];
      }
#pragma unroll
      for (int sl = 0; sl < QS; ++sl)
        if (8 * sl + h < m) cstore<T>::st(Yout, (int64_t)(8 * sl + h) * k + cq, qv[sl]);
    }
  }
  __syncthreads();   // the arena and the carry are reused by the next site
  return k;
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(CM_WG, 3) void k_zipup(TTView w, int w_slots, TTView x, TTView y, double tol, int cap,
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
      // operator n is train n of w (w_slots trains)
      if (n < 1 || n > CM_MAX_N || n >= w_slots || y.n[b] != n || w.n[n] != n) c = CM_E_INVALID;
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
      if (!last && pair_site_fits<T>(sd, chicap, zlds_bytes<T>()))
        k = (p <= 32 && m <= 32) ? zip_site_pair<T, 4, 8>(lds_arena, sd, Wl, Al, C, Yout, delta2, chicap, &code_sh)
            : (p <= 64 && m <= 32) ? zip_site_pair<T, 8, 4>(lds_arena, sd, Wl, Al, C, Yout, delta2, chicap, &code_sh)
            : p <= 64            ? zip_site_pair<T, 12, 4>(lds_arena, sd, Wl, Al, C, Yout, delta2, chicap, &code_sh)
            : m <= 16            ? zip_site_pair<T, 8, 2>(lds_arena, sd, Wl, Al, C, Yout, delta2, chicap, &code_sh)
            : m <= 24            ? zip_site_pair<T, 12, 2>(lds_arena, sd, Wl, Al, C, Yout, delta2, chicap, &code_sh)
            : m <= 32            ? zip_site_pair<T, 16, 2>(lds_arena, sd, Wl, Al, C, Yout, delta2, chicap, &code_sh)
                                 : zip_site_pair<T, SM, 2>(lds_arena, sd, Wl, Al, C, Yout, delta2, chicap, &code_sh);
      else if (need <= (size_t)zlds_bytes<T>())
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

// Validates the arguments of cm_sfft_apply and launches the zip-up over `ws` (one persistent
// workgroup per slab of cm_zip_slab_bytes(cap_rank) bytes, at most one per instance).
static cm_status zip_apply(const cm_tt_batch *w_by_n, const cm_tt_batch *x, double tol, int cap_rank, cm_tt_batch *y,
                           int32_t *status, void *ws, size_t ws_bytes, void *stream) {
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
  hipStream_t s = (hipStream_t)stream;
  TTView vw = tt_view(w_by_n), vx = tt_view(x), vy = tt_view(y);
  CM_HIP_CHECK(cm_allow_lds(k_zipup<float2>, zlds_bytes<float2>()));
  CM_HIP_CHECK(cm_allow_lds(k_zipup<double2>, zlds_bytes<double2>()));
  if (x->dtype == CM_C64)
    hipLaunchKernelGGL(k_zipup<float2>, dim3(slots), dim3(CM_WG), zlds_bytes<float2>(), s, vw, w_by_n->batch, vx, vy,
                       tol, cap_rank, batch, status, (char *)ws, slab, mc);
  else
    hipLaunchKernelGGL(k_zipup<double2>, dim3(slots), dim3(CM_WG), zlds_bytes<double2>(), s, vw, w_by_n->batch, vx,
                       vy, tol, cap_rank, batch, status, (char *)ws, slab, mc);
  CM_LAUNCH_CHECK();
  y->flags = CM_TT_LEFT_ORTHO;
  return CM_OK;
}

extern "C" cm_status cm_sfft_apply(const cm_tt_batch *w_by_n, const cm_tt_batch *x, double tol, int cap_rank,
                                   cm_tt_batch *y, int32_t *status, void *ws, size_t ws_bytes, void *stream) {
  return zip_apply(w_by_n, x, tol, cap_rank, y, status, ws, ws_bytes, stream);
}

// ---- allocation-free variant -----------------------------------------------------------
// The zip-up's per-workgroup slabs come from a fixed device array instead of a caller
// workspace. In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (each device holds
// its own copy of the array) and only that address is passed to kernels. The kernel writes
// every slab word it reads for an instance before reading it, so nothing needs clearing
// between calls; calls that overlap on one device share the array and race.
constexpr size_t ZIP_NOALLOC_BYTES = (size_t)256 << 20;
static __device__ __align__(256) char scratch[ZIP_NOALLOC_BYTES];

namespace {
constexpr int ZIP_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[ZIP_MAX_DEVICES] = {};

cm_status zip_scratch(void **out) {
  int dev = 0;
  CM_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= ZIP_MAX_DEVICES) return CM_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    CM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return CM_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CM_OK;
}
}  // namespace

extern "C" size_t cm_sfft_apply_noalloc_scratch_bytes(void) { return ZIP_NOALLOC_BYTES; }

extern "C" cm_status cm_sfft_apply_noalloc(const cm_tt_batch *w_by_n, const cm_tt_batch *x, double tol, int cap_rank,
                                           cm_tt_batch *y, int32_t *status, void *stream) {
  if (cap_rank < 1 || cap_rank > 64) return CM_E_INVALID;
  if (cm_zip_slab_bytes(cap_rank) > ZIP_NOALLOC_BYTES) return CM_E_UNSUPPORTED;
  if (x && x->batch == 0) return zip_apply(w_by_n, x, tol, cap_rank, y, status, nullptr, 0, stream);
  void *ptr = nullptr;
  const cm_status e = zip_scratch(&ptr);
  if (e != CM_OK) return e;
  return zip_apply(w_by_n, x, tol, cap_rank, y, status, ptr, ZIP_NOALLOC_BYTES, stream);
}
