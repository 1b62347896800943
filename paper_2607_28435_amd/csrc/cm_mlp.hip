// Pricing surrogate network (a project addition; the paper has no learned component):
// forward, backward, MSE, Adam and the gate. Layer equations and the parameter layout are
// in cm.h.
//
// The 256 x 256 layers are GEMMs on BF16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32
// accumulation. Forward and backward-data use k_gemm_ws (the weight matrix stays in LDS for
// a persistent workgroup that streams 32-row tiles of activations); the weight gradients use
// k_gemm (64 x 64 output tiles as four 32 x 32 wave tiles, 32-deep K slices of both operands
// staged in LDS as BF16, split-K over the batch). An operand that comes from FP32
// activations is split into hi + lo BF16 parts (two MFMAs per step), so its rounding error
// is ~2^-16 instead of 2^-8. Operand lane layout (32x32x16): lane l holds
// A[l % 32][8 (l / 32) + i] and B[8 (l / 32) + i][l % 32], i < 8; accumulator v of lane l is
// C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
#include "cm_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NW = CM_MLP_WIDTH;
constexpr int NIN = CM_MLP_NIN;
constexpr int OFF_W1 = 0, OFF_B1 = 1792, OFF_W5 = 199424, OFF_B5 = 199680;
__host__ __device__ constexpr int off_w(int l) { return l == 2 ? 2048 : l == 3 ? 67840 : 133632; }
__host__ __device__ constexpr int off_b(int l) { return l == 2 ? 67584 : l == 3 ? 133376 : 199168; }
static_assert(OFF_B5 + 1 == CM_MLP_NPARAMS, "parameter layout");

// The BF16 copies of W2..W4 (w_bf16) are kept in MFMA fragment order: the eight weights
// W_l[n][k8 .. k8 + 7] (k8 a multiple of 8) are lane 32 ((k8 / 8) mod 2) + n mod 32 of the
// 64-lane, 1 KB block (n / 32) 16 + k8 / 16, which is what lane of a 32 x 32 x 16 MFMA
// A fragment holds them. One neuron block's fragment for one K step is then one contiguous
// 1 KB read (eight full cache lines) rather than 32 pieces of 32 rows.
constexpr int WFB = 512;   // weights per fragment block
__host__ __device__ constexpr int wfrag(int n, int k) {
  return ((((n >> 5) * 16 + (k >> 4)) * 64 + ((k >> 3) & 1) * 32 + (n & 31)) << 3) + (k & 7);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
// SiLU from the hardware exp2 and reciprocal (a few ulps): for the activation operand of the
// layer GEMMs, whose hi + lo BF16 split keeps about 2^-16 of it anyway. Large |z| behave:
// exp2 overflows to inf and the reciprocal to 0 (z -> -inf), or exp2 goes to 0 (z -> +inf).
__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}
__device__ __forceinline__ float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// float -> bf16 bits, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ GEMM
constexpr int GT = 64;        // tile edge
constexpr int KC = 32;        // K slice staged per step
constexpr int KP = KC + 8;    // LDS row pitch (bf16 elements): 80 bytes, 16-byte aligned rows

enum { A_ROWMAJOR = 0, A_COLMAJOR = 1 };        // A[m lda + k] or A[k lda + m]  (FP32)
enum { B_F32_KN = 0, B_BF16_NK = 1, B_BF16_KN = 2 };  // B[k ldb + n] fp32, B[n ldb + k] bf16, B[k ldb + n] bf16
enum { F_NONE = 0, F_SILU = 1 };
enum { E_BIAS_STORE = 0, E_DSILU_STORE = 1, E_ATOMIC_ADD = 2 };

struct GemmArgs {
  const float *A;
  int lda;
  const void *B;
  int ldb;
  int M, N, K, kspan;   // kspan: K range per blockIdx.z
  float *C;
  int ldc;
  const float *bias;    // E_BIAS_STORE
  const float *Z;       // E_DSILU_STORE: multiply by silu'(Z[m ldc + n])
};

template <int AL, int AF, bool ASPLIT, int BK, int BF, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[2][GT][KP];
  __shared__ __align__(16) uint16_t Bs[GT][KP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int n0 = blockIdx.x * GT, m0 = blockIdx.y * GT;
  const int kbeg = blockIdx.z * g.kspan;
  const int kend = min(g.K, kbeg + g.kspan);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    // ---- stage A (64 x 32)
    if (AL == A_ROWMAJOR) {
      const int m = tid >> 2, k8 = (tid & 3) * 8;
      const int gm = m0 + m;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gk = k0 + k8 + i;
        float v = (gm < g.M && gk < kend) ? g.A[(int64_t)gm * g.lda + gk] : 0.0f;
        if (AF == F_SILU) v = silu_f(v);
        const uint16_t hi = f2bf(v);
        As[0][m][k8 + i] = hi;
        if (ASPLIT) As[1][m][k8 + i] = f2bf(v - bf2f(hi));
      }
    } else {
      const int k = tid >> 3, m8 = (tid & 7) * 8;
      const int gk = k0 + k;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gm = m0 + m8 + i;
        float v = (gm < g.M && gk < kend) ? g.A[(int64_t)gk * g.lda + gm] : 0.0f;
        if (AF == F_SILU) v = silu_f(v);
        const uint16_t hi = f2bf(v);
        As[0][m8 + i][k] = hi;
        if (ASPLIT) As[1][m8 + i][k] = f2bf(v - bf2f(hi));
      }
    }
    // ---- stage B (32 x 64) as Bs[n][k]
    if (BK == B_BF16_NK) {
      const int n = tid >> 2, k8 = (tid & 3) * 8;
      const int gn = n0 + n;
      const uint16_t *Bb = (const uint16_t *)g.B;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gk = k0 + k8 + i;
        Bs[n][k8 + i] = (gn < g.N && gk < kend) ? Bb[(int64_t)gn * g.ldb + gk] : (uint16_t)0;
      }
    } else {
      const int k = tid >> 3, n8 = (tid & 7) * 8;
      const int gk = k0 + k;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int gn = n0 + n8 + i;
        uint16_t h = 0;
        if (gn < g.N && gk < kend) {
          if (BK == B_BF16_KN) {
            h = ((const uint16_t *)g.B)[(int64_t)gk * g.ldb + gn];
          } else {
            float v = ((const float *)g.B)[(int64_t)gk * g.ldb + gn];
            if (BF == F_SILU) v = silu_f(v);
            h = f2bf(v);
          }
        }
        Bs[n8 + i][k] = h;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      const int kq = kk + 8 * (lane >> 5);
      const s16x8 bv = *(const s16x8 *)&Bs[wn * 32 + (lane & 31)][kq];
      const s16x8 av = *(const s16x8 *)&As[0][wm * 32 + (lane & 31)][kq];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                    acc, 0, 0, 0);
      if (ASPLIT) {
        const s16x8 al = *(const s16x8 *)&As[1][wm * 32 + (lane & 31)][kq];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al),
                                                      __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // ---- epilogue
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int n = n0 + wn * 32 + (lane & 31);
    if (m < g.M && n < g.N) {
      float* c = g.C + (int64_t)m * g.ldc + n;
      if (EPI == E_BIAS_STORE) *c = acc[v] + g.bias[n];
      else if (EPI == E_DSILU_STORE) *c = acc[v] * silu_grad_f(g.Z[(int64_t)m * g.ldc + n]);
      else atomicAdd(c, acc[v]);
    }
  }
}

// Weight-stationary layer for the batch dimension: C[M x 256] = epi(op(A) W'), with the
// whole 256 x 256 BF16 weight matrix held in LDS (Ws[n][k], 132 KB) for the workgroup's
// lifetime and the workgroup looping over 32-row tiles of A. Each wave computes 32 rows x 64
// columns (two 32 x 32 accumulators); it reads its A operand straight from global memory
// (FP32, split into hi + lo BF16 in registers; the four waves read the same rows, which
// the L1 serves).
//   W_NK: W' = W^T, Ws[n][k] = W[n][k]   (forward: z = a W^T + b)
//   W_KN: W' = W,   Ws[n][k] = W[k][n]   (backward data: delta W)
enum { W_NK = 0, W_KN = 1 };
constexpr int WSP = NW + 8;   // LDS row pitch of Ws (bf16): 528 bytes, 16-byte aligned

// Up to WS_TILES row tiles are in flight per workgroup: wave w computes columns
// 128 (w % 2) .. +127 of tiles blockIdx.x + (w / 2 + WS_TILES i) gridDim.x, so the LDS copy of
// the weights serves 16 waves (four per SIMD) on large batches while small batches still
// spread one tile per workgroup over the CUs; each activation element is transformed
// (SiLU, hi/lo split) by the two waves of its tile.
constexpr int WS_TILES = 8;
constexpr int WS_THREADS = 1024;

template <int WL, int AF, int EPI>
__global__ __launch_bounds__(WS_THREADS) void k_gemm_ws(const float *__restrict__ A, const uint16_t *__restrict__ W,
                                                        int M, float *__restrict__ C, const float *__restrict__ bias,
                                                        const float *__restrict__ Z) {
  extern __shared__ __align__(16) uint16_t Ws[];   // [NW][WSP]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // W is in fragment order: 16-byte piece c holds row 32 (c / 1024) + c mod 32, columns
  // 16 ((c / 64) mod 16) + 8 ((c / 32) mod 2) .. +7
  if (WL == W_NK) {
    for (int c = tid; c < NW * NW / 8; c += WS_THREADS) {
      const int blk = c >> 6, ln = c & 63;
      const int n = 32 * (blk >> 4) + (ln & 31), k8 = 16 * (blk & 15) + 8 * (ln >> 5);
      *(uint4 *)&Ws[n * WSP + k8] = *(const uint4 *)&W[8 * c];
    }
  } else {
    for (int e = tid; e < NW * NW; e += WS_THREADS) {
      const int blk = e >> 9, ln = (e >> 3) & 63;
      const int row = 32 * (blk >> 4) + (ln & 31), col = 16 * (blk & 15) + 8 * (ln >> 5) + (e & 7);
      Ws[col * WSP + row] = W[e];
    }
  }
  __syncthreads();
  const int ntiles = (M + 31) / 32;
  const int col0 = (wave & 1) * 128;
  for (int t = blockIdx.x + (wave >> 1) * gridDim.x; t < ntiles; t += gridDim.x * WS_TILES) {
    const int row = t * 32 + (lane & 31);
    const bool rok = row < M;
    f32x16 acc[4];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[h][v] = 0.0f;
    const float *arow = A + (int64_t)(rok ? row : 0) * NW;
#pragma unroll 2
    for (int kk = 0; kk < NW; kk += 16) {
      const int kq = kk + 8 * (lane >> 5);
      float a[8];
      if (rok) {
        const float4 x0 = *(const float4 *)&arow[kq], x1 = *(const float4 *)&arow[kq + 4];
        a[0] = x0.x; a[1] = x0.y; a[2] = x0.z; a[3] = x0.w; a[4] = x1.x; a[5] = x1.y; a[6] = x1.z; a[7] = x1.w;
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = 0.0f;
      }
      s16x8 ah, al;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        // hi + lo BF16 parts by the hardware conversion (v_cvt_pk_bf16_f32); the split only
        // has to represent v, so its rounding mode does not matter
        const float v = (AF == F_SILU) ? silu_fast(a[i]) : a[i];
        const uint16_t h = __builtin_bit_cast(uint16_t, (__bf16)v);
        ah[i] = (short)h;
        al[i] = (short)__builtin_bit_cast(uint16_t, (__bf16)(v - bf2f(h)));
      }
      const bf16x8 AH = __builtin_bit_cast(bf16x8, ah), AL = __builtin_bit_cast(bf16x8, al);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const s16x8 b = *(const s16x8 *)&Ws[(col0 + 32 * h + (lane & 31)) * WSP + kq];
        acc[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AH, __builtin_bit_cast(bf16x8, b), acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AL, __builtin_bit_cast(bf16x8, b), acc[h], 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = t * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (m < M) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int n = col0 + 32 * h + (lane & 31);
          const float val = acc[h][v];
          float *c = C + (int64_t)m * NW + n;
          if (EPI == E_BIAS_STORE) *c = val + bias[n];
          else *c = val * silu_grad_f(Z[(int64_t)m * NW + n]);
        }
      }
    }
  }
}
constexpr size_t WS_LDS = sizeof(uint16_t) * NW * WSP;

// ------------------------------------------------------------------ fused inference
// The whole network for tiles of FM = 64 queries, with no activation leaving the CU. Each
// layer is computed transposed, Z^T = W A^T: the weights are the MFMA's A operand (32 output
// neurons x 16 inputs per fragment, 16-byte loads of W rows from L2, where the three
// 256 x 256 BF16 matrices stay) and the activations its B operand, read from LDS, where a
// tile's activations live as their hi and lo BF16 parts (Ah, Al: [query][neuron], 68 KB per
// tile). A wave computes neurons 64 w .. 64 w + 63 for all 64 queries of its tile: four
// 32 x 32 accumulators, K in steps of 16, the A fragments loaded a few steps ahead, all hi
// products of a step before the lo products. An accumulator lane holds four consecutive
// neurons of one query per group, so the epilogue (bias, SiLU, hi / lo split) converts in
// pairs and stores eight-byte packets. The first layer (7 -> 256, FP32 weights) is three
// MFMAs per block with both operands split into hi and lo parts (W_hi x_hi + W_hi x_lo +
// W_lo x_hi: relative error ~2^-16, below the hidden layers' own); the last folds
// W5 silu(z4) into per-query partial sums.
//
// A workgroup is two groups of four waves, each with a tile of its own, and a tile goes
// through six phases: (0) the previous tile's output fold, then layer 1 and its epilogue,
// (1) layer 2's MFMAs, (2) its epilogue, (3) layer 3's MFMAs, (4) its epilogue, (5) layer
// 4's MFMAs. Group 1 runs one phase behind group 0 and one barrier of the whole workgroup
// ends every phase, so the two waves that share a SIMD (wave w of each group) alternate:
// one issues MFMAs while the other runs its VALU epilogue. The barrier also orders each
// group's own LDS traffic: a phase's epilogue writes the activations the next phase's MFMAs
// read, after every wave of the group has read the previous layer's.
constexpr int FM = 64;               // queries per tile
constexpr int FQB = FM / 32;         // query blocks
constexpr int FP = NW + 8;           // LDS row pitch (bf16): 528 bytes, 16-byte aligned
constexpr size_t FUSED_LDS = sizeof(uint16_t) * 2 * 2 * FM * FP;   // two tiles, hi and lo
constexpr int FPD = 3;               // K steps between a weight fragment's load and its use
constexpr int FPH = 6;               // phases per tile

__device__ __forceinline__ void split8(const float *v, s16x8 &hi, s16x8 &lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint16_t h = __builtin_bit_cast(uint16_t, (__bf16)v[i]);
    hi[i] = (short)h;
    lo[i] = (short)__builtin_bit_cast(uint16_t, (__bf16)(v[i] - bf2f(h)));
  }
}

__global__ __launch_bounds__(512, 1) void k_mlp_fused(const float *__restrict__ x, int B, const float *__restrict__ p,
                                                   const uint16_t *__restrict__ wbf, cm_mlp net,
                                                   float *__restrict__ y) {
  extern __shared__ __align__(16) uint16_t fl[];
  __shared__ float bsh[4][NW];   // b1..b4
  __shared__ float w5s[NW];
  __shared__ float ys[2][4][FM];  // per-group, per-wave partial outputs
  const int tid = threadIdx.x, lane = tid & 63;
  const int grp = tid >> 8, w = (tid >> 6) & 3, gtid = tid & 255;
  const int l32 = lane & 31, hi32 = lane >> 5;
  uint16_t *Ah = fl + grp * 2 * FM * FP, *Al = Ah + FM * FP;
  for (int e = tid; e < NW; e += 512) {
    bsh[0][e] = p[OFF_B1 + e];
    bsh[1][e] = p[off_b(2) + e];
    bsh[2][e] = p[off_b(3) + e];
    bsh[3][e] = p[off_b(4) + e];
    w5s[e] = p[OFF_W5 + e];
  }
  // first-layer A fragments: W1[n][k], n = 64 w + 32 mb + l32, k = 8 hi32 + i (k < 7; zero
  // beyond), split into hi and lo
  bf16x8 w1h[2], w1l[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    float v[8];
    const int n = 64 * w + 32 * mb + l32;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 8 * hi32 + i;
      v[i] = k < NIN ? p[OFF_W1 + n * NIN + k] : 0.0f;
    }
    s16x8 h, l;
    split8(v, h, l);
    w1h[mb] = __builtin_bit_cast(bf16x8, h);
    w1l[mb] = __builtin_bit_cast(bf16x8, l);
  }
  __syncthreads();
  // the tiles of group g are 2 blockIdx.x + g + i stride, i = 0, 1, ...
  const int ntiles = (B + FM - 1) / FM;
  const int stride = 2 * gridDim.x;
  const int f0 = 2 * blockIdx.x, f1 = f0 + 1;
  const int n0 = f0 < ntiles ? (ntiles - 1 - f0) / stride + 1 : 0;
  const int n1 = f1 < ntiles ? (ntiles - 1 - f1) / stride + 1 : 0;
  const int nmine = grp ? n1 : n0;
  // a group's own steps: FPH per tile, then the last tile's fold (phase 0) and output
  // (phase 1); group 1 starts one step late. Every wave runs the same number of barriers.
  const int last0 = n0 ? FPH * n0 + 2 : 0, last1 = n1 ? 1 + FPH * n1 + 2 : 0;
  const int nsteps = last0 > last1 ? last0 : last1;
  f32x16 acc[2][FQB];
  s16x8 ar0[FPD], ar1[FPD];
  // accumulators start at the layer's bias: element v of block mb is neuron
  // 64 w + 32 mb + 8 (v / 4) + 4 hi32 + v mod 4, the same for both query blocks
  auto bias_init = [&](const float *bias) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      f32x16 bz;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 b4 = *(const float4 *)&bias[64 * w + 32 * mb + 8 * g + 4 * hi32];
        bz[4 * g] = b4.x;
        bz[4 * g + 1] = b4.y;
        bz[4 * g + 2] = b4.z;
        bz[4 * g + 3] = b4.w;
      }
#pragma unroll
      for (int qb = 0; qb < FQB; ++qb) acc[mb][qb] = bz;
    }
  };
  for (int st = 0; st < nsteps; ++st) {
    const int ls = st - grp;
    if (ls >= 0 && ls < FPH * nmine + 2) {
      const int i = ls / FPH, ph = ls - FPH * i;
      const int q0 = (f0 + grp + i * stride) * FM;   // this step's tile (while i < nmine)
      if (ph & 1) {
        if (ph == 1 && i > 0 && gtid < FM && q0 - stride * FM + gtid < B) {
          const int t = gtid;
          y[q0 - stride * FM + t] = ((ys[grp][0][t] + ys[grp][1][t]) + (ys[grp][2][t] + ys[grp][3][t])) + p[OFF_B5];
        }
        if (i < nmine) {
          // layers 2, 3, 4 at phases 1, 3, 5
          const uint16_t *W = wbf + (int64_t)(ph >> 1) * NW * NW;
          bias_init(bsh[1 + (ph >> 1)]);
          // A fragment of neuron block 2 w + mb at K step ks: W[n][16 ks + 8 hi32 .. +7],
          // n = 64 w + 32 mb + l32, one contiguous 1 KB block of the fragment-ordered copy,
          // read from L2 FPD steps ahead into a ring indexed statically by the unrolled K loop
          const uint16_t *wrow0 = W + (int64_t)(2 * w) * 16 * WFB + 8 * lane;
          const uint16_t *wrow1 = wrow0 + 16 * WFB;
          // B fragments of query block qb at K step kk: Ah / Al[q][kk + 8 hi32 .. +7], q = 32 qb + l32
          const int boff = l32 * FP + 8 * hi32;
          s16x8 bhn[FQB], bln[FQB];
#pragma unroll
          for (int qb = 0; qb < FQB; ++qb) {
            bhn[qb] = *(const s16x8 *)&Ah[boff + 32 * qb * FP];
            bln[qb] = *(const s16x8 *)&Al[boff + 32 * qb * FP];
          }
#pragma unroll
          for (int ks = 0; ks < NW / 16; ++ks) {
            const int kk = 16 * ks;
            const bf16x8 A0 = __builtin_bit_cast(bf16x8, ar0[ks % FPD]), A1 = __builtin_bit_cast(bf16x8, ar1[ks % FPD]);
            if (ks + FPD < NW / 16) {
              ar0[ks % FPD] = *(const s16x8 *)(wrow0 + (ks + FPD) * WFB);
              ar1[ks % FPD] = *(const s16x8 *)(wrow1 + (ks + FPD) * WFB);
            }
            s16x8 bh[FQB], bl[FQB];
#pragma unroll
            for (int qb = 0; qb < FQB; ++qb) {
              bh[qb] = bhn[qb];
              bl[qb] = bln[qb];
            }
            if (kk + 16 < NW) {   // next step's activations, in flight during this step's MFMAs
#pragma unroll
              for (int qb = 0; qb < FQB; ++qb) {
                bhn[qb] = *(const s16x8 *)&Ah[boff + 32 * qb * FP + kk + 16];
                bln[qb] = *(const s16x8 *)&Al[boff + 32 * qb * FP + kk + 16];
              }
            }
#pragma unroll
            for (int qb = 0; qb < FQB; ++qb) {
              const bf16x8 BH = __builtin_bit_cast(bf16x8, bh[qb]);
              acc[0][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, BH, acc[0][qb], 0, 0, 0);
              acc[1][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, BH, acc[1][qb], 0, 0, 0);
            }
#pragma unroll
            for (int qb = 0; qb < FQB; ++qb) {
              const bf16x8 BL = __builtin_bit_cast(bf16x8, bl[qb]);
              acc[0][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, BL, acc[0][qb], 0, 0, 0);
              acc[1][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, BL, acc[1][qb], 0, 0, 0);
            }
          }
        }
      } else {
        if (ph == 0) {
          if (i > 0) {
            // the previous tile's y[q] = b5 + sum_n W5[n] silu(z4[n][q]) over this lane's 32
            // neurons; the two half waves hold the same queries' other neurons
#pragma unroll
            for (int qb = 0; qb < FQB; ++qb) {
              float sacc = 0.0f;
#pragma unroll
              for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                  const int n = 64 * w + 32 * mb + 8 * (v >> 2) + 4 * hi32 + (v & 3);
                  sacc += w5s[n] * silu_fast(acc[mb][qb][v]);
                }
              const float s2 = sacc + __shfl_xor(sacc, 32, 64);
              if (hi32 == 0) ys[grp][w][32 * qb + l32] = s2;
            }
          }
          if (i < nmine) {
            // layer 1: B fragments xn[q][k], q = 32 qb + l32, k = 8 hi32 + i
            bf16x8 xh[FQB], xl[FQB];
#pragma unroll
            for (int qb = 0; qb < FQB; ++qb) {
              const int q = q0 + 32 * qb + l32;
              float v[8];
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                const int k = 8 * hi32 + j;
                v[j] = (k < NIN && q < B) ? (x[(int64_t)q * NIN + k] - net.shift[k]) * net.scale[k] : 0.0f;
              }
              s16x8 h, l;
              split8(v, h, l);
              xh[qb] = __builtin_bit_cast(bf16x8, h);
              xl[qb] = __builtin_bit_cast(bf16x8, l);
            }
            bias_init(bsh[0]);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
              for (int qb = 0; qb < FQB; ++qb) {
                acc[mb][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1h[mb], xh[qb], acc[mb][qb], 0, 0, 0);
                acc[mb][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1h[mb], xl[qb], acc[mb][qb], 0, 0, 0);
                acc[mb][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1l[mb], xh[qb], acc[mb][qb], 0, 0, 0);
              }
          }
        }
        if (i < nmine) {
          {
            // the next phase's first weight fragments, in flight during this epilogue
            const uint16_t *wrow0 = wbf + (int64_t)(ph >> 1) * NW * NW + (int64_t)(2 * w) * 16 * WFB + 8 * lane;
            const uint16_t *wrow1 = wrow0 + 16 * WFB;
#pragma unroll
            for (int s = 0; s < FPD; ++s) {
              ar0[s] = *(const s16x8 *)(wrow0 + s * WFB);
              ar1[s] = *(const s16x8 *)(wrow1 + s * WFB);
            }
          }
          // epilogue of layers 1, 2, 3 at phases 0, 2, 4: neurons 64 w + 32 mb + 8 g + 4 hi32 + j
          // (j < 4) of query 32 qb + l32 are acc[mb][qb][4 g + j], bias included
#pragma unroll
          for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int qb = 0; qb < FQB; ++qb)
#pragma unroll
              for (int g = 0; g < 4; ++g) {
                const int n = 64 * w + 32 * mb + 8 * g + 4 * hi32;
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = silu_fast(acc[mb][qb][4 * g + j]);
                uint16_t h[4], lo[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  h[j] = __builtin_bit_cast(uint16_t, (__bf16)v[j]);
                  lo[j] = __builtin_bit_cast(uint16_t, (__bf16)(v[j] - bf2f(h[j])));
                }
                const int off = (32 * qb + l32) * FP + n;
                *(uint2 *)&Ah[off] = make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
                *(uint2 *)&Al[off] = make_uint2(lo[0] | ((uint32_t)lo[1] << 16), lo[2] | ((uint32_t)lo[3] << 16));
              }
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ small layers
// Z1[b][n] = b1[n] + sum_i W1[n][i] xn[b][i]
__global__ void k_mlp_in(const float *__restrict__ x, int B, const float *__restrict__ p, cm_mlp net,
                         float *__restrict__ Z1) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * NW) return;
  const int b = (int)(e / NW), n = (int)(e % NW);
  float acc = p[OFF_B1 + n];
#pragma unroll
  for (int i = 0; i < NIN; ++i) acc += p[OFF_W1 + n * NIN + i] * ((x[(int64_t)b * NIN + i] - net.shift[i]) * net.scale[i]);
  Z1[e] = acc;
}

// y[b] = b5 + sum_n W5[n] silu(Z4[b][n]); one wavefront per row
__global__ void k_mlp_out(const float *__restrict__ Z4, int B, const float *__restrict__ p, float *__restrict__ y) {
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  float acc = 0.0f;
  for (int n = lane; n < NW; n += 64) acc += p[OFF_W5 + n] * silu_f(Z4[(int64_t)b * NW + n]);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) y[b] = acc + p[OFF_B5];
}

// delta4[b][n] = dy[b] W5[n] silu'(Z4[b][n])
__global__ void k_out_back(const float *__restrict__ Z4, const float *__restrict__ dy, int B,
                           const float *__restrict__ p, float *__restrict__ d4) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * NW) return;
  const int b = (int)(e / NW), n = (int)(e % NW);
  d4[e] = dy[b] * p[OFF_W5 + n] * silu_grad_f(Z4[e]);
}

// out[n] += sum_{b in chunk} w[b] f(X[b][n])  (w = NULL: weight 1); blockDim = 256 (one
// thread per column), blockIdx.x = row chunk
template <int F>
__global__ void k_colsum(const float *__restrict__ X, const float *__restrict__ w, int B, int rows_per,
                         float *__restrict__ out) {
  const int n = threadIdx.x;
  const int b0 = blockIdx.x * rows_per, b1 = min(B, b0 + rows_per);
  float acc = 0.0f;
  for (int b = b0; b < b1; ++b) {
    float v = X[(int64_t)b * NW + n];
    if (F == F_SILU) v = silu_f(v);
    acc += (w ? w[b] : 1.0f) * v;
  }
  atomicAdd(out + n, acc);
}

// gb5 += sum_b dy[b]
__global__ void k_sum(const float *__restrict__ v, int B, float *__restrict__ out) {
  float acc = 0.0f;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) acc += v[b];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

// gW1[n][i] += sum_b d1[b][n] xn[b][i], gb1[n] += sum_b d1[b][n]
__global__ void k_in_back(const float *__restrict__ d1, const float *__restrict__ x, int B, int rows_per, cm_mlp net,
                          float *__restrict__ grad) {
  const int n = threadIdx.x;
  const int b0 = blockIdx.x * rows_per, b1 = min(B, b0 + rows_per);
  float gw[NIN], gb = 0.0f;
#pragma unroll
  for (int i = 0; i < NIN; ++i) gw[i] = 0.0f;
  for (int b = b0; b < b1; ++b) {
    const float d = d1[(int64_t)b * NW + n];
    gb += d;
#pragma unroll
    for (int i = 0; i < NIN; ++i) gw[i] += d * ((x[(int64_t)b * NIN + i] - net.shift[i]) * net.scale[i]);
  }
#pragma unroll
  for (int i = 0; i < NIN; ++i) atomicAdd(grad + OFF_W1 + n * NIN + i, gw[i]);
  atomicAdd(grad + OFF_B1 + n, gb);
}

__global__ void k_fill(float *__restrict__ a, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, int B, float *__restrict__ dy,
                      float *__restrict__ loss) {
  float acc = 0.0f;
  const float inv = 1.0f / (float)B;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    const float r = y[b] - t[b];
    dy[b] = 2.0f * r * inv;
    acc += r * r * inv;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, acc);
}

// BF16 copies of W2..W4 live contiguously in w_bf16, layer l's copy at (l - 2) * 65536 in
// fragment order
__device__ __forceinline__ int bf16_slot(int i) {
  for (int l = 2; l <= 4; ++l)
    if (i >= off_w(l) && i < off_w(l) + NW * NW) {
      const int j = i - off_w(l);
      return (l - 2) * NW * NW + wfrag(j / NW, j % NW);
    }
  return -1;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float bc1, float bc2,
                       uint16_t *__restrict__ wbf) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    const int s = bf16_slot(i);
    if (s >= 0) wbf[s] = f2bf(pi);
  }
}

__global__ void k_sync_bf16(const float *__restrict__ p, uint16_t *__restrict__ wbf) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 3 * NW * NW; e += gridDim.x * blockDim.x) {
    const int l = 2 + e / (NW * NW), i = e % (NW * NW);
    wbf[(l - 2) * NW * NW + wfrag(i / NW, i % NW)] = f2bf(p[off_w(l) + i]);
  }
}

struct GateBox {
  float lo[NIN], hi[NIN];
};

// Validation error table of the gate: cell (iT, ik) of an nT x nk grid over the trusted
// box's (T, k) rectangle holds the largest |network - SFFT| / S0 seen there.
struct GateCells {
  const float *err;
  int nT, nk;
  float tol;
};

__global__ void k_gate(const float *__restrict__ x, const float *__restrict__ z, int B, GateBox box, float r,
                       float tol, float out_eps, GateCells cells, float *__restrict__ price,
                       int32_t *__restrict__ accept) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    const float xi = x[(int64_t)b * NIN + i];
    ok = ok && (xi >= box.lo[i]) && (xi <= box.hi[i]);
  }
  const float T = x[(int64_t)b * NIN + 5], k = x[(int64_t)b * NIN + 6];
  const float lower = fmaxf(0.0f, 1.0f - expf(k - r * T));
  const float yb = out_eps > 0.0f ? expf(z[b]) - out_eps : z[b];
  const float res = fmaxf(fmaxf(lower - yb, yb - 1.0f), 0.0f);
  if (ok && cells.err) {
    // the query's (T, k) cell; in-box queries map into [0, n) (the upper edges clamp)
    const float fT = (T - box.lo[5]) / (box.hi[5] - box.lo[5]), fk = (k - box.lo[6]) / (box.hi[6] - box.lo[6]);
    const int iT = min(cells.nT - 1, max(0, (int)(fT * (float)cells.nT)));
    const int ik = min(cells.nk - 1, max(0, (int)(fk * (float)cells.nk)));
    ok = cells.err[iT * cells.nk + ik] <= cells.tol;
  }
  if (price) price[b] = yb;
  accept[b] = (ok && res <= tol && yb == yb) ? 1 : 0;
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

extern "C" size_t cm_mlp_act_bytes(int B) { return B > 0 ? (size_t)4 * B * NW * sizeof(float) : 0; }

static bool net_ok(const cm_mlp *net) { return net && net->params && net->w_bf16; }

extern "C" cm_status cm_mlp_sync_bf16(const cm_mlp *net, void *stream) {
  if (!net_ok(net)) return CM_E_INVALID;
  hipLaunchKernelGGL(k_sync_bf16, dim3(256), dim3(256), 0, (hipStream_t)stream, net->params, net->w_bf16);
  CM_LAUNCH_CHECK();
  return CM_OK;
}

// persistent workgroups for the weight-stationary layers: at most one per CU (132 KB of LDS each)
static int ws_grid(int M) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  const int tiles = (M + 31) / 32;
  return tiles < cus ? tiles : cus;
}

extern "C" cm_status cm_mlp_forward(const cm_mlp *net, const float *x, int B, float *y, float *acts,
                                    size_t acts_bytes, void *stream) {
  if (!net_ok(net) || !x || !y || B < 0) return CM_E_INVALID;
  if (B == 0) return CM_OK;
  if ((int64_t)B * NW > INT32_MAX) return CM_E_UNSUPPORTED;
  const bool keep = acts && acts_bytes >= cm_mlp_act_bytes(B);
  hipStream_t s = (hipStream_t)stream;
  if (!keep) {
    // inference: the fused kernel, one persistent workgroup (two tiles in flight) per CU
    CM_HIP_CHECK(cm_allow_lds(k_mlp_fused, FUSED_LDS));
    const int ntiles = (B + FM - 1) / FM;
    int cus = 0;
    int dev = 0;
    CM_HIP_CHECK(hipGetDevice(&dev));
    CM_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int pairs = (ntiles + 1) / 2;
    const int grid = pairs < cus ? pairs : cus;
    hipLaunchKernelGGL(k_mlp_fused, dim3(grid), dim3(512), FUSED_LDS, s, x, B, net->params, net->w_bf16, *net, y);
    CM_LAUNCH_CHECK();
    return CM_OK;
  }
  float *Z[4];
  for (int l = 0; l < 4; ++l) Z[l] = acts + (int64_t)(keep ? l : (l & 1)) * B * NW;
  CM_HIP_CHECK(cm_allow_lds(k_gemm_ws<W_NK, F_SILU, E_BIAS_STORE>, WS_LDS));
  hipLaunchKernelGGL(k_mlp_in, dim3(grid_for((int64_t)B * NW, 256)), dim3(256), 0, s, x, B, net->params, *net, Z[0]);
  CM_LAUNCH_CHECK();
  for (int l = 2; l <= 4; ++l) {
    hipLaunchKernelGGL((k_gemm_ws<W_NK, F_SILU, E_BIAS_STORE>), dim3(ws_grid(B)), dim3(WS_THREADS), WS_LDS, s, Z[l - 2],
                       net->w_bf16 + (int64_t)(l - 2) * NW * NW, B, Z[l - 1], net->params + off_b(l),
                       (const float *)nullptr);
    CM_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_mlp_out, dim3(grid_for(B, 4)), dim3(256), 0, s, Z[3], B, net->params, y);
  CM_LAUNCH_CHECK();
  return CM_OK;
}

extern "C" cm_status cm_mlp_backward(const cm_mlp *net, const float *x, const float *acts, const float *dy, int B,
                                     float *grad, void *ws, size_t ws_bytes, void *stream) {
  if (!net_ok(net) || !x || !acts || !dy || !grad || B < 0) return CM_E_INVALID;
  if (B == 0) return CM_OK;
  if (!ws || ws_bytes < cm_mlp_act_bytes(B) / 2) return CM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const float *Z[4];
  for (int l = 0; l < 4; ++l) Z[l] = acts + (int64_t)l * B * NW;
  float *D[2] = {(float *)ws, (float *)ws + (int64_t)B * NW};
  const float *p = net->params;
  CM_HIP_CHECK(cm_allow_lds(k_gemm_ws<W_KN, F_NONE, E_DSILU_STORE>, WS_LDS));
  hipLaunchKernelGGL(k_fill, dim3(256), dim3(256), 0, s, grad, (int64_t)CM_MLP_NPARAMS, 0.0f);
  hipLaunchKernelGGL(k_out_back, dim3(grid_for((int64_t)B * NW, 256)), dim3(256), 0, s, Z[3], dy, B, p, D[0]);
  const int rows_per = 64;
  const unsigned chunks = grid_for(B, rows_per);
  hipLaunchKernelGGL(k_colsum<F_SILU>, dim3(chunks), dim3(NW), 0, s, Z[3], dy, B, rows_per, grad + OFF_W5);
  hipLaunchKernelGGL(k_sum, dim3(64), dim3(256), 0, s, dy, B, grad + OFF_B5);
  CM_LAUNCH_CHECK();
  // split-K over the batch for the weight gradients: about 256 rows per workgroup
  const int kspan = 256;
  const unsigned ksplit = grid_for(B, kspan);
  int cur = 0;
  for (int l = 4; l >= 2; --l) {
    const float *dl = D[cur];
    {  // gW_l[m][n] += sum_b delta_l[b][m] silu(Z_{l-1}[b][n])
      GemmArgs g{};
      g.A = dl; g.lda = NW;
      g.B = Z[l - 2]; g.ldb = NW;
      g.M = NW; g.N = NW; g.K = B; g.kspan = kspan;
      g.C = grad + off_w(l); g.ldc = NW;
      hipLaunchKernelGGL((k_gemm<A_COLMAJOR, F_NONE, true, B_F32_KN, F_SILU, E_ATOMIC_ADD>),
                         dim3(NW / GT, NW / GT, ksplit), dim3(256), 0, s, g);
    }
    hipLaunchKernelGGL(k_colsum<F_NONE>, dim3(chunks), dim3(NW), 0, s, dl, (const float *)nullptr, B, rows_per,
                       grad + off_b(l));
    // delta_{l-1}[b][n] = (sum_k delta_l[b][k] W_l[k][n]) silu'(Z_{l-1}[b][n])
    hipLaunchKernelGGL((k_gemm_ws<W_KN, F_NONE, E_DSILU_STORE>), dim3(ws_grid(B)), dim3(WS_THREADS), WS_LDS, s, dl,
                       net->w_bf16 + (int64_t)(l - 2) * NW * NW, B, D[cur ^ 1], (const float *)nullptr, Z[l - 2]);
    CM_LAUNCH_CHECK();
    cur ^= 1;
  }
  hipLaunchKernelGGL(k_in_back, dim3(chunks), dim3(NW), 0, s, D[cur], x, B, rows_per, *net, grad);
  CM_LAUNCH_CHECK();
  return CM_OK;
}

extern "C" cm_status cm_mlp_mse(const float *y, const float *t, int B, float *dy, float *loss, void *stream) {
  if (!y || !t || !dy || B < 0) return CM_E_INVALID;
  if (B == 0) return CM_OK;
  hipLaunchKernelGGL(k_mse, dim3(grid_for(B, 256) < 1024 ? grid_for(B, 256) : 1024), dim3(256), 0,
                     (hipStream_t)stream, y, t, B, dy, loss);
  CM_LAUNCH_CHECK();
  return CM_OK;
}

extern "C" cm_status cm_adam_step(const cm_mlp *net, const float *grad, float *m, float *v, int step, float lr,
                                  float beta1, float beta2, float eps, void *stream) {
  if (!net_ok(net) || !grad || !m || !v || step < 1) return CM_E_INVALID;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f)) return CM_E_INVALID;
  const float bc1 = 1.0f - powf(beta1, (float)step), bc2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(CM_MLP_NPARAMS, 256)), dim3(256), 0, (hipStream_t)stream, net->params,
                     grad, m, v, (int)CM_MLP_NPARAMS, lr, beta1, beta2, eps, bc1, bc2, net->w_bf16);
  CM_LAUNCH_CHECK();
  return CM_OK;
}

extern "C" cm_status cm_surrogate_gate(const float *x, const float *z, int B, const float *lo, const float *hi,
                                       float r, float res_tol, float out_eps, const float *cell_err, int nT, int nk,
                                       float err_tol, float *price, int32_t *accept, void *stream) {
  if (!x || !z || !lo || !hi || !accept || B < 0 || !(out_eps >= 0.0f)) return CM_E_INVALID;
  if (cell_err && (nT < 1 || nk < 1 || nT > 4096 || nk > 4096 || !(err_tol >= 0.0f))) return CM_E_INVALID;
  if (B == 0) return CM_OK;
  GateBox box;
  for (int i = 0; i < NIN; ++i) {
    box.lo[i] = lo[i];
    box.hi[i] = hi[i];
  }
  if (cell_err && !(box.hi[5] > box.lo[5] && box.hi[6] > box.lo[6])) return CM_E_INVALID;
  GateCells cells{cell_err, nT, nk, err_tol};
  hipLaunchKernelGGL(k_gate, dim3(grid_for(B, 256)), dim3(256), 0, (hipStream_t)stream, x, z, B, box, r, res_tol,
                     out_eps, cells, price, accept);
  CM_LAUNCH_CHECK();
  return CM_OK;
}
