// cm_tt_round: in-place TT rounding (the recompression of Section 3.1, after Oseledets
// 2011) of every train in a batch, one workgroup per train, FP64 factorisations.
// One wavefront per train: the factorisations are chains of small dependent steps, so
// barriers over a single wave and more trains per CU beat wider workgroups.
#define CM_WG 64
#include "cm_tt.h"

namespace {
__host__ __device__ inline size_t al256r(size_t x) { return (x + 255) & ~(size_t)255; }
// LDS arena per workgroup: small on purpose. The sweep is a chain of latency-bound steps, so
// more resident workgroups per CU (their matrices then live in the L2-cached slab) beat
// LDS-resident matrices with three workgroups per CU: measured 16.0 -> 7.3 ms for 4096
// trains at n = 24. 7.5 KB plus the 2.1 KB of static LDS lets 16 workgroups (the four waves
// per SIMD that 128 VGPRs allow) share a CU's 160 KB; with 8 KB only 15 fit, and a batch of
// 16 per CU ran its last sixteenth as a second wave.
constexpr int RLDS = 7680;
// Workspace of one persistent workgroup: its hot matrices (Y, X, Z, L, R, C of cap d cap
// elements and the Jacobi pair of cap^2) and, apart from them, the orthogonalised train of the
// first sweep (n_max cores). The hot blocks of all workgroups sit next to each other at the
// start of the workspace and the trains after them, so that the thousands of concurrently
// resident workgroups touch one dense region instead of one scattered slab each (measured:
// the latency of a bond's product grew from 17 K to 250 K cycles between 256 and 4096
// resident workgroups with one slab per workgroup).
__host__ __device__ inline size_t round_hot_bytes(int d, int cap) {
  const size_t mat = (size_t)cap * d * cap;
  return al256r(sizeof(double2) * (6 * mat + 2 * (size_t)cap * cap));
}
__host__ __device__ inline size_t round_tt_bytes(int n_max, int d, int cap) {
  return al256r(sizeof(double2) * (size_t)cap * d * cap * n_max);
}
__host__ __device__ inline size_t round_slab_bytes(int n_max, int d, int cap) {
  return round_hot_bytes(d, cap) + round_tt_bytes(n_max, d, cap);
}
}  // namespace

template <typename T>
__global__ __launch_bounds__(CM_WG, 4) void k_tt_round(TTView t, int batch, double tol, int cap, int incap,
                                                    double *__restrict__ err_out, int32_t *__restrict__ status,
                                                    char *__restrict__ ws, int n_max, int dtype, int skip_a) {
  extern __shared__ __align__(16) char lds_arena[];
  __shared__ la::Sh sh;
  __shared__ int code_sh;
  const int tid = threadIdx.x;
  const size_t hot = round_hot_bytes(t.d, incap);
  double2 *mats = (double2 *)(ws + (size_t)blockIdx.x * hot);
  RoundScratch rs;
  rs.core_cap = (int64_t)incap * t.d * incap;
  rs.tt = (double2 *)(ws + (size_t)gridDim.x * hot + (size_t)blockIdx.x * round_tt_bytes(n_max, t.d, incap));
  rs.Y = mats; rs.X = mats + rs.core_cap; rs.Z = mats + 2 * rs.core_cap;
  rs.L = mats + 3 * rs.core_cap; rs.R = mats + 4 * rs.core_cap; rs.C = mats + 5 * rs.core_cap;
  rs.S = mats + 6 * rs.core_cap;
  rs.J = rs.S + (int64_t)incap * incap;
  for (int b = blockIdx.x; b < batch; b += gridDim.x) {
    const int n = t.n[b];
    if (tid == 0) {
      int c = CM_OK;
      if (n < 1 || n > n_max) c = CM_E_INVALID;
      else
        for (int l = 0; l <= n; ++l)
          if (t.rk(b)[l] < 1 || t.rk(b)[l] > incap) c = CM_E_INVALID;
      code_sh = c;
    }
    __syncthreads();
    if (code_sh != CM_OK) {
      if (tid == 0) { if (status) status[b] = code_sh; if (err_out) err_out[b] = NAN; }
      __syncthreads();
      continue;
    }
    CoreSrc src;
    src.cores = t.cores; src.off = t.off + (int64_t)b * CM_MAX_N; src.ranks = t.rk(b); src.dtype = dtype;
    const double e = round_train_auto<T>(n, t.d, src, tol, cap, (T *)t.cores, t.off + (int64_t)b * CM_MAX_N,
                                         t.rk(b), rs, lds_arena, RLDS, sh, &code_sh, skip_a != 0);
    __syncthreads();
    if (tid == 0) {
      if (status) status[b] = code_sh;
      if (err_out) err_out[b] = e;
    }
    __syncthreads();
  }
}

extern "C" size_t cm_round_slab_bytes(int n_max, int d, int cap) { return round_slab_bytes(n_max, d, cap); }
extern "C" int cm_slots_for_ws(int op, int batch, int n_max, int cap_rank, int dtype, size_t ws_bytes);

extern "C" cm_status cm_tt_round(cm_tt_batch *t, double tol, int cap_rank, double *err_out, int32_t *status,
                                 void *ws, size_t ws_bytes, void *stream) {
  if (!t || !(tol >= 0.0) || cap_rank < 1 || cap_rank > 64) return CM_E_INVALID;
  if (t->batch < 0 || t->n_max < 1 || t->n_max > CM_MAX_N) return CM_E_INVALID;
  if (t->dtype != CM_C64 && t->dtype != CM_C128) return CM_E_INVALID;
  if (t->d_out < 1 || t->d_in < 1 || t->d_out * t->d_in > 4) return CM_E_INVALID;
  if (t->cap_rank < 1 || t->cap_rank > 64) return CM_E_UNSUPPORTED;
  if (t->batch == 0) return CM_OK;
  // one workgroup per workspace slab (cm_workspace_bytes gives the default count)
  const int slots = cm_slots_for_ws(CM_OP_TT_ROUND, t->batch, t->n_max, t->cap_rank, t->dtype, ws ? ws_bytes : 0);
  if (slots < 1) return CM_E_INVALID;
  const int d = t->d_out * t->d_in;
  const size_t lds = RLDS;
  TTView v = tt_view(t);
  hipStream_t s = (hipStream_t)stream;
  const int skip = (t->flags & CM_TT_LEFT_ORTHO) ? 1 : 0;
  CM_HIP_CHECK(cm_allow_lds(k_tt_round<float2>, lds));
  CM_HIP_CHECK(cm_allow_lds(k_tt_round<double2>, lds));
  if (t->dtype == CM_C64)
    hipLaunchKernelGGL(k_tt_round<float2>, dim3(slots), dim3(CM_WG), lds, s, v, t->batch, tol, cap_rank, t->cap_rank,
                       err_out, status, (char *)ws, t->n_max, t->dtype, skip);
  else
    hipLaunchKernelGGL(k_tt_round<double2>, dim3(slots), dim3(CM_WG), lds, s, v, t->batch, tol, cap_rank, t->cap_rank,
                       err_out, status, (char *)ws, t->n_max, t->dtype, skip);
  CM_LAUNCH_CHECK();
  t->flags = CM_TT_RIGHT_ORTHO;
  return CM_OK;
}
