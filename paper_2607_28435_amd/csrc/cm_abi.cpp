// Host-side helpers of the C ABI: capacity layout, workspace sizes, status strings.
#include <stddef.h>
#include <stdint.h>

#include "../../include/cm.h"

extern "C" size_t cm_qtt_slab_bytes(int n_max, int cap);
extern "C" size_t cm_mpo_ws_bytes(int n, int cap);
extern "C" size_t cm_zip_slab_bytes(int cap);
extern "C" size_t cm_round_slab_bytes(int n_max, int d, int cap);
extern "C" size_t cm_fft_ws_bytes(int batch, int n, int dtype, int gather);
extern "C" size_t cm_sample_ws_bytes(int batch, int n_max, int cap_rank);

// Workgroups kept resident by the batched sweep kernels (each processes trains
// blockIdx.x, blockIdx.x + slots, ...). Four per compute unit of a 256-CU device.
extern "C" int cm_slots_for(int batch) {
  const int max_slots = 2048;
  return batch < max_slots ? batch : max_slots;
}

static int64_t ipow_cap(int base, int e, int64_t cap) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) {
    v *= base;
    if (v >= cap) return cap;
  }
  return v;
}

extern "C" int64_t cm_tt_layout(int n, int d_out, int d_in, int cap_rank, int64_t *off) {
  if (n < 1 || n > CM_MAX_N || d_out < 1 || d_in < 1 || cap_rank < 1) return -1;
  const int d = d_out * d_in;
  // bond l holds at most min(cap_rank, d^l) (boundary bonds are 1); the right-hand bound
  // d^(n-l) is not imposed because the zip-up's intermediate bonds may exceed it
  int64_t total = 0;
  for (int l = 0; l < n; ++l) {
    const int64_t rl = (l == 0) ? 1 : ipow_cap(d, l, cap_rank);
    const int64_t rr = (l == n - 1) ? 1 : ipow_cap(d, l + 1, cap_rank);
    if (off) off[l] = total;
    total += rl * d * rr;
  }
  return total;
}

extern "C" size_t cm_workspace_bytes(int op, int batch, int n_max, int cap_rank, int dtype) {
  if (batch < 1 || n_max < 1 || n_max > CM_MAX_N) return 0;
  if (dtype != CM_C64 && dtype != CM_C128) return 0;
  const size_t slots = (size_t)cm_slots_for(batch);
  switch (op) {
    case CM_OP_QFT_MPO:
      // `batch` operators built in one call (cm_qft_mpo: 1), slabs sized for n_max, then
      // one 256-byte block of status words
      if (cap_rank < 1 || cap_rank > 64 || batch > CM_MAX_N) return 0;
      return (size_t)batch * cm_mpo_ws_bytes(n_max, cap_rank) + 256;
    case CM_OP_BUILD_QTT:
      if (cap_rank < 1 || cap_rank > 64) return 0;
      return slots * cm_qtt_slab_bytes(n_max, cap_rank);
    case CM_OP_SFFT_APPLY:
      if (cap_rank < 1 || cap_rank > 64) return 0;
      return slots * cm_zip_slab_bytes(cap_rank);
    case CM_OP_TT_ROUND:
      if (cap_rank < 1 || cap_rank > 64) return 0;
      return slots * cm_round_slab_bytes(n_max, 4, cap_rank);
    case CM_OP_FFT_PRICE:
      return cm_fft_ws_bytes(batch, n_max, dtype, 1);
    case CM_OP_SAMPLE:
      if (cap_rank < 1 || cap_rank > 256) return 0;
      return cm_sample_ws_bytes(batch, n_max, cap_rank);
    default:
      return 0;
  }
}

// Persistent workgroups for a sweep op: one per workspace slab, at most one per instance.
extern "C" int cm_slots_for_ws(int op, int batch, int n_max, int cap_rank, int dtype, size_t ws_bytes) {
  const size_t slab = cm_workspace_bytes(op, 1, n_max, cap_rank, dtype);
  if (slab == 0 || batch < 1) return 0;
  size_t s = ws_bytes / slab;
  if (s > (size_t)batch) s = (size_t)batch;
  if (s > 65535) s = 65535;
  return (int)s;
}

extern "C" const char *cm_status_str(cm_status s) {
  switch (s) {
    case CM_OK: return "ok";
    case CM_E_INVALID: return "invalid argument";
    case CM_E_MOMENT: return "damping moment E[S_T^(alpha+1)] is infinite";
    case CM_E_RANKCAP: return "bond dimension cap reached above tolerance";
    case CM_E_NOCONV: return "iteration did not converge";
    case CM_E_NONFINITE: return "non-finite value";
    case CM_E_HIP: return "HIP runtime error";
    case CM_E_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

extern "C" const char *cm_version(void) { return "cm-sfft 0.1 (gfx950)"; }
