// Internal helpers shared by the HIP sources of libcm: complex arithmetic on
// float2/double2, typed views of a cm_tt_batch, launch-status plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/cm.h"

// Threads per workgroup of the sweep kernels. A source file may define it before including
// this header: each .hip file is compiled to its own device code object, so the
// factorisation routines are instantiated per file with that file's workgroup size.
#ifndef CM_WG
#define CM_WG 256
#endif

// ------------------------------------------------------------------ complex helpers
__host__ __device__ __forceinline__ double2 cmk(double re, double im) { return make_double2(re, im); }
__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ __forceinline__ double2 ccmul(double2 a, double2 b) {
  return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ __forceinline__ double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ __forceinline__ double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  double d = b.x * b.x + b.y * b.y;
  return cmk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
// fused a += b * c
__host__ __device__ __forceinline__ void cfma(double2 &a, double2 b, double2 c) {
  a.x = fma(b.x, c.x, a.x); a.x = fma(-b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y); a.y = fma(b.y, c.x, a.y);
}
// a += conj(b) * c
__host__ __device__ __forceinline__ void ccfma(double2 &a, double2 b, double2 c) {
  a.x = fma(b.x, c.x, a.x); a.x = fma(b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y); a.y = fma(-b.y, c.x, a.y);
}

__host__ __device__ __forceinline__ float2 fadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 fmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ void ffma(float2 &a, float2 b, float2 c) {
  a.x = fmaf(b.x, c.x, a.x); a.x = fmaf(-b.y, c.y, a.x);
  a.y = fmaf(b.x, c.y, a.y); a.y = fmaf(b.y, c.x, a.y);
}

// storage <-> FP64 conversion
template <typename T> struct cstore;
template <> struct cstore<float2> {
  __device__ __forceinline__ static double2 ld(const float2 *p, int64_t i) {
    float2 v = p[i]; return cmk((double)v.x, (double)v.y);
  }
  __device__ __forceinline__ static void st(float2 *p, int64_t i, double2 v) {
    p[i] = make_float2((float)v.x, (float)v.y);
  }
};
template <> struct cstore<double2> {
  __device__ __forceinline__ static double2 ld(const double2 *p, int64_t i) { return p[i]; }
  __device__ __forceinline__ static void st(double2 *p, int64_t i, double2 v) { p[i] = v; }
};

// ------------------------------------------------------------------ TT batch view
struct TTView {
  const int32_t *n;
  int32_t *ranks;
  const int64_t *off;
  void *cores;
  int d;  // d_out * d_in
  __device__ __forceinline__ int len(int b) const { return n[b]; }
  __device__ __forceinline__ int32_t *rk(int b) const { return ranks + (int64_t)b * CM_RANKS_STRIDE; }
  __device__ __forceinline__ int64_t coff(int b, int l) const { return off[(int64_t)b * CM_MAX_N + l]; }
};

static inline TTView tt_view(const cm_tt_batch *t) {
  TTView v;
  v.n = t->n; v.ranks = t->ranks; v.off = t->core_off; v.cores = t->cores; v.d = t->d_out * t->d_in;
  return v;
}

// instance status: first error wins
__device__ __forceinline__ void set_status(int32_t *status, int b, int code) {
  if (status && code != CM_OK) atomicCAS(status + b, (int32_t)CM_OK, (int32_t)code);
}

// ------------------------------------------------------------------ phase reduction
// The error-free transforms below must not be fused with neighbouring operations: with
// contraction enabled, a product feeding `hi - floor(hi)` becomes one FMA that already
// carries the product's rounding error, which the low part then adds a second time.
// Error-free product a*b = p + e (fma based).
__host__ __device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
#pragma clang fp contract(off)
  p = a * b;
  e = fma(a, b, -p);
}
// Fractional part (in [0,1)) of x = hi + lo where hi is a double and lo small.
__host__ __device__ __forceinline__ double frac2(double hi, double lo) {
#pragma clang fp contract(off)
  double f = hi - floor(hi);
  f += lo;
  f -= floor(f);
  return f;
}

// Allows a kernel to take more than the default dynamic LDS (gfx950 has 160 KB per CU).
template <typename K>
static inline hipError_t cm_allow_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define CM_HIP_CHECK(expr)                                         \
  do {                                                             \
    hipError_t _e = (expr);                                        \
    if (_e != hipSuccess) return CM_E_HIP;                         \
  } while (0)

#define CM_LAUNCH_CHECK()                                          \
  do {                                                             \
    hipError_t _e = hipGetLastError();                             \
    if (_e != hipSuccess) return CM_E_HIP;                         \
  } while (0)
