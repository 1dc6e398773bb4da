// Shared device/host helpers for the recovery kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;

#define REVO_HIP_TRY(expr)                                                   \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      fprintf(stderr, "revo: %s failed: %s (%s:%d)\n", #expr,                \
              hipGetErrorString(e_), __FILE__, __LINE__);                    \
      return -5; /* REVO_EDEVICE */                                          \
    }                                                                        \
  } while (0)

namespace revo {

// Operand precisions of the matrix products.
enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP8 = 2 };  // P_FP8: FP8 block products, BF16 elsewhere

// ----------------------------------------------------------------------------
// operand element traits: storage type in HBM/LDS, element size and the
// 32x32 MFMA that consumes it.  Every MFMA step takes KPL contiguous
// elements per lane; lane half h (lanes 32..63) supplies the upper half of
// the step's k slots.
// ----------------------------------------------------------------------------
struct OpF32 {
  typedef float T;
  static constexpr int KPL = 1;            // k elements per lane per MFMA
  static constexpr int BK = 32;            // k per LDS stage (128-byte rows)
  typedef float frag;
  __device__ static inline frag load(const T* p) { return *p; }
  __device__ static inline void mma(f32x16& acc, frag a, frag b) {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
  __device__ static inline T from_float(float x) { return x; }
};

struct OpBF16 {
  typedef __bf16 T;
  static constexpr int KPL = 8;
  static constexpr int BK = 64;
  typedef bf16x8 frag;
  __device__ static inline frag load(const T* p) { return *reinterpret_cast<const bf16x8*>(p); }
  __device__ static inline void mma(f32x16& acc, frag a, frag b) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  __device__ static inline T from_float(float x) { return (__bf16)x; }
};

typedef __attribute__((ext_vector_type(8))) int i32x8;

// OCP FP8 E4M3 (bias 7, max 448): conversions saturate at +-448.
__device__ inline uint32_t e4m3x4(float a, float b, float c, float d) {
  a = fminf(fmaxf(a, -448.0f), 448.0f);
  b = fminf(fmaxf(b, -448.0f), 448.0f);
  c = fminf(fmaxf(c, -448.0f), 448.0f);
  d = fminf(fmaxf(d, -448.0f), 448.0f);
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, v, true);
  return (uint32_t)v;
}
__device__ inline uint8_t e4m3(float a) { return (uint8_t)(e4m3x4(a, 0.0f, 0.0f, 0.0f) & 0xFF); }

// FP8 operands: 32 E4M3 values per lane per MFMA step (two 16-byte reads),
// unit block scales (E8M0 exponent 127).
struct OpFP8 {
  typedef uint8_t T;
  static constexpr int KPL = 32;
  static constexpr int BK = 64;   // one MFMA step per stage (decoder products have K = 192)
  typedef i32x8 frag;
  __device__ static inline void mma(f32x16& acc, frag a, frag b) {
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
  }
  __device__ static inline T from_float(float x) { return e4m3(x); }
};

__device__ inline float to_float(float x) { return x; }
__device__ inline float to_float(__bf16 x) { return (float)x; }

// 32x32 accumulator layout (C/D of a 32x32 MFMA): lane l holds column
// (l & 31) and, in register i, row (i / 4) * 8 + (l / 32) * 4 + (i % 4).
__device__ inline int acc_row(int i, int lane) { return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3); }

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline long long cdivll(long long a, long long b) { return (a + b - 1) / b; }

}  // namespace revo
