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
enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP8 = 2 };

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

__device__ inline float to_float(float x) { return x; }
__device__ inline float to_float(__bf16 x) { return (float)x; }

// 32x32 accumulator layout (C/D of a 32x32 MFMA): lane l holds column
// (l & 31) and, in register i, row (i / 4) * 8 + (l / 32) * 4 + (i % 4).
__device__ inline int acc_row(int i, int lane) { return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3); }

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline long long cdivll(long long a, long long b) { return (a + b - 1) / b; }

}  // namespace revo
