// Row LayerNorm, the loss-mask composite and small conversion kernels.
#include "kernels.h"

namespace revo {

namespace {

// One wave per row: FP32 mean and biased variance over D features (D <= 512, even),
// then (x - mean) / sqrt(var + 1e-6) * g + b, stored as the next product's
// operand type.  With reqs set, output row i is request r's target-tubelet
// token i - head_off (rows of the last tubelet only, for the head).
template <class T>
__global__ __launch_bounds__(256) void layernorm_kernel(const float* __restrict__ x, const float* __restrict__ g,
                                                        const float* __restrict__ b, T* __restrict__ y, int rows,
                                                        int D, const ReqDesc* reqs, int nreq,
                                                        const int* dyn_rows, const int* dyn_nreq) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (dyn_rows) rows = *dyn_rows;
  if (dyn_nreq) nreq = *dyn_nreq;
  if (row >= rows) return;
  int src = row;
  if (reqs) {
    const int r = find_req_head(reqs, nreq, row);
    const ReqDesc& d = reqs[r];
    src = d.tok_off + (d.J - 1) * d.P + (row - d.head_off);
  }
  // float2 chunks (D is even): 512-byte loads per wave instruction
  const float2* xr = reinterpret_cast<const float2*>(x + (size_t)src * D);
  const int D2 = D >> 1;
  float2 v[4];
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = lane + 64 * i;
    v[i] = c < D2 ? xr[c] : make_float2(0.0f, 0.0f);
    s += v[i].x + v[i].y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const float mean = s / (float)D;
  float q = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = lane + 64 * i;
    if (c < D2) {
      const float t0 = v[i].x - mean, t1 = v[i].y - mean;
      q += t0 * t0 + t1 * t1;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
  const float rstd = 1.0f / sqrtf(q / (float)D + 1e-6f);
  T* yr = y + (size_t)row * D;
  const float2* g2 = reinterpret_cast<const float2*>(g);
  const float2* b2 = reinterpret_cast<const float2*>(b);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = lane + 64 * i;
    if (c < D2) {
      const float2 gg = g2[c], bb = b2[c];
      const float y0 = (v[i].x - mean) * rstd * gg.x + bb.x;
      const float y1 = (v[i].y - mean) * rstd * gg.y + bb.y;
      if constexpr (sizeof(T) == 2) {
        *reinterpret_cast<bf16x2*>(yr + 2 * c) = bf16x2{(__bf16)y0, (__bf16)y1};
      } else {
        *reinterpret_cast<float2*>(yr + 2 * c) = make_float2(y0, y1);
      }
    }
  }
}

// The same LayerNorm with a group of L lanes per row and V float4 per lane
// (D = 4 L V), so a wave holds 64 / L rows and every load is 16 bytes.
template <class T, int L, int V>
__global__ __launch_bounds__(256) void layernorm_rows_kernel(const float* __restrict__ x, const float* __restrict__ g,
                                                             const float* __restrict__ b, T* __restrict__ y, int rows,
                                                             const ReqDesc* reqs, int nreq, const int* dyn_rows,
                                                             const int* dyn_nreq) {
  constexpr int D = 4 * L * V;
  const int j = threadIdx.x & (L - 1);
  const int row = blockIdx.x * (256 / L) + (threadIdx.x / L);
  if (dyn_rows) rows = *dyn_rows;
  if (dyn_nreq) nreq = *dyn_nreq;
  if (row >= rows) return;
  int src = row;
  if (reqs) {
    const int r = find_req_head(reqs, nreq, row);
    const ReqDesc& d = reqs[r];
    src = d.tok_off + (d.J - 1) * d.P + (row - d.head_off);
  }
  const float4* xr = reinterpret_cast<const float4*>(x + (size_t)src * D);
  float4 v[V];
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    v[i] = xr[j + L * i];
    s += (v[i].x + v[i].y) + (v[i].z + v[i].w);
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const float mean = s * (1.0f / (float)D);
  float q = 0.0f;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    v[i].x -= mean; v[i].y -= mean; v[i].z -= mean; v[i].w -= mean;
    q += (v[i].x * v[i].x + v[i].y * v[i].y) + (v[i].z * v[i].z + v[i].w * v[i].w);
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) q += __shfl_xor(q, o);
  const float rstd = 1.0f / sqrtf(q * (1.0f / (float)D) + 1e-6f);
  const float4* g4 = reinterpret_cast<const float4*>(g);
  const float4* b4 = reinterpret_cast<const float4*>(b);
  T* yr = y + (size_t)row * D;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int c = j + L * i;
    const float4 gg = g4[c], bb = b4[c];
    const float y0 = v[i].x * rstd * gg.x + bb.x, y1 = v[i].y * rstd * gg.y + bb.y;
    const float y2 = v[i].z * rstd * gg.z + bb.z, y3 = v[i].w * rstd * gg.w + bb.w;
    if constexpr (sizeof(T) == 2) {
      *reinterpret_cast<bf16x4*>(yr + 4 * c) = bf16x4{(__bf16)y0, (__bf16)y1, (__bf16)y2, (__bf16)y3};
    } else {
      *reinterpret_cast<float4*>(yr + 4 * c) = make_float4(y0, y1, y2, y3);
    }
  }
}

// Final frame of one request: lost pixels take the clamped prediction
// (RGB in [0, 1], depth in [0, 65535] mm) quantised half-to-even, received
// pixels are copied unchanged.  A request without a mask is a clean frame
// and is copied; composite == 0 gives every pixel the prediction.
__global__ __launch_bounds__(256) void composite_kernel(const ReqDesc* __restrict__ reqs, int C, int composite,
                                                        const int* dyn_nreq) {
  if (dyn_nreq && (int)blockIdx.y >= *dyn_nreq) return;
  const ReqDesc& d = reqs[blockIdx.y];
  const int npix = d.H * d.W;
  for (int pix = blockIdx.x * 256 + threadIdx.x; pix < npix; pix += gridDim.x * 256) {
  const bool lost = d.mask != nullptr && (composite == 0 || d.mask[pix] != 0);
  const void* recv = d.frames[d.nframes - 1];
  if (C == 3) {
    const uint8_t* rv = (const uint8_t*)recv + (size_t)pix * 3;
    uint8_t* oi = (uint8_t*)d.out_i;
    float* of = d.out_f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t e = (size_t)pix * 3 + c;
      if (lost) {
        const float p = fminf(fmaxf(d.pred[e], 0.0f), 1.0f);
        if (of) of[e] = p;
        if (oi) oi[e] = (uint8_t)rintf(255.0f * p);
      } else {
        const uint8_t u = rv[c];
        if (of) of[e] = (float)u / 255.0f;
        if (oi) oi[e] = u;
      }
    }
  } else {
    const uint16_t* rv = (const uint16_t*)recv;
    uint16_t* oi = (uint16_t*)d.out_i;
    if (lost) {
      const float p = fminf(fmaxf(4000.0f * d.pred[pix], 0.0f), 65535.0f);
      if (d.out_f) d.out_f[pix] = p;
      if (oi) oi[pix] = (uint16_t)rintf(p);
    } else {
      const uint16_t u = rv[pix];
      if (d.out_f) d.out_f[pix] = (float)u;
      if (oi) oi[pix] = u;
    }
  }
  }
}

// LayerNorm as above, stored as FP8 E4M3 of the result / (*out_scale).
__global__ __launch_bounds__(256) void layernorm_fp8_kernel(const float* __restrict__ x, const float* __restrict__ g,
                                                            const float* __restrict__ b, uint8_t* __restrict__ y,
                                                            const float* __restrict__ out_scale, int rows, int D,
                                                            const int* dyn_rows) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (dyn_rows) rows = *dyn_rows;
  if (row >= rows) return;
  const float* xr = x + (size_t)row * D;
  float v[8];
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int c = lane + 64 * i;
    v[i] = c < D ? xr[c] : 0.0f;
    s += v[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const float mean = s / (float)D;
  float q = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int c = lane + 64 * i;
    const float t = c < D ? v[i] - mean : 0.0f;
    q += t * t;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
  const float rstd = 1.0f / sqrtf(q / (float)D + 1e-6f);
  const float inv = 1.0f / *out_scale;
  uint8_t* yr = y + (size_t)row * D;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int c = lane + 64 * i;
    if (c < D) yr[c] = e4m3(((v[i] - mean) * rstd * g[c] + b[c]) * inv);
  }
}

// The FP8 LayerNorm with a group of L lanes per row and V float4 per lane
// (D = 4 L V): E4M3 of the normalised value / (*out_scale), four bytes per
// store.
template <int L, int V>
__global__ __launch_bounds__(256) void layernorm_rows_fp8_kernel(const float* __restrict__ x,
                                                                 const float* __restrict__ g,
                                                                 const float* __restrict__ b, uint8_t* __restrict__ y,
                                                                 const float* __restrict__ out_scale, int rows,
                                                                 const int* dyn_rows) {
  constexpr int D = 4 * L * V;
  const int j = threadIdx.x & (L - 1);
  const int row = blockIdx.x * (256 / L) + (threadIdx.x / L);
  if (dyn_rows) rows = *dyn_rows;
  if (row >= rows) return;
  const float4* xr = reinterpret_cast<const float4*>(x + (size_t)row * D);
  float4 v[V];
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    v[i] = xr[j + L * i];
    s += (v[i].x + v[i].y) + (v[i].z + v[i].w);
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const float mean = s * (1.0f / (float)D);
  float q = 0.0f;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    v[i].x -= mean; v[i].y -= mean; v[i].z -= mean; v[i].w -= mean;
    q += (v[i].x * v[i].x + v[i].y * v[i].y) + (v[i].z * v[i].z + v[i].w * v[i].w);
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) q += __shfl_xor(q, o);
  const float rstd = 1.0f / sqrtf(q * (1.0f / (float)D) + 1e-6f);
  const float inv = 1.0f / *out_scale;
  const float4* g4 = reinterpret_cast<const float4*>(g);
  const float4* b4 = reinterpret_cast<const float4*>(b);
  uint32_t* yr = reinterpret_cast<uint32_t*>(y + (size_t)row * D);
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int c = j + L * i;
    const float4 gg = g4[c], bb = b4[c];
    yr[c] = e4m3x4((v[i].x * rstd * gg.x + bb.x) * inv, (v[i].y * rstd * gg.y + bb.y) * inv,
                   (v[i].z * rstd * gg.z + bb.z) * inv, (v[i].w * rstd * gg.w + bb.w) * inv);
  }
}

// One block per row: row absmax, scale = absmax / 448, E4M3 of w / scale.
__global__ __launch_bounds__(256) void quantize_rows_kernel(const float* __restrict__ w, int cols,
                                                            uint8_t* __restrict__ w8, float* __restrict__ scale) {
  __shared__ float red[4];
  const float* wr = w + (size_t)blockIdx.x * cols;
  float m = 0.0f;
  for (int c = threadIdx.x; c < cols; c += 256) m = fmaxf(m, fabsf(wr[c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const float sc = m > 0.0f ? m / 448.0f : 1.0f;
  if (threadIdx.x == 0) scale[blockIdx.x] = sc;
  const float inv = 1.0f / sc;
  for (int c = threadIdx.x; c < cols; c += 256) w8[(size_t)blockIdx.x * cols + c] = e4m3(wr[c] * inv);
}

// max |x| of 256 threads into one atomicMax per block (non-negative floats
// order as their bits)
__device__ inline void block_max_to(float m, unsigned* __restrict__ slot) {
  __shared__ float red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(slot, __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
}

__device__ inline float absmax8(const uint4& u, float m) {
  const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    m = fmaxf(m, fabsf(__uint_as_float(w[i] << 16)));
    m = fmaxf(m, fabsf(__uint_as_float(w[i] & 0xFFFF0000u)));
  }
  return m;
}

// max |x| over the live rows of every request (the alignment gaps between
// requests are skipped): 16-byte loads over each request's contiguous rows,
// grid-stride, one atomic per block.  D is a multiple of 8.
__global__ __launch_bounds__(256) void absmax_kernel(const __bf16* __restrict__ x, int D,
                                                     const ReqDesc* __restrict__ reqs, int nreq,
                                                     unsigned* __restrict__ slot) {
  float m = 0.0f;
  const long long stride = (long long)gridDim.x * 256;
  for (int r = 0; r < nreq; ++r) {
    const uint4* p = reinterpret_cast<const uint4*>(x + (size_t)reqs[r].tok_off * D);
    const long long n = (long long)reqs[r].J * reqs[r].P * D / 8;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) m = absmax8(p[i], m);
  }
  block_max_to(m, slot);
}

// Per head (grid.y): max |.| of Q and K over the live token rows, and of V
// over the same tokens' V^T columns (BF16 V^T rows keep keys with bits 2
// and 3 swapped).  slots: Q maxima [heads], then K, then V.
__global__ __launch_bounds__(256) void attn_absmax_kernel(const __bf16* __restrict__ q, const __bf16* __restrict__ k,
                                                          const __bf16* __restrict__ vt, int heads, int ld,
                                                          const ReqDesc* __restrict__ reqs, int nreq,
                                                          unsigned* __restrict__ slots) {
  const int h = blockIdx.y;
  float mq = 0.0f, mk = 0.0f, mv = 0.0f;
  const long long stride = (long long)gridDim.x * 256;
  for (int r = 0; r < nreq; ++r) {
    const int t0 = reqs[r].tok_off, N = reqs[r].J * reqs[r].P;
    const size_t off = ((size_t)h * ld + t0) * 64;
    const uint4* qp = reinterpret_cast<const uint4*>(q + off);
    const uint4* kp = reinterpret_cast<const uint4*>(k + off);
    const long long n8 = (long long)N * 8;  // 16-byte chunks of N rows of 64
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n8; i += stride) {
      mq = absmax8(qp[i], mq);
      mk = absmax8(kp[i], mk);
    }
    const __bf16* vh = vt + (size_t)h * 64 * ld;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < 64LL * N; i += stride) {
      const int d = (int)(i / N), t = t0 + (int)(i - (long long)d * N);
      const int col = (t & ~12) | ((t & 4) << 1) | ((t & 8) >> 1);
      mv = fmaxf(mv, fabsf((float)vh[(size_t)d * ld + col]));
    }
  }
  block_max_to(mq, slots + h);
  __syncthreads();
  block_max_to(mk, slots + heads + h);
  __syncthreads();
  block_max_to(mv, slots + 2 * heads + h);
}

__global__ void attn_scales_kernel(const unsigned* __restrict__ absmax, int* __restrict__ exps,
                                   float* __restrict__ inv, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float x = __uint_as_float(absmax[i]) / 448.0f;
  int e = 0;
  if (x > 0.0f) {
    // ceil(log2 x) from the bits: the exponent, plus one unless x is a power of two
    const unsigned b = __float_as_uint(x);
    const int E = (int)((b >> 23) & 0xFF);
    e = E == 0 ? -126 : E - 127 + ((b & 0x7FFFFF) ? 1 : 0);
  }
  exps[i] = 127 + e;
  inv[i] = ldexpf(1.0f, -e);
}

__global__ void scales_kernel(const unsigned* __restrict__ absmax, float* __restrict__ scale, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const float m = __uint_as_float(absmax[i]);
    scale[i] = m > 0.0f ? m / 448.0f : 1.0f;
  }
}

template <class T>
__global__ void convert_kernel(const float* __restrict__ src, T* __restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

__global__ void convert_fp8_kernel(const float* __restrict__ src, uint8_t* __restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = e4m3(src[i]);
}

__global__ void zero_kernel(uint4* __restrict__ p, long long n16) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void zero_tail_kernel(uint8_t* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

int launch_layernorm(Prec out_prec, const float* x, const float* g, const float* b, void* y, int rows, int D,
                     const ReqDesc* reqs, int nreq, hipStream_t s, const int* dyn_rows, const int* dyn_nreq) {
  if (rows <= 0) return 0;
  if (D > 512 || (D & 1)) return -22;
  // the widths of the two networks (16-byte aligned operands): three float4
  // per lane, 2 or 4 rows per wave
#define REVO_LN_ROWS(L_)                                                                                          \
  do {                                                                                                            \
    const dim3 gr(cdiv(rows, 256 / (L_)));                                                                        \
    if (out_prec == P_BF16)                                                                                       \
      layernorm_rows_kernel<__bf16, L_, 3><<<gr, 256, 0, s>>>(x, g, b, (__bf16*)y, rows, reqs, nreq, dyn_rows,     \
                                                              dyn_nreq);                                          \
    else                                                                                                          \
      layernorm_rows_kernel<float, L_, 3><<<gr, 256, 0, s>>>(x, g, b, (float*)y, rows, reqs, nreq, dyn_rows,       \
                                                             dyn_nreq);                                           \
    return hipGetLastError() == hipSuccess ? 0 : -5;                                                              \
  } while (0)
  const bool al16 = (((uintptr_t)x | (uintptr_t)g | (uintptr_t)b | (uintptr_t)y) & 15) == 0;
  if (al16 && D == 384) REVO_LN_ROWS(32);
  if (al16 && D == 192) REVO_LN_ROWS(16);
#undef REVO_LN_ROWS
  dim3 grid(cdiv(rows, 4));
  if (out_prec == P_BF16)
    layernorm_kernel<__bf16><<<grid, 256, 0, s>>>(x, g, b, (__bf16*)y, rows, D, reqs, nreq, dyn_rows, dyn_nreq);
  else
    layernorm_kernel<float><<<grid, 256, 0, s>>>(x, g, b, (float*)y, rows, D, reqs, nreq, dyn_rows, dyn_nreq);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_composite(const ReqDesc* reqs, int nreq, int channels, int max_pixels, int composite, hipStream_t s,
                     const int* dyn_nreq) {
  if (nreq <= 0 || max_pixels <= 0) return 0;
  const int bx = cdiv(max_pixels, 256) < 1024 ? cdiv(max_pixels, 256) : 1024;  // grid-stride beyond
  composite_kernel<<<dim3(bx, nreq), 256, 0, s>>>(reqs, channels, composite, dyn_nreq);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_convert(Prec prec, const float* src, void* dst, long long n, hipStream_t s) {
  if (n <= 0) return 0;
  const unsigned blocks = (unsigned)cdivll(n, 256);
  if (prec == P_BF16) convert_kernel<__bf16><<<blocks, 256, 0, s>>>(src, (__bf16*)dst, n);
  else if (prec == P_FP32) convert_kernel<float><<<blocks, 256, 0, s>>>(src, (float*)dst, n);
  else if (prec == P_FP8) convert_fp8_kernel<<<blocks, 256, 0, s>>>(src, (uint8_t*)dst, n);
  else return -95;
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_layernorm_fp8(const float* x, const float* g, const float* b, uint8_t* y, const float* out_scale,
                         int rows, int D, hipStream_t s, const int* dyn_rows) {
  if (rows <= 0) return 0;
  if (D > 512 || !out_scale) return -22;
  // the widths of the two networks (16-byte aligned inputs, 4-byte aligned
  // output): three float4 per lane, 2 or 4 rows per wave
  const bool al = ((((uintptr_t)x | (uintptr_t)g | (uintptr_t)b) & 15) | ((uintptr_t)y & 3)) == 0;
  if (al && D == 384) {
    layernorm_rows_fp8_kernel<32, 3><<<cdiv(rows, 8), 256, 0, s>>>(x, g, b, y, out_scale, rows, dyn_rows);
    return hipGetLastError() == hipSuccess ? 0 : -5;
  }
  if (al && D == 192) {
    layernorm_rows_fp8_kernel<16, 3><<<cdiv(rows, 16), 256, 0, s>>>(x, g, b, y, out_scale, rows, dyn_rows);
    return hipGetLastError() == hipSuccess ? 0 : -5;
  }
  layernorm_fp8_kernel<<<cdiv(rows, 4), 256, 0, s>>>(x, g, b, y, out_scale, rows, D, dyn_rows);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_quantize_rows(const float* w, int rows, int cols, uint8_t* w8, float* scale, hipStream_t s) {
  if (rows <= 0) return 0;
  quantize_rows_kernel<<<rows, 256, 0, s>>>(w, cols, w8, scale);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_absmax(const __bf16* x, int rows, int D, const ReqDesc* reqs, int nreq, unsigned* slot, hipStream_t s) {
  if (rows <= 0) return 0;
  if (D % 8) return -22;
  absmax_kernel<<<cdiv(rows, 256) < 1024 ? cdiv(rows, 256) : 1024, 256, 0, s>>>(x, D, reqs, nreq, slot);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_attn_absmax(const __bf16* q, const __bf16* k, const __bf16* vt, int heads, int ld, int rows,
                       const ReqDesc* reqs, int nreq, unsigned* slots, hipStream_t s) {
  if (rows <= 0) return 0;
  attn_absmax_kernel<<<dim3(cdiv(rows, 256) < 256 ? cdiv(rows, 256) : 256, heads), 256, 0, s>>>(q, k, vt, heads, ld,
                                                                                            reqs, nreq, slots);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_attn_scales(const unsigned* absmax, int* exps, float* inv, int n, hipStream_t s) {
  if (n <= 0) return 0;
  attn_scales_kernel<<<cdiv(n, 256), 256, 0, s>>>(absmax, exps, inv, n);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_scales_from_absmax(const unsigned* absmax, float* scale, int n, hipStream_t s) {
  if (n <= 0) return 0;
  scales_kernel<<<cdiv(n, 256), 256, 0, s>>>(absmax, scale, n);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_fill_zero(void* p, long long bytes, hipStream_t s) {
  if (bytes <= 0) return 0;
  const long long n16 = bytes / 16;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && n16 > 0)
    zero_kernel<<<(unsigned)cdivll(n16, 256), 256, 0, s>>>((uint4*)p, n16);
  const long long done = ((reinterpret_cast<uintptr_t>(p) & 15) == 0) ? n16 * 16 : 0;
  if (bytes > done)
    zero_tail_kernel<<<(unsigned)cdivll(bytes - done, 256), 256, 0, s>>>((uint8_t*)p + done, bytes - done);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace revo
