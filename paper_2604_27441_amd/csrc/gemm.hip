// MFMA GEMM for every linear step of the recovery network, with the
// tubelet-embedding gather fused into its operand loader and the bias /
// GELU / residual / positional-embedding / head-split / unpatchify work fused
// into its epilogue.
//
// Product: C^T[n][m] = sum_k W[n][k] * X[m][k] (weights [out][in], tokens
// [M][K], both K-contiguous).  Weights feed the MFMA's A operand and tokens
// its B operand, so each lane ends up owning one token and runs of four
// consecutive output features: epilogue stores are 8/16-byte row segments.
//
// Tile: 128 tokens x BN features x one K stage (128 bytes per operand row;
// 64 for FP8), 4 waves in a 2 x 2 grid, LDS double-buffered, row pitch padded
// by 16 bytes.
#include <type_traits>

#include "kernels.h"

namespace revo {

namespace {

constexpr int BM = 128;
constexpr int NT = 256;


// Four consecutive results of one row; inv = 1 / (output scale) for FP8.
template <class T> struct Vec4;
template <> struct Vec4<float> {
  __device__ static void store(float* p, const float v[4], float) {
    *reinterpret_cast<f32x4*>(p) = f32x4{v[0], v[1], v[2], v[3]};
  }
};
template <> struct Vec4<__bf16> {
  __device__ static void store(__bf16* p, const float v[4], float) {
    *reinterpret_cast<bf16x4*>(p) = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
  }
};
template <> struct Vec4<uint8_t> {
  __device__ static void store(uint8_t* p, const float v[4], float inv) {
    *reinterpret_cast<uint32_t*>(p) = e4m3x4(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
  }
};
template <class T> __device__ inline T out_cast(float v, float inv);
template <> __device__ inline float out_cast<float>(float v, float) { return v; }
template <> __device__ inline __bf16 out_cast<__bf16>(float v, float) { return (__bf16)v; }
template <> __device__ inline uint8_t out_cast<uint8_t>(float v, float inv) { return e4m3(v * inv); }

template <class Op> __device__ inline typename Op::frag frag_of(const uint4& u, int g);
template <> __device__ inline float frag_of<OpF32>(const uint4& u, int g) {
  const uint32_t w = g == 0 ? u.x : g == 1 ? u.y : g == 2 ? u.z : u.w;
  return __uint_as_float(w);
}
template <> __device__ inline bf16x8 frag_of<OpBF16>(const uint4& u, int) {
  return __builtin_bit_cast(bf16x8, u);
}
__device__ inline i32x8 frag_fp8(const uint4& lo, const uint4& hi) {
  return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
}

// erf(x) by Abramowitz & Stegun, Handbook of Mathematical Functions, 7.1.26
// (|error| <= 1.5e-7): branch-free, so the lanes of a wave never diverge.
__device__ inline float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
                              0.254829592f);
  const float r = 1.0f - poly * __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
  return copysignf(r, x);
}

__device__ inline float gelu_erf(float v) { return 0.5f * v * (1.0f + erf_as(v * 0.70710678118654752f)); }
// d gelu / dv = Phi(v) + v phi(v)
__device__ inline float gelu_erf_grad(float v) {
  return 0.5f * (1.0f + erf_as(v * 0.70710678118654752f)) +
         v * 0.3989422804014327f * __builtin_amdgcn_exp2f(-0.5f * v * v * 1.4426950408889634f);
}

// sin (odd == 0) or cos (odd == 1) of x for |x| up to a few thousand, without
// scratch memory: x = n (pi/2) + r with a three-part Cody-Waite reduction,
// then the single-precision minimax polynomials of the Cephes library
// (S. L. Moshier) on |r| <= pi/4.
__device__ inline float sincos_small(float x, int odd) {
  const float n = rintf(x * 0.636619772367581343f);
  float r = fmaf(n, -1.5703125f, x);
  r = fmaf(n, -4.837512969970703125e-4f, r);
  r = fmaf(n, -7.54978995489188216e-8f, r);
  const int q = ((int)n + odd) & 3;  // cos(x) = sin(x + pi/2)
  const float z = r * r;
  const float sp = fmaf(fmaf(fmaf(-1.9515295891e-4f, z, 8.3321608736e-3f), z, -1.6666654611e-1f), z * r, r);
  const float cp = fmaf(fmaf(fmaf(2.443315711809948e-5f, z, -1.388731625493765e-3f), z, 4.166664568298827e-2f), z * z,
                        fmaf(-0.5f, z, 1.0f));
  const float v = (q & 1) ? cp : sp;
  return (q & 2) ? -v : v;
}

// Sinusoid of the three-axis positional embedding: column c of a D-wide
// embedding for position s (axis c / (D/3)), sin at even, cos at odd columns,
// frequency 10000^(-2i/(D/3)) for the column pair i.
__device__ inline float pe_value(float s, int c, int d3) {
  const int i2 = (c % d3) >> 1;
  const float freq = exp2f(-(float)(2 * i2) / (float)d3 * 13.287712379549449f);  // log2(10000)
  return sincos_small(s * freq, c & 1);
}

// One 16-byte chunk (E elements) of a tubelet vector: element k of token
// (j, y, x) is frame j*T + t, pixel (16y + py, 16x + px), channel c with
// k = ((t*16 + py)*16 + px)*C + c.  Out-of-frame (padding) pixels and lost
// target pixels read as zero; RGB is scaled by 1/255 and depth by 1/4000 mm.
// A chunk never straddles a patch row (16*C is a multiple of E), so when
// the patch row lies inside the frame and rows are 8-pixel aligned it is
// one contiguous 4..16-byte load.
template <class Op>
__device__ uint4 gather_chunk(const ReqDesc& d, int j, int y, int x, int k, int C) {
  typedef typename Op::T T;
  constexpr int E = 16 / sizeof(T);
  union { uint4 u; T v[E]; } r;
  const int rowlen = 16 * C;
  const int rt = k / rowlen;
  const int o = k - rt * rowlen;
  const int Tt = d.nframes / d.J;
  const int f = j * Tt + (rt >> 4);
  const int Y = 16 * y + (rt & 15);
  const bool target = (f == d.nframes - 1);
  const int X0 = 16 * x;
  float v[E];
  if (Y < d.H && X0 + 16 <= d.W && (d.W & 7) == 0) {
    const size_t rowpix = (size_t)Y * d.W + X0;
    if (C == 3) {
      const uint8_t* src = (const uint8_t*)d.frames[f] + rowpix * 3 + o;
      uint32_t w[E / 4];
      if constexpr (E == 8) {
        const uint2 t = *reinterpret_cast<const uint2*>(src);
        w[0] = t.x; w[1] = t.y;
      } else {
        w[0] = *reinterpret_cast<const uint32_t*>(src);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = (float)((w[e >> 2] >> (8 * (e & 3))) & 0xFF) * (1.0f / 255.0f);
      if (target) {
        const uint8_t* m = d.mask + rowpix;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (m[(o + e) / 3]) v[e] = 0.0f;
      }
    } else {
      const uint16_t* src = (const uint16_t*)d.frames[f] + rowpix + o;
      uint32_t w[E / 2];
      if constexpr (E == 8) {
        const uint4 t = *reinterpret_cast<const uint4*>(src);
        w[0] = t.x; w[1] = t.y; w[2] = t.z; w[3] = t.w;
      } else {
        const uint2 t = *reinterpret_cast<const uint2*>(src);
        w[0] = t.x; w[1] = t.y;
      }
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = (float)((w[e >> 1] >> (16 * (e & 1))) & 0xFFFF) * (1.0f / 4000.0f);
      if (target) {
        const uint8_t* m = d.mask + rowpix + o;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (m[e]) v[e] = 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int oe = o + e;
      const int X = X0 + oe / C;
      const int c = oe - (oe / C) * C;
      v[e] = 0.0f;
      if (Y < d.H && X < d.W) {
        const size_t pix = (size_t)Y * d.W + X;
        if (!(target && d.mask[pix])) {
          if (C == 3) v[e] = (float)((const uint8_t*)d.frames[f])[pix * 3 + c] * (1.0f / 255.0f);
          else v[e] = (float)((const uint16_t*)d.frames[f])[pix] * (1.0f / 4000.0f);
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) r.v[e] = Op::from_float(v[e]);
  return r.u;
}

// Tubelet vectors written out once as a dense [M][K] operand (K = T*16*16*C),
// so the embedding product runs as a plain dense GEMM instead of gathering
// the same pixels again for every N tile.  One thread per 16-byte chunk;
// rows in the alignment gaps between requests are zeros.
template <class Op>
__global__ void tubelet_pack_kernel(const ReqDesc* __restrict__ reqs, int nreq_, const int* dyn_nreq, int M_,
                                    const int* dyn_m, int K, int C, typename Op::T* __restrict__ out) {
  constexpr int E = 16 / sizeof(typename Op::T);
  const int M = dyn_m ? *dyn_m : M_;
  const int nreq = dyn_nreq ? *dyn_nreq : nreq_;
  const int cpr = K / E;
  const long long total = (long long)M * cpr;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(i / cpr);
    const int k = (int)(i - (long long)m * cpr) * E;
    uint4 v = make_uint4(0, 0, 0, 0);
    const int r = find_req_tok(reqs, nreq, m);
    const ReqDesc& d = reqs[r];
    const int t = m - d.tok_off;
    const int j = t / d.P, p = t - (t / d.P) * d.P;
    if (t >= 0 && j < d.J) v = gather_chunk<Op>(d, j, p / d.gx, p - (p / d.gx) * d.gx, k, C);
    *reinterpret_cast<uint4*>(out + (size_t)m * K + k) = v;
  }
}

// Bias (and, for FP8 operands, row-scale x activation-scale) values of the
// output features one lane's accumulators hold: features
// n0 + wn BN/2 + 32 ns + 8 g + 4 half + e.  Fetched as 16-byte vectors
// (bias and scales are 16-byte aligned) all at once, early, instead of once
// per group of four inside the epilogue.
template <int BN>
struct EpiCols {
  f32x4 b[BN / 64][4], s[BN / 64][4];
};
template <class Op, int BN>
__device__ __forceinline__ void epi_load_cols(const GemmArgs& a, int n0, int wn, int half, EpiCols<BN>& c) {
  constexpr bool SC = sizeof(typename Op::T) == 1;
  const float xsc = SC ? *a.xscale : 1.0f;
#pragma unroll
  for (int ns = 0; ns < BN / 64; ++ns)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int n = n0 + wn * (BN / 2) + ns * 32 + g * 8 + half * 4;
      c.b[ns][g] = *reinterpret_cast<const f32x4*>(a.bias + n);
      if constexpr (SC) c.s[ns][g] = *reinterpret_cast<const f32x4*>(a.wscale + n) * xsc;
    }
}

// Epilogue of one 128 x BN tile straight from the accumulators (the head's
// unpatchify scatter), for the tile's rows below Mlive.
template <class Op, int BN, int EPI, class OutT>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& a, f32x16 (&acc)[BN / 64][2], int m0, int n0,
                                              int Mlive, int nreq, int lane, int wave, const EpiCols<BN>& cols) {
  constexpr int NSUB = BN / 64;
  constexpr bool SC = sizeof(typename Op::T) == 1;  // FP8 operands carry row scales
  const int half = lane >> 5, l32 = lane & 31;
  const int wn = wave >> 1, wm = wave & 1;
  const float oinv = a.out_scale ? 1.0f / *a.out_scale : 1.0f;
#pragma unroll
  for (int ms = 0; ms < 2; ++ms) {
    const int m = m0 + wm * 64 + ms * 32 + l32;
    if (m >= Mlive) continue;
    int r = 0, tj = 0, ty = 0, tx = 0;
    if (EPI == EPI_PE) {
      r = find_req_tok(a.reqs, nreq, m);
      const ReqDesc& d = a.reqs[r];
      const int t = m - d.tok_off;
      tj = t / d.P;
      const int p = t - tj * d.P;
      ty = p / d.gx; tx = p - ty * d.gx;
    } else if (EPI == EPI_HEAD) {
      r = find_req_head(a.reqs, nreq, m);
      const ReqDesc& d = a.reqs[r];
      const int p = m - d.head_off;
      ty = p / d.gx; tx = p - ty * d.gx;
    }
#pragma unroll
    for (int ns = 0; ns < NSUB; ++ns) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int n = n0 + wn * (BN / 2) + ns * 32 + g * 8 + half * 4;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[e] = SC ? acc[ns][ms][4 * g + e] * cols.s[ns][g][e] + cols.b[ns][g][e]
                    : acc[ns][ms][4 * g + e] + cols.b[ns][g][e];
        if (EPI == EPI_STORE) {
          Vec4<OutT>::store((OutT*)a.out + (size_t)m * a.ldo + n, v, oinv);
        } else if (EPI == EPI_GELU) {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = gelu_erf(v[e]);
          Vec4<OutT>::store((OutT*)a.out + (size_t)m * a.ldo + n, v, oinv);
        } else if (EPI == EPI_RESIDUAL) {
          float* p = (float*)a.out + (size_t)m * a.ldo + n;
          f32x4 old = *reinterpret_cast<const f32x4*>(a.res ? a.res + (size_t)m * a.ldo + n : p);
          *reinterpret_cast<f32x4*>(p) = f32x4{old[0] + v[0], old[1] + v[1], old[2] + v[2], old[3] + v[3]};
        } else if (EPI == EPI_PE) {
          const ReqDesc& d = a.reqs[r];
          const int d3 = a.N / 3;
          const int axis = n / d3;
          const float s = axis == 0 ? (tj < d.J ? d.tau[tj] : 0.0f) : axis == 1 ? (float)ty : (float)tx;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] += pe_value(s, n + e, d3);
          float* p = (float*)a.out + (size_t)m * a.ldo + n;
          *reinterpret_cast<f32x4*>(p) = f32x4{v[0], v[1], v[2], v[3]};
        } else if (EPI == EPI_QKV) {
          const int D = a.heads * 64;
          const int part = n / D, hd = (n % D) >> 6, dd = n & 63;
          if (part == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] *= a.qscale;
            Vec4<OutT>::store((OutT*)a.q + ((size_t)hd * a.ldqk + m) * 64 + dd, v, 1.0f);
          } else if (part == 1) {
            Vec4<OutT>::store((OutT*)a.k + ((size_t)hd * a.ldqk + m) * 64 + dd, v, 1.0f);
          } else {
            OutT* vt = (OutT*)a.vt + ((size_t)hd * 64 + dd) * a.ldv + m;
#pragma unroll
            for (int e = 0; e < 4; ++e) vt[(size_t)e * a.ldv] = out_cast<OutT>(v[e], 1.0f);
          }
        } else if (EPI == EPI_HEAD) {
          // feature c = (py * 16 + px) * C + ch; the two channel counts get
          // constant divisors
          const ReqDesc& d = a.reqs[r];
          auto put = [&](auto Cc) {
            constexpr int C = decltype(Cc)::value;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int c = n + e;
              const int py = c / (16 * C), px = (c / C) & 15, ch = c % C;
              const int Y = 16 * ty + py, Xp = 16 * tx + px;
              if (Y < d.H && Xp < d.W) d.pred[((size_t)Y * d.W + Xp) * C + ch] = v[e];
            }
          };
          if (a.channels == 3) put(std::integral_constant<int, 3>{});
          else put(std::integral_constant<int, 1>{});
        }
      }
    }
  }
}

// LDS bytes of the staged epilogue: a row-major [BM][BN] tile of the output
// type, or for the V part of the QKV product a transposed [BN][BM] tile
// (rows padded by 16 bytes).
template <int BN, class OutT, int BM_ = BM>
constexpr int epi_stage_bytes() {
  return BM_ * (BN * (int)sizeof(OutT) + 16) > BN * (BM_ * (int)sizeof(OutT) + 16)
             ? BM_ * (BN * (int)sizeof(OutT) + 16)
             : BN * (BM_ * (int)sizeof(OutT) + 16);
}

// Epilogue through LDS: the accumulators (lane = token, runs of four
// features) go into a tile after the scale / bias / fused step, and the
// workgroup then writes whole output rows in 16-byte chunks, so every store
// instruction covers contiguous row segments instead of one short piece per
// token.  The V part of the QKV product is staged transposed and written as
// contiguous token runs of V^T.  smem must hold epi_stage_bytes<BN, OutT, BM_>().
// The tile is BM_ tokens x BN features over 2 WM_ waves, wave w covering
// tokens (w % WM_) 64 .. +63 and features (w / WM_) BN/2 .. +BN/2-1.
template <class Op, int BN, int EPI, class OutT, int BM_ = BM, int WM_ = 2>
__device__ __forceinline__ void gemm_epilogue_staged(const GemmArgs& a, f32x16 (&acc)[BN / 64][2], int m0, int n0,
                                                     int Mlive, int nreq, int tid, uint8_t* smem,
                                                     const EpiCols<BN>& cols, bool active = true) {
  constexpr int NT_ = 128 * WM_;
  constexpr int NSUB = BN / 64;
  constexpr int TPB = BN * (int)sizeof(OutT) + 16;   // row pitch (bytes), row-major tile
  constexpr int TPV = BM_ * (int)sizeof(OutT) + 16;  // row pitch (bytes), transposed V tile
  constexpr int EO = 16 / (int)sizeof(OutT);          // output elements per 16-byte chunk
  const int lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int wn = wave / WM_, wm = wave % WM_;
  const float oinv = a.out_scale ? 1.0f / *a.out_scale : 1.0f;
  const int D = EPI == EPI_QKV ? a.heads * 64 : 1;
  const int part = EPI == EPI_QKV ? n0 / D : 0;  // tiles never straddle Q | K | V
  const bool vtile = EPI == EPI_QKV && part == 2;
  constexpr bool SC = sizeof(typename Op::T) == 1;  // FP8 operands carry row scales
  __syncthreads();  // every wave is done with the operand tiles
  // (threads beyond the tile's 2 WM_ waves, !active, only join the barriers)
  if (active) {
#pragma unroll
  for (int ms = 0; ms < 2; ++ms) {
    const int ml = wm * 64 + ms * 32 + l32;
    const int m = m0 + ml;
    int r = 0, tj = 0, ty = 0, tx = 0;
    if (EPI == EPI_PE) {
      r = find_req_tok(a.reqs, nreq, m);
      const ReqDesc& d = a.reqs[r];
      const int t = m - d.tok_off;
      tj = t / d.P;
      const int p = t - tj * d.P;
      ty = p / d.gx; tx = p - ty * d.gx;
    }
#pragma unroll
    for (int ns = 0; ns < NSUB; ++ns) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int nl = wn * (BN / 2) + ns * 32 + g * 8 + half * 4;
        const int n = n0 + nl;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[e] = SC ? acc[ns][ms][4 * g + e] * cols.s[ns][g][e] + cols.b[ns][g][e]
                    : acc[ns][ms][4 * g + e] + cols.b[ns][g][e];
        if (EPI == EPI_GELU) {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = gelu_erf(v[e]);
        } else if (EPI == EPI_PE) {
          const ReqDesc& d = a.reqs[r];
          const int d3 = a.N / 3;
          const int axis = n / d3;
          const float s = axis == 0 ? (tj < d.J ? d.tau[tj] : 0.0f) : axis == 1 ? (float)ty : (float)tx;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] += pe_value(s, n + e, d3);
        } else if (EPI == EPI_QKV && part == 0) {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] *= a.qscale;
        }
        // E4M3 Q / K / V^T of the FP8 attention: each head's own scale
        const float hinv = (EPI == EPI_QKV && sizeof(OutT) == 1) ? a.head_inv[part * a.heads + ((n % D) >> 6)] : oinv;
        if (vtile) {
          // 2-byte V^T (BF16 attention): within each group of 16 tokens the
          // column index has bits 2 and 3 swapped, the order in which a
          // lane's eight probabilities meet the P V product; 1-byte V^T (FP8
          // attention): fp8_vt_col order within groups of 64
          const int mc = sizeof(OutT) == 2 ? (ml & ~12) | ((ml & 4) << 1) | ((ml & 8) >> 1)
                                           : (sizeof(OutT) == 1 ? fp8_vt_col(ml) : ml);
#pragma unroll
          for (int e = 0; e < 4; ++e) reinterpret_cast<OutT*>(smem + (nl + e) * TPV)[mc] = out_cast<OutT>(v[e], hinv);
        } else {
          Vec4<OutT>::store(reinterpret_cast<OutT*>(smem + ml * TPB) + nl, v, hinv);
        }
      }
    }
  }
  }
  __syncthreads();
  if (!active) return;
  if (vtile) {
    // V^T rows: EO consecutive columns per 16-byte chunk; a 2-byte chunk
    // can hold permuted tokens up to the end of its group of 16 (a 1-byte
    // one up to the end of its group of 64), so it is written whole while
    // its group starts below Mlive
    const int Mcol = sizeof(OutT) == 2 ? (Mlive + 15) & ~15 : (sizeof(OutT) == 1 ? (Mlive + 63) & ~63 : Mlive);
    for (int i = tid; i < BN * (BM_ / EO); i += NT_) {
      const int nl = i / (BM_ / EO), c = (i - nl * (BM_ / EO)) * EO;
      const int m = m0 + c;
      if (m >= Mcol) continue;
      const int n = n0 + nl;
      const int hd = (n - 2 * D) >> 6, dd = n & 63;
      OutT* dst = (OutT*)a.vt + ((size_t)hd * 64 + dd) * a.ldv + m;
      const OutT* src = reinterpret_cast<const OutT*>(smem + nl * TPV) + c;
      if (m + EO <= Mcol) {
        *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
      } else {
        for (int e = 0; m + e < Mcol; ++e) dst[e] = src[e];
      }
    }
    return;
  }
  constexpr int CPRO = BN / EO;
  if constexpr (EPI == EPI_GELU_PRE || EPI == EPI_GELU_BWD) {
    static_assert(sizeof(OutT) == 4, "FP32 outputs");
    static_assert(BM_ * CPRO % NT_ == 0, "whole chunks per thread");
    constexpr int IT = BM_ * CPRO / NT_;
    // EPI_GELU_BWD: every pre-activation chunk of this thread is loaded
    // before the first store
    f32x4 pv[EPI == EPI_GELU_BWD ? IT : 1];
    if constexpr (EPI == EPI_GELU_BWD) {
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = tid + it * NT_;
        const int rl = i / CPRO, c = (i - rl * CPRO) * EO;
        const int m = m0 + rl;
        pv[it] = m < Mlive ? *reinterpret_cast<const f32x4*>(a.pre + (size_t)m * a.ldo + n0 + c) : f32x4{};
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = tid + it * NT_;
      const int rl = i / CPRO, c = (i - rl * CPRO) * EO;
      const int m = m0 + rl;
      if (m >= Mlive) continue;
      const f32x4 v = *reinterpret_cast<const f32x4*>(smem + rl * TPB + c * (int)sizeof(OutT));
      f32x4 r;
      if constexpr (EPI == EPI_GELU_PRE) {
        *reinterpret_cast<f32x4*>(a.pre + (size_t)m * a.ldo + n0 + c) = v;
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = gelu_erf(v[e]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = v[e] * gelu_erf_grad(pv[it][e]);
      }
      *reinterpret_cast<f32x4*>((float*)a.out + (size_t)m * a.ldo + n0 + c) = r;
    }
    return;
  }
  if constexpr (EPI == EPI_RESIDUAL) {
    // every residual chunk of this thread is loaded before the first add and
    // store (a load after a store to the same buffer would otherwise wait
    // out one memory round trip per chunk)
    static_assert(BM_ * CPRO % NT_ == 0, "whole chunks per thread");
    constexpr int IT = BM_ * CPRO / NT_;
    const float* rsrc = a.res ? a.res : (const float*)a.out;
    f32x4 res[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = tid + it * NT_;
      const int rl = i / CPRO, c = (i - rl * CPRO) * EO;
      const int m = m0 + rl;
      res[it] = m < Mlive ? *reinterpret_cast<const f32x4*>(rsrc + (size_t)m * a.ldo + n0 + c) : f32x4{};
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = tid + it * NT_;
      const int rl = i / CPRO, c = (i - rl * CPRO) * EO;
      const int m = m0 + rl;
      if (m >= Mlive) continue;
      const f32x4 v = *reinterpret_cast<const f32x4*>(smem + rl * TPB + c * (int)sizeof(OutT));
      *reinterpret_cast<f32x4*>((float*)a.out + (size_t)m * a.ldo + n0 + c) = res[it] + v;
    }
    return;
  }
  for (int i = tid; i < BM_ * CPRO; i += NT_) {
    const int rl = i / CPRO, c = (i - rl * CPRO) * EO;
    const int m = m0 + rl;
    if (m >= Mlive) continue;
    const int n = n0 + c;
    const uint4 val = *reinterpret_cast<const uint4*>(smem + rl * TPB + c * (int)sizeof(OutT));
    if (EPI == EPI_QKV) {
      const int hd = (n - part * D) >> 6, dd = n & 63;
      OutT* dst = (OutT*)(part == 0 ? a.q : a.k) + ((size_t)hd * a.ldqk + m) * 64 + dd;
      *reinterpret_cast<uint4*>(dst) = val;
    } else {
      *reinterpret_cast<uint4*>((OutT*)a.out + (size_t)m * a.ldo + n) = val;
    }
  }
}

// KS = 2 (FP32 products of at most one workgroup per CU): 8 waves, the
// second four taking the second half of every stage's k steps into
// accumulators of their own, added to the first four's through LDS before
// the epilogue, so each SIMD holds two waves
template <class Op, int BN, int EPI, int XM, class OutT, int KS = 1>
__global__ __launch_bounds__(NT * KS, KS == 1 ? 2 : 1) void gemm_kernel(const GemmArgs a) {
  typedef typename Op::T T;
  static_assert(KS == 1 || (KS == 2 && EPI != EPI_HEAD), "K split: staged epilogues only");
  constexpr int NT_ = NT * KS;
  constexpr int BK = Op::BK;
  constexpr int E = 16 / sizeof(T);               // elements per 16-byte chunk
  constexpr int CPR = BK * sizeof(T) / 16;        // chunks per stage row
  constexpr int PITCH = (BK * sizeof(T) + 16) / sizeof(T);  // LDS row pitch, padded by 16 bytes
  constexpr int XC = BM * CPR / NT_;
  constexpr int WC = BN * CPR / NT_;
  static_assert(XC * NT_ == BM * CPR && WC * NT_ == BN * CPR, "whole chunks per thread");
  constexpr int NSUB = BN / 64;
  constexpr int FB = Op::KPL * sizeof(T);          // operand bytes per lane per MFMA step
  constexpr int G = FB >= 16 ? 1 : 16 / FB;        // MFMA steps per 16-byte LDS read
  constexpr int STEPS = BK / (2 * Op::KPL);
  // operand stages, reused by the staged epilogue once the K loop is done
  constexpr int OPB = (2 * BM * PITCH + 2 * BN * PITCH) * (int)sizeof(T);
  constexpr int EPB = EPI == EPI_HEAD ? 0 : epi_stage_bytes<BN, OutT>();
  __shared__ __attribute__((aligned(16))) uint8_t smem[OPB > EPB ? OPB : EPB];
  T(*xs)[BM * PITCH] = reinterpret_cast<T(*)[BM * PITCH]>(smem);
  T(*ws)[BN * PITCH] = reinterpret_cast<T(*)[BN * PITCH]>(smem + 2 * BM * PITCH * sizeof(T));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  // Workgroups go round-robin to the 8 XCDs, each with its own L2.  Give
  // XCD x a contiguous range of tiles, ordered with the N tile fastest, so
  // the N tiles that reuse one block of activation rows run together on one
  // XCD and read those rows from its L2 instead of HBM.
  const int gn = a.N / BN;
  const int ntiles = gridDim.x;
  const int L = blockIdx.x;
  const int xcd = L & 7, per = ntiles >> 3, rem = ntiles & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (L >> 3);
  const int m0 = (tile / gn) * BM;
  const int n0 = (tile - (tile / gn) * gn) * BN;
  const int Mlive = a.dyn_m ? *a.dyn_m : a.M;
  const int nreq = a.dyn_nreq ? *a.dyn_nreq : a.nreq;
  if (m0 >= Mlive) return;  // grid sized for a capacity
  const int KT = a.K / BK;
  const T* __restrict__ W = (const T*)a.W;
  const T* __restrict__ X = (const T*)a.X;

  // gather: token coordinates of this thread's rows
  int g_req[XC], g_j[XC], g_y[XC], g_x[XC];
  if (XM == X_GATHER) {
#pragma unroll
    for (int i = 0; i < XC; ++i) {
      const int m = m0 + (tid + i * NT_) / CPR;
      g_req[i] = -1;
      if (m < Mlive) {
        const int r = find_req_tok(a.reqs, nreq, m);
        const ReqDesc& d = a.reqs[r];
        const int t = m - d.tok_off;
        const int j = t / d.P, p = t - (t / d.P) * d.P;
        // rows past the request's J * P tokens are alignment gaps: zero
        if (j < d.J) { g_req[i] = r; g_j[i] = j; g_y[i] = p / d.gx; g_x[i] = p - (p / d.gx) * d.gx; }
      }
    }
  }

  // per-thread chunk coordinates within a stage
  int c_row[XC > WC ? XC : WC], c_k[XC > WC ? XC : WC];
#pragma unroll
  for (int i = 0; i < (XC > WC ? XC : WC); ++i) {
    c_row[i] = (tid + i * NT_) / CPR;
    c_k[i] = ((tid + i * NT_) % CPR) * E;
  }
  // two register sets of stage operands: the loads for stage k+2 are
  // issued while stage k is multiplied, so two stages of compute cover the
  // memory latency
  uint4 xr0[XC], wr0[WC], xr1[XC], wr1[WC];
  // Dense operands come in through buffer loads: a per-thread byte offset
  // and a scalar one per stage, and activation rows at or past Mlive fall
  // outside the descriptor's range and read as zeros, so no lane branches
  // around a load (the host keeps both operands below 2 GiB).
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)W, (short)0, a.N * a.K * (int)sizeof(T), 0x00020000);
  const __amdgpu_buffer_rsrc_t xrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, XM == X_DENSE ? Mlive * a.K * (int)sizeof(T) : 0,
                                        0x00020000);
  int xoff[XC], woff[WC];
#pragma unroll
  for (int i = 0; i < XC; ++i) xoff[i] = ((m0 + c_row[i]) * a.K + c_k[i]) * (int)sizeof(T);
#pragma unroll
  for (int i = 0; i < WC; ++i) woff[i] = ((n0 + c_row[i]) * a.K + c_k[i]) * (int)sizeof(T);
#define REVO_GEMM_LOAD(kt_, XR, WR)                                                                          \
  do {                                                                                                       \
    const int k0_ = (kt_) * BK;                                                                              \
    _Pragma("unroll") for (int i = 0; i < XC; ++i) {                                                         \
      if (XM == X_DENSE) {                                                                                   \
        XR[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(                             \
                                              xrs, xoff[i], k0_ * (int)sizeof(T), 0));                       \
      } else {                                                                                               \
        XR[i] = g_req[i] >= 0                                                                                \
                    ? gather_chunk<Op>(a.reqs[g_req[i]], g_j[i], g_y[i], g_x[i], k0_ + c_k[i], a.channels)   \
                    : make_uint4(0, 0, 0, 0);                                                                \
      }                                                                                                      \
    }                                                                                                        \
    _Pragma("unroll") for (int i = 0; i < WC; ++i)                                                           \
      WR[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(                               \
                                            wrs, woff[i], k0_ * (int)sizeof(T), 0));                         \
  } while (0)
#define REVO_GEMM_STORE(buf_, XR, WR)                                                                        \
  do {                                                                                                       \
    _Pragma("unroll") for (int i = 0; i < XC; ++i)                                                           \
      *reinterpret_cast<uint4*>(&xs[buf_][c_row[i] * PITCH + c_k[i]]) = XR[i];                               \
    _Pragma("unroll") for (int i = 0; i < WC; ++i)                                                           \
      *reinterpret_cast<uint4*>(&ws[buf_][c_row[i] * PITCH + c_k[i]]) = WR[i];                               \
  } while (0)

  // waves 4..7 (KS = 2) repeat waves 0..3's tile positions on the other k steps
  const int wq = wave & 3, kgrp = KS == 1 ? 0 : wave >> 2;
  const int wn = wq >> 1, wm = wq & 1;
  static_assert(STEPS % (KS * G) == 0, "whole LDS reads per k group");
  f32x16 acc[NSUB][2];
#pragma unroll
  for (int i = 0; i < NSUB; ++i) { acc[i][0] = f32x16{}; acc[i][1] = f32x16{}; }

  // one K stage from LDS buffer buf_ into the accumulators
#define REVO_GEMM_COMPUTE(buf_)                                                                              \
  _Pragma("unroll") for (int s0 = 0; s0 < STEPS / KS; s0 += G) {                                            \
    const int koff = half * (BK / 2) + (kgrp * (STEPS / KS) + s0) * Op::KPL;                                 \
    if constexpr (FB == 32) {                                                                                \
      uint4 wf[NSUB][2], xf[2][2];                                                                           \
      _Pragma("unroll") for (int ns = 0; ns < NSUB; ++ns) {                                                  \
        const T* p = &ws[buf_][(wn * (BN / 2) + ns * 32 + l32) * PITCH + koff];                              \
        wf[ns][0] = reinterpret_cast<const uint4*>(p)[0];                                                    \
        wf[ns][1] = reinterpret_cast<const uint4*>(p)[1];                                                    \
      }                                                                                                      \
      _Pragma("unroll") for (int ms = 0; ms < 2; ++ms) {                                                     \
        const T* p = &xs[buf_][(wm * 64 + ms * 32 + l32) * PITCH + koff];                                    \
        xf[ms][0] = reinterpret_cast<const uint4*>(p)[0];                                                    \
        xf[ms][1] = reinterpret_cast<const uint4*>(p)[1];                                                    \
      }                                                                                                      \
      _Pragma("unroll") for (int ns = 0; ns < NSUB; ++ns)                                                    \
        _Pragma("unroll") for (int ms = 0; ms < 2; ++ms)                                                     \
          Op::mma(acc[ns][ms], frag_fp8(wf[ns][0], wf[ns][1]), frag_fp8(xf[ms][0], xf[ms][1]));              \
    } else {                                                                                                 \
      uint4 wf[NSUB], xf[2];                                                                                 \
      _Pragma("unroll") for (int ns = 0; ns < NSUB; ++ns)                                                    \
        wf[ns] = *reinterpret_cast<const uint4*>(&ws[buf_][(wn * (BN / 2) + ns * 32 + l32) * PITCH + koff]); \
      _Pragma("unroll") for (int ms = 0; ms < 2; ++ms)                                                       \
        xf[ms] = *reinterpret_cast<const uint4*>(&xs[buf_][(wm * 64 + ms * 32 + l32) * PITCH + koff]);       \
      _Pragma("unroll") for (int g = 0; g < G; ++g)                                                          \
        _Pragma("unroll") for (int ns = 0; ns < NSUB; ++ns)                                                  \
          _Pragma("unroll") for (int ms = 0; ms < 2; ++ms)                                                   \
            Op::mma(acc[ns][ms], frag_of<Op>(wf[ns], g), frag_of<Op>(xf[ms], g));                            \
    }                                                                                                        \
  }

  // stage k sits in LDS buffer k % 2 and, before that, in register set k % 2
  // (prefetches past the last stage re-read the last stage; those copies
  // are never stored)
  REVO_GEMM_LOAD(0, xr0, wr0);
  REVO_GEMM_LOAD(KT > 1 ? 1 : 0, xr1, wr1);
  REVO_GEMM_STORE(0, xr0, wr0);
  __syncthreads();
  // (the scheduling barriers keep each prefetch ahead of the multiplies
  // it is meant to overlap)
  for (int kt = 0; kt < KT; kt += 2) {
    REVO_GEMM_LOAD(kt + 2 < KT ? kt + 2 : KT - 1, xr0, wr0);
    __builtin_amdgcn_sched_barrier(0);
    REVO_GEMM_COMPUTE(0)
    if (kt + 1 >= KT) break;
    REVO_GEMM_STORE(1, xr1, wr1);
    __syncthreads();
    REVO_GEMM_LOAD(kt + 3 < KT ? kt + 3 : KT - 1, xr1, wr1);
    __builtin_amdgcn_sched_barrier(0);
    REVO_GEMM_COMPUTE(1)
    if (kt + 2 >= KT) break;
    REVO_GEMM_STORE(0, xr0, wr0);
    __syncthreads();
  }
#undef REVO_GEMM_LOAD
#undef REVO_GEMM_STORE
#undef REVO_GEMM_COMPUTE

  if constexpr (KS == 2) {
    // the second k group's accumulators into the first's, lane by lane
    // (identical fragment layouts), through the operand stages' LDS
    static_assert(4 * NSUB * 2 * 16 * 64 * 4 <= (OPB > EPB ? OPB : EPB), "reduction fits the stages");
    float* red = reinterpret_cast<float*>(smem);
    __syncthreads();  // every wave is done with the operand stages
    if (kgrp == 1) {
#pragma unroll
      for (int ns = 0; ns < NSUB; ++ns)
#pragma unroll
        for (int ms = 0; ms < 2; ++ms)
#pragma unroll
          for (int j = 0; j < 16; ++j) red[(((wq * NSUB + ns) * 2 + ms) * 16 + j) * 64 + lane] = acc[ns][ms][j];
    }
    __syncthreads();
    if (kgrp == 0) {
#pragma unroll
      for (int ns = 0; ns < NSUB; ++ns)
#pragma unroll
        for (int ms = 0; ms < 2; ++ms)
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[ns][ms][j] += red[(((wq * NSUB + ns) * 2 + ms) * 16 + j) * 64 + lane];
    }
  }
  const bool act = kgrp == 0;
  // bias (and scale) vectors fetched together after the K loop: this
  // kernel has no registers to hold them through it
  EpiCols<BN> cols;
  epi_load_cols<Op, BN>(a, n0, wn, half, cols);
  if constexpr (EPI == EPI_HEAD) {
    gemm_epilogue<Op, BN, EPI, OutT>(a, acc, m0, n0, Mlive, nreq, lane, wave, cols);
  } else {
    gemm_epilogue_staged<Op, BN, EPI, OutT>(a, acc, m0, n0, Mlive, nreq, tid, smem, cols, act);
  }
}


// ---------------------------------------------------------------------------
// Dense BF16 and FP8 form: operand stages go from HBM straight into LDS
// (buffer loads with the LDS as destination) in a ring of NS stages, so no
// registers hold stages in flight and no LDS stores are issued.  A stage row
// is 128 bytes of K (64 BF16 or 128 E4M3 values), unpadded; 16-byte chunk c
// of row r sits at byte gswz(r, c), slot c ^ ((r >> 1) & 7), which spreads the
// 32 rows one fragment read touches over all banks.
__device__ __forceinline__ int gswz(int r, int c) { return r * 128 + ((c ^ ((r >> 1) & 7)) << 4); }

// One 16-byte-per-lane buffer load into LDS: lane L's bytes land at lds + 16 L
// (lds is wave-uniform).  Kept out of line of the kernel template's body: the
// host pass drops a kernel template's launch stub when the builtin sits there.
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, const void* lds, int vo, int so) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)lds, 16, vo, so, 0, 0);
}

// s_waitcnt vmcnt(N_): at most N_ of this wave's vector loads still in flight.
template <int N_>
__device__ __forceinline__ void wait_vm() {
  static_assert(N_ >= 0 && N_ < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N_ & 15) | ((N_ >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// One 128-byte K stage from LDS into the accumulators: all 16 fragment
// reads, then the products.  BF16: four 32x32x16 steps, lane half h taking
// chunk 4h + s of step s.  FP8: two 32x32x64 steps, lane half h taking chunks
// 4s + 2h and 4s + 2h + 1 (32 consecutive k, the layout of the register-staged
// kernel).  The operand pointers are restrict-qualified, so the reads carry
// alias scopes and the compiler does not hold them behind the ring's loads
// still in flight (the kernel orders those with vmcnt waits and barriers).
template <class Op, int BN>
__device__ __forceinline__ void gemm_dma_stage(const uint8_t* __restrict__ xb, const uint8_t* __restrict__ wb,
                                               f32x16 (&acc)[BN / 64][2], int wn, int wm, int half, int l32) {
  constexpr int NSUB = BN / 64;
  uint4 wf[4][NSUB], xf[4][2];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    // chunk read at s: BF16 step s; FP8 step s / 2, part s % 2
    const int ch = sizeof(typename Op::T) == 2 ? half * 4 + s : (s >> 1) * 4 + half * 2 + (s & 1);
#pragma unroll
    for (int ns = 0; ns < NSUB; ++ns)
      wf[s][ns] = *reinterpret_cast<const uint4*>(wb + gswz(wn * (BN / 2) + ns * 32 + l32, ch));
#pragma unroll
    for (int ms = 0; ms < 2; ++ms)
      xf[s][ms] = *reinterpret_cast<const uint4*>(xb + gswz(wm * 64 + ms * 32 + l32, ch));
  }
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (sizeof(typename Op::T) == 2) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int ns = 0; ns < NSUB; ++ns)
#pragma unroll
        for (int ms = 0; ms < 2; ++ms)
          Op::mma(acc[ns][ms], __builtin_bit_cast(bf16x8, wf[s][ns]), __builtin_bit_cast(bf16x8, xf[s][ms]));
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int ns = 0; ns < NSUB; ++ns)
#pragma unroll
        for (int ms = 0; ms < 2; ++ms)
          Op::mma(acc[ns][ms], frag_fp8(wf[2 * s][ns], wf[2 * s + 1][ns]), frag_fp8(xf[2 * s][ms], xf[2 * s + 1][ms]));
  }
}

// Tile BM_ tokens x BN features, 2 WM_ waves (each 64 x BN/2), NS stages of
// 128 bytes of K.
template <class Op, int BN, int EPI, class OutT, int NS, int BM_, int WM_>
__global__ __launch_bounds__(128 * WM_, 512 / (128 * WM_)) void gemm_dma_kernel(const GemmArgs a) {
  typedef typename Op::T T;
  constexpr int BK = 128 / (int)sizeof(T);  // K per stage
  constexpr int E = 16 / (int)sizeof(T);    // K per 16-byte chunk
  constexpr int NW = 2 * WM_;                         // waves
  constexpr int XR = BM_ / NW, WR = BN / NW;          // stage rows each wave loads
  constexpr int XI = XR / 8, WI = WR / 8;             // 8-row loads per wave per stage
  static_assert(XI >= 1 && WI >= 1 && BM_ == 64 * WM_, "tile geometry");
  constexpr int SX = BM_ * 128, SW = BN * 128;        // bytes per X / W stage
  constexpr int OPB = NS * (SX + SW);
  constexpr int EPB = epi_stage_bytes<BN, OutT, BM_>();
  // X stages at stg + b SX, W stages at stg + NS SX + b SW; the epilogue
  // reuses the whole array
  __shared__ __attribute__((aligned(16))) uint8_t stg[OPB > EPB ? OPB : EPB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  // XCD-aware tile order, as in gemm_kernel
  const int gn = a.N / BN;
  const int ntiles = gridDim.x;
  const int L = blockIdx.x;
  const int xcd = L & 7, per = ntiles >> 3, rem = ntiles & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (L >> 3);
  const int m0 = (tile / gn) * BM_;
  const int n0 = (tile - (tile / gn) * gn) * BN;
  const int Mlive = a.dyn_m ? *a.dyn_m : a.M;
  const int nreq = a.dyn_nreq ? *a.dyn_nreq : a.nreq;
  if (m0 >= Mlive) return;
  const int KT = a.K / BK;

  // rows at or past Mlive are outside the descriptor's range: they read as
  // zeros and only ever reach outputs that are not stored
  const __amdgpu_buffer_rsrc_t wrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.W, (short)0, a.N * a.K * (int)sizeof(T), 0x00020000);
  const __amdgpu_buffer_rsrc_t xrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.X, (short)0, Mlive * a.K * (int)sizeof(T), 0x00020000);
  // wave w fills rows w XR .. (w+1) XR - 1 of the X stage (likewise for W),
  // 8 rows per load; lane L fills slot L % 8 of row L / 8 of its group
  int xo[XI], wo[WI];
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int rr = wave * XR + 8 * j + (lane >> 3);
    xo[j] = ((m0 + rr) * a.K + ((lane & 7) ^ ((rr >> 1) & 7)) * E) * (int)sizeof(T);
  }
#pragma unroll
  for (int j = 0; j < WI; ++j) {
    const int rr = wave * WR + 8 * j + (lane >> 3);
    wo[j] = ((n0 + rr) * a.K + ((lane & 7) ^ ((rr >> 1) & 7)) * E) * (int)sizeof(T);
  }
#define REVO_GD_FETCH(kt_, buf_)                                                                         \
  do {                                                                                                   \
    _Pragma("unroll") for (int j = 0; j < XI; ++j)                                                       \
      dma16(xrs, stg + (buf_) * SX + (wave * XR + 8 * j) * 128, xo[j], (kt_) * 128);                      \
    _Pragma("unroll") for (int j = 0; j < WI; ++j)                                                       \
      dma16(wrs, stg + NS * SX + (buf_) * SW + (wave * WR + 8 * j) * 128, wo[j], (kt_) * 128);            \
  } while (0)

  const int wn = wave / WM_, wm = wave % WM_;
  f32x16 acc[BN / 64][2];
#pragma unroll
  for (int i = 0; i < BN / 64; ++i) { acc[i][0] = f32x16{}; acc[i][1] = f32x16{}; }
  EpiCols<BN> cols;  // in flight during the K loop
  epi_load_cols<Op, BN>(a, n0, wn, half, cols);

  // stage k goes to buffer k % NS; loads past the last stage re-read it
  // into a free buffer, which keeps the wait counts static
#pragma unroll
  for (int i = 0; i < NS - 1; ++i) REVO_GD_FETCH(i < KT ? i : KT - 1, i);
  // the ring is unrolled NS times so that every buffer index is a constant
  for (int kt = 0; kt < KT;) {
#pragma unroll
    for (int b = 0; b < NS; ++b) {
      wait_vm<(NS - 2) * (XI + WI)>();  // this wave's part of stage kt is in LDS
      // every wave's part is, and stage kt-1's buffer is free (a plain
      // barrier: the fence of __syncthreads would also wait for the younger
      // stage loads)
      asm volatile("s_barrier" ::: "memory");
      REVO_GD_FETCH(kt + NS - 1 < KT ? kt + NS - 1 : KT - 1, (b + NS - 1) % NS);
      gemm_dma_stage<Op, BN>(stg + b * SX, stg + NS * SX + b * SW, acc, wn, wm, half, l32);
      if (++kt >= KT) break;
    }
  }
  wait_vm<0>();  // no load still writes LDS when the epilogue reuses it
#undef REVO_GD_FETCH
  gemm_epilogue_staged<Op, BN, EPI, OutT, BM_, WM_>(a, acc, m0, n0, Mlive, nreq, tid, stg, cols);
}

template <class Op, int EPI, int XM, class OutT>
int launch_t(const GemmArgs& a, hipStream_t s) {
  const int gm = cdiv(a.M, BM);
  // buffer-load byte offsets are 32-bit: both operands, with X padded to
  // whole row tiles, stay below 2 GiB
  const long long esz = sizeof(typename Op::T);
  if ((long long)gm * BM * a.K * esz >= (1LL << 31) || (long long)a.N * a.K * esz >= (1LL << 31)) return -22;
  // Dense BF16 products (all but the head) and FP8 products whose K is a
  // multiple of 128 take the LDS-ring kernel, two stages: 128 x 128 tiles over
  // 4 waves, or, for 64-wide feature tiles, 256 x 64 tiles over 8 waves
  // (measured faster on the decoder's products)
  constexpr bool RING = XM == X_DENSE && EPI != EPI_HEAD && sizeof(typename Op::T) <= 2;
  if constexpr (RING) {
    if (sizeof(typename Op::T) == 2 || a.K % 128 == 0) {
      if (a.N % 128 == 0) {
        gemm_dma_kernel<Op, 128, EPI, OutT, 2, 128, 2><<<dim3(gm * (a.N / 128)), 256, 0, s>>>(a);
        return hipGetLastError() == hipSuccess ? 0 : -5;
      }
      const int gm2 = cdiv(a.M, 256);
      if ((long long)gm2 * 256 * a.K * esz >= (1LL << 31)) return -22;
      gemm_dma_kernel<Op, 64, EPI, OutT, 2, 256, 4><<<dim3(gm2 * (a.N / 64)), 512, 0, s>>>(a);
      return hipGetLastError() == hipSuccess ? 0 : -5;
    }
  }
  if constexpr (RING && sizeof(typename Op::T) == 2) {
    return -22;  // not reached: every BF16 dense product takes the ring
  } else {
    // the gather loader's per-row token coordinates leave no registers for a
    // 128-wide tile with two prefetched stages.  Dense products take 128-wide
    // tiles unless 64-wide ones (twice as many, half the work each) spread
    // better over the 256 CUs: the busiest CU then holds fewer feature columns
    if constexpr (XM == X_DENSE && sizeof(typename Op::T) == 4 && EPI != EPI_HEAD) {
      // FP32 products of at most one 64-wide workgroup per CU: eight waves
      // that split each stage's k steps, two per SIMD instead of one
      if ((long long)gm * (a.N / 64) <= 256) {
        gemm_kernel<Op, 64, EPI, XM, OutT, 2><<<gm * (a.N / 64), 2 * NT, 0, s>>>(a);
        return hipGetLastError() == hipSuccess ? 0 : -5;
      }
    }
    if constexpr (XM == X_DENSE) {
      const long long t128 = (long long)gm * (a.N / 128);
      const bool wide = a.N % 128 == 0 && (2 * t128 + 255) / 256 >= 2 * ((t128 + 255) / 256);
      if (wide) {
        gemm_kernel<Op, 128, EPI, XM, OutT><<<gm * (a.N / 128), NT, 0, s>>>(a);
        return hipGetLastError() == hipSuccess ? 0 : -5;
      }
    }
    gemm_kernel<Op, 64, EPI, XM, OutT><<<gm * (a.N / 64), NT, 0, s>>>(a);
    return hipGetLastError() == hipSuccess ? 0 : -5;
  }
}

template <class Op>
int launch_op(int epi, int xmode, const GemmArgs& a, hipStream_t s) {
  typedef typename Op::T T;
  if (xmode == X_GATHER) {
    if (epi != EPI_PE) return -22;
    return launch_t<Op, EPI_PE, X_GATHER, float>(a, s);
  }
  switch (epi) {
    case EPI_STORE: return launch_t<Op, EPI_STORE, X_DENSE, T>(a, s);
    case EPI_RESIDUAL: return launch_t<Op, EPI_RESIDUAL, X_DENSE, float>(a, s);
    case EPI_GELU: return launch_t<Op, EPI_GELU, X_DENSE, T>(a, s);
    case EPI_QKV: return launch_t<Op, EPI_QKV, X_DENSE, T>(a, s);
    case EPI_PE: return launch_t<Op, EPI_PE, X_DENSE, float>(a, s);
    case EPI_HEAD: return launch_t<Op, EPI_HEAD, X_DENSE, float>(a, s);
    case EPI_GELU_PRE:
    case EPI_GELU_BWD:
      if constexpr (sizeof(T) == 4) {
        if (epi == EPI_GELU_PRE) return launch_t<Op, EPI_GELU_PRE, X_DENSE, float>(a, s);
        return launch_t<Op, EPI_GELU_BWD, X_DENSE, float>(a, s);
      }
      return -22;
  }
  return -22;
}

// FP8 operands: Q/K/V and plain stores come out in BF16 (attention runs in
// BF16), GELU results in FP8 for the next product, residuals and PE in FP32.
int launch_fp8(int epi, const GemmArgs& a, hipStream_t s) {
  switch (epi) {
    case EPI_STORE: return launch_t<OpFP8, EPI_STORE, X_DENSE, __bf16>(a, s);
    case EPI_RESIDUAL: return launch_t<OpFP8, EPI_RESIDUAL, X_DENSE, float>(a, s);
    case EPI_GELU: return launch_t<OpFP8, EPI_GELU, X_DENSE, uint8_t>(a, s);
    case EPI_QKV:
      // E4M3 Q / K / V^T for the FP8 attention, BF16 for the BF16 one
      if (a.head_inv) return launch_t<OpFP8, EPI_QKV, X_DENSE, uint8_t>(a, s);
      return launch_t<OpFP8, EPI_QKV, X_DENSE, __bf16>(a, s);
    case EPI_PE: return launch_t<OpFP8, EPI_PE, X_DENSE, float>(a, s);
  }
  return -22;
}

}  // namespace

int launch_tubelet_pack(Prec prec, const GemmArgs& a, void* out, hipStream_t s) {
  if (a.M <= 0) return 0;
  const int E = prec == P_FP32 ? 4 : 8;
  if (a.K % E || !out) return -22;
  const long long chunks = (long long)a.M * (a.K / E);
  const int grid = (int)(chunks / 256 + 1 < 65536 ? chunks / 256 + 1 : 65536);
  if (prec == P_FP32)
    tubelet_pack_kernel<OpF32><<<grid, 256, 0, s>>>(a.reqs, a.nreq, a.dyn_nreq, a.M, a.dyn_m, a.K, a.channels,
                                                    (float*)out);
  else
    tubelet_pack_kernel<OpBF16><<<grid, 256, 0, s>>>(a.reqs, a.nreq, a.dyn_nreq, a.M, a.dyn_m, a.K, a.channels,
                                                     (__bf16*)out);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_gemm(Prec prec, int epi, int xmode, const GemmArgs& a, hipStream_t s) {
  if (a.M <= 0) return 0;
  if (a.N % 64 != 0) return -22;
  // the epilogue reads bias and row scales as 16-byte vectors
  if (((uintptr_t)a.bias | (uintptr_t)a.wscale) & 15) return -22;
  // the head's unpatchify knows RGB and depth pixels
  if (epi == EPI_HEAD && a.channels != 3 && a.channels != 1) return -22;
  // the FP32 GELU epilogues move pre-activations as 16-byte vectors
  if (epi == EPI_GELU_PRE || epi == EPI_GELU_BWD) {
    if (prec != P_FP32 || xmode != X_DENSE || !a.pre || ((uintptr_t)a.pre & 15) || a.ldo % 4) return -22;
  }
  if (epi == EPI_RESIDUAL && a.res && (((uintptr_t)a.res & 15) || a.ldo % 4)) return -22;
  if (prec == P_BF16) {
    if (a.K % OpBF16::BK != 0) return -22;
    return launch_op<OpBF16>(epi, xmode, a, s);
  }
  if (prec == P_FP32) {
    if (a.K % OpF32::BK != 0) return -22;
    return launch_op<OpF32>(epi, xmode, a, s);
  }
  if (prec == P_FP8) {
    if (a.K % OpFP8::BK != 0 || xmode != X_DENSE || !a.wscale || !a.xscale) return -22;
    if (epi == EPI_GELU && !a.out_scale) return -22;
    return launch_fp8(epi, a, s);
  }
  return -95;
}

}  // namespace revo
