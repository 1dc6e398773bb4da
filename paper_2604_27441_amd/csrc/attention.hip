// Joint space-time flash attention over the tokens of one request
// (softmax(Q K^T / sqrt(64)) V per head, with an online softmax over key
// blocks), the dominant step of the recovery network.
//
// Each wave owns 32 queries.  Scores are computed transposed, S^T = K Q^T,
// so that the 32x32 MFMA accumulator puts one query per lane (lanes l and
// l+32 hold disjoint halves of the keys): the running max, the rescale of
// the output and the row sum stay lane-local, with one cross-half exchange
// per key block.  The output is also accumulated transposed, O^T = V^T P^T,
// so the probabilities feed the MFMA straight from the score registers; V
// is stored transposed ([head][dim][token]) by the QKV epilogue for that.
// Q arrives pre-scaled by log2(e)/8, so probabilities are exp2(s - m).
// K and V^T blocks of 64 keys are double-buffered in LDS.
#include "kernels.h"

namespace revo {

namespace {

constexpr int NT = 256;
constexpr int QT = 128;   // queries per workgroup (4 waves x 32)
constexpr int KB = 64;    // keys per block
constexpr float NEG_BIG = -1.0e30f;

template <class Op>
__global__ __launch_bounds__(NT, 2) void attn_kernel(const AttnArgs a) {
  typedef typename Op::T T;
  constexpr int E = 16 / sizeof(T);          // elements per 16-byte chunk
  constexpr int PITCH = 64 + E;              // padded row pitch in elements
  constexpr int CPR = 64 / E;                // 16-byte chunks per 64-element row
  constexpr int LC = KB * CPR / NT;          // chunks per thread per tile
  __shared__ __attribute__((aligned(16))) T ks[2][KB * PITCH];   // [key][dim]
  __shared__ __attribute__((aligned(16))) T vs[2][64 * PITCH];   // [dim][key]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int w = a.work[blockIdx.x];
  const int r = w >> 16, qt = w & 0xFFFF;
  const int hd = blockIdx.y;
  const ReqDesc& d = a.reqs[r];
  const int N = d.J * d.P;
  const int base = d.tok_off;
  const int q_local = qt * QT + wave * 32 + l32;
  const int q = base + q_local;

  const T* __restrict__ Kg = (const T*)a.k + ((size_t)hd * a.ldqk + base) * 64;
  const T* __restrict__ Vg = (const T*)a.vt + (size_t)hd * 64 * a.ldv + base;

  // Q^T fragment: this lane's query, dims [half*32, half*32 + 32)
  constexpr int QCH = 32 / E;
  uint4 qf[QCH];
  {
    // queries past the request (ragged last tile) load row `base`; never stored
    const T* qp = (const T*)a.q + ((size_t)hd * a.ldqk + (q_local < N ? q : base)) * 64 + half * 32;
#pragma unroll
    for (int i = 0; i < QCH; ++i) qf[i] = reinterpret_cast<const uint4*>(qp)[i];
  }

  uint4 kr[LC], vr[LC];
  auto load_block = [&](int kb) {
#pragma unroll
    for (int i = 0; i < LC; ++i) {
      const int c = tid + i * NT, row = c / CPR, cc = c % CPR;
      kr[i] = *reinterpret_cast<const uint4*>(Kg + (size_t)(kb + row) * 64 + cc * E);
      vr[i] = *reinterpret_cast<const uint4*>(Vg + (size_t)row * a.ldv + kb + cc * E);
    }
  };
  auto store_block = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LC; ++i) {
      const int c = tid + i * NT, row = c / CPR, cc = c % CPR;
      *reinterpret_cast<uint4*>(&ks[buf][row * PITCH + cc * E]) = kr[i];
      *reinterpret_cast<uint4*>(&vs[buf][row * PITCH + cc * E]) = vr[i];
    }
  };

  f32x16 oacc[2] = {f32x16{}, f32x16{}};
  float m_run = NEG_BIG, l_run = 0.0f;
  const int nkb = (N + KB - 1) / KB;

  load_block(0);
  store_block(0);
  __syncthreads();
  for (int b = 0; b < nkb; ++b) {
    const int buf = b & 1;
    const int kb = b * KB;
    if (b + 1 < nkb) load_block(kb + KB);

    // S^T = K Q^T for two 32-key subtiles
    f32x16 sacc[2] = {f32x16{}, f32x16{}};
#pragma unroll
    for (int kc = 0; kc < QCH; ++kc) {          // one 16-byte chunk of dims per lane
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        const uint4 kf = *reinterpret_cast<const uint4*>(&ks[buf][(st * 32 + l32) * PITCH + half * 32 + kc * E]);
        if constexpr (sizeof(T) == 2) {
          Op::mma(sacc[st], __builtin_bit_cast(bf16x8, kf), __builtin_bit_cast(bf16x8, qf[kc]));
        } else {
          Op::mma(sacc[st], __uint_as_float(kf.x), __uint_as_float(qf[kc].x));
          Op::mma(sacc[st], __uint_as_float(kf.y), __uint_as_float(qf[kc].y));
          Op::mma(sacc[st], __uint_as_float(kf.z), __uint_as_float(qf[kc].z));
          Op::mma(sacc[st], __uint_as_float(kf.w), __uint_as_float(qf[kc].w));
        }
      }
    }

    // online softmax (lane-local per query, halves exchanged once)
    float mloc = NEG_BIG;
    const bool ragged = kb + KB > N;
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (ragged && kb + st * 32 + acc_row(i, lane) >= N) sacc[st][i] = NEG_BIG;
        mloc = fmaxf(mloc, sacc[st][i]);
      }
    mloc = fmaxf(mloc, __shfl_xor(mloc, 32));
    const float m_new = fmaxf(m_run, mloc);
    const float alpha = exp2f(m_run - m_new);
    m_run = m_new;
    float lsum = 0.0f;
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float p = exp2f(sacc[st][i] - m_new);
        sacc[st][i] = p;
        lsum += p;
      }
    l_run = l_run * alpha + lsum;
#pragma unroll
    for (int ds = 0; ds < 2; ++ds)
#pragma unroll
      for (int i = 0; i < 16; ++i) oacc[ds][i] *= alpha;

    // O^T += V^T P^T, contraction over the block's keys
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          // registers 8g..8g+7 hold keys st*32 + g*16 + {half*4 + 0..3, 8 + half*4 + 0..3}
          bf16x8 pf;
#pragma unroll
          for (int e = 0; e < 8; ++e) pf[e] = (__bf16)sacc[st][8 * g + e];
          const int key = st * 32 + g * 16 + half * 4;
#pragma unroll
          for (int ds = 0; ds < 2; ++ds) {
            const T* vrow = &vs[buf][(ds * 32 + l32) * PITCH];
            const uint2 lo = *reinterpret_cast<const uint2*>(vrow + key);
            const uint2 hi = *reinterpret_cast<const uint2*>(vrow + key + 8);
            const uint4 vv = make_uint4(lo.x, lo.y, hi.x, hi.y);
            Op::mma(oacc[ds], __builtin_bit_cast(bf16x8, vv), pf);
          }
        }
      } else {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          // registers 4g..4g+3 hold keys st*32 + g*8 + half*4 + 0..3
          const int key = st * 32 + g * 8 + half * 4;
#pragma unroll
          for (int ds = 0; ds < 2; ++ds) {
            const uint4 vv = *reinterpret_cast<const uint4*>(&vs[buf][(ds * 32 + l32) * PITCH + key]);
            Op::mma(oacc[ds], __uint_as_float(vv.x), sacc[st][4 * g + 0]);
            Op::mma(oacc[ds], __uint_as_float(vv.y), sacc[st][4 * g + 1]);
            Op::mma(oacc[ds], __uint_as_float(vv.z), sacc[st][4 * g + 2]);
            Op::mma(oacc[ds], __uint_as_float(vv.w), sacc[st][4 * g + 3]);
          }
        }
      }
    }
    if (b + 1 < nkb) store_block(buf ^ 1);
    __syncthreads();
  }

  const float l_tot = l_run + __shfl_xor(l_run, 32);
  if (q_local < N) {
    const float inv = 1.0f / l_tot;
    T* op = (T*)a.o + (size_t)q * (a.heads * 64) + hd * 64;
#pragma unroll
    for (int ds = 0; ds < 2; ++ds)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int dim = ds * 32 + g * 8 + half * 4;
        if constexpr (sizeof(T) == 2) {
          *reinterpret_cast<bf16x4*>(op + dim) =
              bf16x4{(__bf16)(oacc[ds][4 * g] * inv), (__bf16)(oacc[ds][4 * g + 1] * inv),
                     (__bf16)(oacc[ds][4 * g + 2] * inv), (__bf16)(oacc[ds][4 * g + 3] * inv)};
        } else {
          *reinterpret_cast<f32x4*>(op + dim) =
              f32x4{oacc[ds][4 * g] * inv, oacc[ds][4 * g + 1] * inv, oacc[ds][4 * g + 2] * inv,
                    oacc[ds][4 * g + 3] * inv};
        }
      }
  }
}

}  // namespace

int launch_attention(Prec prec, const AttnArgs& a, hipStream_t s) {
  if (a.nwork <= 0) return 0;
  dim3 grid(a.nwork, a.heads);
  if (prec == P_BF16) attn_kernel<OpBF16><<<grid, NT, 0, s>>>(a);
  else if (prec == P_FP32) attn_kernel<OpF32><<<grid, NT, 0, s>>>(a);
  else return -95;
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace revo
