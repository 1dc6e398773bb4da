// Joint space-time flash attention over the tokens of one request
// (softmax(Q K^T / sqrt(64)) V per head, with an online softmax over key
// blocks), the dominant step of the recovery network.
//
// Each wave owns 32 queries.  Scores are computed transposed, S^T = K Q^T,
// so that the 32x32 MFMA accumulator puts one query per lane (lanes l and
// l+32 hold disjoint halves of the keys): the running max, the row sum and
// the rescale of the output stay lane-local, with one cross-half exchange
// (v_permlane32_swap) per key block.  The output is also accumulated
// transposed, O^T = V^T P^T, so the probabilities feed the MFMA straight
// from the score registers; V is stored transposed ([head][dim][token]) by
// the QKV epilogue for that.  Q arrives pre-scaled by log2(e)/8, so
// probabilities are exp2(s - m).
//
// The final division by the row sum makes the result independent of the
// max subtracted before exp2, so any max that keeps the probabilities finite
// will do.  The first block sets it; after that (BF16) the score products
// accumulate onto a register block holding -max, so they come out already
// shifted and the softmax is a bare exp2 per score.  BF16 rows first run a
// pass that never changes that max and takes no block max at all; if some
// row sum of the workgroup reaches 2^64 (or is not finite) the workgroup
// repeats its rows in a pass that raises the max lazily: a query keeps its
// max until a block's scores exceed it by more than 8 (in log2 units), so
// probabilities stay below 2^8 and the output rescale is skipped for almost
// every block.  FP32 rows always use the lazy form.  Only the last key block
// of a request checks key bounds.
// K and V^T blocks of 64 keys are double-buffered in LDS.  BF16 blocks go
// from HBM straight into LDS (buffer loads with an LDS destination, no
// registers in between) with swizzled, unpadded rows; FP32 blocks pass
// through registers.  Loads take scalar per-block offsets, and the block
// loop runs two blocks per trip so both LDS buffers have fixed addresses.
#include <string.h>

#include <mutex>

#include "kernels.h"

namespace revo {

namespace {

constexpr int NT = 256;
constexpr int QT = 128;   // queries per workgroup (4 waves x 32)
constexpr int KB = 64;    // keys per block
constexpr float NEG_BIG = -1.0e30f;
constexpr float LAZY = 8.0f;

// One 16-byte-per-lane buffer load into LDS (lane L's bytes at lds + 16 L).
__device__ __forceinline__ void dma16_att(__amdgpu_buffer_rsrc_t rs, const void* lds, int vo, int so) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)lds, 16, vo, so, 0, 0);
}

// s_waitcnt vmcnt(N_): at most N_ of this wave's vector memory loads in flight.
template <int N_>
__device__ __forceinline__ void wait_vm_att() {
  static_assert(N_ >= 0 && N_ < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N_ & 15) | ((N_ >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// max / sum of a value and its partner lane (l ^ 32)
__device__ __forceinline__ float xhalf_max(float x) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float xhalf_sum(float x) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <class T>
struct AttnTile {
  static constexpr int E = 16 / sizeof(T);   // elements per 16-byte chunk
  // BF16 tiles arrive by DMA (whole 128-byte rows, unpadded, chunks
  // swizzled); FP32 rows are padded by one chunk
  static constexpr int PITCH = sizeof(T) == 2 ? 64 : 64 + E;  // LDS row pitch (elements)
  static constexpr int CPR = 64 / E;         // 16-byte chunks per 64-element row
  static constexpr int LC = KB * CPR / NT;   // chunks per thread per tile (FP32)
  static constexpr int QCH = 32 / E;         // Q chunks per lane
};

// BF16 K and V^T tiles: row r (a key of K, a dimension of V^T) holds its
// eight 16-byte chunks with chunk c at slot c ^ ((r >> 1) & 7), so the 16
// rows read by one 16-lane phase of a b128 read cover all 64 banks.
__device__ __forceinline__ int swz(int row, int chunk) { return row * 64 + ((chunk ^ ((row >> 1) & 7)) << 3); }

// One 64-key block for one wave: scores, online softmax, P V accumulation.
template <class Op, bool MASK, bool FIRST, bool FAST>
__device__ __forceinline__ void attn_block(const typename Op::T* __restrict__ kt, const typename Op::T* __restrict__ vt,
                                           const uint4 (&qf)[AttnTile<typename Op::T>::QCH], f32x16 (&oacc)[2],
                                           f32x16& negm, float& m_run, float& l_run, int lane, int kvalid) {
  typedef typename Op::T T;
  typedef AttnTile<T> A;
  const int half = lane >> 5, l32 = lane & 31;
  // BF16: after the first block the score products start from -m_run (all
  // 16 registers of negm), so they come out already shifted by the max
  constexpr bool SHIFTED = sizeof(T) == 2 && !FIRST;

  // S^T = K Q^T for two 32-key subtiles
  f32x16 sacc[2];
  if constexpr (SHIFTED) {
    sacc[0] = negm;
    sacc[1] = negm;
  } else {
    sacc[0] = f32x16{};
    sacc[1] = f32x16{};
  }
  if constexpr (sizeof(T) == 2) {
    // all eight K fragments in flight before the first product
    uint4 kf[A::QCH][2];
#pragma unroll
    for (int kc = 0; kc < A::QCH; ++kc)
#pragma unroll
      for (int st = 0; st < 2; ++st) kf[kc][st] = *reinterpret_cast<const uint4*>(kt + swz(st * 32 + l32, half * 4 + kc));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kc = 0; kc < A::QCH; ++kc)
#pragma unroll
      for (int st = 0; st < 2; ++st)
        Op::mma(sacc[st], __builtin_bit_cast(bf16x8, kf[kc][st]), __builtin_bit_cast(bf16x8, qf[kc]));
  }
#pragma unroll
  for (int kc = 0; kc < A::QCH; ++kc) {
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      if constexpr (sizeof(T) == 4) {
        const uint4 kf = *reinterpret_cast<const uint4*>(kt + (st * 32 + l32) * A::PITCH + half * 32 + kc * A::E);
        Op::mma(sacc[st], __uint_as_float(kf.x), __uint_as_float(qf[kc].x));
        Op::mma(sacc[st], __uint_as_float(kf.y), __uint_as_float(qf[kc].y));
        Op::mma(sacc[st], __uint_as_float(kf.z), __uint_as_float(qf[kc].z));
        Op::mma(sacc[st], __uint_as_float(kf.w), __uint_as_float(qf[kc].w));
      }
    }
  }
  if constexpr (MASK) {
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (st * 32 + acc_row(i, lane) >= kvalid) sacc[st][i] = NEG_BIG;
  }

  // FAST (BF16, after the first block): the max stays where the first block
  // put it and no block max is taken; the caller checks the row sums after
  // the last block instead
  if constexpr (!(SHIFTED && FAST)) {
    // block max of this query
    float m0 = fmaxf(fmaxf(sacc[0][0], sacc[0][1]), sacc[0][2]);
    float m1 = fmaxf(fmaxf(sacc[1][0], sacc[1][1]), sacc[1][2]);
#pragma unroll
    for (int i = 3; i < 15; i += 2) {
      m0 = fmaxf(fmaxf(m0, sacc[0][i]), sacc[0][i + 1]);
      m1 = fmaxf(fmaxf(m1, sacc[1][i]), sacc[1][i + 1]);
    }
    float mloc = fmaxf(fmaxf(m0, sacc[0][15]), fmaxf(m1, sacc[1][15]));
    mloc = xhalf_max(mloc);
    if constexpr (FIRST) {
      // nothing accumulated yet: take this block's max as it is
      m_run = mloc;
      if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int i = 0; i < 16; ++i) negm[i] = -mloc;
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
          for (int i = 0; i < 16; ++i) sacc[st][i] -= mloc;
      }
    } else if constexpr (SHIFTED) {
      // mloc is relative to m_run here
      const bool grow = mloc > LAZY;
      if (__any(grow)) {
        const float d = grow ? mloc : 0.0f;
        const float alpha = __builtin_amdgcn_exp2f(-d);
        m_run += d;
        l_run *= alpha;
        oacc[0] *= alpha;
        oacc[1] *= alpha;
#pragma unroll
        for (int i = 0; i < 16; ++i) negm[i] = -m_run;
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
          for (int i = 0; i < 16; ++i) sacc[st][i] -= d;
        // keep the rescale inside this (rarely taken) branch instead of letting
        // it become unconditional work with a selected factor
        asm volatile("" : "+v"(oacc[0]), "+v"(oacc[1]), "+v"(sacc[0]), "+v"(sacc[1]), "+v"(negm));
      }
    } else {
      const bool grow = mloc > m_run + LAZY;
      if (__any(grow)) {
        const float m_new = grow ? mloc : m_run;
        const float alpha = __builtin_amdgcn_exp2f(m_run - m_new);
        m_run = m_new;
        l_run *= alpha;
        oacc[0] *= alpha;
        oacc[1] *= alpha;
        asm volatile("" : "+v"(oacc[0]), "+v"(oacc[1]));
      }
    }
  }

  // O^T += V^T P^T, contraction over the block's keys
  if constexpr (sizeof(T) == 2) {
    // row sum from the bf16-rounded probabilities that also feed the MFMA
    const bf16x2 one = {(__bf16)1.0f, (__bf16)1.0f};
    float ls0 = l_run, ls1 = 0.0f;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        // registers 8g..8g+7 hold keys st*32 + g*16 + {half*4 + 0..3, 8 + half*4 + 0..3};
        // V^T rows hold keys with bits 2 and 3 swapped, so those keys are the
        // 8 contiguous elements at st*32 + g*16 + half*8
        bf16x8 pf;
#pragma unroll
        for (int e = 0; e < 8; ++e) pf[e] = (__bf16)__builtin_amdgcn_exp2f(sacc[st][8 * g + e]);
        ls0 = __builtin_amdgcn_fdot2_f32_bf16(bf16x2{pf[0], pf[1]}, one, ls0, false);
        ls1 = __builtin_amdgcn_fdot2_f32_bf16(bf16x2{pf[2], pf[3]}, one, ls1, false);
        ls0 = __builtin_amdgcn_fdot2_f32_bf16(bf16x2{pf[4], pf[5]}, one, ls0, false);
        ls1 = __builtin_amdgcn_fdot2_f32_bf16(bf16x2{pf[6], pf[7]}, one, ls1, false);
        const int pos = st * 32 + g * 16 + half * 8;
#pragma unroll
        for (int ds = 0; ds < 2; ++ds) {
          const uint4 vv = *reinterpret_cast<const uint4*>(vt + swz(ds * 32 + l32, pos >> 3));
          Op::mma(oacc[ds], __builtin_bit_cast(bf16x8, vv), pf);
        }
      }
    }
    l_run = ls0 + ls1;
  } else {
    float ls0 = 0.0f, ls1 = 0.0f;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        sacc[st][i] = __builtin_amdgcn_exp2f(sacc[st][i] - m_run);
        sacc[st][i + 1] = __builtin_amdgcn_exp2f(sacc[st][i + 1] - m_run);
        ls0 += sacc[st][i];
        ls1 += sacc[st][i + 1];
      }
    }
    l_run += ls0 + ls1;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        // registers 4g..4g+3 hold keys st*32 + g*8 + half*4 + 0..3
        const int key = st * 32 + g * 8 + half * 4;
#pragma unroll
        for (int ds = 0; ds < 2; ++ds) {
          const uint4 vv = *reinterpret_cast<const uint4*>(vt + (ds * 32 + l32) * A::PITCH + key);
          Op::mma(oacc[ds], __uint_as_float(vv.x), sacc[st][4 * g + 0]);
          Op::mma(oacc[ds], __uint_as_float(vv.y), sacc[st][4 * g + 1]);
          Op::mma(oacc[ds], __uint_as_float(vv.z), sacc[st][4 * g + 2]);
          Op::mma(oacc[ds], __uint_as_float(vv.w), sacc[st][4 * g + 3]);
        }
      }
    }
  }
}

template <class Op>
__global__ __launch_bounds__(NT, sizeof(typename Op::T) == 2 ? 3 : 2) void attn_kernel(const AttnArgs a) {
  typedef typename Op::T T;
  typedef AttnTile<T> A;
  // two K stages [key][dim], two V^T stages [dim][key], then a flag.  One
  // LDS object only: with a second one the compiler attaches alias scopes to
  // the stage loads and then waits for every prefetch before reading.
  __shared__ __attribute__((aligned(16))) T kv[4 * KB * A::PITCH + 16 / sizeof(T)];
  T(*ks)[KB * A::PITCH] = reinterpret_cast<T(*)[KB * A::PITCH]>(kv);
  T(*vs)[KB * A::PITCH] = ks + 2;
  int& redo = *reinterpret_cast<int*>(kv + 4 * KB * A::PITCH);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5;
  // Workgroups are dispatched round-robin over the 8 XCDs (each with its own
  // L2).  Remap so that XCD x runs a contiguous range of (head, q-tile) work:
  // the q-tiles of one request and head then share its K/V in one L2.
  const int nwork = a.dyn_nwork ? *a.dyn_nwork : a.nwork;
  const int G = nwork * a.heads;
  const int L = blockIdx.x;
  if (L >= G) return;  // grid sized for a capacity
  const int xcd = L & 7, per = G >> 3, rem = G & 7;
  const int Lr = xcd * per + (xcd < rem ? xcd : rem) + (L >> 3);
  const int hd = Lr / nwork;
  const int w = a.work[Lr - hd * nwork];
  const int r = w >> 16, qt = w & (ATTN_TARGET_TILE - 1);
  const ReqDesc& d = a.reqs[r];
  const int N = d.J * d.P;
  const int base = d.tok_off;
  // target-tubelet tiles (the last block, whose other queries feed nothing)
  const int q0 = (w & ATTN_TARGET_TILE) ? (d.J - 1) * d.P : 0;
  const int q_local = q0 + qt * QT + wave * 32 + (lane & 31);
  const int q = base + q_local;

  const T* __restrict__ Kg = (const T*)a.k + ((size_t)hd * a.ldqk + base) * 64;
  const T* __restrict__ Vg = (const T*)a.vt + (size_t)hd * 64 * a.ldv + base;

  // Q^T fragment: this lane's query, dims [half*32, half*32 + 32); queries
  // past the request (ragged last tile) load row `base` and are never stored
  uint4 qf[A::QCH];
  {
    const T* qp = (const T*)a.q + ((size_t)hd * a.ldqk + (q_local < N ? q : base)) * 64 + half * 32;
#pragma unroll
    for (int i = 0; i < A::QCH; ++i) qf[i] = reinterpret_cast<const uint4*>(qp)[i];
  }

  const __amdgpu_buffer_rsrc_t krs =
      __builtin_amdgcn_make_buffer_rsrc((void*)Kg, (short)0, (a.ldqk - base) * 64 * (int)sizeof(T), 0x00020000);
  const __amdgpu_buffer_rsrc_t vrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)Vg, (short)0, (64 * a.ldv - base) * (int)sizeof(T), 0x00020000);
  // Stage loads for key block kb_ into LDS buffer buf_: FETCH starts them,
  // LAND completes them (the caller then synchronises the workgroup).
  //  BF16: buffer loads straight into LDS.  Wave w fills rows 16w .. 16w+15
  //  of the K and V^T tiles, 8 rows (1 KB, 16 bytes per lane) per load; lane
  //  L takes row 16w + 8j + L / 8 and the chunk whose swizzled slot is L % 8.
  //  V^T arrives with bits 2 and 3 of the key index already swapped within
  //  each group of 16 keys (the QKV epilogue writes it so; requests start on
  //  16-key boundaries), so a lane's eight probabilities meet one 16-byte read.
  //  FP32: 16-byte loads into registers, then LDS stores.
  constexpr int R = NT / A::CPR;
  const int c_row = tid / A::CPR;
  const int c_col = (tid % A::CPR) * A::E;
  int kvo[2], vvo[2];
  if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int rr = wave * 16 + 8 * j + (lane >> 3);
      const int cc = (lane & 7) ^ ((rr >> 1) & 7);
      kvo[j] = (rr * 64 + cc * 8) * (int)sizeof(T);
      vvo[j] = (rr * a.ldv + cc * 8) * (int)sizeof(T);
    }
  } else {
    kvo[0] = (c_row * 64 + c_col) * (int)sizeof(T);
    vvo[0] = (c_row * a.ldv + c_col) * (int)sizeof(T);
  }
  uint4 kr0, kr1, kr2, kr3, vr0, vr1, vr2, vr3;
#define REVO_ATTN_LOAD1(kb_, i_, kr_, vr_)                                                                       \
  {                                                                                                              \
    auto k_ = __builtin_amdgcn_raw_buffer_load_b128(krs, kvo[0], ((kb_) + (i_) * R) * 64 * (int)sizeof(T), 0);  \
    auto v_ = __builtin_amdgcn_raw_buffer_load_b128(vrs, vvo[0], ((i_) * R * a.ldv + (kb_)) * (int)sizeof(T), 0); \
    kr_ = make_uint4(k_[0], k_[1], k_[2], k_[3]);                                                                \
    vr_ = make_uint4(v_[0], v_[1], v_[2], v_[3]);                                                                \
  }
#define REVO_ATTN_STORE1(buf_, i_, kr_, vr_)                                                          \
  {                                                                                                   \
    *reinterpret_cast<uint4*>(&ks[buf_][(c_row + (i_) * R) * A::PITCH + c_col]) = kr_;                \
    *reinterpret_cast<uint4*>(&vs[buf_][(c_row + (i_) * R) * A::PITCH + c_col]) = vr_;                \
  }
#define REVO_ATTN_DMA(rs_, lds_, vo_, so_)                                                            \
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_, (__attribute__((address_space(3))) void*)(lds_), 16, \
                                           vo_, so_, 0, 0)
#define REVO_ATTN_FETCH(kb_, buf_)                                                                    \
  if constexpr (sizeof(T) == 2) {                                                                     \
    REVO_ATTN_DMA(krs, &ks[buf_][(wave * 16) * 64], kvo[0], (kb_) * 64 * (int)sizeof(T));             \
    REVO_ATTN_DMA(krs, &ks[buf_][(wave * 16 + 8) * 64], kvo[1], (kb_) * 64 * (int)sizeof(T));         \
    REVO_ATTN_DMA(vrs, &vs[buf_][(wave * 16) * 64], vvo[0], (kb_) * (int)sizeof(T));                  \
    REVO_ATTN_DMA(vrs, &vs[buf_][(wave * 16 + 8) * 64], vvo[1], (kb_) * (int)sizeof(T));              \
  } else {                                                                                            \
    REVO_ATTN_LOAD1(kb_, 0, kr0, vr0)                                                                 \
    REVO_ATTN_LOAD1(kb_, 1, kr1, vr1)                                                                 \
    REVO_ATTN_LOAD1(kb_, 2, kr2, vr2)                                                                 \
    REVO_ATTN_LOAD1(kb_, 3, kr3, vr3)                                                                 \
  }
#define REVO_ATTN_LAND(buf_)                                                                          \
  if constexpr (sizeof(T) == 2) {                                                                     \
    __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0): this wave's loads are in LDS */                  \
  } else {                                                                                            \
    REVO_ATTN_STORE1(buf_, 0, kr0, vr0)                                                               \
    REVO_ATTN_STORE1(buf_, 1, kr1, vr1)                                                               \
    REVO_ATTN_STORE1(buf_, 2, kr2, vr2)                                                               \
    REVO_ATTN_STORE1(buf_, 3, kr3, vr3)                                                               \
  }
  static_assert(sizeof(T) == 2 || A::LC == 4, "FP32: 4 chunks per thread");

  f32x16 oacc[2];
  f32x16 negm;
  float m_run, l_run;
  const int nkb = (N + KB - 1) / KB;
  const int nfull = N / KB;
  // One pass over the key blocks.  FAST passes (BF16) keep the first block's
  // max for the whole row (see attn_block); SAFE passes update it lazily.
  // Written out in the kernel body (not a called function) so that the
  // compiler keeps seeing the two LDS stages as distinct and does not wait
  // for the prefetch before reading the current stage.
#define REVO_ATTN_STEP(b_, buf_, fast_)                                                               \
  {                                                                                                   \
    const int kn_ = (b_) + 1 < nkb ? ((b_) + 1) * KB : (b_) * KB;                                     \
    REVO_ATTN_FETCH(kn_, buf_ ^ 1);                                                                   \
    attn_block<Op, false, false, fast_>(ks[buf_], vs[buf_], qf, oacc, negm, m_run, l_run, lane, KB);  \
    REVO_ATTN_LAND(buf_ ^ 1);                                                                         \
    __syncthreads();                                                                                  \
  }
#define REVO_ATTN_PASS(fast_)                                                                             \
  {                                                                                                       \
    oacc[0] = f32x16{};                                                                                   \
    oacc[1] = f32x16{};                                                                                   \
    m_run = 0.0f;                                                                                         \
    l_run = 0.0f;                                                                                         \
    REVO_ATTN_FETCH(0, 0);                                                                                \
    REVO_ATTN_LAND(0);                                                                                    \
    __syncthreads();                                                                                      \
    if (nfull == 0) {                                                                                     \
      /* a single, ragged block */                                                                        \
      attn_block<Op, true, true, fast_>(ks[0], vs[0], qf, oacc, negm, m_run, l_run, lane, N);             \
    } else {                                                                                              \
      /* the first block sets the max; the prefetch of the next block (or, at the end, a re-read of its   \
         own block into the idle buffer, which is then never read) overlaps it */                         \
      REVO_ATTN_FETCH(nkb > 1 ? KB : 0, 1);                                                               \
      attn_block<Op, false, true, fast_>(ks[0], vs[0], qf, oacc, negm, m_run, l_run, lane, KB);           \
      REVO_ATTN_LAND(1);                                                                                  \
      __syncthreads();                                                                                    \
      int b = 1;                                                                                          \
      for (; b + 1 < nfull; b += 2) {                                                                     \
        REVO_ATTN_STEP(b, 1, fast_)                                                                       \
        REVO_ATTN_STEP(b + 1, 0, fast_)                                                                   \
      }                                                                                                   \
      if (b < nfull) REVO_ATTN_STEP(b, 1, fast_)                                                          \
      if (nfull < nkb) /* ragged last block, already in LDS */                                            \
        attn_block<Op, true, false, fast_>(ks[nfull & 1], vs[nfull & 1], qf, oacc, negm, m_run, l_run, lane, \
                                           N - nfull * KB);                                               \
    }                                                                                                     \
  }
  if constexpr (sizeof(T) == 2) {
    // A FAST pass is exact as long as no probability overflowed: every
    // probability of a lane's keys is at most that lane's row sum, so row sums
    // below 2^64 bound them all (and the output by 2^64 max|v|).  Otherwise
    // (or on NaN) the whole workgroup repeats the row in a SAFE pass.
    if (tid == 0) redo = 0;  // ordered before any write by the pass's first barrier
    REVO_ATTN_PASS(true)
    if (__any(!(l_run < 0x1p64f)) && lane == 0) redo = 1;
    __syncthreads();
    if (redo) REVO_ATTN_PASS(false)  // every wave is past its last block
  } else {
    REVO_ATTN_PASS(false)
  }
#undef REVO_ATTN_PASS
#undef REVO_ATTN_STEP
#undef REVO_ATTN_LOAD1
#undef REVO_ATTN_STORE1
#undef REVO_ATTN_DMA
#undef REVO_ATTN_FETCH
#undef REVO_ATTN_LAND

  // The output goes through LDS (the K stages are free once every wave is
  // past its last block) so that whole 64-dim query rows are written in
  // 16-byte chunks rather than one short piece per query row.
  const float l_tot = xhalf_sum(l_run);
  const int ql = wave * 32 + (lane & 31);  // this lane's query within the tile
  if (sizeof(T) == 4 && a.lse && lane < 32 && q_local < N)
    a.lse[(size_t)hd * a.ldqk + q] = m_run + log2f(l_tot);  // P = exp2(s - lse)
  uint8_t* st = reinterpret_cast<uint8_t*>(kv);
  __syncthreads();
  if (a.o_scale) {
    // FP8 output for an FP8 output projection
    constexpr int RB = 64 + 16;  // bytes per staged row
    const float inv = 1.0f / (l_tot * *a.o_scale);
#pragma unroll
    for (int ds = 0; ds < 2; ++ds)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int dim = ds * 32 + g * 8 + half * 4;
        *reinterpret_cast<uint32_t*>(st + ql * RB + dim) = e4m3x4(oacc[ds][4 * g] * inv, oacc[ds][4 * g + 1] * inv,
                                                                  oacc[ds][4 * g + 2] * inv, oacc[ds][4 * g + 3] * inv);
      }
    __syncthreads();
    for (int i = tid; i < QT * 4; i += NT) {
      const int row = i >> 2, c = (i & 3) * 16;
      const int qr = q0 + qt * QT + row;
      if (qr < N)
        *reinterpret_cast<uint4*>((uint8_t*)a.o + (size_t)(base + qr) * (a.heads * 64) + hd * 64 + c) =
            *reinterpret_cast<const uint4*>(st + row * RB + c);
    }
  } else {
    constexpr int RB = 64 * (int)sizeof(T) + 16;
    constexpr int EC = 16 / (int)sizeof(T);  // elements per 16-byte chunk
    static_assert(QT * RB <= (int)sizeof(kv), "output tile fits the K and V stages");
    const float inv = 1.0f / l_tot;
#pragma unroll
    for (int ds = 0; ds < 2; ++ds)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int dim = ds * 32 + g * 8 + half * 4;
        T* sp = reinterpret_cast<T*>(st + ql * RB) + dim;
        if constexpr (sizeof(T) == 2) {
          *reinterpret_cast<bf16x4*>(sp) =
              bf16x4{(__bf16)(oacc[ds][4 * g] * inv), (__bf16)(oacc[ds][4 * g + 1] * inv),
                     (__bf16)(oacc[ds][4 * g + 2] * inv), (__bf16)(oacc[ds][4 * g + 3] * inv)};
        } else {
          *reinterpret_cast<f32x4*>(sp) = f32x4{oacc[ds][4 * g] * inv, oacc[ds][4 * g + 1] * inv,
                                                oacc[ds][4 * g + 2] * inv, oacc[ds][4 * g + 3] * inv};
        }
      }
    __syncthreads();
    for (int i = tid; i < QT * (64 / EC); i += NT) {
      const int row = i / (64 / EC), c = (i - row * (64 / EC)) * EC;
      const int qr = q0 + qt * QT + row;
      if (qr < N)
        *reinterpret_cast<uint4*>((T*)a.o + (size_t)(base + qr) * (a.heads * 64) + hd * 64 + c) =
            *reinterpret_cast<const uint4*>(st + row * RB + c * (int)sizeof(T));
    }
  }
}

// ---- FP8 form ----------------------------------------------------------------
//
// Q, K and V^T are OCP E4M3 with per-head power-of-two scales 2^eq, 2^ek,
// 2^ev, applied exactly by the scaled 32x32x64 FP8 MFMA (E8M0 block scales),
// so the score products come out in the BF16 kernel's units (log2 scale,
// onto the -max register block).  The probabilities are E4M3 with unit
// scale; the max is raised lazily as in the safe pass above, which keeps
// them at most 2^8 (E4M3 holds up to 448).  The row sums are those of the
// E4M3 probabilities, taken by one more product per block (a ones row
// against P^T) instead of VALU adds.  A head dimension of 64 is one product
// step: per 64-key block a wave issues 2 score, 2 P V and 1 row-sum products.  K rows and V^T rows are
// 64 bytes in LDS, 16-byte chunk c of row r at slot c ^ ((r >> 2) & 3), so
// the 16 rows one read phase touches cover all banks.  V^T columns are in
// fp8_vt_col order within each group of 64 keys (requests start on
// 64-token boundaries), so a lane's probabilities are its 32 consecutive k.

__device__ __forceinline__ int swz8(int row, int chunk) { return row * 64 + ((chunk ^ ((row >> 2) & 3)) << 4); }

__device__ __forceinline__ f32x16 mfma_fp8(const i32x8& a, const i32x8& b, const f32x16& c, int sa, int sb) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
}

__device__ __forceinline__ i32x8 load_frag8(const uint8_t* __restrict__ t, int row, int half) {
  const uint4 lo = *reinterpret_cast<const uint4*>(t + swz8(row, 2 * half));
  const uint4 hi = *reinterpret_cast<const uint4*>(t + swz8(row, 2 * half + 1));
  return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
}

template <bool MASK, bool FIRST>
__device__ __forceinline__ void fp8_block(const uint8_t* __restrict__ kt, const uint8_t* __restrict__ vt,
                                          const i32x8& qf, const i32x8& ones, f32x16 (&oacc)[2], f32x16& lacc,
                                          f32x16& negm, float& m_run, int lane, int kvalid, int eqk_q, int eqk_k,
                                          int ev) {
  const int half = lane >> 5, l32 = lane & 31;
  i32x8 kf[2];
#pragma unroll
  for (int st = 0; st < 2; ++st) kf[st] = load_frag8(kt, st * 32 + l32, half);
  __builtin_amdgcn_sched_barrier(0);
  f32x16 sacc[2];
#pragma unroll
  for (int st = 0; st < 2; ++st) sacc[st] = mfma_fp8(kf[st], qf, FIRST ? f32x16{} : negm, eqk_k, eqk_q);
  if constexpr (MASK) {
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (st * 32 + acc_row(i, lane) >= kvalid) sacc[st][i] = NEG_BIG;
  }
  float m0 = fmaxf(fmaxf(sacc[0][0], sacc[0][1]), sacc[0][2]);
  float m1 = fmaxf(fmaxf(sacc[1][0], sacc[1][1]), sacc[1][2]);
#pragma unroll
  for (int i = 3; i < 15; i += 2) {
    m0 = fmaxf(fmaxf(m0, sacc[0][i]), sacc[0][i + 1]);
    m1 = fmaxf(fmaxf(m1, sacc[1][i]), sacc[1][i + 1]);
  }
  const float mloc = xhalf_max(fmaxf(fmaxf(m0, sacc[0][15]), fmaxf(m1, sacc[1][15])));
  if constexpr (FIRST) {
    m_run = mloc;
#pragma unroll
    for (int i = 0; i < 16; ++i) negm[i] = -mloc;
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int i = 0; i < 16; ++i) sacc[st][i] -= mloc;
  } else {
    // mloc is relative to m_run: raise the max only past LAZY
    const bool grow = mloc > LAZY;
    if (__any(grow)) {
      const float d = grow ? mloc : 0.0f;
      const float alpha = __builtin_amdgcn_exp2f(-d);
      m_run += d;
      oacc[0] *= alpha;
      oacc[1] *= alpha;
      lacc *= alpha;
#pragma unroll
      for (int i = 0; i < 16; ++i) negm[i] = -m_run;
#pragma unroll
      for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int i = 0; i < 16; ++i) sacc[st][i] -= d;
      asm volatile("" : "+v"(oacc[0]), "+v"(oacc[1]), "+v"(lacc), "+v"(sacc[0]), "+v"(sacc[1]), "+v"(negm));
    }
  }
  // probabilities: byte j = 16 st + i of the lane's 32 (fp8_vt_col order).
  // Every exponent is at most LAZY = 8, so p lies in [0, 256], inside the
  // E4M3 range: the conversion needs no saturation (the clamp to +-448 would
  // change no value)
  static_assert(LAZY <= 8.0f, "probabilities below the E4M3 maximum");
  i32x8 pf;
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      float p[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) p[e] = __builtin_amdgcn_exp2f(sacc[st][4 * g + e]);
      int v = __builtin_amdgcn_cvt_pk_fp8_f32(p[0], p[1], 0, false);
      pf[st * 4 + g] = __builtin_amdgcn_cvt_pk_fp8_f32(p[2], p[3], v, true);
    }
#pragma unroll
  for (int ds = 0; ds < 2; ++ds) oacc[ds] = mfma_fp8(load_frag8(vt, ds * 32 + l32, half), pf, oacc[ds], ev, 127);
  // row sums of the E4M3 probabilities on the matrix core: a block whose
  // row 0 is all ones (the other rows zero) times P^T
  lacc = mfma_fp8(ones, pf, lacc, 127, 127);
}

__global__ __launch_bounds__(NT, 3) void attn_fp8_kernel(const AttnArgs a) {
  constexpr int TB = KB * 64;  // bytes per K or V^T tile
  __shared__ __attribute__((aligned(16))) uint8_t kv[4 * TB];
  uint8_t* ks = kv;
  uint8_t* vs = kv + 2 * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5;
  const int nwork = a.dyn_nwork ? *a.dyn_nwork : a.nwork;
  const int G = nwork * a.heads;
  const int L = blockIdx.x;
  if (L >= G) return;
  const int xcd = L & 7, per = G >> 3, rem = G & 7;
  const int Lr = xcd * per + (xcd < rem ? xcd : rem) + (L >> 3);
  const int hd = Lr / nwork;
  const int w = a.work[Lr - hd * nwork];
  const int r = w >> 16, qt = w & (ATTN_TARGET_TILE - 1);
  const ReqDesc& d = a.reqs[r];
  const int N = d.J * d.P;
  const int base = d.tok_off;
  const int q0 = (w & ATTN_TARGET_TILE) ? (d.J - 1) * d.P : 0;
  const int q_local = q0 + qt * QT + wave * 32 + (lane & 31);
  const int q = base + q_local;
  // E8M0 scale operands (127 + e)
  const int sq = a.qkv_exp[hd], sk = a.qkv_exp[a.heads + hd], sv = a.qkv_exp[2 * a.heads + hd];

  const uint8_t* Kg = (const uint8_t*)a.k + ((size_t)hd * a.ldqk + base) * 64;
  const uint8_t* Vg = (const uint8_t*)a.vt + (size_t)hd * 64 * a.ldv + base;
  i32x8 qf;
  {
    const uint4* qp = reinterpret_cast<const uint4*>((const uint8_t*)a.q + ((size_t)hd * a.ldqk + (q_local < N ? q : base)) * 64 + half * 32);
    const uint4 lo = qp[0], hi = qp[1];
    qf = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
  }
  const __amdgpu_buffer_rsrc_t krs =
      __builtin_amdgcn_make_buffer_rsrc((void*)Kg, (short)0, (a.ldqk - base) * 64, 0x00020000);
  const __amdgpu_buffer_rsrc_t vrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)Vg, (short)0, 64 * a.ldv - base, 0x00020000);
  // wave w fills rows 16w .. 16w+15 of the K and V^T tiles (1 KB, 16 bytes
  // per lane); lane L takes row 16w + L / 4 and the chunk whose swizzled
  // slot is L % 4
  const int rr = wave * 16 + (lane >> 2);
  const int cc = (lane & 3) ^ ((rr >> 2) & 3);
  const int kvo = rr * 64 + cc * 16;
  const int vvo = rr * a.ldv + cc * 16;
  auto fetch = [&](int kb, int buf) {
    dma16_att(krs, ks + buf * TB + wave * 16 * 64, kvo, kb * 64);
    dma16_att(vrs, vs + buf * TB + wave * 16 * 64, vvo, kb);
  };
  f32x16 oacc[2], lacc, negm;
  oacc[0] = f32x16{};
  oacc[1] = f32x16{};
  lacc = f32x16{};
  negm = f32x16{};
  float m_run = 0.0f;
  // row 0 of the row-sum block: E4M3 ones (0x38) from lanes 0 and 32
  const int one8 = (lane & 31) == 0 ? 0x38383838 : 0;
  const i32x8 ones = {one8, one8, one8, one8, one8, one8, one8, one8};
  const int nkb = (N + KB - 1) / KB;
  const int nfull = N / KB;
  fetch(0, 0);
  wait_vm_att<0>();
  __syncthreads();
  if (nfull == 0) {
    fp8_block<true, true>(ks, vs, qf, ones, oacc, lacc, negm, m_run, lane, N, sq, sk, sv);
  } else {
    fetch(nkb > 1 ? KB : 0, 1);
    fp8_block<false, true>(ks, vs, qf, ones, oacc, lacc, negm, m_run, lane, KB, sq, sk, sv);
    wait_vm_att<0>();
    __syncthreads();
    int b = 1;
    for (; b + 1 < nfull; b += 2) {
      fetch((b + 1) * KB, 0);
      fp8_block<false, false>(ks + TB, vs + TB, qf, ones, oacc, lacc, negm, m_run, lane, KB, sq, sk, sv);
      wait_vm_att<0>();
      __syncthreads();
      fetch(b + 2 < nkb ? (b + 2) * KB : (b + 1) * KB, 1);
      fp8_block<false, false>(ks, vs, qf, ones, oacc, lacc, negm, m_run, lane, KB, sq, sk, sv);
      wait_vm_att<0>();
      __syncthreads();
    }
    if (b < nfull) {
      fetch(b + 1 < nkb ? (b + 1) * KB : b * KB, 0);
      fp8_block<false, false>(ks + TB, vs + TB, qf, ones, oacc, lacc, negm, m_run, lane, KB, sq, sk, sv);
      wait_vm_att<0>();
      __syncthreads();
    }
    if (nfull < nkb)  // ragged last block, already in LDS
      fp8_block<true, false>(ks + (nfull & 1) * TB, vs + (nfull & 1) * TB, qf, ones, oacc, lacc, negm, m_run, lane,
                             N - nfull * KB, sq, sk, sv);
  }
  // output through LDS in whole 64-dim rows (the tiles are free once every
  // wave is past its last block)
  // the row sum of query l % 32 sits in register 0 of lane l % 32 (row 0 of
  // the block); lanes 32..63 hold rows 4..7, all zero
  const float l_tot = xhalf_sum(lane < 32 ? lacc[0] : 0.0f);
  const int ql = wave * 32 + (lane & 31);
  uint8_t* st = kv;
  __syncthreads();
  if (a.o_scale) {
    constexpr int RB = 64 + 16;
    static_assert(QT * RB <= 4 * TB, "output tile fits the stages");
    const float inv = 1.0f / (l_tot * *a.o_scale);
#pragma unroll
    for (int ds = 0; ds < 2; ++ds)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int dim = ds * 32 + g * 8 + half * 4;
        *reinterpret_cast<uint32_t*>(st + ql * RB + dim) = e4m3x4(oacc[ds][4 * g] * inv, oacc[ds][4 * g + 1] * inv,
                                                                  oacc[ds][4 * g + 2] * inv, oacc[ds][4 * g + 3] * inv);
      }
    __syncthreads();
    for (int i = tid; i < QT * 4; i += NT) {
      const int row = i >> 2, c = (i & 3) * 16;
      const int qr = q0 + qt * QT + row;
      if (qr < N)
        *reinterpret_cast<uint4*>((uint8_t*)a.o + (size_t)(base + qr) * (a.heads * 64) + hd * 64 + c) =
            *reinterpret_cast<const uint4*>(st + row * RB + c);
    }
  } else {
    // BF16 output: two passes of 64 queries through the 16 KB of stages
    constexpr int RB = 64 * 2 + 16;
    const float inv = 1.0f / l_tot;
    for (int pass = 0; pass < 2; ++pass) {
      if ((wave >> 1) == pass) {
        const int qp = ql - pass * 64;
#pragma unroll
        for (int ds = 0; ds < 2; ++ds)
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int dim = ds * 32 + g * 8 + half * 4;
            *reinterpret_cast<bf16x4*>(reinterpret_cast<__bf16*>(st + qp * RB) + dim) =
                bf16x4{(__bf16)(oacc[ds][4 * g] * inv), (__bf16)(oacc[ds][4 * g + 1] * inv),
                       (__bf16)(oacc[ds][4 * g + 2] * inv), (__bf16)(oacc[ds][4 * g + 3] * inv)};
          }
      }
      __syncthreads();
      for (int i = tid; i < 64 * 8; i += NT) {
        const int row = i >> 3, c = (i & 7) * 8;
        const int qr = q0 + qt * QT + pass * 64 + row;
        if (qr < N)
          *reinterpret_cast<uint4*>((__bf16*)a.o + (size_t)(base + qr) * (a.heads * 64) + hd * 64 + c) =
              *reinterpret_cast<const uint4*>(st + row * RB + c * 2);
      }
      __syncthreads();
    }
  }
}

}  // namespace

int launch_attention(Prec prec, const AttnArgs& a, hipStream_t s) {
  if (a.nwork <= 0) return 0;
  dim3 grid(a.nwork * a.heads);
  if (prec == P_FP8 && a.qkv_exp) attn_fp8_kernel<<<grid, NT, 0, s>>>(a);
  else if (prec == P_BF16 || prec == P_FP8) attn_kernel<OpBF16><<<grid, NT, 0, s>>>(a);  // uncalibrated FP8 form: BF16
  else if (prec == P_FP32 && !a.o_scale) attn_kernel<OpF32><<<grid, NT, 0, s>>>(a);
  else return -95;
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

// ---- Attention without allocation ------------------------------------------
//
// The one-request form of the attention kernel needs a request descriptor
// and a q-tile work list in device memory.  This variant keeps both in a
// file-scope device array (one copy per device, held until the process
// ends): a small kernel on the caller's stream writes them, then the
// attention kernel reads them.  Calls on one stream are ordered; calls that
// overlap on one device (other streams, other threads) share the array and
// race.

namespace {

constexpr size_t NOALLOC_DESC_BYTES = 256;
static_assert(sizeof(ReqDesc) <= NOALLOC_DESC_BYTES, "request descriptor slot too small");
constexpr size_t NOALLOC_BYTES = NOALLOC_DESC_BYTES + sizeof(int) * (ATTN_NOALLOC_MAX_TILES + 1);
constexpr int NOALLOC_MAX_DEVICES = 64;

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Descriptor of one request covering every token (one tubelet of ntok
// tokens, no frames) and the work list 0 .. ntile-1; every value the
// attention kernel reads is rewritten, so nothing needs clearing first.
__global__ void attn_noalloc_setup_kernel(unsigned char* ws, int ntok, int ntile) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ReqDesc* d = reinterpret_cast<ReqDesc*>(ws);
    d->tok_off = 0; d->head_off = 0;
    d->H = 1; d->W = ntok; d->gy = 1; d->gx = ntok; d->P = ntok;
    d->J = 1; d->nframes = 1; d->pad_ = 0;
    for (int f = 0; f < REVO_MAX_FRAMES; ++f) { d->tau[f] = 0.f; d->frames[f] = nullptr; }
    d->mask = nullptr; d->pred = nullptr; d->out_i = nullptr; d->out_f = nullptr;
  }
  int* work = reinterpret_cast<int*>(ws + NOALLOC_DESC_BYTES);
  if (i < ntile) work[i] = i;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

// Device address of this device's copy of the array, looked up once per
// device (the array's name is not a device address in host code).
int noalloc_workspace(unsigned char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return -5;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -5;
    g_noalloc_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_noalloc_ptr[dev]);
  return 0;
}

}  // namespace

int launch_attention_noalloc(Prec prec, const void* q, const void* k, const void* vt, void* o, int heads, int ntok,
                             int ld, hipStream_t s) {
  const int ntile = (ntok + 127) / 128;
  if (ntok <= 0 || ntile > ATTN_NOALLOC_MAX_TILES) return -7;
  unsigned char* ws = nullptr;
  if (int rc = noalloc_workspace(&ws)) return rc;
  attn_noalloc_setup_kernel<<<(ntile + 255) / 256, 256, 0, s>>>(ws, ntok, ntile);
  if (hipGetLastError() != hipSuccess) return -5;
  AttnArgs a;
  memset(&a, 0, sizeof(a));
  a.q = q; a.k = k; a.vt = vt; a.o = o; a.heads = heads; a.ldqk = ld; a.ldv = ld;
  a.reqs = reinterpret_cast<const ReqDesc*>(ws); a.nreq = 1;
  a.work = reinterpret_cast<const int*>(ws + NOALLOC_DESC_BYTES); a.nwork = ntile;
  return launch_attention(prec, a, s);
}

}  // namespace revo
