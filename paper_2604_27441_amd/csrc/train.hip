// Kernels of the pretraining step (backward pass and Adam) of the recovery
// network: the RGB objective MSE + alpha TV on the raw prediction of the
// target frame (Sec. 3.4.2 RGB loss equation, used for both models in
// pretraining), reverse-mode gradients of every layer, and Adam (Sec. 4;
// Kingma & Ba 2015, Algorithm 1).  FP32 throughout.
#include "train.h"

#include <cstring>

namespace revo {

namespace {

constexpr int TB = 256;

// ---- transposes and column sums ---------------------------------------------

// out[c][r] = in[r][c] for every block of the list, one 64 x 64 tile per
// workgroup: the descriptor is the last one whose first tile is at or below
// the workgroup's (a binary search over the list)
__global__ __launch_bounds__(TB) void transpose_batch_kernel(const TrDesc* __restrict__ list, int n) {
  __shared__ float t[64][65];
  const int tile = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (list[mid].tile0 <= tile) lo = mid;
    else hi = mid - 1;
  }
  const TrDesc d = list[lo];
  const int tc = (d.cols + 63) / 64, tl = tile - d.tile0;
  const int r0 = (tl / tc) * 64, c0 = (tl - (tl / tc) * tc) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int r = r0 + i, c = c0 + tx;
    t[i][tx] = (r < d.rows && c < d.cols) ? d.in[(size_t)r * d.ld_in + c] : 0.0f;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int c = c0 + i, r = r0 + tx;
    if (c < d.cols && r < d.rows) d.out[(size_t)c * d.ld_out + r] = t[tx][i];
  }
}

// out[i] = sum over b of part[b n + i]: b in groups of 8 (added as a
// pairwise tree, the groups in order; eight loads in flight); with v4
// (n a multiple of 4, both arrays 16-byte aligned) four consecutive i per
// thread
__global__ __launch_bounds__(TB) void sum_chunks_kernel(const float* __restrict__ part, int nb, long long n,
                                                        float* __restrict__ out, bool v4) {
  if (v4) {
    const long long n4 = n >> 2;
    const float4* p4 = reinterpret_cast<const float4*>(part);
    for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n4; i += (long long)gridDim.x * TB) {
      float4 s = {0.0f, 0.0f, 0.0f, 0.0f};
      int b = 0;
      for (; b + 8 <= nb; b += 8) {
        float4 t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = p4[(size_t)(b + u) * n4 + i];
        s.x += ((t[0].x + t[1].x) + (t[2].x + t[3].x)) + ((t[4].x + t[5].x) + (t[6].x + t[7].x));
        s.y += ((t[0].y + t[1].y) + (t[2].y + t[3].y)) + ((t[4].y + t[5].y) + (t[6].y + t[7].y));
        s.z += ((t[0].z + t[1].z) + (t[2].z + t[3].z)) + ((t[4].z + t[5].z) + (t[6].z + t[7].z));
        s.w += ((t[0].w + t[1].w) + (t[2].w + t[3].w)) + ((t[4].w + t[5].w) + (t[6].w + t[7].w));
      }
      for (; b < nb; ++b) {
        const float4 t = p4[(size_t)b * n4 + i];
        s.x += t.x; s.y += t.y; s.z += t.z; s.w += t.w;
      }
      reinterpret_cast<float4*>(out)[i] = s;
    }
    return;
  }
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB) {
    float s = 0.0f;
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
      float t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = part[(size_t)(b + u) * n + i];
      s += ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    }
    for (; b < nb; ++b) s += part[(size_t)b * n + i];
    out[i] = s;
  }
}

// out[c] = sum of the block partials: 64 columns x 4 lanes per block, lane
// l taking blocks l, l + 4, ... in groups of 8 (added as a pairwise tree,
// the groups in order; eight loads in flight), then the four lanes in order
__global__ __launch_bounds__(TB) void colsum_final_kernel(const float* __restrict__ part, int nchunk, int cols,
                                                          float* __restrict__ out) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), l = threadIdx.x >> 6;
  float s = 0.0f;
  if (c < cols) {
    int i = l;
    for (; i + 28 < nchunk; i += 32) {
      float t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = part[(size_t)(i + 4 * u) * cols + c];
      s += ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    }
    for (; i < nchunk; i += 4) s += part[(size_t)i * cols + c];
  }
  red[l][threadIdx.x & 63] = s;
  __syncthreads();
  if (l == 0 && c < cols)
    out[c] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// ---- weight gradients ------------------------------------------------------------

// part[c][o][i] = sum over the rows m of chunk c (rows c kc .. c kc + kc - 1
// below `rows`) of dy[m][o] x[m][i] for every chunk c; with bpart, the tiles of
// the first input columns also write bpart[c][o] = the same rows' sum of
// dy[m][o].  Both operands are read as they lie (token rows, features
// contiguous), so no transposed copies are made.  Tile 128 (o) x 128 (i) on
// 4 waves of 64 x 64 (2 x 2 FP32 32x32x2 MFMA blocks); stages of 16 rows of
// each operand double-buffered in LDS, the next stage fetched into registers
// during the current one's products.  One launch can hold two layers over
// the same rows (independent products of one block's backward pass): the
// tiles from tile1 on belong to the second.
struct WgradLayer {
  const float* dy;
  const float* x;
  int nout, nin, ldy, ldx;
  float* part;
  float* bpart;
  long long pstride, bstride;  // elements from one chunk's part / bpart to the next
};
struct WgradArgs {
  WgradLayer l0, l1;
  int tile1;  // the first tile of l1 (the grid's width with one layer)
  int rows, kc;
};

__global__ __launch_bounds__(TB, 2) void wgrad_kernel(const WgradArgs args) {
  constexpr int R = 16, P = 160;  // rows per stage; row pitch (half-waves read rows 2s and 2s + 1 on disjoint banks)
  __shared__ __attribute__((aligned(16))) float sy[2][R][P], sx[2][R][P];
  // Workgroups go round-robin to the 8 XCDs, each with its own L2: give XCD
  // x a contiguous range of (chunk, tile) pairs, tile fastest, so the tiles
  // that read one chunk's rows share that XCD's L2 instead of every L2
  // fetching them from HBM
  const int nwg = gridDim.x * gridDim.y, L = blockIdx.y * gridDim.x + blockIdx.x;
  const int xcd = L & 7, per = nwg >> 3, rem = nwg & 7;
  const int q = xcd * per + (xcd < rem ? xcd : rem) + (L >> 3);
  const int chunk = q / (int)gridDim.x, tall = q - chunk * (int)gridDim.x;
  const bool second = tall >= args.tile1;
  const WgradLayer a = second ? args.l1 : args.l0;
  const int tile = tall - (second ? args.tile1 : 0);
  const int gi = (a.nin + 127) / 128;
  const int o0 = (tile / gi) * 128, i0 = (tile - (tile / gi) * gi) * 128;
  const int m0 = chunk * args.kc, m1 = min(args.rows, m0 + args.kc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5, l32 = lane & 31;
  const int wo = wave >> 1, wi = wave & 1;
  // loader: rows tid / 32 and tid / 32 + 8 of the stage, columns 4 (tid %
  // 32) .. +3 of the tile, so the 32 lanes of a half-wave move 512
  // contiguous bytes of one row (coalesced loads, conflict-free LDS stores).
  // Buffer loads: the descriptors end at the chunk's last row, so rows past
  // it read as zeros without a branch.  Columns past the matrix (a partial
  // last tile) read the next row or zeros; they only reach outputs and bias
  // sums that are not stored.
  const int lr = tid >> 5, lc = (tid & 31) * 4;
  const __amdgpu_buffer_rsrc_t yrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.dy, (short)0, m1 * a.ldy * (int)sizeof(float), 0x00020000);
  const __amdgpu_buffer_rsrc_t xrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.x, (short)0, m1 * a.ldx * (int)sizeof(float), 0x00020000);
  const bool bias = a.bpart && i0 == 0;
  float4 ry[2], rx[2];
  float bs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  auto fetch = [&](int r0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int m = r0 + lr + 8 * h;
      const int yo = (m * a.ldy + o0 + lc) * (int)sizeof(float), xo = (m * a.ldx + i0 + lc) * (int)sizeof(float);
      ry[h] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(yrs, yo, 0, 0));
      rx[h] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(xrs, xo, 0, 0));
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      *reinterpret_cast<float4*>(&sy[b][lr + 8 * h][lc]) = ry[h];
      *reinterpret_cast<float4*>(&sx[b][lr + 8 * h][lc]) = rx[h];
      if (bias) { bs[0] += ry[h].x; bs[1] += ry[h].y; bs[2] += ry[h].z; bs[3] += ry[h].w; }
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u) { acc[u][0] = f32x16{}; acc[u][1] = f32x16{}; }
  const int nst = (m1 - m0 + R - 1) / R;
  if (nst > 0) {
    fetch(m0);
    put(0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int b = st & 1;
    if (st + 1 < nst) fetch(m0 + (st + 1) * R);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const int r = 2 * k + half;
      const float y0 = sy[b][r][64 * wo + l32], y1 = sy[b][r][64 * wo + 32 + l32];
      const float x0 = sx[b][r][64 * wi + l32], x1 = sx[b][r][64 * wi + 32 + l32];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(y0, x0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(y0, x1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(y1, x0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(y1, x1, acc[1][1], 0, 0, 0);
    }
    if (st + 1 < nst) put(b ^ 1);
    __syncthreads();
  }
  float* out = a.part + (size_t)chunk * a.pstride;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = i0 + 64 * wi + 32 * v + l32;
      if (i >= a.nin) continue;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int o = o0 + 64 * wo + 32 * u + acc_row(j, lane);
        if (o < a.nout) out[(size_t)o * a.nin + i] = acc[u][v][j];
      }
    }
  if (bias) {
    // the 8 loader rows' sums of each column (rows r and r + 8 of every
    // stage), added in row order
    float* red = &sx[0][0][0];  // [8][128]: free after the last barrier
#pragma unroll
    for (int e = 0; e < 4; ++e) red[lr * 128 + lc + e] = bs[e];
    __syncthreads();
    if (tid < 128 && o0 + tid < a.nout) {
      float t = 0.0f;
      for (int r = 0; r < 8; ++r) t += red[r * 128 + tid];
      a.bpart[(size_t)chunk * a.bstride + o0 + tid] = t;
    }
  }
}

// ---- LayerNorm backward -------------------------------------------------------------
//
// y = xhat g + b with xhat = (x - mean) rstd.  One wave per row, 16 waves
// per block: dx = rstd (dy g - mean(dy g) - xhat mean(dy g xhat)), added
// to din into dout (the same buffer or, without rowmap, another one).  The gain and shift gradients are column sums over the rows of
// xhat dy and dy: each block writes its 16 rows' sums (in row order),
// part[block][d] (gain) and part[block][D + d] (shift), which
// colsum_final_kernel then adds over the blocks in order.  With rowmap, row i
// of dy belongs to row rowmap[i] of x and dres.
constexpr int LN_WAVES = 16, LN_TB = 64 * LN_WAVES;
__global__ __launch_bounds__(LN_TB) void ln_bwd_kernel(const float* __restrict__ x, const float* __restrict__ g,
                                                       const float* __restrict__ dy, const float* din,
                                                       float* dout, float* __restrict__ part, int rows, int D,
                                                       const int* __restrict__ rowmap) {
  constexpr int MAXE = 8;  // D <= 512
  __shared__ float red[LN_WAVES][64 * MAXE];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * LN_WAVES + wave;
  float pg[MAXE], pb[MAXE];  // this row's xhat dy and dy (zeros past the rows)
#pragma unroll
  for (int e = 0; e < MAXE; ++e) { pg[e] = 0.0f; pb[e] = 0.0f; }
  if (row < rows) {
    const int xr = rowmap ? rowmap[row] : row;
    const float* xp = x + (size_t)xr * D;
    const float* dp = dy + (size_t)row * D;
    float xv[MAXE], gv[MAXE];
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int d = lane + 64 * e;
      xv[e] = d < D ? xp[d] : 0.0f;
      pb[e] = d < D ? dp[d] : 0.0f;
      s += xv[e];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const float mean = s / D;
    float v = 0.0f;
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int d = lane + 64 * e;
      const float c = d < D ? xv[e] - mean : 0.0f;
      v += c * c;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const float rstd = 1.0f / sqrtf(v / D + 1e-6f);
    float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int d = lane + 64 * e;
      const float xh = d < D ? (xv[e] - mean) * rstd : 0.0f;
      gv[e] = d < D ? pb[e] * g[d] : 0.0f;
      s1 += gv[e];
      s2 += gv[e] * xh;
      pg[e] = xh * pb[e];
      xv[e] = xh;
    }
    for (int o = 32; o > 0; o >>= 1) {
      s1 += __shfl_xor(s1, o);
      s2 += __shfl_xor(s2, o);
    }
    const float m1 = s1 / D, m2 = s2 / D;
    const float* ri = din + (size_t)xr * D;
    float* ro = dout + (size_t)xr * D;
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int d = lane + 64 * e;
      if (d < D) ro[d] = ri[d] + rstd * (gv[e] - m1 - xv[e] * m2);
    }
  }
  float* out = part + (size_t)blockIdx.x * 2 * D;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k) __syncthreads();  // the gain sums have been read
#pragma unroll
    for (int e = 0; e < MAXE; ++e) red[wave][lane + 64 * e] = k ? pb[e] : pg[e];
    __syncthreads();
    for (int c = threadIdx.x; c < D; c += LN_TB) {
      float t = 0.0f;
      for (int w = 0; w < LN_WAVES; ++w) t += red[w][c];
      out[k * D + c] = t;
    }
  }
}

// ---- loss ---------------------------------------------------------------------------
//
// Per frame b: MSE(pred, gt) + alpha (mean |x forward difference| + mean |y
// forward difference|) of pred, averaged over the batch.  dpred is the
// gradient of that batch loss (sign(0) = 0 for the absolute values);
// part[block] the block's share of the loss.  gt: u8 HWC (C = 3, / 255) or
// u16 HW (C = 1, / 4000 mm).
__global__ __launch_bounds__(TB) void pretrain_loss_kernel(const float* __restrict__ pred, const void* __restrict__ gt,
                                                           int B, int H, int W, int C, float alpha,
                                                           float* __restrict__ dpred, double* __restrict__ part) {
  __shared__ double red[TB / 64];
  const long long per = (long long)H * W * C;
  const long long n = per * B;
  const float inv_n = 1.0f / (float)per;
  const float inv_h = W > 1 ? 1.0f / (float)((long long)H * (W - 1) * C) : 0.0f;
  const float inv_v = H > 1 ? 1.0f / (float)((long long)(H - 1) * W * C) : 0.0f;
  const float inv_b = 1.0f / (float)B;
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB) {
    const long long f = i / per, r = i - f * per;
    const long long px = r / C;
    const int y = (int)(px / W), x = (int)(px - (long long)y * W);
    const float p = pred[i];
    const float gv = C == 3 ? (float)((const uint8_t*)gt)[i] * (1.0f / 255.0f)
                            : (float)((const uint16_t*)gt)[i] * (1.0f / 4000.0f);
    const float e = p - gv;
    float d = 2.0f * e * inv_n;
    float l = e * e * inv_n;
    auto sgn = [](float v) { return v > 0.0f ? 1.0f : (v < 0.0f ? -1.0f : 0.0f); };
    if (x + 1 < W) {
      const float t = pred[i + C] - p;
      l += alpha * fabsf(t) * inv_h;
      d -= alpha * sgn(t) * inv_h;
    }
    if (x > 0) d += alpha * sgn(p - pred[i - C]) * inv_h;
    if (y + 1 < H) {
      const float t = pred[i + (long long)W * C] - p;
      l += alpha * fabsf(t) * inv_v;
      d -= alpha * sgn(t) * inv_v;
    }
    if (y > 0) d += alpha * sgn(p - pred[i - (long long)W * C]) * inv_v;
    dpred[i] = d * inv_b;
    acc += (double)l;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < TB / 64; ++w) s += red[w];
    part[blockIdx.x] = s * (1.0 / B);
  }
}

// Head gradient rows: dhead[i][c] for compact target row i and slot column
// c = (py 16 + px) C + ch takes dpred at pixel (16 ty + py, 16 tx + px),
// channel ch of the row's request (0 outside the frame and past Mh).
__global__ __launch_bounds__(TB) void head_grad_kernel(const ReqDesc* __restrict__ reqs, int nreq, int Mh, int Mh_pad,
                                                       int C, const float* __restrict__ dpred, long long frame_elems,
                                                       float* __restrict__ dhead) {
  const int cols = 256 * C;
  const long long n = (long long)Mh_pad * cols;
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB) {
    const int row = (int)(i / cols), c = (int)(i - (long long)row * cols);
    float v = 0.0f;
    if (row < Mh) {
      const int r = find_req_head(reqs, nreq, row);
      const ReqDesc& d = reqs[r];
      const int p = row - d.head_off;
      const int ty = p / d.gx, tx = p - ty * d.gx;
      const int ch = c % C, px = (c / C) & 15, py = c / (16 * C);
      const int Y = 16 * ty + py, X = 16 * tx + px;
      if (Y < d.H && X < d.W) v = dpred[(long long)r * frame_elems + ((long long)Y * d.W + X) * C + ch];
    }
    dhead[i] = v;
  }
}

// ---- attention backward ---------------------------------------------------------------
//
// Forward: Q arrives scaled, qs = q log2(e) / 8, and P_ij = exp2(qs_i . k_j -
// lse_i) with lse the base-2 log of the row's normaliser.  With dO the
// output gradient and Dv_i = dO_i . O_i, the gradient with respect to the
// natural scores s_ij = q_i . k_j / 8 is dS_ij = P_ij (dO_i . v_j - Dv_i);
// then dq_i = sum_j dS_ij k_j / 8, dk_j = sum_i dS_ij q_i / 8 =
// sum_i dS_ij qs_i / log2(e), dv_j = sum_i P_ij dO_i.  Blocks of 64 queries x
// 64 keys; each of 256 threads holds a 4 x 4 piece of a tile.

// Dv[h][t] = sum_d dO[t][h 64 + d] O[t][h 64 + d]
__global__ __launch_bounds__(TB) void attn_bwd_dot_kernel(const float* __restrict__ o, const float* __restrict__ dout,
                                                          int M, int heads, int ld, float* __restrict__ dv) {
  const int wave = (blockIdx.x * TB + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (wave >= M * heads) return;
  const int t = wave / heads, h = wave - t * heads;
  const size_t off = (size_t)t * heads * 64 + h * 64 + lane;
  float s = o[off] * dout[off];
  for (int k = 32; k > 0; k >>= 1) s += __shfl_xor(s, k);
  if (lane == 0) dv[(size_t)h * ld + t] = s;
}

struct AttnBwdArgs {
  const float* q;     // [heads][ld][64], scaled by log2(e) / 8
  const float* k;     // [heads][ld][64]
  const float* vt;    // [heads][64][ld]
  const float* dout;  // [M][heads 64]
  const float* lse;   // [heads][ld]
  const float* dv;    // [heads][ld]
  float* dqkv;        // [M][3 heads 64]: dq | dk | dv, head-major
  int heads, ld;
  const ReqDesc* reqs;
  const int* work;    // (request << 16) | 64-row block
  int nwork;
};

__device__ __forceinline__ f32x16 mfma_f32(float a, float b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// The tiles are products of 64 x 64 blocks over 64 (head dimension, queries
// or keys), on FP32 32x32x2 MFMAs: lane l supplies A[l % 32][k] and B[k][l %
// 32] for k = 2 step + l / 32, and holds C[row(i, l)][l % 32] (acc_row).
// Each of the 4 waves takes one 32 x 32 tile per product.  The operand a
// wave reuses for every block of the loop stays in registers (32 values per
// matrix); the loop's next block is fetched into registers while the current
// one is multiplied, and stored to LDS once the current one is consumed.

// 16 values per thread of a 64 x 64 tile of a [rows][pitch] matrix (row
// offset r0, rows at or past rmax read as zeros): thread t takes rows
// t / 64 + 4 j, column t % 64.  Buffer loads whose descriptor ends at row
// rmax give the zeros without a branch.
__device__ __forceinline__ void fetch_rows(float (&r)[16], const float* __restrict__ src, int pitch, int r0, int rmax) {
  const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, rmax * pitch * (int)sizeof(float), 0x00020000);
#pragma unroll
  for (int j = 0; j < 16; ++j)
    r[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, ((r0 + rb + 4 * j) * pitch + c) * 4, 0, 0));
}
__device__ __forceinline__ void store_rows(float (*t)[65], const float (&r)[16]) {
  const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 16; ++j) t[rb + 4 * j][c] = r[j];
}
// The same from V^T [64][ld]: thread t takes dimensions t / 64 + 4 j of key
// c0 + t % 64; store_cols writes t[key][d].  Keys past the request read
// what the padded V^T holds there (zeros or other requests' finite values):
// every product that takes them is masked by a select.
__device__ __forceinline__ void fetch_cols(float (&r)[16], const float* __restrict__ vt, int ld, int c0) {
  const int c = threadIdx.x & 63, db = threadIdx.x >> 6;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)vt, (short)0, 64 * ld * (int)sizeof(float), 0x00020000);
#pragma unroll
  for (int j = 0; j < 16; ++j)
    r[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, ((db + 4 * j) * ld + c0 + c) * 4, 0, 0));
}
__device__ __forceinline__ void store_cols(float (*t)[65], const float (&r)[16]) {
  const int c = threadIdx.x & 63, db = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 16; ++j) t[c][db + 4 * j] = r[j];
}

// dK and dV of one 64-key block of one (request, head), looping over the
// request's query blocks.  Per block: wave (qc, kt) forms the 32 x 32 piece
// of S = Qs K^T and dP = dO V^T (K and V rows of its keys in registers), P
// and dS go through LDS; wave (kt, dt) accumulates dV += P^T dO and
// dK += dS^T Qs over the block's 64 queries.
__global__ __launch_bounds__(TB, 2) void attn_bwd_dkdv_kernel(const AttnBwdArgs a) {
  __shared__ float Qs[64][65], Ds[64][65], Pt[64][65], dSt[64][65];
  __shared__ float lse_s[64], dv_s[64];
  const int h = blockIdx.y;
  const int w = a.work[blockIdx.x];
  const ReqDesc& d = a.reqs[w >> 16];
  const int N = d.J * d.P, base = d.tok_off;
  const int k0 = (w & 0xFFFF) * 64;
  const int nk = min(64, N - k0);
  const float* qh = a.q + (size_t)h * a.ld * 64;
  const float* doh = a.dout + h * 64;
  const int dpitch = a.heads * 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, l32 = lane & 31;
  const int qc = wave & 1, kt = wave >> 1;   // S / dP piece: queries 32 qc .., keys 32 kt ..
  const int kt2 = wave >> 1, dt = wave & 1;  // dK / dV piece: keys 32 kt2 .., dims 32 dt ..

  // K and V rows of this wave's keys into registers (through LDS)
  float kr[32], vr[32];
  {
    float t0[16], t1[16];
    fetch_rows(t0, a.k + (size_t)h * a.ld * 64, 64, base + k0, base + N);
    fetch_cols(t1, a.vt + (size_t)h * 64 * a.ld, a.ld, base + k0);
    store_rows(Pt, t0);
    store_cols(dSt, t1);
  }
  float pq[16], pd[16], plse = 0.0f, pdv = 0.0f;
  fetch_rows(pq, qh, 64, base, base + N);
  fetch_rows(pd, doh, dpitch, base, base + N);
  if (threadIdx.x < 64 && (int)threadIdx.x < N) {
    plse = a.lse[(size_t)h * a.ld + base + threadIdx.x];
    pdv = a.dv[(size_t)h * a.ld + base + threadIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int st = 0; st < 32; ++st) {
    kr[st] = Pt[32 * kt + l32][2 * st + half];
    vr[st] = dSt[32 * kt + l32][2 * st + half];
  }
  f32x16 gk = {}, gv = {};
  for (int q0 = 0; q0 < N; q0 += 64) {
    const int nq = min(64, N - q0);
    __syncthreads();  // the previous block's Qs, Ds, Pt, dSt are consumed
    store_rows(Qs, pq);
    store_rows(Ds, pd);
    if (threadIdx.x < 64) {
      lse_s[threadIdx.x] = plse;
      dv_s[threadIdx.x] = pdv;
    }
    __syncthreads();
    if (q0 + 64 < N) {
      fetch_rows(pq, qh, 64, base + q0 + 64, base + N);
      fetch_rows(pd, doh, dpitch, base + q0 + 64, base + N);
      if (threadIdx.x < 64 && q0 + 64 + (int)threadIdx.x < N) {
        plse = a.lse[(size_t)h * a.ld + base + q0 + 64 + threadIdx.x];
        pdv = a.dv[(size_t)h * a.ld + base + q0 + 64 + threadIdx.x];
      }
    }
    f32x16 sc = {}, dp = {};
#pragma unroll
    for (int st = 0; st < 32; ++st) {
      const int dd = 2 * st + half;
      sc = mfma_f32(Qs[32 * qc + l32][dd], kr[st], sc);
      dp = mfma_f32(Ds[32 * qc + l32][dd], vr[st], dp);
    }
    const int kl = 32 * kt + l32;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int ql = 32 * qc + acc_row(i, lane);
      const bool ok = ql < nq && kl < nk;
      const float pv = ok ? __builtin_amdgcn_exp2f(sc[i] - lse_s[ql]) : 0.0f;
      Pt[ql][kl] = pv;
      dSt[ql][kl] = ok ? pv * (dp[i] - dv_s[ql]) : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int st = 0; st < 32; ++st) {
      const int qq = 2 * st + half;
      gv = mfma_f32(Pt[qq][32 * kt2 + l32], Ds[qq][32 * dt + l32], gv);
      gk = mfma_f32(dSt[qq][32 * kt2 + l32], Qs[qq][32 * dt + l32], gk);
    }
  }
  const int D = a.heads * 64;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int key = 32 * kt2 + acc_row(i, lane);
    if (key >= nk) continue;
    float* row = a.dqkv + (size_t)(base + k0 + key) * 3 * D;
    row[D + h * 64 + 32 * dt + l32] = gk[i] * 0.69314718055994531f;  // 1 / log2(e)
    row[2 * D + h * 64 + 32 * dt + l32] = gv[i];
  }
}

// dQ of one 64-query block of one (request, head), looping over key blocks.
// Per block: wave (kt, qc) forms S^T = K Qs^T and dP^T = V dO^T (keys as
// rows; Q and dO rows of its queries in registers), dS^T goes through LDS;
// wave (dt, qc2) accumulates dQ^T += K^T dS^T.
__global__ __launch_bounds__(TB, 2) void attn_bwd_dq_kernel(const AttnBwdArgs a) {
  __shared__ float Ks[64][65], Vs[64][65], dSt[64][65];
  const int h = blockIdx.y;
  const int w = a.work[blockIdx.x];
  const ReqDesc& d = a.reqs[w >> 16];
  const int N = d.J * d.P, base = d.tok_off;
  const int q0 = (w & 0xFFFF) * 64;
  const int nq = min(64, N - q0);
  const float* kh = a.k + (size_t)h * a.ld * 64;
  const float* vth = a.vt + (size_t)h * 64 * a.ld;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, l32 = lane & 31;
  const int kt = wave >> 1, qc = wave & 1;   // S^T piece: keys 32 kt .., queries 32 qc ..
  const int dt = wave >> 1, qc2 = wave & 1;  // dQ^T piece: dims 32 dt .., queries 32 qc2 ..
  const int ql = 32 * qc + l32;

  // Q and dO rows of this wave's queries into registers (through LDS)
  float qr[32], dr[32];
  {
    float t0[16], t1[16];
    fetch_rows(t0, a.q + (size_t)h * a.ld * 64, 64, base + q0, base + N);
    fetch_rows(t1, a.dout + h * 64, a.heads * 64, base + q0, base + N);
    store_rows(Ks, t0);
    store_rows(Vs, t1);
  }
  const float lse = ql < nq ? a.lse[(size_t)h * a.ld + base + q0 + ql] : 0.0f;
  const float dvq = ql < nq ? a.dv[(size_t)h * a.ld + base + q0 + ql] : 0.0f;
  float pk[16], pv[16];
  fetch_rows(pk, kh, 64, base, base + N);
  fetch_cols(pv, vth, a.ld, base);
  __syncthreads();
#pragma unroll
  for (int st = 0; st < 32; ++st) {
    qr[st] = Ks[ql][2 * st + half];
    dr[st] = Vs[ql][2 * st + half];
  }
  f32x16 gq = {};
  for (int k0 = 0; k0 < N; k0 += 64) {
    const int nk = min(64, N - k0);
    __syncthreads();  // the previous block's Ks, Vs, dSt are consumed
    store_rows(Ks, pk);
    store_cols(Vs, pv);
    __syncthreads();
    if (k0 + 64 < N) {
      fetch_rows(pk, kh, 64, base + k0 + 64, base + N);
      fetch_cols(pv, vth, a.ld, base + k0 + 64);
    }
    f32x16 sc = {}, dp = {};
#pragma unroll
    for (int st = 0; st < 32; ++st) {
      const int dd = 2 * st + half;
      sc = mfma_f32(Ks[32 * kt + l32][dd], qr[st], sc);
      dp = mfma_f32(Vs[32 * kt + l32][dd], dr[st], dp);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int kl = 32 * kt + acc_row(i, lane);
      const bool ok = ql < nq && kl < nk;
      const float p = ok ? __builtin_amdgcn_exp2f(sc[i] - lse) : 0.0f;
      dSt[kl][ql] = ok ? p * (dp[i] - dvq) : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int st = 0; st < 32; ++st) {
      const int kk = 2 * st + half;
      gq = mfma_f32(Ks[kk][32 * dt + l32], dSt[kk][32 * qc2 + l32], gq);
    }
  }
  const int D = a.heads * 64;
  const int q = 32 * qc2 + l32;
  if (q < nq) {
    float* row = a.dqkv + (size_t)(base + q0 + q) * 3 * D + h * 64 + 32 * dt;
#pragma unroll
    for (int i = 0; i < 16; ++i) row[acc_row(i, lane)] = gq[i] * 0.125f;
  }
}

// ---- Adam ---------------------------------------------------------------------------------

__global__ __launch_bounds__(TB) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                                                  float b1, float b2, float eps, float bc1, float bc2) {
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

int grid_for(long long n) {
  const long long b = (n + TB - 1) / TB;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

int last() { return hipGetLastError() == hipSuccess ? 0 : -5; }

}  // namespace

long long transpose_plan(TrDesc* d, int n) {
  long long tiles = 0;
  for (int i = 0; i < n; ++i) {
    d[i].tile0 = (int)tiles;
    tiles += (long long)cdiv(d[i].rows, 64) * cdiv(d[i].cols, 64);
  }
  return tiles;
}

int launch_transpose_batch(const TrDesc* d, int n, long long tiles, hipStream_t s) {
  if (n <= 0 || tiles <= 0) return 0;
  if (tiles > (1LL << 31) - 1) return -22;
  transpose_batch_kernel<<<(unsigned)tiles, TB, 0, s>>>(d, n);
  return last();
}

int launch_sum_chunks(const float* part, int nb, long long n, float* out, hipStream_t s) {
  // the four-wide form needs 16-byte aligned rows
  const bool v4 = n % 4 == 0 && ((uintptr_t)part & 15) == 0 && ((uintptr_t)out & 15) == 0;
  sum_chunks_kernel<<<grid_for(v4 ? n / 4 : n), TB, 0, s>>>(part, nb, n, out, v4);
  return last();
}

int launch_wgrad2(const WgradJob* jobs, int njobs, int rows, int kc, int nchunk, hipStream_t s) {
  if (njobs < 1 || njobs > 2 || kc <= 0 || nchunk <= 0 || nchunk > 65535 ||
      (size_t)(nchunk - 1) * kc >= (size_t)(rows > 0 ? rows : 1))
    return -22;
  WgradArgs a;
  memset(&a, 0, sizeof(a));
  a.rows = rows; a.kc = kc;
  int tiles = 0;
  for (int j = 0; j < njobs; ++j) {
    const WgradJob& w = jobs[j];
    // buffer-load byte offsets are 32-bit
    if ((long long)rows * (w.ldy > w.ldx ? w.ldy : w.ldx) * 4 + 64 >= (1LL << 31)) return -22;
    if (w.nout % 8 || w.nin % 8 || w.ldy % 4 || w.ldx % 4 || w.ldy < w.nout || w.ldx < w.nin ||
        (nchunk > 1 && (w.pstride < (long long)w.nout * w.nin || (w.bpart && w.bstride < w.nout))) ||
        (((uintptr_t)w.dy | (uintptr_t)w.x) & 15))
      return -22;
    WgradLayer& l = j ? a.l1 : a.l0;
    l.dy = w.dy; l.x = w.x; l.nout = w.nout; l.nin = w.nin; l.ldy = w.ldy; l.ldx = w.ldx;
    l.part = w.part; l.bpart = w.bpart; l.pstride = w.pstride; l.bstride = w.bstride;
    if (j == 1) a.tile1 = tiles;
    tiles += cdiv(w.nout, 128) * cdiv(w.nin, 128);
  }
  if (njobs == 1) a.tile1 = tiles;
  wgrad_kernel<<<dim3(tiles, nchunk), TB, 0, s>>>(a);
  return last();
}

int launch_wgrad(const float* dy, const float* x, int rows, int nout, int nin, int ldy, int ldx, int kc, int nchunk,
                 float* part, long long pstride, float* bpart, long long bstride, hipStream_t s) {
  WgradJob w;
  w.dy = dy; w.x = x; w.nout = nout; w.nin = nin; w.ldy = ldy; w.ldx = ldx;
  w.part = part; w.bpart = bpart; w.pstride = pstride; w.bstride = bstride;
  return launch_wgrad2(&w, 1, rows, kc, nchunk, s);
}

int ln_bwd_blocks(int rows) { return rows > 0 ? cdiv(rows, LN_WAVES) : 1; }

int launch_ln_bwd(const float* x, const float* g, const float* dy, const float* din, float* dout, float* part,
                  int max_blocks, int rows, int D, const int* rowmap, float* gb, hipStream_t s) {
  if (D <= 0 || D > 512 || rows < 0 || (rowmap && din != dout)) return -22;
  const int nblk = ln_bwd_blocks(rows);
  if (nblk > max_blocks) return -22;
  ln_bwd_kernel<<<nblk, LN_TB, 0, s>>>(x, g, dy, din, dout, part, rows, D, rowmap);
  if (int e = last()) return e;
  colsum_final_kernel<<<cdiv(2 * D, 64), TB, 0, s>>>(part, nblk, 2 * D, gb);
  return last();
}

int launch_pretrain_loss(const float* pred, const void* gt, int B, int H, int W, int C, float alpha, float* dpred,
                         double* part, int nblocks, hipStream_t s) {
  pretrain_loss_kernel<<<nblocks, TB, 0, s>>>(pred, gt, B, H, W, C, alpha, dpred, part);
  return last();
}

int launch_head_grad(const ReqDesc* reqs, int nreq, int Mh, int Mh_pad, int C, const float* dpred,
                     long long frame_elems, float* dhead, hipStream_t s) {
  head_grad_kernel<<<grid_for((long long)Mh_pad * 256 * C), TB, 0, s>>>(reqs, nreq, Mh, Mh_pad, C, dpred, frame_elems,
                                                                       dhead);
  return last();
}

int launch_attention_bwd(const float* q, const float* k, const float* vt, const float* o, const float* dout,
                         const float* lse, float* dv, float* dqkv, int M, int heads, int ld, const ReqDesc* reqs,
                         const int* work, int nwork, hipStream_t s) {
  // the block loaders' buffer offsets are 32-bit byte offsets into one head's
  // Q / K / V^T slab or into dout
  if ((long long)ld * 64 * 4 >= (1LL << 31) || (long long)ld * heads * 64 * 4 >= (1LL << 31) || M > ld) return -22;
  attn_bwd_dot_kernel<<<cdiv(M * heads, TB / 64), TB, 0, s>>>(o, dout, M, heads, ld, dv);
  if (int e = last()) return e;
  AttnBwdArgs a;
  a.q = q; a.k = k; a.vt = vt; a.dout = dout; a.lse = lse; a.dv = dv; a.dqkv = dqkv;
  a.heads = heads; a.ld = ld; a.reqs = reqs; a.work = work; a.nwork = nwork;
  attn_bwd_dkdv_kernel<<<dim3(nwork, heads), TB, 0, s>>>(a);
  if (int e = last()) return e;
  attn_bwd_dq_kernel<<<dim3(nwork, heads), TB, 0, s>>>(a);
  return last();
}

int launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2, float eps,
                float bc1, float bc2, hipStream_t s) {
  adam_kernel<<<grid_for(n), TB, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
  return last();
}

}  // namespace revo
