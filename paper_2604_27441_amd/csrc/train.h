// Host launchers of the pretraining-step kernels (train.hip).
#pragma once
#include "kernels.h"

namespace revo {

// One block of a batched transpose: out[c][r] = in[r][c] for r < rows,
// c < cols (row pitches ld_in, ld_out); its 64 x 64 tiles are numbers
// tile0 .. tile0 + cdiv(rows, 64) cdiv(cols, 64) - 1 of the launch.
struct TrDesc {
  const float* in;
  float* out;
  int rows, cols, ld_in, ld_out, tile0;
};
// Fills tile0 of the n descriptors and returns the launch's tile count.
long long transpose_plan(TrDesc* d, int n);
// Every listed transpose in one launch (d: n device-resident descriptors
// in tile0 order, tiles their total).
int launch_transpose_batch(const TrDesc* d, int n, long long tiles, hipStream_t s);
// out[i] = sum_b part[b n + i] for b = 0 .. nb-1 in order.
int launch_sum_chunks(const float* part, int nb, long long n, float* out, hipStream_t s);
// Weight-gradient chunks: part[c pstride + o nin + i] = sum over rows m of
// chunk c (rows c kc .. c kc + kc - 1 below rows) of dy[m][o] x[m][i]; with
// bpart, also bpart[c bstride + o] = the chunk's sum of dy[m][o].  Column
// counts multiple of 8, row pitches of 4, operands 16-byte aligned; every
// chunk holds rows.
int launch_wgrad(const float* dy, const float* x, int rows, int nout, int nin, int ldy, int ldx, int kc, int nchunk,
                 float* part, long long pstride, float* bpart, long long bstride, hipStream_t s);
// One weight-gradient product of launch_wgrad2 (fields as launch_wgrad's).
struct WgradJob {
  const float* dy;
  const float* x;
  int nout, nin, ldy, ldx;
  float* part;
  float* bpart;
  long long pstride, bstride;
};
// One or two weight-gradient products over the same rows and chunks in one
// launch (the tiles of both fill the GPU together).
int launch_wgrad2(const WgradJob* jobs, int njobs, int rows, int kc, int nchunk, hipStream_t s);
// LayerNorm backward (y = LN(x) g + b, eps 1e-6) of rows [0, rows):
// dout[row] = din[row] + dL/dx (din == dout: in place; another buffer only
// without rowmap), gb[0, D) = the gain gradient and gb[D, 2D) the shift
// gradient (column sums over the rows; zeros for rows == 0).  part holds
// ln_bwd_blocks(rows) <= max_blocks partial rows of 2D floats.  With rowmap,
// dy row i belongs to x / din / dout row rowmap[i].
int ln_bwd_blocks(int rows);
int launch_ln_bwd(const float* x, const float* g, const float* dy, const float* din, float* dout, float* part,
                  int max_blocks, int rows, int D, const int* rowmap, float* gb, hipStream_t s);
// Batch loss mean_b [MSE + alpha TV(pred)] and its gradient dpred; part
// receives nblocks partial sums of the loss.
int launch_pretrain_loss(const float* pred, const void* gt, int B, int H, int W, int C, float alpha, float* dpred,
                         double* part, int nblocks, hipStream_t s);
// Dense head-output gradient [Mh_pad][256 C] of the target slot from dpred
// (frames of frame_elems values each, request order).
int launch_head_grad(const ReqDesc* reqs, int nreq, int Mh, int Mh_pad, int C, const float* dpred,
                     long long frame_elems, float* dhead, hipStream_t s);
// Attention backward from the saved forward (q scaled by log2(e)/8, k, v^T,
// o, base-2 log normalisers lse) and dout: dqkv [M][3 heads 64]; dv is a
// [heads][ld] scratch; work lists (request << 16) | 64-row block.
int launch_attention_bwd(const float* q, const float* k, const float* vt, const float* o, const float* dout,
                         const float* lse, float* dv, float* dqkv, int M, int heads, int ld, const ReqDesc* reqs,
                         const int* work, int nwork, hipStream_t s);
int launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2, float eps,
                float bc1, float bc2, hipStream_t s);

}  // namespace revo
