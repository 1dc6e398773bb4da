// Pretraining step of the recovery network (revo_train.h): FP32 forward
// pass that keeps the activations the backward pass needs, the RGB
// objective on the raw prediction (Sec. 3.4.2), reverse-mode gradients of
// every layer, and Adam (Sec. 4).  The forward pass runs the same kernels
// as inference (tubelet packing, GEMM epilogues with bias / positional
// embedding / Q-K-V split, attention, LayerNorm, head unpatchify); the
// backward pass adds transposes, column sums, LayerNorm, GELU and attention
// backward kernels (train.hip).  Every product of the backward pass is an
// FP32 MFMA GEMM: dX = dY W runs on the transposed weights, dW = dY^T X on
// transposed activations.
#include <string.h>

#include <cmath>
#include <vector>

#include "../../include/revo.h"
#include "../../include/revo_train.h"
#include "model.h"
#include "train.h"

using namespace revo;

namespace {

// offsets (in floats) of one linear layer in the weight blob
struct Lin {
  size_t w = 0, b = 0;
  int out = 0, in = 0;
};
struct BlockL {
  size_t ln1g, ln1b, ln2g, ln2b;
  Lin qkv, proj, fc1, fc2;
};
struct Layout {
  Lin emb, e2d, head;
  size_t encg, encb, decg, decb;
  std::vector<BlockL> enc, dec;
  size_t count = 0;
};

// the blob order of the weight file (emb, encoder blocks, enc norm, e2d,
// decoder blocks, dec norm, head; each matrix [out][in] then its bias)
Layout make_layout(int C, int T, int ne, int nd) {
  Layout L;
  size_t pos = 0;
  auto lin = [&](int out, int in) {
    Lin l;
    l.out = out; l.in = in;
    l.w = pos; pos += (size_t)out * in;
    l.b = pos; pos += out;
    return l;
  };
  auto vec = [&](int n) { const size_t o = pos; pos += n; return o; };
  auto block = [&](int D) {
    BlockL b;
    b.ln1g = vec(D); b.ln1b = vec(D);
    b.qkv = lin(3 * D, D);
    b.proj = lin(D, D);
    b.ln2g = vec(D); b.ln2b = vec(D);
    b.fc1 = lin(4 * D, D);
    b.fc2 = lin(D, 4 * D);
    return b;
  };
  const int De = 384, Dd = 192, Lt = T * 256 * C;
  L.emb = lin(De, Lt);
  for (int i = 0; i < ne; ++i) L.enc.push_back(block(De));
  L.encg = vec(De); L.encb = vec(De);
  L.e2d = lin(Dd, De);
  for (int i = 0; i < nd; ++i) L.dec.push_back(block(Dd));
  L.decg = vec(Dd); L.decb = vec(Dd);
  L.head = lin(Lt, Dd);
  L.count = pos;
  return L;
}

// saved activations of one Transformer block
struct BlockAct {
  float *xin, *a1, *q, *k, *vt, *lse, *o, *xmid, *a2, *h1, *g;  // g = GELU(h1), FC2's input
};

}  // namespace

struct revo_trainer {
  int dev = 0;
  hipStream_t s = nullptr;
  int C = 3, T = 2, k = 5, ne = 12, nd = 4, B = 1, H = 0, W = 0;
  int J = 0, gy = 0, gx = 0, P = 0, N = 0, Nal = 0, nfr = 0, Lt = 0;
  int M = 0, Mpad = 0, Mh = 0, Mh_pad = 0, ld = 0;
  int nwork_f = 0, nwork_b = 0, loss_blocks = 0, max_chunks = 0, ln_blocks = 0;
  float lr = 2e-4f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f, alpha = 0.01f;
  long long step = 0;
  Layout L;
  std::vector<void*> allocs;
  float *theta = nullptr, *grad = nullptr, *mom = nullptr, *vel = nullptr, *wT = nullptr, *zero = nullptr;
  ReqDesc* d_reqs = nullptr;
  std::vector<ReqDesc> h_reqs;
  int *d_work_f = nullptr, *d_work_b = nullptr, *d_rowmap = nullptr;
  float *U = nullptr, *xe = nullptr, *ae = nullptr, *zd = nullptr, *ahead = nullptr, *pred = nullptr;
  std::vector<BlockAct> act;  // ne encoder blocks, then nd decoder blocks
  float *dpred = nullptr, *dhead = nullptr, *dahead = nullptr, *lnpart = nullptr, *dxe = nullptr, *dz = nullptr;
  float *dH1 = nullptr, *da = nullptr, *dO = nullptr, *dqkv = nullptr;
  float *part = nullptr, *dvec = nullptr, *splitk = nullptr;
  size_t splitk_elems = 0;
  TrDesc* d_tr = nullptr;  // the weight transposes of a step
  // the weight gradients run on s2 beside the input-gradient chain on s:
  // ev_fork orders s2 after s, ev_p1 / ev_p2 mark a block's first and
  // second dW pair done, ev_join the last dW launch of the step
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_p1 = nullptr, ev_p2 = nullptr, ev_join = nullptr;
  float* dmid = nullptr;  // a block's midpoint gradient
  int ntr = 0;
  long long tr_tiles = 0;
  double* loss_part = nullptr;
  std::vector<double> h_loss_part;
};

namespace {

int alloc(revo_trainer* t, void** p, size_t bytes) {
  if (hipMalloc(p, bytes < 256 ? 256 : bytes) != hipSuccess) return REVO_ENOMEM;
  t->allocs.push_back(*p);
  return hipMemsetAsync(*p, 0, bytes < 256 ? 256 : bytes, t->s) == hipSuccess ? 0 : REVO_EDEVICE;
}
template <class X>
int alloc_n(revo_trainer* t, X** p, size_t n) {
  return alloc(t, reinterpret_cast<void**>(p), n * sizeof(X));
}

int align_up(int x, int a) { return (x + a - 1) / a * a; }

// out[m][n] = sum_k x[m][k] w[n][k] (FP32 GEMM, no bias)
int mm(revo_trainer* t, const float* x, const float* w, float* out, int M, int N, int K, int ldo) {
  GemmArgs a;
  memset(&a, 0, sizeof(a));
  a.M = M; a.N = N; a.K = K; a.X = x; a.W = w; a.bias = t->zero; a.out = out; a.ldo = ldo;
  return launch_gemm(P_FP32, EPI_STORE, X_DENSE, a, t->s);
}

// dW [out][in] = dY^T X over Mrows rows (dY [Mrows][out], X [Mrows][in]),
// db = column sums of dY.  The contraction runs over the token rows, and
// out x in is only a few output tiles, so it is split along the rows into S
// chunks of kc rows (one launch, grid.y = chunk) whose partial products are
// then summed in chunk order.
int weight_grad(revo_trainer* t, const float* dy, const float* x, int Mrows, const Lin& l, float* gblob) {
  int e;
  const int tiles = cdiv(l.out, 128) * cdiv(l.in, 128);
  int S = 512 / tiles;
  if (S > Mrows / 64) S = Mrows / 64;  // at least 64 rows (4 stages) per chunk
  if (S < 1) S = 1;
  const int kc = align_up(cdiv(Mrows, S), 16);
  S = cdiv(Mrows, kc);
  const long long nw = (long long)l.out * l.in;
  if (S == 1) return launch_wgrad(dy, x, Mrows, l.out, l.in, l.out, l.in, kc, 1, gblob + l.w, nw, gblob + l.b, 0, t->s2);
  if (l.b == l.w + (size_t)nw) {
    // the blob keeps a layer's bias right after its weights: chunk c's
    // partial dW and db are laid out the same way, and one sum covers both
    if ((size_t)S * (nw + l.out) > t->splitk_elems) return -22;
    if ((e = launch_wgrad(dy, x, Mrows, l.out, l.in, l.out, l.in, kc, S, t->splitk, nw + l.out, t->splitk + nw,
                          nw + l.out, t->s2)))
      return e;
    return launch_sum_chunks(t->splitk, S, nw + l.out, gblob + l.w, t->s2);
  }
  if ((size_t)S * nw > t->splitk_elems || S > t->max_chunks) return -22;
  if ((e = launch_wgrad(dy, x, Mrows, l.out, l.in, l.out, l.in, kc, S, t->splitk, nw, t->part, l.out, t->s2))) return e;
  if ((e = launch_sum_chunks(t->splitk, S, nw, gblob + l.w, t->s2))) return e;
  return launch_sum_chunks(t->part, S, l.out, gblob + l.b, t->s2);
}

// dW and db of two layers over the same Mrows rows in one launch (two
// independent products of one block's backward pass): the tiles of both
// share the split into S row chunks, then each layer's chunks are summed.
// Both layers keep their bias right after their weights in the blob.
int weight_grad2(revo_trainer* t, const float* dy0, const float* x0, const Lin& l0, const float* dy1,
                 const float* x1, const Lin& l1, int Mrows, float* gblob) {
  int e;
  const Lin* L[2] = {&l0, &l1};
  int tiles = 0;
  for (const Lin* l : L) tiles += cdiv(l->out, 128) * cdiv(l->in, 128);
  int S = 512 / tiles;
  if (S > Mrows / 64) S = Mrows / 64;  // at least 64 rows (4 stages) per chunk
  if (S < 1) S = 1;
  const int kc = align_up(cdiv(Mrows, S), 16);
  S = cdiv(Mrows, kc);
  WgradJob w[2];
  const float* dys[2] = {dy0, dy1};
  const float* xs[2] = {x0, x1};
  size_t off = 0;
  for (int j = 0; j < 2; ++j) {
    const Lin& l = *L[j];
    const long long nw = (long long)l.out * l.in;
    if (l.b != l.w + (size_t)nw) return -22;
    w[j].dy = dys[j]; w[j].x = xs[j]; w[j].nout = l.out; w[j].nin = l.in; w[j].ldy = l.out; w[j].ldx = l.in;
    if (S == 1) {
      w[j].part = gblob + l.w; w[j].pstride = nw; w[j].bpart = gblob + l.b; w[j].bstride = 0;
    } else {
      w[j].part = t->splitk + off; w[j].pstride = nw + l.out;
      w[j].bpart = t->splitk + off + nw; w[j].bstride = nw + l.out;
      off += (size_t)S * (nw + l.out);
    }
  }
  if (off > t->splitk_elems) return -22;
  if ((e = launch_wgrad2(w, 2, Mrows, kc, S, t->s2))) return e;
  if (S == 1) return 0;
  for (int j = 0; j < 2; ++j)
    if ((e = launch_sum_chunks(w[j].part, S, w[j].pstride, gblob + L[j]->w, t->s2))) return e;
  return 0;
}

// dX [Mrows][in] = dY W (dY [Mrows][out]) on the transposed weights
int input_grad(revo_trainer* t, const float* dy, const Lin& l, float* dx, int Mrows) {
  return mm(t, dy, t->wT + l.w, dx, Mrows, l.in, l.out, l.in);
}

// LayerNorm backward of rows [0, rows): adds dL/dx into dres, writes the
// gain and shift gradients
int ln_grad(revo_trainer* t, const float* x, size_t g_off, size_t b_off, const float* dy, const float* din, float* dout,
            int rows, int D, const int* rowmap) {
  if (b_off != g_off + (size_t)D) return -22;  // one sum writes both vectors
  return launch_ln_bwd(x, t->theta + g_off, dy, din, dout, t->lnpart, t->ln_blocks, rows, D, rowmap, t->grad + g_off,
                       t->s);
}

// s2 continues after everything enqueued on s so far
int fork_wgrad(revo_trainer* t) {
  return hipEventRecord(t->ev_fork, t->s) == hipSuccess && hipStreamWaitEvent(t->s2, t->ev_fork, 0) == hipSuccess
             ? 0
             : REVO_EDEVICE;
}
// ev marks the point s2 has reached; s waits for the latest mark of ev
int mark_wgrad(revo_trainer* t, hipEvent_t ev) { return hipEventRecord(ev, t->s2) == hipSuccess ? 0 : REVO_EDEVICE; }
int wait_wgrad(revo_trainer* t, hipEvent_t ev) {
  return hipStreamWaitEvent(t->s, ev, 0) == hipSuccess ? 0 : REVO_EDEVICE;
}

// forward of one block from its input A.xin into xout, saving what the
// backward pass reads (the residual adds read one buffer and write another,
// so no copies of the stream are made)
int block_fwd(revo_trainer* t, const BlockL& b, BlockAct& A, float* xout, int D, int heads) {
  int e;
  hipStream_t s = t->s;
  if ((e = launch_layernorm(P_FP32, A.xin, t->theta + b.ln1g, t->theta + b.ln1b, A.a1, t->Mpad, D, nullptr, 0, s)))
    return e;
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.reqs = t->d_reqs; g.nreq = t->B; g.channels = t->C; g.M = t->Mpad;
  GemmArgs q = g;
  q.X = A.a1; q.K = D; q.N = 3 * D; q.W = t->theta + b.qkv.w; q.bias = t->theta + b.qkv.b;
  q.q = A.q; q.k = A.k; q.vt = A.vt; q.heads = heads; q.ldqk = t->ld; q.ldv = t->ld;
  q.qscale = 1.4426950408889634f / 8.0f;
  if ((e = launch_gemm(P_FP32, EPI_QKV, X_DENSE, q, s))) return e;
  AttnArgs at;
  memset(&at, 0, sizeof(at));
  at.q = A.q; at.k = A.k; at.vt = A.vt; at.o = A.o; at.heads = heads; at.ldqk = t->ld; at.ldv = t->ld;
  at.reqs = t->d_reqs; at.nreq = t->B; at.work = t->d_work_f; at.nwork = t->nwork_f; at.lse = A.lse;
  if ((e = launch_attention(P_FP32, at, s))) return e;
  GemmArgs pr = g;
  pr.X = A.o; pr.K = D; pr.N = D; pr.W = t->theta + b.proj.w; pr.bias = t->theta + b.proj.b;
  pr.res = A.xin; pr.out = A.xmid; pr.ldo = D;
  if ((e = launch_gemm(P_FP32, EPI_RESIDUAL, X_DENSE, pr, s))) return e;
  if ((e = launch_layernorm(P_FP32, A.xmid, t->theta + b.ln2g, t->theta + b.ln2b, A.a2, t->Mpad, D, nullptr, 0, s)))
    return e;
  GemmArgs f1 = g;
  f1.X = A.a2; f1.K = D; f1.N = 4 * D; f1.W = t->theta + b.fc1.w; f1.bias = t->theta + b.fc1.b;
  f1.pre = A.h1; f1.out = A.g; f1.ldo = 4 * D;
  if ((e = launch_gemm(P_FP32, EPI_GELU_PRE, X_DENSE, f1, s))) return e;
  GemmArgs f2 = g;
  f2.X = A.g; f2.K = 4 * D; f2.N = D; f2.W = t->theta + b.fc2.w; f2.bias = t->theta + b.fc2.b;
  f2.res = A.xmid; f2.out = xout; f2.ldo = D;
  return launch_gemm(P_FP32, EPI_RESIDUAL, X_DENSE, f2, s);
}

// backward of one block: dx holds dL/d(block output) and becomes dL/d(input).
// The block's two dW pairs run on s2 while s carries on with the input
// gradients: the first pair reads dx and dH1, the second dmid and dqkv, so
// s waits for the first before it rewrites dx, and for the previous block's
// second before it rewrites dmid and dqkv.  dH1 is rewritten only after
// the previous block's first pair, which s waited for at that block's end.
int block_bwd(revo_trainer* t, const BlockL& b, const BlockAct& A, float* dx, int D, int heads) {
  int e;
  hipStream_t s = t->s;
  const int M = t->Mpad;
  // x_out = xmid + FC2(GELU(FC1(LN2(xmid))))
  {
    // dH1 = (dx W2) gelu'(h1), the GELU backward in the product's epilogue
    GemmArgs a;
    memset(&a, 0, sizeof(a));
    a.M = M; a.N = 4 * D; a.K = D; a.X = dx; a.W = t->wT + b.fc2.w; a.bias = t->zero;
    a.pre = A.h1; a.out = t->dH1; a.ldo = 4 * D;
    if ((e = launch_gemm(P_FP32, EPI_GELU_BWD, X_DENSE, a, s))) return e;
  }
  if ((e = fork_wgrad(t)) || (e = weight_grad2(t, dx, A.g, b.fc2, t->dH1, A.a2, b.fc1, M, t->grad)) ||
      (e = mark_wgrad(t, t->ev_p1)))
    return e;
  if ((e = input_grad(t, t->dH1, b.fc1, t->da, M))) return e;  // da2 = dH1 W1
  if ((e = wait_wgrad(t, t->ev_p2))) return e;                  // the previous block's dmid and dqkv readers
  if ((e = ln_grad(t, A.xmid, b.ln2g, b.ln2b, t->da, dx, t->dmid, M, D, nullptr))) return e;  // d(xmid)
  // xmid = xin + Proj(Attn(LN1(xin)))
  if ((e = input_grad(t, t->dmid, b.proj, t->dO, M))) return e;
  // the attention backward writes the rows of the batch's tokens only; the
  // alignment gaps between requests and past the last one, if any, must read
  // as zero gradient (the buffer is shared by the encoder and decoder widths)
  if (t->Nal != t->N || t->M != M)
    if (hipMemsetAsync(t->dqkv, 0, (size_t)M * 3 * D * 4, s) != hipSuccess) return REVO_EDEVICE;
  if ((e = launch_attention_bwd(A.q, A.k, A.vt, A.o, t->dO, A.lse, t->dvec, t->dqkv, M, heads, t->ld, t->d_reqs,
                                t->d_work_b, t->nwork_b, s)))
    return e;
  if ((e = input_grad(t, t->dqkv, b.qkv, t->da, M))) return e;
  if ((e = fork_wgrad(t)) || (e = weight_grad2(t, t->dmid, A.o, b.proj, t->dqkv, A.a1, b.qkv, M, t->grad)) ||
      (e = mark_wgrad(t, t->ev_p2)))
    return e;
  if ((e = wait_wgrad(t, t->ev_p1))) return e;  // the first pair has read dx
  return ln_grad(t, A.xin, b.ln1g, b.ln1b, t->da, t->dmid, dx, M, D, nullptr);
}

// the transposed weights the dX products read (every layer but the
// embedding, whose input gradient is not needed): one launch per step
int transpose_weights(revo_trainer* t) {
  return launch_transpose_batch(t->d_tr, t->ntr, t->tr_tiles, t->s);
}

int plan_transposes(revo_trainer* t) {
  std::vector<TrDesc> d;
  auto add = [&](size_t off, int rows, int cols) {
    TrDesc x;
    x.in = t->theta + off; x.out = t->wT + off;
    x.rows = rows; x.cols = cols; x.ld_in = cols; x.ld_out = rows; x.tile0 = 0;
    d.push_back(x);
  };
  auto lin = [&](const Lin& l) { add(l.w, l.out, l.in); };
  lin(t->L.e2d);
  // head: only the target time slot's rows take part; their transpose
  // [Dd][256 C] sits at the slot block's own offset
  add(t->L.head.w + (size_t)(t->T - 1) * 256 * t->C * t->L.head.in, 256 * t->C, t->L.head.in);
  for (auto* v : {&t->L.enc, &t->L.dec})
    for (const BlockL& b : *v) {
      lin(b.qkv); lin(b.proj); lin(b.fc1); lin(b.fc2);
    }
  t->tr_tiles = transpose_plan(d.data(), (int)d.size());
  t->ntr = (int)d.size();
  if (int e = alloc_n(t, &t->d_tr, d.size())) return e;
  // on the trainer's stream, after the allocation's clearing; d is local
  if (hipMemcpyAsync(t->d_tr, d.data(), d.size() * sizeof(TrDesc), hipMemcpyHostToDevice, t->s) != hipSuccess)
    return REVO_EDEVICE;
  return hipStreamSynchronize(t->s) == hipSuccess ? 0 : REVO_EDEVICE;
}

int run_step(revo_trainer* t, const revo_train_batch* bt, double* loss_out) {
  int e;
  hipStream_t s = t->s;
  const int De = 384, Dd = 192;
  const size_t esz = t->C == 3 ? 1 : 2;
  const size_t frame_bytes = (size_t)t->H * t->W * t->C * esz;
  // request descriptors: k references oldest first, the target last, padded
  // at the old end with the oldest reference to a multiple of T
  for (int r = 0; r < t->B; ++r) {
    ReqDesc& d = t->h_reqs[r];
    memset(&d, 0, sizeof(d));
    d.tok_off = r * t->Nal; d.head_off = r * t->P;
    d.H = t->H; d.W = t->W; d.gy = t->gy; d.gx = t->gx; d.P = t->P; d.J = t->J; d.nframes = t->nfr;
    const char* refs = (const char*)bt->refs + (size_t)r * t->k * frame_bytes;
    std::vector<const void*> seq;
    std::vector<long long> tim;
    for (int i = 0; i < t->k; ++i) {
      seq.push_back(refs + (size_t)i * frame_bytes);
      tim.push_back(bt->ref_idx[(size_t)r * t->k + i]);
    }
    seq.push_back((const char*)bt->target + (size_t)r * frame_bytes);
    tim.push_back(bt->t_target[r]);
    while ((int)seq.size() % t->T) {
      seq.insert(seq.begin(), seq.front());
      tim.insert(tim.begin(), tim.front());
    }
    for (int f = 0; f < t->nfr; ++f) d.frames[f] = seq[f];
    for (int j = 0; j < t->J; ++j) d.tau[j] = (float)(bt->t_target[r] - tim[(size_t)j * t->T]);
    d.mask = bt->mask + (size_t)r * t->H * t->W;
    d.pred = t->pred + (size_t)r * t->H * t->W * t->C;
  }
  if (hipMemcpyAsync(t->d_reqs, t->h_reqs.data(), t->B * sizeof(ReqDesc), hipMemcpyHostToDevice, s) != hipSuccess)
    return REVO_EDEVICE;

  // ---- forward ----
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.reqs = t->d_reqs; g.nreq = t->B; g.channels = t->C; g.M = t->Mpad;
  g.N = De; g.K = t->Lt; g.W = t->theta + t->L.emb.w; g.bias = t->theta + t->L.emb.b; g.out = t->xe; g.ldo = De;
  if ((e = launch_tubelet_pack(P_FP32, g, t->U, s))) return e;
  // each block reads its input from its own saved buffer: the embedding
  // writes the first encoder block's, every block the next one's and the
  // last block of a stack the stack's output (xe, zd)
  auto enc_in = [&](int i) { return i < t->ne ? t->act[i].xin : t->xe; };
  auto dec_in = [&](int i) { return i < t->nd ? t->act[t->ne + i].xin : t->zd; };
  GemmArgs ge = g;
  ge.X = t->U; ge.out = enc_in(0);
  if ((e = launch_gemm(P_FP32, EPI_PE, X_DENSE, ge, s))) return e;
  for (int i = 0; i < t->ne; ++i)
    if ((e = block_fwd(t, t->L.enc[i], t->act[i], enc_in(i + 1), De, 6))) return e;
  if ((e = launch_layernorm(P_FP32, t->xe, t->theta + t->L.encg, t->theta + t->L.encb, t->ae, t->Mpad, De, nullptr, 0,
                            s)))
    return e;
  GemmArgs e2 = g;
  e2.X = t->ae; e2.K = De; e2.N = Dd; e2.W = t->theta + t->L.e2d.w; e2.bias = t->theta + t->L.e2d.b; e2.out = dec_in(0);
  e2.ldo = Dd;
  if ((e = launch_gemm(P_FP32, EPI_PE, X_DENSE, e2, s))) return e;
  for (int i = 0; i < t->nd; ++i)
    if ((e = block_fwd(t, t->L.dec[i], t->act[t->ne + i], dec_in(i + 1), Dd, 3))) return e;
  if ((e = launch_layernorm(P_FP32, t->zd, t->theta + t->L.decg, t->theta + t->L.decb, t->ahead, t->Mh, Dd, t->d_reqs,
                            t->B, s)))
    return e;
  const size_t slot = (size_t)(t->T - 1) * 256 * t->C;  // target time slot: head rows slot .. slot + 256 C
  GemmArgs hd = g;
  hd.M = t->Mh; hd.X = t->ahead; hd.K = Dd; hd.N = 256 * t->C;
  hd.W = t->theta + t->L.head.w + slot * Dd; hd.bias = t->theta + t->L.head.b + slot;
  if ((e = launch_gemm(P_FP32, EPI_HEAD, X_DENSE, hd, s))) return e;

  // ---- loss ----
  if ((e = launch_pretrain_loss(t->pred, bt->target, t->B, t->H, t->W, t->C, t->alpha, t->dpred, t->loss_part,
                                t->loss_blocks, s)))
    return e;

  // ---- backward ----
  if (hipMemsetAsync(t->grad, 0, t->L.count * 4, s) != hipSuccess) return REVO_EDEVICE;
  if (hipMemsetAsync(t->dz, 0, (size_t)t->Mpad * Dd * 4, s) != hipSuccess) return REVO_EDEVICE;
  if ((e = transpose_weights(t))) return e;
  // the dW launches' marks start out passed (s2 is idle)
  if ((e = fork_wgrad(t)) || (e = mark_wgrad(t, t->ev_p1)) || (e = mark_wgrad(t, t->ev_p2))) return e;
  // head: o = LN_dec(z) W_slot^T + b_slot on the target rows
  if ((e = launch_head_grad(t->d_reqs, t->B, t->Mh, t->Mh_pad, t->C, t->dpred, (long long)t->H * t->W * t->C, t->dhead,
                            s)))
    return e;
  Lin hs;
  hs.out = 256 * t->C; hs.in = Dd;
  hs.w = t->L.head.w + slot * Dd; hs.b = t->L.head.b + slot;
  if ((e = fork_wgrad(t)) || (e = weight_grad(t, t->dhead, t->ahead, t->Mh_pad, hs, t->grad))) return e;
  if ((e = input_grad(t, t->dhead, hs, t->dahead, t->Mh_pad))) return e;
  if ((e = ln_grad(t, t->zd, t->L.decg, t->L.decb, t->dahead, t->dz, t->dz, t->Mh, Dd, t->d_rowmap))) return e;
  for (int i = t->nd - 1; i >= 0; --i)
    if ((e = block_bwd(t, t->L.dec[i], t->act[t->ne + i], t->dz, Dd, 3))) return e;
  // z0 = LN_enc(h) W_e2d^T + b + PE
  if ((e = fork_wgrad(t)) || (e = weight_grad(t, t->dz, t->ae, t->Mpad, t->L.e2d, t->grad))) return e;
  if ((e = input_grad(t, t->dz, t->L.e2d, t->da, t->Mpad))) return e;
  if (hipMemsetAsync(t->dxe, 0, (size_t)t->Mpad * De * 4, s) != hipSuccess) return REVO_EDEVICE;
  if ((e = ln_grad(t, t->xe, t->L.encg, t->L.encb, t->da, t->dxe, t->dxe, t->Mpad, De, nullptr))) return e;
  for (int i = t->ne - 1; i >= 0; --i)
    if ((e = block_bwd(t, t->L.enc[i], t->act[i], t->dxe, De, 6))) return e;
  // h0 = U W_emb^T + b + PE
  if ((e = fork_wgrad(t)) || (e = weight_grad(t, t->dxe, t->U, t->Mpad, t->L.emb, t->grad))) return e;
  // every dW launch is done before Adam reads the gradients
  if ((e = mark_wgrad(t, t->ev_join)) || (e = wait_wgrad(t, t->ev_join))) return e;

  // ---- Adam ----
  t->step += 1;
  const double bc1 = 1.0 - std::pow((double)t->b1, (double)t->step);
  const double bc2 = 1.0 - std::pow((double)t->b2, (double)t->step);
  if ((e = launch_adam(t->theta, t->grad, t->mom, t->vel, (long long)t->L.count, t->lr, t->b1, t->b2, t->eps,
                       (float)bc1, (float)bc2, s)))
    return e;
  if (hipMemcpyAsync(t->h_loss_part.data(), t->loss_part, t->loss_blocks * sizeof(double), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return REVO_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return REVO_EDEVICE;
  if (loss_out) {
    double l = 0.0;
    for (double v : t->h_loss_part) l += v;
    *loss_out = l;
  }
  return 0;
}

int setup(revo_trainer* t, const revo_train_config& c) {
  int e;
  const int De = 384, Dd = 192;
  t->Lt = t->T * 256 * t->C;
  t->L = make_layout(t->C, t->T, t->ne, t->nd);
  t->nfr = (t->k + 1 + t->T - 1) / t->T * t->T;
  t->J = t->nfr / t->T;
  t->gy = cdiv(t->H, 16); t->gx = cdiv(t->W, 16); t->P = t->gy * t->gx;
  t->N = t->J * t->P;
  t->Nal = align_up(t->N, 16);
  t->M = t->B * t->Nal;
  t->Mpad = align_up(t->M, 64);
  t->Mh = t->B * t->P;
  t->Mh_pad = align_up(t->Mh, 64);
  t->ld = t->Mpad + 64;
  t->loss_blocks = 256;
  t->max_chunks = cdiv(t->Mpad > t->Mh_pad ? t->Mpad : t->Mh_pad, 64);  // 64-row dW chunks
  const size_t n = t->L.count;
  if ((e = alloc_n(t, &t->theta, n)) || (e = alloc_n(t, &t->grad, n)) || (e = alloc_n(t, &t->mom, n)) ||
      (e = alloc_n(t, &t->vel, n)) || (e = alloc_n(t, &t->wT, n)) || (e = alloc_n(t, &t->zero, 4096)))
    return e;
  // uploads go on the trainer's stream (non-blocking), behind the clearing
  // of the buffers they fill; the end of set-up synchronizes it
  if (hipMemcpyAsync(t->theta, c.weights, n * 4, hipMemcpyHostToDevice, t->s) != hipSuccess) return REVO_EDEVICE;
  if ((e = alloc_n(t, &t->d_reqs, t->B))) return e;
  t->h_reqs.resize(t->B);
  // work lists: 128-query tiles (forward attention), 64-row blocks (backward)
  std::vector<int> wf, wb, rowmap;
  for (int r = 0; r < t->B; ++r) {
    for (int q = 0; q * 128 < t->N; ++q) wf.push_back((r << 16) | q);
    for (int q = 0; q * 64 < t->N; ++q) wb.push_back((r << 16) | q);
    for (int p = 0; p < t->P; ++p) rowmap.push_back(r * t->Nal + (t->J - 1) * t->P + p);
  }
  t->nwork_f = (int)wf.size();
  t->nwork_b = (int)wb.size();
  if ((e = alloc_n(t, &t->d_work_f, wf.size())) || (e = alloc_n(t, &t->d_work_b, wb.size())) ||
      (e = alloc_n(t, &t->d_rowmap, rowmap.size())))
    return e;
  if (hipMemcpyAsync(t->d_work_f, wf.data(), wf.size() * 4, hipMemcpyHostToDevice, t->s) != hipSuccess ||
      hipMemcpyAsync(t->d_work_b, wb.data(), wb.size() * 4, hipMemcpyHostToDevice, t->s) != hipSuccess ||
      hipMemcpyAsync(t->d_rowmap, rowmap.data(), rowmap.size() * 4, hipMemcpyHostToDevice, t->s) != hipSuccess ||
      hipStreamSynchronize(t->s) != hipSuccess)
    return REVO_EDEVICE;
  const size_t Mp = t->Mpad;
  if ((e = alloc_n(t, &t->U, Mp * t->Lt)) || (e = alloc_n(t, &t->xe, Mp * De)) || (e = alloc_n(t, &t->ae, Mp * De)) ||
      (e = alloc_n(t, &t->zd, Mp * Dd)) || (e = alloc_n(t, &t->ahead, (size_t)t->Mh_pad * Dd)) ||
      (e = alloc_n(t, &t->pred, (size_t)t->B * t->H * t->W * t->C)))
    return e;
  t->act.resize(t->ne + t->nd);
  for (int i = 0; i < t->ne + t->nd; ++i) {
    const int D = i < t->ne ? De : Dd, heads = i < t->ne ? 6 : 3;
    BlockAct& A = t->act[i];
    if ((e = alloc_n(t, &A.xin, Mp * D)) || (e = alloc_n(t, &A.a1, Mp * D)) ||
        (e = alloc_n(t, &A.q, (size_t)heads * t->ld * 64)) || (e = alloc_n(t, &A.k, (size_t)heads * t->ld * 64)) ||
        (e = alloc_n(t, &A.vt, (size_t)heads * t->ld * 64)) || (e = alloc_n(t, &A.lse, (size_t)heads * t->ld)) ||
        (e = alloc_n(t, &A.o, Mp * D)) || (e = alloc_n(t, &A.xmid, Mp * D)) || (e = alloc_n(t, &A.a2, Mp * D)) ||
        (e = alloc_n(t, &A.h1, Mp * 4 * D)) || (e = alloc_n(t, &A.g, Mp * 4 * D)))
      return e;
  }
  const size_t Mx = Mp > (size_t)t->Mh_pad ? Mp : (size_t)t->Mh_pad;
  t->ln_blocks = ln_bwd_blocks((int)Mx);
  const size_t widest = (size_t)(t->Lt > 4 * De ? t->Lt : 4 * De);
  if ((e = alloc_n(t, &t->dpred, (size_t)t->B * t->H * t->W * t->C)) ||
      (e = alloc_n(t, &t->dhead, (size_t)t->Mh_pad * 256 * t->C)) || (e = alloc_n(t, &t->dahead, (size_t)t->Mh_pad * Dd)) ||
      (e = alloc_n(t, &t->lnpart, (size_t)t->ln_blocks * 2 * 512)) || (e = alloc_n(t, &t->dxe, Mp * De)) || (e = alloc_n(t, &t->dz, Mp * Dd)) ||
      (e = alloc_n(t, &t->dH1, Mp * 4 * De)) || (e = alloc_n(t, &t->da, Mp * De)) || (e = alloc_n(t, &t->dmid, Mp * De)) ||
      (e = alloc_n(t, &t->dO, Mp * De)) || (e = alloc_n(t, &t->dqkv, Mp * 3 * De)) ||
      (e = alloc_n(t, &t->part, (size_t)t->max_chunks * widest)) || (e = alloc_n(t, &t->dvec, (size_t)6 * t->ld)) ||
      (e = alloc_n(t, &t->loss_part, t->loss_blocks)))
    return e;
  // split-K partial products: at most 512 / tiles chunks of out x in values
  t->splitk_elems = (size_t)512 * 128 * 128 + (size_t)64 * 1536 * 64;
  if ((e = alloc_n(t, &t->splitk, t->splitk_elems))) return e;
  t->h_loss_part.assign(t->loss_blocks, 0.0);
  if ((e = plan_transposes(t))) return e;
  return hipStreamSynchronize(t->s) == hipSuccess ? 0 : REVO_EDEVICE;
}

}  // namespace

extern "C" {

int revo_train_create(const revo_train_config* cfg, revo_trainer** out) {
  if (!cfg || !out) return REVO_EINVAL;
  *out = nullptr;
  revo_train_config c = *cfg;
  if (c.channels != 3 && c.channels != 1) return REVO_EINVAL;
  if (c.k < 1 || c.k > 7 || c.tubelet < 1 || c.tubelet > 4 || c.batch < 1 || c.height < 1 || c.width < 1)
    return REVO_EINVAL;
  if ((c.k + 1 + c.tubelet - 1) / c.tubelet * c.tubelet > REVO_MAX_FRAMES) return REVO_ENOTSUP;
  if (c.enc_depth == 0) c.enc_depth = 12;
  if (c.dec_depth == 0) c.dec_depth = 4;
  if (c.enc_depth < 0 || c.dec_depth < 0 || c.enc_depth > 64 || c.dec_depth > 64) return REVO_EINVAL;
  if ((long long)c.height * c.width > (1LL << 24) || c.batch > 4096) return REVO_EINVAL;
  const size_t n = weight_count(c.channels, c.tubelet, c.enc_depth, c.dec_depth);
  if (!c.weights || c.n_weights != n) return REVO_EINVAL;
  revo_trainer* t = new revo_trainer();
  t->dev = c.device;
  t->C = c.channels; t->T = c.tubelet; t->k = c.k; t->ne = c.enc_depth; t->nd = c.dec_depth;
  t->B = c.batch; t->H = c.height; t->W = c.width;
  t->lr = c.lr > 0 ? c.lr : 2e-4f;
  t->b1 = c.beta1 > 0 ? c.beta1 : 0.9f;
  t->b2 = c.beta2 > 0 ? c.beta2 : 0.999f;
  t->eps = c.eps > 0 ? c.eps : 1e-8f;
  t->alpha = c.tv_weight > 0 ? c.tv_weight : (c.tv_weight < 0 ? 0.0f : 0.01f);
  int rc = 0;
  if (hipSetDevice(t->dev) != hipSuccess || hipStreamCreateWithFlags(&t->s, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&t->s2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_p1, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_p2, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming) != hipSuccess) {
    rc = REVO_EDEVICE;
  } else {
    rc = setup(t, c);
  }
  if (rc) {
    revo_train_destroy(t);
    return rc;
  }
  *out = t;
  return 0;
}

int revo_train_step(revo_trainer* t, const revo_train_batch* b, double* loss) {
  if (!t || !b || !b->refs || !b->target || !b->mask || !b->ref_idx || !b->t_target) return REVO_EINVAL;
  if (hipSetDevice(t->dev) != hipSuccess) return REVO_EDEVICE;
  const int rc = run_step(t, b, loss);
  if (rc) {
    (void)hipStreamSynchronize(t->s);
    (void)hipStreamSynchronize(t->s2);
  }
  return rc;
}

static int copy_out(revo_trainer* t, const float* src, float* out, size_t n, size_t have) {
  if (!t || !out || n != have) return REVO_EINVAL;
  if (hipSetDevice(t->dev) != hipSuccess) return REVO_EDEVICE;
  if (hipStreamSynchronize(t->s) != hipSuccess || hipStreamSynchronize(t->s2) != hipSuccess ||
      hipMemcpy(out, src, n * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return REVO_EDEVICE;
  return 0;
}

int revo_train_get_weights(revo_trainer* t, float* out, size_t n) {
  return t ? copy_out(t, t->theta, out, n, t->L.count) : REVO_EINVAL;
}
int revo_train_get_grads(revo_trainer* t, float* out, size_t n) {
  return t ? copy_out(t, t->grad, out, n, t->L.count) : REVO_EINVAL;
}
int revo_train_get_pred(revo_trainer* t, float* out, size_t n) {
  return t ? copy_out(t, t->pred, out, n, (size_t)t->B * t->H * t->W * t->C) : REVO_EINVAL;
}

void revo_train_destroy(revo_trainer* t) {
  if (!t) return;
  (void)hipSetDevice(t->dev);
  if (t->s) (void)hipStreamSynchronize(t->s);
  if (t->s2) (void)hipStreamSynchronize(t->s2);
  for (void* p : t->allocs) (void)hipFree(p);
  for (hipEvent_t ev : {t->ev_fork, t->ev_p1, t->ev_p2, t->ev_join})
    if (ev) (void)hipEventDestroy(ev);
  if (t->s2) (void)hipStreamDestroy(t->s2);
  if (t->s) (void)hipStreamDestroy(t->s);
  delete t;
}

}  // extern "C"
