// Device-resident model weights, batch workspaces and the forward pass.
#pragma once
#include <vector>

#include "kernels.h"

namespace revo {

struct BlockW {
  const float *ln1_g, *ln1_b, *qkv_b, *proj_b, *ln2_g, *ln2_b, *fc1_b, *fc2_b;
  const void *qkv_w, *proj_w, *fc1_w, *fc2_w;
  // FP8 form: E4M3 weights and their per-output-row scales
  const uint8_t *qkv_w8 = nullptr, *proj_w8 = nullptr, *fc1_w8 = nullptr, *fc2_w8 = nullptr;
  const float *qkv_s = nullptr, *proj_s = nullptr, *fc1_s = nullptr, *fc2_s = nullptr;
};

// Activation-scale slots of the FP8 form: 4 per block (inputs of qkv, proj,
// fc1, fc2; encoder blocks first) and one for the encoder-to-decoder input.
enum { ACT_QKV = 0, ACT_PROJ = 1, ACT_FC1 = 2, ACT_FC2 = 3 };

struct ModelW {
  int C = 3, T = 2, De = 384, Dd = 192, He = 6, Hd = 3, ne = 12, nd = 4;
  Prec prec = P_BF16;
  float* master = nullptr;  // FP32 blob on the device (biases, LN parameters)
  void* ops = nullptr;      // operand-precision copy of the blob (matrices)
  size_t count = 0;
  const void *emb_w = nullptr, *e2d_w = nullptr, *head_w = nullptr;
  const float *emb_b = nullptr, *e2d_b = nullptr, *head_b = nullptr;
  const float *enc_g = nullptr, *enc_b = nullptr, *dec_g = nullptr, *dec_b = nullptr;
  std::vector<BlockW> enc, dec;
  size_t bytes = 0;
  // FP8 form
  uint8_t* ops8 = nullptr;        // E4M3 copy of the quantised matrices (blob offsets)
  float* wscale = nullptr;        // per-row weight scales
  const uint8_t* e2d_w8 = nullptr;
  const float* e2d_s = nullptr;
  float* act_scale = nullptr;     // [nact] per-tensor activation scales (device)
  unsigned* act_absmax = nullptr; // [nact] calibration maxima (float bits, device)
  int nact = 0;
  // FP8 attention: per block [3][heads] (Q, K, V) calibration maxima,
  // E8M0 exponents (127 + e) and inverse scales 2^-e of the E4M3 operands
  unsigned* attn_absmax = nullptr;
  int* attn_exp = nullptr;
  float* attn_inv = nullptr;
  int nattn = 0;
  int attn_off(bool dec, int block) const { return dec ? 3 * He * ne + 3 * Hd * block : 3 * He * block; }
  bool calibrated = false;
  int tub_len() const { return T * REVO_PATCH * REVO_PATCH * C; }
  int act_slot(bool dec, int block, int kind) const { return 4 * ((dec ? ne : 0) + block) + kind; }
  int act_e2d() const { return 4 * (ne + nd); }
};

size_t weight_count(int C, int T, int ne, int nd);
int model_load(ModelW& m, int C, int T, int ne, int nd, Prec p, const float* host_blob, size_t n, hipStream_t s);
void model_free(ModelW& m);

// Optional per-launch GPU timing with events on the launching stream.
enum ProfKind { PK_ATTN = 0, PK_GEMM = 1, PK_OTHER = 2, PK_FORWARD = 3, PK_N = 4 };
struct Prof {
  bool on = false;
  bool attn_only = false;  // only attention launches and whole passes
  std::vector<hipEvent_t> pool;
  struct Rec { int a, b, kind; double flop; };
  std::vector<Rec> recs;
  int used = 0;
  double ms[PK_N] = {0, 0, 0, 0};
  double flop[PK_N] = {0, 0, 0, 0};
  long long count[PK_N] = {0, 0, 0, 0};
};
int prof_init(Prof& p, int events);
void prof_free(Prof& p);
// Adds the finished batch's records to the totals (call after the stream synchronised).
int prof_collect(Prof& p);

// Activation buffers for one batch of one modality.  Token rows are the
// batch's requests one after the other, each starting at a multiple of 8; q/k/vt carry ld >= cap + 64 rows so
// the last key block of any request stays inside the (zeroed) allocation.
constexpr int WS_SLOTS = 2;    // batches in flight per workspace (host descriptor copies)
constexpr int WS_BUCKETS = 4;  // graph capacity buckets: cap/8, cap/4, cap/2, cap tokens

struct Workspace {
  int cap = 0, head_cap = 0, ld = 0, max_req = 0, max_work = 0;
  Prec prec = P_BF16;
  float* h = nullptr;
  void *a = nullptr, *q = nullptr, *k = nullptr, *vt = nullptr, *o = nullptr, *hid = nullptr, *ahead = nullptr;
  float* z = nullptr;
  ReqDesc* d_reqs = nullptr;
  int* d_work = nullptr;
  int* d_hdr = nullptr;                  // live batch shape (BatchHdr)
  ReqDesc* h_reqs_slot[WS_SLOTS] = {};   // pinned host descriptors, one set per batch in flight
  int* h_work_slot[WS_SLOTS] = {};
  int* h_hdr_slot[WS_SLOTS] = {};
  ReqDesc* h_reqs = nullptr;             // = h_reqs_slot[0] (single-batch callers)
  hipGraphExec_t graph[WS_BUCKETS] = {};
  size_t bytes = 0;
  Prof prof;
};

size_t workspace_bytes(const ModelW& m, int cap, int max_req);
int workspace_alloc(Workspace& w, const ModelW& m, int cap, int max_req, hipStream_t s);
void workspace_free(Workspace& w);

// Tokens of one request at frame size H x W.
int request_tokens(int H, int W, int J);
// Token rows a request starts on: a V^T key group of 16 (BF16 attention) or
// of 64 (FP8 attention).
inline int token_align(Prec p) { return p == P_FP8 ? 64 : 16; }

// Runs the network for w.h_reqs_slot[slot][0 .. nrec) and the composite for
// entries [0 .. nall) (entries nrec.. are clean frames: copy only).  The
// caller fills frames/mask/outputs/size fields; offsets are set here.  The
// slot's host descriptors must not be reused before this batch completes.
// With use_graph (and profiling off) the launches replay a graph captured
// once per capacity bucket; the batch shape then comes from device memory.
// record: run the BF16 network and raise the activation maxima of the FP8
// form's product inputs (calibration); never replayed from a graph.
int forward(const ModelW& m, Workspace& w, int slot, int nrec, int nall, int composite, bool use_graph,
            hipStream_t s, bool record = false);
// Turn the recorded maxima into activation scales and switch the FP8 form on.
int model_finish_calibration(ModelW& m, hipStream_t s);
int model_reset_calibration(ModelW& m, hipStream_t s);

}  // namespace revo
