// Device-side request descriptors and host launchers of the recovery kernels.
#pragma once
#include "common.h"

#define REVO_MAX_FRAMES 9
#define REVO_PATCH 16

namespace revo {

// One request of a batch, as the kernels see it (lives in device memory).
// Token rows of request r are [tok_off, tok_off + J * P): tubelet j, patch
// row y, column x sits at tok_off + j * P + y * gx + x.
struct ReqDesc {
  int tok_off;          // first token row in the batch
  int head_off;         // first row in the compact target-tubelet buffer
  int H, W;             // frame size in pixels
  int gy, gx, P;        // patch grid: ceil(H/16), ceil(W/16), gy * gx
  int J;                // tubelets per request
  int nframes;          // J * T frames, oldest first, the target last
  int pad_;
  float tau[REVO_MAX_FRAMES];           // temporal distance of tubelet j
  const void* frames[REVO_MAX_FRAMES];  // u8 HWC (C = 3) or u16 HW (C = 1)
  const uint8_t* mask;                  // target loss mask, H * W, 1 = lost
  float* pred;                          // H * W * C prediction, model units
  void* out_i;                          // u8 HWC / u16 HW output (nullable)
  float* out_f;                         // float output (nullable)
};

// GEMM epilogues.  The product is C^T[n][m] = sum_k W[n][k] X[m][k].
enum EpiMode {
  EPI_STORE = 0,     // out[m][n] = acc + bias[n]                (OutT)
  EPI_RESIDUAL = 1,  // out[m][n] = res[m][n] + acc + bias[n]   (fp32)
  EPI_GELU = 2,      // out[m][n] = gelu(acc + bias[n])          (OutT)
  EPI_QKV = 3,       // q/k [h][m][64] (q scaled), vt [h][64][ldv]
  EPI_PE = 4,        // out[m][n] = acc + bias[n] + PE(token m, n)  (fp32)
  EPI_HEAD = 5,      // pred pixel of compact target row m, slot column n
  // FP32 operands only (the pretraining step):
  EPI_GELU_PRE = 6,  // pre[m][n] = acc + bias[n], out[m][n] = gelu(pre[m][n])
  EPI_GELU_BWD = 7,  // out[m][n] = (acc + bias[n]) gelu'(pre[m][n])
};

enum XMode {
  X_DENSE = 0,       // X [M][K] row-major
  X_GATHER = 1,      // tubelet vectors gathered from the request's frames
};

// Batch shape in device memory (read by kernels launched with grids sized
// for a capacity, e.g. from a captured graph): rows past the live counts exit.
enum BatchHdr { HDR_M = 0, HDR_MH = 1, HDR_NREC = 2, HDR_NALL = 3, HDR_NWORK = 4, HDR_NWORK_LAST = 5, HDR_N = 8 };

struct GemmArgs {
  int M, N, K;       // M sizes the grid; the live row count is *dyn_m when set
  const int* dyn_m;  // nullable
  const int* dyn_nreq;  // nullable: live request count for the gather / PE / head lookups
  const void* X;     // X_DENSE: [M][K] operand elements
  const void* W;     // [N][K] operand elements
  const float* bias; // [N]
  void* out;         // EPI_STORE / GELU / PE: [M][ldo]; RESIDUAL: fp32 [M][ldo]
  int ldo;
  const float* res;  // EPI_RESIDUAL: out = res + acc + bias ([M][ldo]; nullable: res = out, in place)
  float* pre;        // EPI_GELU_PRE (written) / EPI_GELU_BWD (read): fp32 [M][ldo] pre-activations
  // EPI_QKV
  void* q; void* k; void* vt; int heads; int ldqk; int ldv; float qscale;
  // FP8 operands: acc * wscale[n] * (*xscale) + bias[n]; an FP8 result is
  // stored as value / (*out_scale)
  const float* wscale; const float* xscale; const float* out_scale;
  // EPI_QKV with E4M3 outputs (FP8 attention): per-head inverse scales
  // 2^-e, [3][heads] (Q, K, V); V^T columns in fp8_vt_col order
  const float* head_inv;
  // gather / PE / head
  const ReqDesc* reqs; int nreq; int channels;
};

constexpr int ATTN_TARGET_TILE = 0x8000;

struct AttnArgs {
  const void* q;     // [heads][ldqk rows][64], pre-scaled by log2(e)/sqrt(64)
  const void* k;     // [heads][ldqk rows][64]
  const void* vt;    // [heads][64][ldv]
  void* o;           // [M][heads * 64]
  int heads, ldqk, ldv;
  const ReqDesc* reqs; int nreq;
  // per workgroup: (request << 16) | q-tile, with ATTN_TARGET_TILE set for a
  // q-tile of the request's target tubelet only (queries from (J-1)*P on)
  const int* work;
  int nwork;         // sizes the grid; the live count is *dyn_nwork when set
  const int* dyn_nwork;  // nullable
  const int* dyn_nreq;   // nullable
  const float* o_scale;  // nullable: store o / (*o_scale) as FP8 E4M3
  float* lse;            // nullable (FP32): [heads][ldqk] base-2 log of each query's normaliser
  // FP8 attention: E8M0 exponents (127 + e, scale 2^e) of Q, K, V, [3][heads]
  const int* qkv_exp;
};

// Column position, within its aligned group of 64 keys, at which the FP8
// attention kernel's V^T holds key t: the order in which a lane's 32
// probabilities (two 32-key score subtiles, rows (i / 4) 8 + half 4 + i % 4)
// meet the 32 consecutive k of its half of a 32x32x64 FP8 product.
__host__ __device__ inline int fp8_vt_col(int t) {
  return (t & ~63) | (((t >> 2) & 1) << 5) | (((t >> 5) & 1) << 4) | (((t >> 3) & 3) << 2) | (t & 3);
}

int launch_gemm(Prec prec, int epi, int xmode, const GemmArgs& a, hipStream_t s);
// Tubelet vectors of the requests in a (reqs, nreq, M, K = tubelet length,
// channels, dyn_m / dyn_nreq) written to out as a dense [M][K] operand
// (float for P_FP32, bfloat16 otherwise).
int launch_tubelet_pack(Prec prec, const GemmArgs& a, void* out, hipStream_t s);
int launch_attention(Prec prec, const AttnArgs& a, hipStream_t s);
// Attention of one request of ntok tokens whose descriptor and q-tile work
// list live in a fixed per-device workspace instead of allocated memory:
// no allocation, no host copy, no synchronisation.  At most
// ATTN_NOALLOC_MAX_TILES q-tiles of 128 tokens (-7 beyond).
constexpr int ATTN_NOALLOC_MAX_TILES = ATTN_TARGET_TILE - 1;
int launch_attention_noalloc(Prec prec, const void* q, const void* k, const void* vt, void* o, int heads, int ntok,
                             int ld, hipStream_t s);
// y = LN(x) * g + b over rows of length D.  With reqs set, output row i is
// the target-tubelet token (i - head_off) of the request owning compact row i.
int launch_layernorm(Prec out_prec, const float* x, const float* g, const float* b,
                     void* y, int rows, int D, const ReqDesc* reqs, int nreq, hipStream_t s,
                     const int* dyn_rows = nullptr, const int* dyn_nreq = nullptr);
// Output frames.  Requests with a null mask are clean frames (copied).  With
// composite == 0 every pixel of a recovered frame takes the prediction.
// y = LN(x) * g + b stored as FP8 E4M3 of y / (*out_scale) (FP8 form).
int launch_layernorm_fp8(const float* x, const float* g, const float* b, uint8_t* y, const float* out_scale,
                         int rows, int D, hipStream_t s, const int* dyn_rows = nullptr);
// Per-row FP8 quantisation of a float matrix: scale[r] = max|W[r][:]| / 448
// (1 for an all-zero row), W8[r][c] = E4M3(W[r][c] / scale[r]).
int launch_quantize_rows(const float* w, int rows, int cols, uint8_t* w8, float* scale, hipStream_t s);
// Calibration: atomically raise *slot (float bits) to max |x| over the rows
// of [rows x D] that hold tokens of the batch's requests (alignment gaps skipped).
int launch_absmax(const __bf16* x, int rows, int D, const ReqDesc* reqs, int nreq, unsigned* slot, hipStream_t s);
// scale[i] = absmax[i] / 448 (1 where nothing was recorded).
int launch_scales_from_absmax(const unsigned* absmax, float* scale, int n, hipStream_t s);
// Calibration of the FP8 attention: raise slots[h], slots[heads + h],
// slots[2 heads + h] to max |Q|, |K|, |V| of head h over the live tokens of
// the BF16 buffers q, k [heads][ld][64] and vt [heads][64][ld] (V^T columns
// in the BF16 kernel's bits-2-and-3 order).
int launch_attn_absmax(const __bf16* q, const __bf16* k, const __bf16* vt, int heads, int ld, int rows,
                       const ReqDesc* reqs, int nreq, unsigned* slots, hipStream_t s);
// Power-of-two scales 2^e, e = ceil(log2(absmax / 448)) (0 where nothing was
// recorded): exps[i] = 127 + e (E8M0), inv[i] = 2^-e.
int launch_attn_scales(const unsigned* absmax, int* exps, float* inv, int n, hipStream_t s);
int launch_composite(const ReqDesc* reqs, int nreq, int channels, int max_pixels, int composite, hipStream_t s,
                     const int* dyn_nreq = nullptr);
int launch_convert(Prec prec, const float* src, void* dst, long long n, hipStream_t s);
// Frame metrics of B prediction / ground-truth frames (kind 0 u8, 1 u16, 2
// float; H x W x C each, contiguous); out [B][8] doubles.
int launch_frame_metrics(int kind, const void* pred, const void* gt, int B, int H, int W, int C, double* out,
                         hipStream_t s);
// RGB-D unprojection (depth [B][H][W] u16 mm -> float4 points [B][H][W]) and
// z-buffered rendering of a new view (pose: R|t row-major 3 x 4, intrinsics
// fx, fy, cx, cy; both host arrays).
int launch_unproject(const uint16_t* depth, int B, int H, int W, const float* intr, float* pts, hipStream_t s);
int launch_render_view(const float* pts, const uint8_t* rgb, int B, int H, int W, const float* pose,
                       const float* intr, int Ho, int Wo, unsigned long long* zbuf, uint8_t* rgb_out,
                       uint16_t* depth_out, hipStream_t s);
int launch_fill_zero(void* p, long long bytes, hipStream_t s);

// row -> request lookup over the ascending tok_off (or head_off) values
__device__ inline int find_req_tok(const ReqDesc* r, int n, int m) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (r[mid].tok_off <= m) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ inline int find_req_head(const ReqDesc* r, int n, int m) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (r[mid].head_off <= m) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace revo
