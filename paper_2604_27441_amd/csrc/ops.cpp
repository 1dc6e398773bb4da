// Single-kernel entry points (revo_ops.h): thin launch wrappers over the
// kernels the forward pass uses, for per-kernel checks.
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/revo.h"
#include "../../include/revo_ops.h"
#include "kernels.h"

using namespace revo;

namespace {

bool prec_of(int precision, Prec* p) {
  if (precision == REVO_FP32) { *p = P_FP32; return true; }
  if (precision == REVO_BF16) { *p = P_BF16; return true; }
  return false;
}

int epi_of(int epilogue) {
  switch (epilogue) {
    case REVO_EPI_STORE: return EPI_STORE;
    case REVO_EPI_RESIDUAL: return EPI_RESIDUAL;
    case REVO_EPI_GELU: return EPI_GELU;
  }
  return -1;
}

}  // namespace

extern "C" {

int revo_op_linear(int precision, int epilogue, const void* x, const void* w, const float* bias, void* out, int M,
                   int N, int K, void* stream) {
  Prec p;
  if (!prec_of(precision, &p)) return REVO_ENOTSUP;
  if (M < 0 || N <= 0 || K <= 0 || !x || !w || !bias || !out) return REVO_EINVAL;
  if (N % 64 || K % (p == P_BF16 ? 64 : 32)) return REVO_EINVAL;
  int epi;
  switch (epilogue) {
    case REVO_EPI_STORE: epi = EPI_STORE; break;
    case REVO_EPI_RESIDUAL: epi = EPI_RESIDUAL; break;
    case REVO_EPI_GELU: epi = EPI_GELU; break;
    default: return REVO_EINVAL;
  }
  GemmArgs a;
  memset(&a, 0, sizeof(a));
  a.M = M; a.N = N; a.K = K; a.X = x; a.W = w; a.bias = bias; a.out = out; a.ldo = N;
  return launch_gemm(p, epi, X_DENSE, a, (hipStream_t)stream);
}

int revo_op_linear_fp8(int epilogue, const void* x8, const void* w8, const float* wscale, const float* xscale,
                       const float* bias, void* out, const float* out_scale, int M, int N, int K, void* stream) {
  const int epi = epi_of(epilogue);
  if (epi < 0 || M < 0 || N <= 0 || K <= 0 || !x8 || !w8 || !wscale || !xscale || !bias || !out) return REVO_EINVAL;
  if (N % 64 || K % 64 || (epi == EPI_GELU && !out_scale)) return REVO_EINVAL;
  GemmArgs a;
  memset(&a, 0, sizeof(a));
  a.M = M; a.N = N; a.K = K; a.X = x8; a.W = w8; a.bias = bias; a.out = out; a.ldo = N;
  a.wscale = wscale; a.xscale = xscale; a.out_scale = out_scale;
  return launch_gemm(P_FP8, epi, X_DENSE, a, (hipStream_t)stream);
}

int revo_op_layernorm(int precision, const float* x, const float* g, const float* b, void* y, int rows, int D,
                      void* stream) {
  Prec p;
  if (!prec_of(precision, &p)) return REVO_ENOTSUP;
  if (rows < 0 || D <= 0 || D > 512 || !x || !g || !b || !y) return REVO_EINVAL;
  return launch_layernorm(p, x, g, b, y, rows, D, nullptr, 0, (hipStream_t)stream);
}

int revo_op_attention(int precision, const void* q, const void* k, const void* vt, void* o, int heads, int ntok,
                      int ld, void* stream) {
  Prec p;
  if (!prec_of(precision, &p)) return REVO_ENOTSUP;
  if (heads <= 0 || ntok <= 0 || ld < ntok + 64 || !q || !k || !vt || !o) return REVO_EINVAL;
  if (ld % 16) return REVO_EINVAL;  // 16-byte aligned vt rows, whole key groups of 16
  const int ntile = (ntok + 127) / 128;
  if (ntile >= ATTN_TARGET_TILE) return REVO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // one request covering all tokens; descriptor and work list in device memory
  ReqDesc h;
  memset(&h, 0, sizeof(h));
  h.J = 1; h.P = ntok; h.gy = 1; h.gx = ntok; h.H = 1; h.W = ntok; h.nframes = 1;
  ReqDesc* d = nullptr;
  int* work = nullptr;
  if (hipMalloc(&d, sizeof(ReqDesc)) != hipSuccess) return REVO_ENOMEM;
  if (hipMalloc(&work, ntile * sizeof(int)) != hipSuccess) { (void)hipFree(d); return REVO_ENOMEM; }
  int* hw = new int[ntile];
  for (int i = 0; i < ntile; ++i) hw[i] = i;
  int rc = 0;
  if (hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(work, hw, ntile * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    rc = REVO_EDEVICE;
  delete[] hw;
  if (!rc) {
    AttnArgs a;
    memset(&a, 0, sizeof(a));
    a.q = q; a.k = k; a.vt = vt; a.o = o; a.heads = heads; a.ldqk = ld; a.ldv = ld;
    a.reqs = d; a.nreq = 1; a.work = work; a.nwork = ntile;
    rc = launch_attention(p, a, s);
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = REVO_EDEVICE;
  }
  (void)hipFree(d);
  (void)hipFree(work);
  return rc;
}

int revo_op_attention_fp8(const void* q8, const void* k8, const void* vt8, void* o, int heads, int ntok, int ld,
                          const int* exps, void* stream) {
  if (heads <= 0 || heads > 64 || ntok <= 0 || ld < ntok + 64 || !q8 || !k8 || !vt8 || !o || !exps) return REVO_EINVAL;
  if (ld % 64) return REVO_EINVAL;  // whole 64-key groups of V^T, 16-byte aligned rows
  for (int i = 0; i < 3 * heads; ++i)
    if (exps[i] < -100 || exps[i] > 100) return REVO_EINVAL;
  const int ntile = (ntok + 127) / 128;
  if (ntile >= ATTN_TARGET_TILE) return REVO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  ReqDesc h;
  memset(&h, 0, sizeof(h));
  h.J = 1; h.P = ntok; h.gy = 1; h.gx = ntok; h.H = 1; h.W = ntok; h.nframes = 1;
  std::vector<int> hw(ntile);
  for (int i = 0; i < ntile; ++i) hw[i] = i;
  std::vector<int> he(3 * heads);
  for (int i = 0; i < 3 * heads; ++i) he[i] = 127 + exps[i];
  ReqDesc* d = nullptr;
  int *work = nullptr, *de = nullptr;
  int rc = 0;
  if (hipMalloc(&d, sizeof(ReqDesc)) != hipSuccess || hipMalloc(&work, ntile * sizeof(int)) != hipSuccess ||
      hipMalloc(&de, 3 * heads * sizeof(int)) != hipSuccess)
    rc = REVO_ENOMEM;
  if (!rc && (hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(work, hw.data(), ntile * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(de, he.data(), 3 * heads * sizeof(int), hipMemcpyHostToDevice) != hipSuccess))
    rc = REVO_EDEVICE;
  if (!rc) {
    AttnArgs a;
    memset(&a, 0, sizeof(a));
    a.q = q8; a.k = k8; a.vt = vt8; a.o = o; a.heads = heads; a.ldqk = ld; a.ldv = ld;
    a.reqs = d; a.nreq = 1; a.work = work; a.nwork = ntile; a.qkv_exp = de;
    rc = launch_attention(P_FP8, a, s);
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = REVO_EDEVICE;
  }
  if (d) (void)hipFree(d);
  if (work) (void)hipFree(work);
  if (de) (void)hipFree(de);
  return rc;
}

int revo_op_attention_noalloc(int precision, const void* q, const void* k, const void* vt, void* o, int heads,
                              int ntok, int ld, void* stream) {
  Prec p;
  if (!prec_of(precision, &p)) return REVO_ENOTSUP;
  if (heads <= 0 || ntok <= 0 || ld < ntok + 64 || !q || !k || !vt || !o) return REVO_EINVAL;
  if (ld % 16) return REVO_EINVAL;
  if ((ntok + 127) / 128 > ATTN_NOALLOC_MAX_TILES) return REVO_E2BIG;
  return launch_attention_noalloc(p, q, k, vt, o, heads, ntok, ld, (hipStream_t)stream);
}

int revo_op_convert(int precision, const float* src, void* dst, long long n, void* stream) {
  Prec p;
  if (precision == REVO_FP8) p = P_FP8;
  else if (!prec_of(precision, &p)) return REVO_ENOTSUP;
  if (n < 0 || !src || !dst) return REVO_EINVAL;
  return launch_convert(p, src, dst, n, (hipStream_t)stream);
}

int revo_op_frame_metrics(int kind, const void* pred, const void* gt, int batch, int height, int width,
                          int channels, double* out, void* stream) {
  if (kind < REVO_FRAME_U8 || kind > REVO_FRAME_F32 || batch <= 0 || height < 11 || width < 11 || channels < 1 ||
      channels > 4 || (kind == REVO_FRAME_U16 && channels != 1) || !pred || !gt || !out)
    return REVO_EINVAL;
  return launch_frame_metrics(kind, pred, gt, batch, height, width, channels, out, (hipStream_t)stream);
}

int revo_op_unproject(const unsigned short* depth, int batch, int height, int width, const float* intrinsics,
                      float* points, void* stream) {
  if (batch <= 0 || height <= 0 || width <= 0 || !depth || !intrinsics || !points) return REVO_EINVAL;
  return launch_unproject(depth, batch, height, width, intrinsics, points, (hipStream_t)stream);
}

int revo_op_render_view(const float* points, const unsigned char* rgb, int batch, int height, int width,
                        const float* pose, const float* intrinsics, int out_height, int out_width,
                        unsigned long long* zbuf, unsigned char* rgb_out, unsigned short* depth_out, void* stream) {
  if (batch <= 0 || height <= 0 || width <= 0 || out_height <= 0 || out_width <= 0 || !points || !rgb || !pose ||
      !intrinsics || !zbuf || !rgb_out || !depth_out)
    return REVO_EINVAL;
  return launch_render_view(points, rgb, batch, height, width, pose, intrinsics, out_height, out_width, zbuf, rgb_out,
                            depth_out, (hipStream_t)stream);
}

}  // extern "C"
