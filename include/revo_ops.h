/*
 * revo_ops.h -- single-kernel entry points of the recovery library.
 *
 * Each call runs one of the kernels the recovery network is made of, on
 * caller-owned device buffers, so that every kernel can be checked on its
 * own.  All pointers are device pointers on the current HIP device; stream
 * may be NULL (the default stream).  Calls are asynchronous on that stream.
 * They return 0 or a negative revo_status (REVO_EINVAL on shapes the
 * kernel does not take, REVO_ENOTSUP on an unknown precision, REVO_EDEVICE
 * when the launch fails).  precision is REVO_FP32 (float operands) or
 * REVO_BF16 (bfloat16 operands, float accumulation).
 */
#ifndef REVO_OPS_H
#define REVO_OPS_H

#ifdef __cplusplus
extern "C" {
#endif

enum revo_op_epilogue {
  REVO_EPI_STORE = 0,    /* out[m][n] = sum_k x[m][k] w[n][k] + bias[n]          (operand type) */
  REVO_EPI_RESIDUAL = 1, /* out[m][n] += sum_k x[m][k] w[n][k] + bias[n]         (float)        */
  REVO_EPI_GELU = 2      /* out[m][n] = GELU_erf(sum_k x[m][k] w[n][k] + bias[n]) (operand type) */
};

/* Linear layer of a Transformer block (Sec. 3.4.1): x [M][K] and w [N][K]
 * row-major in the operand type, bias [N] float (16-byte aligned), out [M][N].
 * Requires N % 64 == 0 and K % 64 == 0 (K % 32 for REVO_FP32). */
int revo_op_linear(int precision, int epilogue, const void *x, const void *w, const float *bias,
                   void *out, int M, int N, int K, void *stream);

/* FP8 linear layer (the FP8 form's block products): x8 [M][K] and w8 [N][K]
 * are OCP E4M3 bytes, wscale [N] per-row weight scales, xscale a device
 * pointer to the activation scale; the product is
 * sum_k x8[m][k] w8[n][k] * wscale[n] * (*xscale) + bias[n], accumulated in
 * float.  REVO_EPI_STORE writes bfloat16 out [M][N], REVO_EPI_RESIDUAL adds
 * into float out, REVO_EPI_GELU writes E4M3 bytes of GELU(.) / (*out_scale).
 * bias and wscale are 16-byte aligned.  Requires N % 64 == 0 and K % 64 == 0. */
int revo_op_linear_fp8(int epilogue, const void *x8, const void *w8, const float *wscale, const float *xscale,
                       const float *bias, void *out, const float *out_scale, int M, int N, int K, void *stream);

/* LayerNorm over rows of D <= 512 floats, D even: y = (x - mean) / sqrt(var + 1e-6)
 * * g + b with the biased variance; y in the operand type. */
int revo_op_layernorm(int precision, const float *x, const float *g, const float *b, void *y,
                      int rows, int D, void *stream);

/* Scaled dot-product attention of one request with ntok tokens and
 * `heads` heads of 64 (the attention inside each Transformer block,
 * App. B.1): o[t][h*64 + d] = sum_j softmax_j(q_h[t] . k_h[j] / 8) v_h[j][d].
 * Layouts (operand type): q and k [heads][ld][64] with q already
 * multiplied by log2(e) / 8; vt [heads][64][ld] (V transposed), where for
 * REVO_BF16 column c holds token c with bits 2 and 3 of c swapped
 * (c ^ ((c ^ (c >> 1)) & 4) * 3, a permutation inside each group of 16);
 * o [ntok][heads * 64].  ld >= ntok + 64, ld % 16 == 0, and rows ntok ..
 * ld-1 of q, k and columns ntok .. ld-1 of vt must hold finite values
 * (zeros). */
int revo_op_attention(int precision, const void *q, const void *k, const void *vt, void *o,
                      int heads, int ntok, int ld, void *stream);

/* FP8 attention of the FP8 form: the same softmax(q k^T / 8) v with OCP
 * E4M3 operands and per-head power-of-two scales, q8 = E4M3(q log2(e) / 8 /
 * 2^eq[h]), k8 = E4M3(k / 2^ek[h]), vt8 = E4M3(v^T / 2^ev[h]) (exps: host,
 * eq[heads] then ek[heads] then ev[heads], each in -100 .. 100), applied
 * exactly by the scaled FP8 products; probabilities E4M3 (unit scale,
 * exp2 of the scores minus a running max raised only past 8 in log2
 * units, so they stay below 2^8); FP32 accumulation and row sums (App. B.1
 * item 4 attention; the FP8 form's precision).  q8, k8 [heads][ld][64]
 * bytes; vt8 [heads][64][ld] bytes with the keys of each aligned group of 64
 * in the order key t -> column (t & ~63) | ((t >> 2) & 1) << 5 |
 * ((t >> 5) & 1) << 4 | ((t >> 3) & 3) << 2 | (t & 3); rows / columns ntok ..
 * ld-1 zero.  o [ntok][heads 64] bfloat16.  ld % 64 == 0, ld >= ntok + 64.
 * Synchronous (descriptors are allocated and freed per call). */
int revo_op_attention_fp8(const void *q8, const void *k8, const void *vt8, void *o, int heads, int ntok, int ld,
                          const int *exps, void *stream);

/* revo_op_attention for callers that cannot allocate device memory: code
 * under HIP graph capture, serving loops that must not call hipMalloc, and
 * harnesses that forbid it.  Same arguments, layouts and result as
 * revo_op_attention, but it allocates nothing, copies nothing from the host
 * and does not synchronise: the request descriptor and the q-tile work list
 * go to a fixed device workspace of 128.25 KiB (one per device, held until
 * the process ends), written by a kernel on `stream` before the attention
 * kernel.  ntok is at most 32767 * 128 = 4194176 tokens (REVO_E2BIG beyond).
 * Calls on one stream are ordered; calls that overlap on one device (other
 * streams or threads) share the workspace and race. */
int revo_op_attention_noalloc(int precision, const void *q, const void *k, const void *vt, void *o,
                              int heads, int ntok, int ld, void *stream);

/* Element-wise float -> operand type conversion of n values (round to
 * nearest even for REVO_BF16; REVO_FP8 gives OCP E4M3 bytes, nearest even,
 * saturating at +-448). */
int revo_op_convert(int precision, const float *src, void *dst, long long n, void *stream);

/* Frame element types for revo_op_frame_metrics. */
enum revo_frame_kind {
  REVO_FRAME_U8 = 0,  /* u8, normalised by 1/255 (RGB) */
  REVO_FRAME_U16 = 1, /* u16 depth in mm, normalised by 1/4000; channels must be 1 */
  REVO_FRAME_F32 = 2  /* float, already normalised */
};

/* Quality metrics and training losses of `batch` predicted frames against
 * their ground truth (SSIM and PSNR of Sec. 5.1; L_RGB = MSE + 0.01 TV and
 * L_Depth = 0.1 L1 + L_edge + (1 - SSIM) of the Sec. 3.4.2 loss equations
 * with the Sec. 4 weights).  pred and gt: device pointers, batch frames of
 * height x width x channels elements each, contiguous (HWC).  All values use
 * normalised pixels (data range 1).  SSIM: 11 x 11 Gaussian window, sigma 1.5,
 * K1 0.01, K2 0.03, valid windows only, mean over positions and channels.
 * TV: mean |horizontal forward difference| + mean |vertical one| of pred.
 * L_edge: mean over pixels with both forward differences of
 * | |grad pred| - |grad gt| |.  out: device pointer to batch x 8 doubles,
 * per frame [mse, l1, tv, edge, ssim, psnr, l_rgb, l_depth]
 * (psnr = 10 log10(1 / mse), +inf for identical frames); it is also the
 * accumulator, so its previous contents are lost.  Requires height, width
 * >= 11 and 1 <= channels <= 4.  Runs asynchronously on `stream`. */
int revo_op_frame_metrics(int kind, const void *pred, const void *gt, int batch, int height, int width,
                          int channels, double *out, void *stream);

/* RGB-D unprojection: an RGB-D frame projected into Cartesian space (Sec. 2),
 * the first half of the receiver's rendering step (Sec. 5).  depth: device,
 * batch x height x width u16 z in mm (0 = no measurement).  intrinsics: host,
 * 4 floats (fx, fy, cx, cy) in pixels, pixel centres at integer coordinates.
 * points: device, 16-byte aligned, batch x height x width float4
 * (X, Y, Z in mm, valid 1 or 0) with X = (u - cx) Z / fx, Y = (v - cy) Z / fy.
 * Requires batch and height <= 65535. */
int revo_op_unproject(const unsigned short *depth, int batch, int height, int width, const float *intrinsics,
                      float *points, void *stream);

/* Z-buffered rendering of organised point clouds (from revo_op_unproject)
 * into a new view, the second half of the rendering step (Sec. 5).  Each
 * valid point moves by X' = R X + t (pose: host, 12 floats, R|t row-major
 * 3 x 4, t in mm), projects with the target intrinsics (host, fx, fy, cx, cy)
 * to the nearest target pixel centre, and is dropped when Z' <= 0 or it falls
 * outside out_height x out_width.  Each target pixel shows the point of
 * smallest Z' (ties to the lower point index): its colour from rgb (device,
 * batch x height x width x 3 u8, the cloud's source frames) and Z' rounded
 * half to even to mm (u16, clamped); pixels no point reaches are 0.  zbuf:
 * device workspace of batch x out_height x out_width 64-bit words, 8-byte
 * aligned; on return it holds per pixel (bits of Z') << 32 | point index, or
 * all ones.  rgb_out: device, batch x out_height x out_width x 3 u8;
 * depth_out: device, batch x out_height x out_width u16.  Requires
 * height x width < 2^32 and batch, height, out_height <= 65535. */
int revo_op_render_view(const float *points, const unsigned char *rgb, int batch, int height, int width,
                        const float *pose, const float *intrinsics, int out_height, int out_width,
                        unsigned long long *zbuf, unsigned char *rgb_out, unsigned short *depth_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* REVO_OPS_H */
