/*
 * revo.h -- C ABI of the MI355X neural loss-recovery library.
 *
 * The library runs ReVo's post-decode neural loss recovery (Sec. 3.4.1 of
 * the paper): for a frame whose packets were partly lost, it takes the k
 * closest clean frames of the same stream and modality plus the corrupted
 * frame and returns a reconstructed frame.  RGB and depth have separate
 * models of the same architecture (Sec. 3.4.2).  The same clean references
 * are reused for every corrupted frame until a new clean frame arrives,
 * with the temporal distance to the target fed to the network (Sec. 3.4.1).
 * Intact frames bypass recovery (Sec. 3.1 overview): a request without a
 * loss mask is a clean frame, it updates the reference set and its output
 * is a copy.  The decoder thread hands frames over and the display thread
 * collects them (Sec. 4 receiver threads): submit and poll may be called
 * from different threads.
 *
 * Model ("ViViT-S/16" reading of Sec. 3.4.1, App. B.1, App. B.3): tubelets
 * of T frames x 16 x 16 pixels, encoder 384 wide x 12 pre-LN blocks x 6
 * heads (MLP 1536), decoder 192 x 4 x 3 (MLP 768), joint space-time
 * attention over all tokens of a request, a fixed three-axis sinusoidal
 * positional embedding (temporal distance, patch row, patch column), and a
 * head emitting the target frame's pixels.  Inputs are RGB u8/255 and
 * depth u16 mm / 4000; lost target pixels are zero-filled (Sec. 3.3).
 *
 * Errors are negative return codes (revo_status).  Per-request failures
 * are reported in revo_completion.status / .error.
 */
#ifndef REVO_H
#define REVO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define REVO_ABI_VERSION 1

typedef struct revo_ctx revo_ctx; /* opaque: device memory, weights, rings, worker thread */

enum revo_status {
  REVO_OK = 0,
  REVO_EAGAIN = 1,       /* queue full: poll, then submit again */
  REVO_EINVAL = -22,     /* bad argument */
  REVO_ENOMEM = -12,     /* device memory or HBM budget exhausted */
  REVO_EDEVICE = -5,     /* HIP runtime error */
  REVO_ENOREF = -61,     /* recovery asked for before any clean frame of the stream */
  REVO_ENOTSUP = -95,    /* configuration the library does not support */
  REVO_ESHUTDOWN = -108, /* context is being destroyed */
  REVO_E2BIG = -7        /* size beyond a fixed workspace (revo_op_attention_noalloc) */
};

enum revo_precision {
  REVO_FP32 = 0,  /* FP32 operands, FP32 MFMA */
  REVO_BF16 = 1,  /* BF16 operands, FP32 accumulation, FP32 residual/LN/softmax/composite */
  REVO_FP8 = 2    /* OCP FP8 E4M3 operands for the block products (qkv, proj, fc1, fc2) and the
                     encoder-to-decoder projection, with per-output-row weight scales and
                     per-tensor activation scales from a calibration pass (revo_calibrate);
                     embedding, attention and head in BF16; FP32 accumulation, residual, LN
                     statistics and composite.  Until calibrated it computes as REVO_BF16. */
};

enum revo_completion_status {
  REVO_DONE = 0,    /* outputs written */
  REVO_SHED = 1,    /* deadline could not be met; nothing written (display repeats the last frame) */
  REVO_FAILED = 2   /* see revo_completion.error */
};

/* revo_request.flags */
#define REVO_DEVICE_PTRS 0x1u /* every pointer of the request is a device pointer on cfg.device */
#define REVO_HOLD 0x2u        /* keep queued: batch with the next submit that lacks this flag */

/* revo_config.flags */
#define REVO_CFG_SHED 0x1u    /* shed requests whose deadline cannot be met */
#define REVO_CFG_PROFILE 0x2u /* time every kernel launch with HIP events (see revo_get_stats) */
#define REVO_CFG_ONE_STREAM 0x4u /* run the RGB and depth networks one after the other on one stream
                                   (default: two streams that overlap on the GPU) */
#define REVO_CFG_GRAPHS 0x8u  /* replay each network as a HIP graph captured once per token-capacity
                                 bucket (cap/8, cap/4, cap/2, cap); ignored with REVO_CFG_PROFILE or
                                 REVO_CFG_PROFILE_ATTN */
#define REVO_CFG_PROFILE_ATTN 0x10u /* time only the attention launches and whole network passes
                                       with HIP events: about 34 events per pass instead of one pair
                                       per kernel, so the timing barely perturbs throughput */

typedef struct revo_config {
  int device;                 /* HIP device ordinal */
  int precision;              /* revo_precision */
  int k;                      /* clean reference frames per recovery, 1..7 (paper: 5, App. B.3) */
  int tubelet;                /* frames per tubelet T, 1..4 (paper: 2, App. B.3); (k+1) padded to a
                                 multiple of T with the oldest frame, at most 9 frames in all */
  int enc_depth;              /* encoder blocks; 0 = 12 */
  int dec_depth;              /* decoder blocks; 0 = 4 */
  int composite;              /* 1 = replace lost pixels only; 0 = raw clamped prediction everywhere */
  int max_streams;            /* conference streams holding reference state (0 = 64) */
  int max_batch;              /* requests per batch (0 = 16) */
  int max_batch_tokens;       /* tokens per batch per modality (0 = from hbm_budget_bytes, else 43200) */
  size_t hbm_budget_bytes;    /* cap on weights + workspaces + reference rings + staging (0 = none) */
  float fps;                  /* default deadline is arrival + 1/fps (0 = 30) */
  const float *weights_rgb;   /* host FP32 blob, layout below; copied at create */
  size_t n_weights_rgb;
  const float *weights_depth; /* host FP32 blob for the depth model */
  size_t n_weights_depth;
  unsigned flags;             /* REVO_CFG_* */
  void *hip_stream;           /* optional hipStream_t of the caller: each submit's input copies are
                                 ordered after the work already enqueued on it (NULL: inputs must
                                 be complete when submit is called) */
} revo_config;

/*
 * Weight blob layout, per modality (C = 3 RGB, 1 depth; L = T*256*C; every
 * matrix row-major [out][in], each followed by its bias):
 *   emb.w [384][L] emb.b [384]
 *   enc_depth x { ln1.g ln1.b [384]  qkv.w [1152][384] qkv.b [1152]
 *                 proj.w [384][384] proj.b [384]  ln2.g ln2.b [384]
 *                 fc1.w [1536][384] fc1.b [1536]  fc2.w [384][1536] fc2.b [384] }
 *   enc_norm.g enc_norm.b [384]   e2d.w [192][384] e2d.b [192]
 *   dec_depth x { same with 192 wide, qkv 576, MLP 768 }
 *   dec_norm.g dec_norm.b [192]   head.w [L][192] head.b [L]
 * qkv output columns are Q | K | V, each with heads of 64 contiguous.
 * Tubelet vector element ((t*16 + py)*16 + px)*C + c is frame t of the
 * tubelet at patch pixel (py, px), channel c.
 */

typedef struct revo_request {
  unsigned stream_id;             /* < max_streams */
  long long frame_index;          /* decode order index; temporal distance = target - reference */
  int width, height;              /* frame size in pixels (>= 16 x 16, <= 4096 x 4096) */
  unsigned flags;                 /* REVO_DEVICE_PTRS, REVO_HOLD */
  const unsigned char *rgb;       /* H x W x 3 u8, or NULL: no RGB in this request */
  const unsigned char *mask_rgb;  /* H x W u8, 1 = pixel lost; NULL = clean RGB frame */
  const unsigned short *depth;    /* H x W u16 millimetres, or NULL */
  const unsigned char *mask_depth;/* H x W u8; NULL = clean depth frame */
  unsigned char *rgb_out;         /* H x W x 3 u8 output (may be NULL) */
  unsigned short *depth_out;      /* H x W u16 output (may be NULL) */
  float *rgb_out_f32;             /* optional H x W x 3 float output in [0, 1] */
  float *depth_out_f32;           /* optional H x W float output in mm */
  long long deadline_ns;          /* CLOCK_MONOTONIC; 0 = submit time + 1/fps */
} revo_request;

typedef struct revo_completion {
  unsigned long long ticket;
  unsigned stream_id;
  long long frame_index;
  int status;                     /* revo_completion_status */
  int error;                      /* revo_status when status == REVO_FAILED */
  long long submit_ns, done_ns;   /* CLOCK_MONOTONIC */
} revo_completion;

/* Fill cfg with the paper's configuration: k = 5 references and T = 2 frame
 * tubelets (App. B.3), 12 + 4 blocks, BF16, composite on, 30 fps (the
 * receiver's frame budget, Sec. 3.3 Eq. 1).  Weights must still be set. */
void revo_config_default(revo_config *cfg);

/* Number of floats in one modality's weight blob (channels 3 or 1; the RGB
 * and depth models are separate, Sec. 3.4.2).  0 for invalid arguments. */
size_t revo_weight_count(int channels, int tubelet, int enc_depth, int dec_depth);

/* Create a context on cfg->device: uploads and converts both models'
 * weights (Sec. 3.4.1 architecture, one model per modality, Sec. 3.4.2),
 * sizes the workspaces from max_batch_tokens or hbm_budget_bytes, starts the
 * worker and completion threads (the receiver's recovery thread, Sec. 4).
 * The weight blobs are copied; the caller keeps ownership.  *out is set on
 * success.  Errors: REVO_EINVAL (bad k, tubelet, depths or weights),
 * REVO_ENOTSUP (precision), REVO_EDEVICE (no such device, HIP failure),
 * REVO_ENOMEM (device memory, or a budget below the weights and the
 * smallest workspace). */
int revo_recover_create(const revo_config *cfg, revo_ctx **out);

/* Queue one frame (RGB and/or depth) of one stream: the recovery module's
 * input is the k closest clean frames of the stream plus the corrupted
 * frame, and its output the reconstructed frame (Sec. 3.4.1); intact frames
 * bypass recovery (Sec. 3.1).  Non-blocking with respect to the GPU work:
 * inputs are copied into library staging before it returns, so input
 * buffers may be reused at once; output buffers must stay valid until poll
 * reports the ticket.  A modality with a mask is recovered against the
 * stream's clean references as they stand at this submit; a modality
 * without a mask becomes the newest clean reference (a resolution change
 * resets the stream's references) and is copied to the output.  Recovered
 * frames never become references (Sec. 3.4.1, reference reuse).
 * Returns REVO_OK and sets *ticket; REVO_EAGAIN when the queue is full or
 * the HBM budget has no room for the request's staging and prediction
 * buffers (poll, then retry); REVO_ENOREF when a modality is to be
 * recovered but no clean frame of that stream and modality at this size
 * was submitted before it; REVO_EINVAL for bad sizes or pointers.  A clean
 * frame whose reference update fails later (device memory) completes with
 * status REVO_FAILED, and a recovery queued behind it with error
 * REVO_ENOREF. */
int revo_recover_submit(revo_ctx *ctx, const revo_request *req, unsigned long long *ticket);

/* Collect up to max completions, waiting up to timeout_us (0 = no wait,
 * -1 = wait for at least one): the display thread's side of the receiver
 * (Sec. 4).  Outputs of a reported ticket are complete.  Returns the count
 * (>= 0) or REVO_EINVAL. */
int revo_recover_poll(revo_ctx *ctx, revo_completion *out, int max, int timeout_us);

/* Drain queued and in-flight work (completions are posted but no longer
 * collectable), stop the threads and free every device allocation. */
void revo_recover_destroy(revo_ctx *ctx);

/* FP8 calibration (REVO_FP8 contexts only; REVO_ENOTSUP otherwise).  The
 * paper states no inference precision; the FP8 form's static activation
 * scales come from this pass.
 * phase = 1: wait for queued work, clear the recorded maxima; recoveries
 * submitted afterwards run in BF16 and raise the per-tensor maximum of every
 * FP8 product input over their tokens.  phase = 0: wait for queued work, set
 * each activation scale to maximum / 448 and run later recoveries in FP8.
 * Both block the caller until the queue and the GPU are drained. */
int revo_calibrate(revo_ctx *ctx, int phase);

/* Counters of a context.  The *_ms and *_flop fields are filled only with
 * REVO_CFG_PROFILE: GPU time between HIP events recorded on the stream of
 * each launch, and algorithmic FLOPs (2 per multiply-add of the layer's
 * definition: attention 4 * N^2 * 64 per head and request, a linear layer
 * 2 * tokens * out * in; alignment rows and padding excluded). */
typedef struct revo_stats {
  long long batches;                /* batches run */
  long long served, shed, failed;   /* completions by status */
  long long attn_launches;          /* flash-attention kernel launches */
  double attn_ms, attn_flop;
  long long gemm_launches;          /* linear-layer launches (embedding, blocks, e2d, head) */
  double gemm_ms, gemm_flop;
  long long other_launches;         /* LayerNorm and composite launches */
  double other_ms;
  double forward_ms;                /* whole forward passes, both modalities summed */
  long long hbm_fixed_bytes;        /* weights + workspaces (always filled, never reset) */
  long long hbm_pool_bytes;         /* reference rings + staging held in the pool, cached blocks included */
} revo_stats;

/* Copy the counters into *out; reset = 1 zeroes them afterwards. */
int revo_get_stats(revo_ctx *ctx, revo_stats *out, int reset);

/* Static text for a revo_status code ("unknown error" otherwise). */
const char *revo_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* REVO_H */
