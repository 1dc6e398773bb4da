/*
 * revo_train.h -- pretraining step of the recovery network (C ABI).
 *
 * The paper pretrains each model on frames with randomly masked pixels,
 * with the RGB objective L_RGB = MSE + alpha * TV (Sec. 3.4.2, RGB loss
 * equation) for both the RGB and the depth model ("Robustness Across
 * Codecs" paragraph), alpha = 0.01, Adam at learning rate 2e-4 (Sec. 4).
 *
 * One trainer holds one modality's model (channels 3: RGB u8, 1: depth u16
 * mm) at a fixed batch shape, in FP32: master weights, gradients, Adam
 * moments and the activations the backward pass needs, all in device
 * memory.  A step runs the forward pass on the batch (references plus the
 * clean target whose masked pixels the input zero-fills), the loss
 *   L = (1/B) sum_b [ mean((pred_b - gt_b)^2) + alpha * TV(pred_b) ]
 * on the raw prediction of the target frame (model units: RGB / 255, depth
 * / 4000 mm; TV = mean |x forward difference| + mean |y forward
 * difference|), the gradient of every parameter, and one Adam update
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * (Kingma & Ba 2015, Algorithm 1).
 *
 * Errors are negative revo_status codes (revo.h).
 */
#ifndef REVO_TRAIN_H
#define REVO_TRAIN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct revo_trainer revo_trainer; /* opaque: device buffers and stream */

typedef struct {
  int device;
  int channels;              /* 3 (RGB, u8 frames) or 1 (depth, u16 mm frames) */
  int k;                     /* clean references per sample (1..7) */
  int tubelet;               /* T (1..4); k + 1 frames padded to a multiple of T */
  int enc_depth, dec_depth;  /* blocks (0: 12 and 4) */
  int batch;                 /* samples per step */
  int height, width;         /* frame size of every sample */
  float lr, beta1, beta2, eps;  /* Adam (0: 2e-4, 0.9, 0.999, 1e-8) */
  float tv_weight;           /* alpha (0: 0.01; negative: no TV term) */
  const float *weights;      /* host: initial FP32 blob, revo_weight_count(channels, tubelet, ...) values */
  size_t n_weights;
} revo_train_config;

typedef struct {
  /* device pointers, contiguous, sample-major:
   *   refs     [batch][k][height][width][channels]  u8 (RGB) or u16 (depth), oldest first
   *   target   [batch][height][width][channels]     the clean target frame (same type)
   *   mask     [batch][height][width]               u8, 1 = masked (zero-filled in the input)
   *   ref_idx  host [batch][k] frame indices, t_target host [batch]: the positional
   *            embedding's temporal distances t_target - t_ref (Sec. 3.4.1) */
  const void *refs;
  const void *target;
  const unsigned char *mask;
  const long long *ref_idx;
  const long long *t_target;
} revo_train_batch;

/* Creates a trainer; copies the weights.  REVO_EINVAL on bad shapes,
 * REVO_ENOMEM when device memory runs out. */
int revo_train_create(const revo_train_config *cfg, revo_trainer **out);

/* One step (forward, loss, backward, Adam) on the trainer's stream; returns
 * when it has finished.  *loss receives L before the update (nullable).
 * The batch buffers need only stay valid during the call. */
int revo_train_step(revo_trainer *t, const revo_train_batch *batch, double *loss);

/* Copies the current FP32 weights (n = the blob size) to host memory. */
int revo_train_get_weights(revo_trainer *t, float *out, size_t n);
/* Copies the gradient of the last step (blob layout) to host memory. */
int revo_train_get_grads(revo_trainer *t, float *out, size_t n);
/* Copies the last step's raw predictions [batch][height][width][channels]
 * (model units) to host memory. */
int revo_train_get_pred(revo_trainer *t, float *out, size_t n);

void revo_train_destroy(revo_trainer *t);

#ifdef __cplusplus
}
#endif

#endif /* REVO_TRAIN_H */
