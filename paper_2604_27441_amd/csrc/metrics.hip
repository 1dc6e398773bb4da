// Frame quality metrics and the per-modality training losses for a batch of
// prediction / ground-truth frames: SSIM and PSNR (Sec. 5.1), MSE, L1, TV,
// the gradient-magnitude edge loss, L_RGB = MSE + 0.01 TV and
// L_Depth = 0.1 L1 + L_edge + (1 - SSIM) (Sec. 3.4.2 loss equations, Sec. 4
// weights).  Values are normalised first (u8 / 255, u16 / 4000 mm, float as
// given), so the data range is 1.
//
// One tiled pass over each frame channel adds FP64 partial sums into the
// caller's output (which doubles as the accumulator): squared and absolute
// error, the two TV sums, the edge sum and the SSIM sum (separable 11 x 11
// Gaussian, sigma 1.5, valid windows only).  A finishing kernel turns the six
// sums into the eight reported values.
#include <math.h>

#include "kernels.h"

namespace revo {

namespace {

constexpr int MT = 256;
enum { FM_SQ = 0, FM_ABS, FM_TVX, FM_TVY, FM_EDGE, FM_SSIM };
constexpr int FM_OUT = 8;  // values per frame in the output

struct SsimWeights {
  float w[11];
};

// Element i of a frame buffer as stored (u8 0..255, u16 mm, float).
template <int KIND>
__device__ __forceinline__ float fm_raw(const void* base, long long i) {
  if constexpr (KIND == 0) return (float)static_cast<const uint8_t*>(base)[i];
  else if constexpr (KIND == 1) return (float)static_cast<const uint16_t*>(base)[i];
  else return static_cast<const float*>(base)[i];
}

// Sum NV per-thread values over the workgroup (wave shuffles, then LDS) and
// add the totals into dst[0 .. NV-1] in FP64.
template <int NV>
__device__ __forceinline__ void fm_accumulate(const float (&v)[NV], double* dst) {
  __shared__ float red[NV][MT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    float s = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < MT / 64; ++w) t += (double)red[threadIdx.x][w];
    atomicAdd(dst + threadIdx.x, t);
  }
}

__global__ void fm_zero_kernel(double* __restrict__ out, int n) {
  const int i = blockIdx.x * MT + threadIdx.x;
  if (i < n) out[i] = 0.0;
}

// One pass per frame channel: blockIdx.y picks (frame, channel), and each
// workgroup walks tiles of TH x TW pixels.  A tile's pixels plus a 10-pixel
// halo go to LDS as stored values (zeros past the frame); the next tile's
// pixels are fetched into registers while this one is processed.  From the
// tile come
//  - the pixel terms of its own pixels: squared and absolute error, the two
//    TV sums and the edge sum, on stored values (integer differences are
//    exact; the finishing kernel applies the normalisation);
//  - SSIM at its window positions below (H - 10, W - 10): the five Gaussian
//    moments (of x, y, x^2, y^2, xy) filtered along rows, four outputs per
//    thread from a register window over 16-byte LDS reads, into LDS, then
//    along columns, four rows per thread.  SSIM is unchanged by the scale
//    when C1 and C2 are taken in stored units, so c1 = (0.01 L)^2 and
//    c2 = (0.03 L)^2 with L the stored data range.
template <int KIND>
__global__ __launch_bounds__(MT, 3) void fm_frame_kernel(const void* __restrict__ P, const void* __restrict__ G,
                                                         int H, int W, int C, SsimWeights wt, float c1, float c2,
                                                         double* __restrict__ out) {
  constexpr int TH = 16, TW = 64, IH = TH + 10, IW = TW + 12;  // IW: 74 used, padded to 16-byte rows
  constexpr int NL = (IH * IW + MT - 1) / MT;                  // tile elements per thread
  __shared__ __attribute__((aligned(16))) float pl[2][IH][IW];
  __shared__ __attribute__((aligned(16))) float hm[5][IH][TW];
  const int tid = threadIdx.x;
  const int b = blockIdx.y / C, c = blockIdx.y - b * C;
  const long long off = (long long)b * H * W * C + c;
  const int ntx = (W + TW - 1) / TW, nt = ntx * ((H + TH - 1) / TH);
  float xr[NL], yr[NL];
  auto fetch = [&](int t) {
    const int ty = t / ntx;
    const int i0 = ty * TH, j0 = (t - ty * ntx) * TW;
#pragma unroll
    for (int n = 0; n < NL; ++n) {
      const int e = tid + n * MT;
      const int r = e / IW, q = e - r * IW;
      const int i = i0 + r, j = j0 + q;
      xr[n] = yr[n] = 0.0f;
      if (e < IH * IW && q < TW + 10 && i < H && j < W) {
        const long long k = off + ((long long)i * W + j) * C;
        xr[n] = fm_raw<KIND>(P, k);
        yr[n] = fm_raw<KIND>(G, k);
      }
    }
  };
  float sq = 0.0f, ab = 0.0f, tvx = 0.0f, tvy = 0.0f, edge = 0.0f, ss = 0.0f;
  if (blockIdx.x < nt) fetch(blockIdx.x);
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int ty = t / ntx;
    const int i0 = ty * TH, j0 = (t - ty * ntx) * TW;
    __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
    for (int n = 0; n < NL; ++n) {
      const int e = tid + n * MT;
      if (e < IH * IW) {
        const int r = e / IW, q = e - r * IW;
        pl[0][r][q] = xr[n];
        pl[1][r][q] = yr[n];
      }
    }
    __syncthreads();
    if (t + gridDim.x < nt) fetch(t + gridDim.x);  // in flight during this tile
    // pixel terms; forward differences exist for j < W-1 and i < H-1
    for (int e = tid; e < TH * TW; e += MT) {
      const int r = e / TW, q = e - r * TW;
      const int i = i0 + r, j = j0 + q;
      if (i >= H || j >= W) continue;
      const float p = pl[0][r][q], g = pl[1][r][q];
      const float d = p - g;
      sq += d * d;
      ab += fabsf(d);
      const bool hx = j + 1 < W, hy = i + 1 < H;
      float pdx = 0.0f, pdy = 0.0f, gdx = 0.0f, gdy = 0.0f;
      if (hx) {
        pdx = pl[0][r][q + 1] - p;
        gdx = pl[1][r][q + 1] - g;
        tvx += fabsf(pdx);
      }
      if (hy) {
        pdy = pl[0][r + 1][q] - p;
        gdy = pl[1][r + 1][q] - g;
        tvy += fabsf(pdy);
      }
      if (hx && hy) edge += fabsf(sqrtf(pdx * pdx + pdy * pdy) - sqrtf(gdx * gdx + gdy * gdy));
    }
    // row filter: item (r, group of 4 columns)
    for (int e = tid; e < IH * (TW / 4); e += MT) {
      const int r = e / (TW / 4), q0 = (e - r * (TW / 4)) * 4;
      float x[16], y[16];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 f = *reinterpret_cast<const float4*>(&pl[0][r][q0 + 4 * u]);
        const float4 h = *reinterpret_cast<const float4*>(&pl[1][r][q0 + 4 * u]);
        x[4 * u] = f.x; x[4 * u + 1] = f.y; x[4 * u + 2] = f.z; x[4 * u + 3] = f.w;
        y[4 * u] = h.x; y[4 * u + 1] = h.y; y[4 * u + 2] = h.z; y[4 * u + 3] = h.w;
      }
      float o[5][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float mx = 0.0f, my = 0.0f, xx = 0.0f, yy = 0.0f, xy = 0.0f;
#pragma unroll
        for (int m = 0; m < 11; ++m) {
          const float a = x[u + m], bb = y[u + m], w = wt.w[m];
          mx += w * a;
          my += w * bb;
          xx += w * (a * a);
          yy += w * (bb * bb);
          xy += w * (a * bb);
        }
        o[0][u] = mx; o[1][u] = my; o[2][u] = xx; o[3][u] = yy; o[4][u] = xy;
      }
#pragma unroll
      for (int k = 0; k < 5; ++k)
        *reinterpret_cast<float4*>(&hm[k][r][q0]) = make_float4(o[k][0], o[k][1], o[k][2], o[k][3]);
    }
    __syncthreads();
    // column filter and SSIM: item (group of 4 rows, column), one per thread
    {
      const int q = tid & (TW - 1), r0 = (tid >> 6) * 4;
      float mo[5][4];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        float v[14];
#pragma unroll
        for (int m = 0; m < 14; ++m) v[m] = hm[k][r0 + m][q];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          float a = 0.0f;
#pragma unroll
          for (int m = 0; m < 11; ++m) a += wt.w[m] * v[u + m];
          mo[k][u] = a;
        }
      }
      const int j = j0 + q;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + r0 + u;
        if (i >= H - 10 || j >= W - 10) continue;
        const float mx = mo[0][u], my = mo[1][u];
        const float sxx = mo[2][u] - mx * mx, syy = mo[3][u] - my * my, sxy = mo[4][u] - mx * my;
        ss += ((2.0f * mx * my + c1) * (2.0f * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2));
      }
    }
  }
  const float v[6] = {sq, ab, tvx, tvy, edge, ss};
  fm_accumulate<6>(v, out + (long long)b * FM_OUT + FM_SQ);
}

// Sums -> means and the derived values, in place:
// [mse, l1, tv, edge, ssim, psnr, l_rgb, l_depth].  `scale` normalises the
// pixel pass's stored-value sums.
__global__ void fm_finish_kernel(double* __restrict__ out, int B, int H, int W, int C, double scale) {
  const int b = blockIdx.x * MT + threadIdx.x;
  if (b >= B) return;
  double* o = out + (long long)b * FM_OUT;
  const double n = (double)H * W * C;
  const double mse = o[FM_SQ] * scale * scale / n, l1 = o[FM_ABS] * scale / n;
  const double tv =
      scale * (o[FM_TVX] / ((double)H * (W - 1) * C) + o[FM_TVY] / ((double)(H - 1) * W * C));
  const double edge = o[FM_EDGE] * scale / ((double)(H - 1) * (W - 1) * C);
  const double ssim = o[FM_SSIM] / ((double)(H - 10) * (W - 10) * C);
  o[0] = mse;
  o[1] = l1;
  o[2] = tv;
  o[3] = edge;
  o[4] = ssim;
  o[5] = mse > 0.0 ? 10.0 * log10(1.0 / mse) : INFINITY;
  o[6] = mse + 0.01 * tv;
  o[7] = 0.1 * l1 + edge + (1.0 - ssim);
}

}  // namespace

int launch_frame_metrics(int kind, const void* pred, const void* gt, int B, int H, int W, int C, double* out,
                         hipStream_t s) {
  if (B <= 0 || H < 11 || W < 11 || !pred || !gt || !out) return -22;
  if (kind < 0 || kind > 2 || C < 1 || C > 4 || (kind == 1 && C != 1)) return -22;
  if ((long long)B * C > 65535 || (long long)cdiv(W, 64) * cdiv(H, 16) > (1LL << 30)) return -22;
  // the Gaussian window in double, rounded once
  SsimWeights wt;
  double w[11], sum = 0.0;
  for (int a = 0; a < 11; ++a) sum += (w[a] = exp(-(double)((a - 5) * (a - 5)) / (2.0 * 1.5 * 1.5)));
  for (int a = 0; a < 11; ++a) wt.w[a] = (float)(w[a] / sum);
  // SSIM constants in stored units (data range 255, 4000 mm or 1)
  const double range = kind == 0 ? 255.0 : kind == 1 ? 4000.0 : 1.0;
  const float c1 = (float)(0.01 * range * 0.01 * range), c2 = (float)(0.03 * range * 0.03 * range);
  // about 1536 workgroups in all (three per CU, two rounds), each walking
  // several tiles
  const int nt = cdiv(W, 64) * cdiv(H, 16);
  const int per = cdiv(1536, B * C);
  const dim3 grid(per < nt ? per : nt, B * C);
  fm_zero_kernel<<<cdiv(B * FM_OUT, MT), MT, 0, s>>>(out, B * FM_OUT);
  if (kind == 0) fm_frame_kernel<0><<<grid, MT, 0, s>>>(pred, gt, H, W, C, wt, c1, c2, out);
  else if (kind == 1) fm_frame_kernel<1><<<grid, MT, 0, s>>>(pred, gt, H, W, C, wt, c1, c2, out);
  else fm_frame_kernel<2><<<grid, MT, 0, s>>>(pred, gt, H, W, C, wt, c1, c2, out);
  const double scale = kind == 0 ? 1.0 / 255.0 : kind == 1 ? 1.0 / 4000.0 : 1.0;
  fm_finish_kernel<<<cdiv(B, MT), MT, 0, s>>>(out, B, H, W, C, scale);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace revo
