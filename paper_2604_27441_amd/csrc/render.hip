// RGB-D unprojection and z-buffered rendering of a new view: the receiver
// step after recovery, which turns each recovered RGB-D pair into 3-D points
// (an RGB-D frame projected into Cartesian space, Sec. 2) and renders them
// for a viewpoint (Sec. 5 microbenchmarks).
//
// Pinhole camera, pixel centres at integer coordinates, depth = z in mm
// (0 = no measurement).  Unprojection writes an organised cloud, one float4
// (X, Y, Z, valid) per pixel.  Rendering moves each point by X' = R X + t,
// projects it to the nearest target pixel centre and keeps, per pixel, the
// point of smallest Z' (ties to the lower index) with a 64-bit atomic min on
// (bits of Z', point index): positive floats order like their bit patterns.
// A resolve pass then writes the winner's colour and Z' rounded to mm.
#include <math.h>

#include "kernels.h"

namespace revo {

namespace {

constexpr int RT = 256;

struct Intr {
  float fx, fy, cx, cy;
};
struct Pose {
  float r[9], t[3];
};

// grid (columns / RT, rows, frames)
__global__ __launch_bounds__(RT) void unproject_kernel(const uint16_t* __restrict__ depth, int H, int W, Intr k,
                                                       float4* __restrict__ pts) {
  const int u = blockIdx.x * RT + threadIdx.x;
  if (u >= W) return;
  const int v = blockIdx.y;
  const long long i = ((long long)blockIdx.z * H + v) * W + u;
  const float z = (float)depth[i];
  pts[i] = make_float4(((float)u - k.cx) * z / k.fx, ((float)v - k.cy) * z / k.fy, z, z > 0.0f ? 1.0f : 0.0f);
}

__global__ void zbuf_clear_kernel(unsigned long long* __restrict__ zbuf, long long n) {
  const long long i = (long long)blockIdx.x * RT + threadIdx.x;
  if (i < n) zbuf[i] = ~0ull;
}

// grid (source columns / RT, source rows, frames)
__global__ __launch_bounds__(RT) void splat_kernel(const float4* __restrict__ pts, int H, int W, Pose P, Intr k,
                                                   int Ho, int Wo, unsigned long long* __restrict__ zbuf) {
  const int u = blockIdx.x * RT + threadIdx.x;
  if (u >= W) return;
  const unsigned n = (unsigned)(blockIdx.y * W + u);
  const float4 p = pts[(long long)blockIdx.z * H * W + n];
  if (!(p.w > 0.0f)) return;
  const float x = P.r[0] * p.x + P.r[1] * p.y + P.r[2] * p.z + P.t[0];
  const float y = P.r[3] * p.x + P.r[4] * p.y + P.r[5] * p.z + P.t[1];
  const float z = P.r[6] * p.x + P.r[7] * p.y + P.r[8] * p.z + P.t[2];
  if (!(z > 0.0f)) return;
  const float fu = k.fx * x / z + k.cx + 0.5f, fv = k.fy * y / z + k.cy + 0.5f;
  if (!(fu >= 0.0f && fu < (float)Wo && fv >= 0.0f && fv < (float)Ho)) return;
  const int iu = (int)floorf(fu), iv = (int)floorf(fv);
  if (iu >= Wo || iv >= Ho) return;  // fu just below Wo can round up to it
  const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | n;
  atomicMin(zbuf + ((long long)blockIdx.z * Ho + iv) * Wo + iu, key);
}

// grid (target columns / RT, target rows, frames)
__global__ __launch_bounds__(RT) void resolve_kernel(const unsigned long long* __restrict__ zbuf,
                                                     const uint8_t* __restrict__ rgb, int H, int W, int Ho, int Wo,
                                                     uint8_t* __restrict__ rgb_out, uint16_t* __restrict__ depth_out) {
  const int u = blockIdx.x * RT + threadIdx.x;
  if (u >= Wo) return;
  const long long o = ((long long)blockIdx.z * Ho + blockIdx.y) * Wo + u;
  const unsigned long long key = zbuf[o];
  uint8_t c0 = 0, c1 = 0, c2 = 0;
  uint16_t d = 0;
  if (key != ~0ull) {
    const long long n = (long long)blockIdx.z * H * W + (unsigned)(key & 0xffffffffu);
    c0 = rgb[3 * n]; c1 = rgb[3 * n + 1]; c2 = rgb[3 * n + 2];
    d = (uint16_t)fminf(rintf(__uint_as_float((unsigned)(key >> 32))), 65535.0f);
  }
  rgb_out[3 * o] = c0; rgb_out[3 * o + 1] = c1; rgb_out[3 * o + 2] = c2;
  depth_out[o] = d;
}

}  // namespace

int launch_unproject(const uint16_t* depth, int B, int H, int W, const float* intr, float* pts, hipStream_t s) {
  if (B <= 0 || H <= 0 || W <= 0 || B > 65535 || H > 65535 || !depth || !intr || !pts) return -22;
  if (((uintptr_t)pts & 15) || intr[0] == 0.0f || intr[1] == 0.0f) return -22;
  const Intr k{intr[0], intr[1], intr[2], intr[3]};
  unproject_kernel<<<dim3(cdiv(W, RT), H, B), RT, 0, s>>>(depth, H, W, k, reinterpret_cast<float4*>(pts));
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int launch_render_view(const float* pts, const uint8_t* rgb, int B, int H, int W, const float* pose,
                       const float* intr, int Ho, int Wo, unsigned long long* zbuf, uint8_t* rgb_out,
                       uint16_t* depth_out, hipStream_t s) {
  if (B <= 0 || H <= 0 || W <= 0 || Ho <= 0 || Wo <= 0 || B > 65535 || H > 65535 || Ho > 65535) return -22;
  if ((long long)H * W > 0xffffffffLL || !pts || !rgb || !pose || !intr || !zbuf || !rgb_out || !depth_out) return -22;
  if (((uintptr_t)pts & 15) || ((uintptr_t)zbuf & 7) || ((uintptr_t)depth_out & 1)) return -22;
  Pose P;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) P.r[3 * i + j] = pose[4 * i + j];
    P.t[i] = pose[4 * i + 3];
  }
  const Intr k{intr[0], intr[1], intr[2], intr[3]};
  const long long nz = (long long)B * Ho * Wo;
  if (cdivll(nz, RT) > 0x7fffffffLL) return -22;
  zbuf_clear_kernel<<<(unsigned)cdivll(nz, RT), RT, 0, s>>>(zbuf, nz);
  splat_kernel<<<dim3(cdiv(W, RT), H, B), RT, 0, s>>>(reinterpret_cast<const float4*>(pts), H, W, P, k, Ho, Wo, zbuf);
  resolve_kernel<<<dim3(cdiv(Wo, RT), Ho, B), RT, 0, s>>>(zbuf, rgb, H, W, Ho, Wo, rgb_out, depth_out);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace revo
