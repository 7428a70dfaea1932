// Scene residency and per-view projection (Sec. 3.1): covariance from scale
// and rotation, EWA projection to a 2D conic, tile rectangle, depth key.
// Every quantity that decides structure (visibility, rectangle, key, conic)
// is computed by a fixed sequence of FP32 operations (no contraction), so it
// is identical on any IEEE-754 machine that evaluates the same sequence.
#include "lv_internal.h"

namespace lv {

// Sigma = R diag(s)^2 R^T of the normalised quaternion (w, x, y, z), upper
// triangle (00, 01, 02, 11, 12, 22).  Scene layout, 48 bytes per Gaussian:
//   p0 = (mu_x, mu_y, mu_z, opacity), p1 = (S00, S01, S02, S11), p2 = (S12, S22, 0, 0)
__global__ void scene_derive_kernel(const float* __restrict__ means, const float* __restrict__ scales,
                                    const float* __restrict__ quats, const float* __restrict__ opacity,
                                    int64_t n, float4* __restrict__ p0, float4* __restrict__ p1,
                                    float4* __restrict__ p2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* q = quats + 4 * i;
  const float* s = scales + 3 * i;
  float q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  float n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
  float w = 1.0f, x = 0.0f, y = 0.0f, z = 0.0f;
  if (n2 > 0.0f) {
    float nr = sqrtf(n2);
    w = q0 / nr;
    x = q1 / nr;
    y = q2 / nr;
    z = q3 / nr;
  }
  float R[9];
  R[0] = 1.0f - 2.0f * (y * y + z * z);
  R[1] = 2.0f * (x * y - w * z);
  R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z);
  R[4] = 1.0f - 2.0f * (x * x + z * z);
  R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y);
  R[7] = 2.0f * (y * z + w * x);
  R[8] = 1.0f - 2.0f * (x * x + y * y);
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int c = 0; c < 3; c++) M[3 * r + c] = R[3 * r + c] * s[c];
  float S[6];
  const int I[6] = {0, 0, 0, 1, 1, 2}, J[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int e = 0; e < 6; e++) {
    const float* a = M + 3 * I[e];
    const float* b = M + 3 * J[e];
    S[e] = (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
  }
  p0[i] = make_float4(means[3 * i], means[3 * i + 1], means[3 * i + 2], opacity[i]);
  p1[i] = make_float4(S[0], S[1], S[2], S[3]);
  p2[i] = make_float4(S[4], S[5], 0.0f, 0.0f);
}

hipError_t launch_scene_derive(const float* means, const float* scales, const float* quats,
                               const float* opacity, int64_t n, float4* p0, float4* p1, float4* p2,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(scene_derive_kernel, dim3((unsigned)blocks), dim3(256), 0, s, means, scales,
                     quats, opacity, n, p0, p1, p2);
  return hipGetLastError();
}

// One thread per (view, Gaussian).  Outputs:
//   key  = FP32 bits of z_c for visible Gaussians, 0xFFFFFFFF otherwise
//   val  = Gaussian index (the payload of the depth sort)
//   rect = tile rectangle packed as (x0 | y0 << 16, x1 | y1 << 16)
//   cnt  = number of tiles in the rectangle (0 if not visible)
//   rec  = conic record (see Rec)
__global__ void preprocess_kernel(const float4* __restrict__ p0, const float4* __restrict__ p1,
                                  const float4* __restrict__ p2, int64_t n,
                                  const Cam* __restrict__ cams, const ViewGeom* __restrict__ geom,
                                  Rec* __restrict__ rec, uint32_t* __restrict__ key,
                                  uint32_t* __restrict__ val, uint2* __restrict__ rect,
                                  uint32_t* __restrict__ cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int v = blockIdx.y;
  if (i >= n) return;
  int64_t o = (int64_t)v * n + i;
  const Cam& c = cams[v];
  const ViewGeom g = geom[v];
  float4 a0 = p0[i], a1 = p1[i], a2 = p2[i];
  val[o] = (uint32_t)i;
  key[o] = 0xFFFFFFFFu;
  cnt[o] = 0u;
  rect[o] = make_uint2(0u, 0u);
  rec[o].r1 = make_float4(0.0f, 0.0f, -1.0f, -1.0f);

  float mx = a0.x, my = a0.y, mz = a0.z, op = a0.w;
  float xc = ((c.R[0] * mx + c.R[1] * my) + c.R[2] * mz) + c.t[0];
  float yc = ((c.R[3] * mx + c.R[4] * my) + c.R[5] * mz) + c.t[1];
  float zc = ((c.R[6] * mx + c.R[7] * my) + c.R[8] * mz) + c.t[2];
  if (!(zc > c.znear)) return;
  float ix = xc / zc, iy = yc / zc;
  float ux = c.fx * ix + c.cx, uy = c.fy * iy + c.cy;
  float limx = kClamp * ((0.5f * (float)g.W) / c.fx);
  float limy = kClamp * ((0.5f * (float)g.H) / c.fy);
  float tx = fminf(limx, fmaxf(-limx, ix));
  float ty = fminf(limy, fmaxf(-limy, iy));
  float j00 = c.fx / zc, j11 = c.fy / zc;
  float j02 = -(j00 * tx), j12 = -(j11 * ty);
  float T[6];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    T[k] = j00 * c.R[k] + j02 * c.R[6 + k];
    T[3 + k] = j11 * c.R[3 + k] + j12 * c.R[6 + k];
  }
  const float S[9] = {a1.x, a1.y, a1.z, a1.y, a1.w, a2.x, a1.z, a2.x, a2.y};
  float V[6];
#pragma unroll
  for (int r = 0; r < 2; r++)
#pragma unroll
    for (int k = 0; k < 3; k++)
      V[3 * r + k] = (T[3 * r] * S[k] + T[3 * r + 1] * S[3 + k]) + T[3 * r + 2] * S[6 + k];
  float sa = ((V[0] * T[0] + V[1] * T[1]) + V[2] * T[2]) + kDilate;
  float sb = (V[0] * T[3] + V[1] * T[4]) + V[2] * T[5];
  float sc = ((V[3] * T[3] + V[4] * T[4]) + V[5] * T[5]) + kDilate;
  float det = sa * sc - sb * sb;
  if (!(det > 0.0f)) return;
  float h = 0.5f * (sa + sc), dd = 0.5f * (sa - sc);
  float lam = h + sqrtf(dd * dd + sb * sb);
  float r = ceilf(3.0f * sqrtf(lam));
  float fx0 = floorf((ux - r) / (float)kTile);
  float fx1 = floorf((ux + r) / (float)kTile) + 1.0f;
  float fy0 = floorf((uy - r) / (float)kTile);
  float fy1 = floorf((uy + r) / (float)kTile) + 1.0f;
  int x0 = (int)fminf(fmaxf(fx0, 0.0f), (float)g.TX), x1 = (int)fminf(fmaxf(fx1, 0.0f), (float)g.TX);
  int y0 = (int)fminf(fmaxf(fy0, 0.0f), (float)g.TY), y1 = (int)fminf(fmaxf(fy1, 0.0f), (float)g.TY);
  if (x1 <= x0 || y1 <= y0) return;

  float A = -0.5f * (sc / det);
  float B = sb / det;
  float C = -0.5f * (sa / det);
  // Culling bound: alpha >= 1/255 needs -(A dx^2 + B dx dy + C dy^2) <=
  // ln(opacity * 255); tau adds generous slack so that rounding of the
  // exponent can never make a skipped pixel count.  -1: never reachable.
  float tau = op >= kAlphaMin ? (logf(op / kAlphaMin) + 0.01f) * 1.01f : -1.0f;
  key[o] = __float_as_uint(zc);
  cnt[o] = (uint32_t)((x1 - x0) * (y1 - y0));
  rect[o] = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
  rec[o].r0 = make_float4(ux, uy, A, B);
  rec[o].r1 = make_float4(C, op, tau, 0.0f);
}

hipError_t launch_preprocess(const float4* p0, const float4* p1, const float4* p2, int64_t n,
                             const Cam* cams, const ViewGeom* geom, int m, Rec* rec,
                             uint32_t* key, uint32_t* val, uint2* rect, uint32_t* cnt,
                             hipStream_t s) {
  if (n == 0 || m == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)blocks, (unsigned)m), dim3(256), 0, s, p0,
                     p1, p2, n, cams, geom, rec, key, val, rect, cnt);
  return hipGetLastError();
}

}  // namespace lv
