// Scene residency and per-view projection (Sec. 3.1): covariance from scale
// and rotation, EWA projection to a 2D conic, tile rectangle, depth key.
// Every quantity that decides structure (visibility, rectangle, key, conic)
// is computed by a fixed sequence of FP32 operations (no contraction), so it
// is identical on any IEEE-754 machine that evaluates the same sequence.
#include "lv_internal.h"

namespace lv {

// Scene layout, 48 bytes per Gaussian:
//   p0 = (mu_x, mu_y, mu_z, opacity), p1 = normalised quaternion (w, x, y, z),
//   p2 = (s_x, s_y, s_z, 0).
// The covariance Sigma = M M^T, M = R diag(s), is never formed: projection
// builds the 2D covariance from T M (see preprocess_kernel).
__global__ void scene_derive_kernel(const float* __restrict__ means, const float* __restrict__ scales,
                                    const float* __restrict__ quats, const float* __restrict__ opacity,
                                    int64_t n, float4* __restrict__ p0, float4* __restrict__ p1,
                                    float4* __restrict__ p2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* q = quats + 4 * i;
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
  p0[i] = make_float4(means[3 * i], means[3 * i + 1], means[3 * i + 2], opacity[i]);
  p1[i] = make_float4(w, x, y, z);
  p2[i] = make_float4(scales[3 * i], scales[3 * i + 1], scales[3 * i + 2], 0.0f);
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

__global__ void gather_scene_kernel(const float4* __restrict__ c0, const float4* __restrict__ c1,
                                    const float4* __restrict__ c2, const uint32_t* __restrict__ perm,
                                    int64_t n, float4* __restrict__ p0, float4* __restrict__ p1,
                                    float4* __restrict__ p2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  p0[i] = c0[j];
  p1[i] = c1[j];
  p2[i] = c2[j];
}

hipError_t launch_gather_scene(const float4* c0, const float4* c1, const float4* c2,
                               const uint32_t* perm, int64_t n, float4* p0, float4* p1, float4* p2,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_scene_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c0, c1, c2,
                     perm, n, p0, p1, p2);
  return hipGetLastError();
}

// Error-free transformations for the projected centre.  Pixel coordinates
// reach ~10^3 px, where one FP32 ulp (6e-5 px) already shifts the exponent of
// a compact Gaussian by ~1e-4, so the centre is carried as hi + lo: TwoSum
// (Knuth), TwoProduct by fma, the compensated dot product Dot2 (Ogita, Rump,
// Oishi, SIAM J. Sci. Comput. 26(6), 2005) for x_c = R x_w + t, a corrected
// quotient x_c / z_c and a compensated affine map u = f i + c.  lo keeps its
// 8 leading significand bits so that the two low parts pack into one word.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

__device__ __forceinline__ void dot3(const float* r, float m0, float m1, float m2, float t, float& hi,
                                     float& lo) {
  float p, s, h, q, e;
  two_prod(r[0], m0, p, s);
  two_prod(r[1], m1, h, q);
  two_sum(p, h, p, e);
  s = s + (q + e);
  two_prod(r[2], m2, h, q);
  two_sum(p, h, p, e);
  s = s + (q + e);
  two_sum(p, t, p, e);
  s = s + e;
  hi = p + s;
  lo = s - (hi - p);
}

// hi + lo = f (xh + xl) / (zh + zl) + c; returns lo's upper 16 bits.
__device__ __forceinline__ uint32_t center(float f, float c, float xh, float xl, float zh, float zl,
                                           float& hi) {
  const float q = xh / zh;
  float r = __builtin_fmaf(-q, zh, xh);
  r = (r + xl) - q * zl;
  const float ql = r / zh;
  float p, e, sm, g;
  two_prod(f, q, p, e);
  e = __builtin_fmaf(f, ql, e);
  two_sum(p, c, sm, g);
  g = g + e;
  hi = sm + g;
  return __float_as_uint(g - (hi - sm)) >> 16;
}

// a b - c d to within ~1.5 ulp (Kahan's algorithm).
__device__ __forceinline__ float diff_prod(float a, float b, float c, float d) {
  const float w = c * d;
  const float e = __builtin_fmaf(-c, d, w);
  return __builtin_fmaf(a, b, -w) + e;
}

// One thread per (view, Gaussian).  Outputs:
//   key  = FP32 bits of z_c for visible Gaussians, 0xFFFFFFFF otherwise
//   val  = Gaussian index (the payload of the depth sort)
//   rect = tile rectangle packed as (x0 | y0 << 16, x1 | y1 << 16)
//   cnt  = number of tiles in the rectangle (0 if not visible)
//   rec  = centre and conic record (see Rec)
__global__ void preprocess_kernel(const float4* __restrict__ p0, const float4* __restrict__ p1,
                                  const float4* __restrict__ p2, int64_t n,
                                  const Cam* __restrict__ cams, const ViewGeom* __restrict__ geom,
                                  Rec* __restrict__ rec, uint32_t* __restrict__ key,
                                  uint2* __restrict__ rect) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int v = blockIdx.y;
  if (i >= n) return;
  int64_t o = (int64_t)v * n + i;
  const Cam& c = cams[v];
  const ViewGeom g = geom[v];
  float4 a0 = p0[i], a1 = p1[i], a2 = p2[i];
  key[o] = 0xFFFFFFFFu;
  rect[o] = make_uint2(0u, 0u);
  rec[o].r1 = make_float4(0.0f, 0.0f, -1.0f, -1.0f);

  float mx = a0.x, my = a0.y, mz = a0.z, op = a0.w;
  float xc, xl, yc, yl, zc, zl;
  dot3(c.R, mx, my, mz, c.t[0], xc, xl);
  dot3(c.R + 3, mx, my, mz, c.t[1], yc, yl);
  dot3(c.R + 6, mx, my, mz, c.t[2], zc, zl);
  if (!(zc > c.znear)) return;
  float ix = xc / zc, iy = yc / zc;
  float ux, uy;
  const uint32_t uxl = center(c.fx, c.cx, xc, xl, zc, zl, ux);
  const uint32_t uyl = center(c.fy, c.cy, yc, yl, zc, zl, uy);
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
  // M = R diag(s) of the normalised quaternion, V = T M, 2D covariance
  // [[sa, sb], [sb, sc]] = V V^T + 0.3 I; det by Lagrange's identity
  // |v0|^2 |v1|^2 - (v0.v1)^2 = |v0 x v1|^2, a sum of squares.
  const float qw = a1.x, qx = a1.y, qy = a1.z, qz = a1.w;
  float R[9];
  R[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
  R[1] = 2.0f * (qx * qy - qw * qz);
  R[2] = 2.0f * (qx * qz + qw * qy);
  R[3] = 2.0f * (qx * qy + qw * qz);
  R[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
  R[5] = 2.0f * (qy * qz - qw * qx);
  R[6] = 2.0f * (qx * qz - qw * qy);
  R[7] = 2.0f * (qy * qz + qw * qx);
  R[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
  const float sv[3] = {a2.x, a2.y, a2.z};
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int k = 0; k < 3; k++) M[3 * r + k] = R[3 * r + k] * sv[k];
  float V[6];
#pragma unroll
  for (int r = 0; r < 2; r++)
#pragma unroll
    for (int k = 0; k < 3; k++)
      V[3 * r + k] = (T[3 * r] * M[k] + T[3 * r + 1] * M[3 + k]) + T[3 * r + 2] * M[6 + k];
  const float n0 = (V[0] * V[0] + V[1] * V[1]) + V[2] * V[2];
  const float n1 = (V[3] * V[3] + V[4] * V[4]) + V[5] * V[5];
  const float sb = (V[0] * V[3] + V[1] * V[4]) + V[2] * V[5];
  const float sa = n0 + kDilate, sc = n1 + kDilate;
  const float k0 = diff_prod(V[1], V[5], V[2], V[4]);
  const float k1 = diff_prod(V[2], V[3], V[0], V[5]);
  const float k2 = diff_prod(V[0], V[4], V[1], V[3]);
  const float det = (((k0 * k0 + k1 * k1) + k2 * k2) + kDilate * (n0 + n1)) + kDilate * kDilate;
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

  // Exponent -d^T Sigma2^-1 d / 2 = -((L11 dx + L12 dy)^2 + (L22 dy)^2):
  // the conditional variance of x given y, then the marginal of y.
  const float L11 = sqrtf((0.5f * sc) / det);
  const float L12 = -((sb / sc) * L11);
  const float L22 = sqrtf(0.5f / sc);
  // Culling bound: alpha >= 1/255 needs (L11 dx + L12 dy)^2 + (L22 dy)^2 <=
  // ln(opacity * 255); tau adds generous slack so that rounding of the
  // exponent can never make a skipped pixel count.  -1: never reachable.
  float tau = op >= kAlphaMin ? (logf(op / kAlphaMin) + 0.01f) * 1.01f : -1.0f;
  key[o] = __float_as_uint(zc);
  rect[o] = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
  rec[o].r0 = make_float4(ux, uy, L11, L12);
  rec[o].r1 = make_float4(L22, op, tau, __uint_as_float(uxl | (uyl << 16)));
}

hipError_t launch_preprocess(const float4* p0, const float4* p1, const float4* p2, int64_t n,
                             const Cam* cams, const ViewGeom* geom, int m, Rec* rec,
                             uint32_t* key, uint2* rect, hipStream_t s) {
  if (n == 0 || m == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)blocks, (unsigned)m), dim3(256), 0, s, p0,
                     p1, p2, n, cams, geom, rec, key, rect);
  return hipGetLastError();
}

}  // namespace lv
