// Blend-and-accumulate (Sec. 3.2, Eq. 3 / Eq. 5): for every tile of every
// view, walk the tile's depth-ordered Gaussians front to back, form the
// alpha-blending weight w_i(p) = alpha_i(p) T_i(p) of each Gaussian at each
// pixel (Eq. 1), and scatter w_i(p) F(p) and w_i(p) into the per-Gaussian
// accumulators U_i and beta_i.  W is never materialised.
//
// One workgroup = one wave64 = one 8x8 quadrant of a 16x16 tile (one pixel
// per lane) x one group of DG channels.  Waves never wait for each other: no
// barriers, a wave retires as soon as its 64 pixels are done.  Per step of 32
// Gaussians of the tile's list:
//   0. lane j loads Gaussian j's record (vector loads, all in flight
//      together) and tests whether its alpha >= 1/255 region can touch the
//      quadrant (exact minimum of the conic over the quadrant, conservative
//      slack); a ballot gives the step's hit mask;
//   A. walk: each lane evaluates the hit Gaussians for its pixel in order
//      (record fields broadcast with readlane), keeping w in VGPRs;
//   B. accumulate and scatter: per hit Gaussian with some w > 0, the wave
//      visits those lanes and sums w * F (DG = 64: one channel per lane, w by
//      readlane, eight feature reads in flight; DG < 64: 64/DG pixel slots of
//      DG channels, w by permute, slots reduced by shuffles), then issues one
//      global atomic per channel and one compensated update of beta.
#include "lv_internal.h"

namespace lv {

namespace {

template <lv_dtype DT>
__device__ __forceinline__ float load_feature(const void* map, int64_t idx, float scale) {
  if constexpr (DT == LV_F32) {
    return static_cast<const float*>(map)[idx];
  } else if constexpr (DT == LV_BF16) {
    uint32_t b = static_cast<const uint16_t*>(map)[idx];
    return __uint_as_float(b << 16);
  } else {
    uint32_t b = static_cast<const uint8_t*>(map)[idx];
    uint32_t e = (b >> 3) & 0xFu, mt = b & 7u;
    float mag = e ? __uint_as_float(((e + 120u) << 23) | (mt << 20)) : (float)mt * 0x1.0p-9f;
    return ((b & 0x80u) ? -mag : mag) * scale;
  }
}

// Can -power(d) <= tau hold for some d in the rectangle [X0,X1] x [Y0,Y1]
// (offsets from the Gaussian's centre)?  -power = a dx^2 + b dx dy + c dy^2 is
// convex with its minimum at 0, so outside the rectangle its minimum over the
// rectangle lies on an edge; each edge is a 1D quadratic with a clamped vertex.
__device__ __forceinline__ bool region_hits(float4 r0, float4 r1, float X0, float X1, float Y0,
                                            float Y1) {
  const float tau = r1.z;
  if (!(tau >= 0.0f)) return false;
  if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return true;
  const float a = -r0.z, b = -r0.w, c = -r1.x;
  const float h2c = 0.5f / c, h2a = 0.5f / a;
  float dy0 = fminf(fmaxf(-b * X0 * h2c, Y0), Y1);
  float dy1 = fminf(fmaxf(-b * X1 * h2c, Y0), Y1);
  float dx0 = fminf(fmaxf(-b * Y0 * h2a, X0), X1);
  float dx1 = fminf(fmaxf(-b * Y1 * h2a, X0), X1);
  float q0 = (a * X0 + b * dy0) * X0 + c * dy0 * dy0;
  float q1 = (a * X1 + b * dy1) * X1 + c * dy1 * dy1;
  float q2 = a * dx0 * dx0 + (b * dx0 + c * Y0) * Y0;
  float q3 = a * dx1 * dx1 + (b * dx1 + c * Y1) * Y1;
  return fminf(fminf(q0, q1), fminf(q2, q3)) <= tau;
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}

// Sum over the 64 lanes of the wave with DPP (within rows: quad swaps and
// mirrors; across rows: row broadcasts), returned as a wave-uniform value.
__device__ __forceinline__ float wave_sum(float x) {
  x += dpp_f<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
  x += dpp_f<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
  x += dpp_f<0x141, 0xF>(x);  // row_half_mirror
  x += dpp_f<0x140, 0xF>(x);  // row_mirror
  x += dpp_f<0x142, 0xA>(x);  // row_bcast:15 into rows 1, 3
  x += dpp_f<0x143, 0xC>(x);  // row_bcast:31 into rows 2, 3
  return readlane_f(x, 63);
}

template <lv_dtype DT, int DG, bool FLDS>
__global__ __launch_bounds__(64) void blend_kernel(
    const Rec* __restrict__ rec, const uint32_t* __restrict__ ids, const uint2* __restrict__ ranges,
    const ViewGeom* __restrict__ geom, const void* const* __restrict__ maps,
    const float* __restrict__ fp8_scales, int view_base, int64_t n, int D, int tiles_stride,
    float* __restrict__ U, float2* __restrict__ beta, uint32_t* __restrict__ counts,
    unsigned long long* __restrict__ stats) {
  constexpr int G = kChunk;
  constexpr int SLOTS = 64 / DG;  // pixel slots per wave in step B
  extern __shared__ float Fs[];   // [64][DG] when FLDS

  const int v = blockIdx.y, quad = blockIdx.x & 3, tile = blockIdx.x >> 2, cg = blockIdx.z;
  const ViewGeom g = geom[v];
  if (tile >= g.TX * g.TY) return;
  const uint2 rg = ranges[(int64_t)v * tiles_stride + tile];
  if (rg.y <= rg.x) return;
  const int lane = threadIdx.x;
  const int tx = tile % g.TX, ty = tile / g.TX;
  const int qx = tx * kTile + (quad & 1) * 8, qy = ty * kTile + (quad >> 1) * 8;
  if (qx >= g.W || qy >= g.H) return;  // quadrant entirely outside the image
  const int px = qx + (lane & 7), py = qy + (lane >> 3);
  const bool inside = px < g.W && py < g.H;
  const int c0 = cg * DG;
  const int dv = D - c0 < DG ? D - c0 : DG;  // valid channels in this group
  const void* map = maps[v];
  float fsc = 1.0f;  // FP8 scale of this lane's channel
  const int slot = lane / DG, ch = lane - slot * DG;
  if constexpr (DT == LV_FP8_E4M3) {
    if (ch < dv) fsc = fp8_scales[(int64_t)(view_base + v) * D + c0 + ch];
  }

  if constexpr (FLDS) {
    // this quadrant's features for channels [c0, c0 + dv); pixel p = lane index
    for (int e = lane; e < 64 * DG; e += 64) {
      int p = e / DG, c = e - p * DG;
      int gx = qx + (p & 7), gy = qy + (p >> 3);
      float val = 0.0f;
      if (c < dv && gx < g.W && gy < g.H) {
        float sc = 1.0f;
        if constexpr (DT == LV_FP8_E4M3) sc = fp8_scales[(int64_t)(view_base + v) * D + c0 + c];
        val = load_feature<DT>(map, ((int64_t)gy * g.W + gx) * D + c0 + c, sc);
      }
      Fs[e] = val;
    }
    __syncthreads();
  }
  // feature of channel ch at the wave's pixel l
  auto feat = [&](int l) -> float {
    if constexpr (FLDS) {
      return Fs[l * DG + ch];
    } else {
      const int gx = qx + (l & 7), gy = qy + (l >> 3);
      if (ch >= dv || gx >= g.W || gy >= g.H) return 0.0f;
      return load_feature<DT>(map, ((int64_t)gy * g.W + gx) * D + c0 + ch, fsc);
    }
  };

  const Rec* vrec = rec + (int64_t)v * n;
  const float pxf = (float)px + 0.5f, pyf = (float)py + 0.5f;
  const float qx0 = (float)qx + 0.5f, qx1 = (float)qx + 7.5f;
  const float qy0 = (float)qy + 0.5f, qy1 = (float)qy + 7.5f;
  float T = 1.0f;
  bool alive = inside;
  uint32_t ncontrib = 0;  // this pixel's counted Gaussians (statistics only)

  for (uint32_t base = rg.x; base < rg.y; base += G) {
    if (__ballot(alive) == 0ull) break;
    const int cnt = (int)(rg.y - base < (uint32_t)G ? rg.y - base : (uint32_t)G);

    // ---- 0: records of this step, one per lane; quadrant test
    float4 q0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), q1 = make_float4(0.0f, 0.0f, -1.0f, 0.0f);
    uint32_t my_id = 0;
    if (lane < cnt) {
      my_id = ids[base + lane];
      q0 = vrec[my_id].r0;
      q1 = vrec[my_id].r1;
    }
    const bool lane_hit =
        lane < cnt && region_hits(q0, q1, qx0 - q0.x, qx1 - q0.x, qy0 - q0.y, qy1 - q0.y);
    const uint64_t hits = __ballot(lane_hit);

    // ---- A: walk
    float wv[G];
#pragma unroll
    for (int j = 0; j < G; j++) {
      wv[j] = 0.0f;
      if ((hits >> j) & 1ull) {
        const float ux = readlane_f(q0.x, j), uy = readlane_f(q0.y, j);
        const float A = readlane_f(q0.z, j), B = readlane_f(q0.w, j);
        const float C = readlane_f(q1.x, j), op = readlane_f(q1.y, j);
        // branch-free: every lane evaluates, selects keep the walk exact
        float dx = pxf - ux, dy = pyf - uy;
        float pw = (B * dx) * dy;
        pw = __builtin_fmaf(C * dy, dy, pw);
        pw = __builtin_fmaf(A * dx, dx, pw);
        pw = fminf(pw, 0.0f);
        const float al = fminf(kAlphaMax, op * exp32(pw));
        const bool ok = alive && al >= kAlphaMin;
        const float Tn = T * (1.0f - al);
        const bool stop = ok && Tn < kTEps;
        const bool take = ok && !stop;
        wv[j] = take ? al * T : 0.0f;
        T = take ? Tn : T;
        alive = alive && !stop;
        ncontrib += take ? 1u : 0u;
      }
    }

    // ---- B: accumulate and scatter, one Gaussian at a time
#pragma unroll
    for (int j = 0; j < G; j++) {
      if ((hits >> j) & 1ull) {
        const uint64_t msk = __ballot(wv[j] > 0.0f);
        if (msk) {
          float acc = 0.0f, ws;
          if constexpr (SLOTS == 1) {
            // rows of 8 pixels of the quadrant that hold a contribution; within
            // an active row every pixel is visited (w = 0 adds nothing): lanes
            // and LDS offsets are compile-time constants, no scalar bit loops
            const int wj = __float_as_int(wv[j]);
#pragma unroll
            for (int r = 0; r < 8; r++) {
              if ((msk >> (8 * r)) & 0xFFull) {
                float wl[8], fv[8];
#pragma unroll
                for (int k = 0; k < 8; k++) {
                  wl[k] = __int_as_float(__builtin_amdgcn_readlane(wj, 8 * r + k));
                  fv[k] = feat(8 * r + k);
                }
#pragma unroll
                for (int k = 0; k < 8; k++) acc = __builtin_fmaf(wl[k], fv[k], acc);
              }
            }
            ws = wave_sum(wv[j]);
          } else {
            // slot s takes the pixels p = s (mod SLOTS) of the wave
            uint64_t sel = 0ull;
#pragma unroll
            for (int k = 0; k < 64; k += SLOTS) sel |= 1ull << k;
            uint64_t mm = msk & (sel << slot);
            float wsl = 0.0f;
            while (__ballot(mm != 0ull)) {
              const bool has = mm != 0ull;
              const int l = has ? (int)__builtin_ctzll(mm) : 0;
              if (has) mm &= mm - 1ull;
              const float wl = __shfl(wv[j], l, 64);  // every lane takes part
              if (has) {
                acc = __builtin_fmaf(wl, feat(l), acc);
                wsl += wl;
              }
            }
#pragma unroll
            for (int o = DG; o < 64; o <<= 1) {
              acc += __shfl_down(acc, o, 64);
              wsl += __shfl_down(wsl, o, 64);
            }
            ws = wsl;
          }
          const uint32_t gid = (uint32_t)__builtin_amdgcn_readlane((int)my_id, j);
          if (lane < dv && acc != 0.0f) unsafeAtomicAdd(&U[(int64_t)gid * D + c0 + lane], acc);
          if (lane == 0 && cg == 0) {
            twosum_atomic_add(&beta[gid], ws);
            if (counts) atomicAdd(&counts[gid], (uint32_t)__popcll(msk));
          }
        }
      }
    }
  }
  if (counts && cg == 0) {
    // covered pixels and contributions of this quadrant
    const uint64_t covered = __ballot(ncontrib != 0u);
    uint64_t s = ncontrib;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) {
      atomicAdd(&stats[1], (unsigned long long)s);
      atomicAdd(&stats[0], (unsigned long long)__popcll(covered));
    }
  }
}

template <lv_dtype DT, int DG, bool FLDS>
hipError_t launch_blend_dg(const BlendArgs& a, int m, int max_tiles, hipStream_t s) {
  size_t lds = FLDS ? sizeof(float) * 64 * DG : 0;
  int groups = (a.D + DG - 1) / DG;
  hipLaunchKernelGGL((blend_kernel<DT, DG, FLDS>), dim3(max_tiles * 4, m, groups), dim3(64), lds, s,
                     a.rec, a.ids, a.ranges, a.geom, a.maps, a.fp8_scales, a.view_base, a.n, a.D,
                     a.tiles_stride, a.U, a.beta, a.counts, a.stats);
  return hipGetLastError();
}

template <lv_dtype DT>
hipError_t launch_blend_t(const BlendArgs& a, int m, int max_tiles, hipStream_t s) {
  if (a.D <= 1) return launch_blend_dg<DT, 1, true>(a, m, max_tiles, s);
  if (a.D <= 2) return launch_blend_dg<DT, 2, true>(a, m, max_tiles, s);
  if (a.D <= 4) return launch_blend_dg<DT, 4, true>(a, m, max_tiles, s);
  if (a.D <= 8) return launch_blend_dg<DT, 8, true>(a, m, max_tiles, s);
  if (a.D <= 16) return launch_blend_dg<DT, 16, true>(a, m, max_tiles, s);
  if (a.D <= 32) return launch_blend_dg<DT, 32, true>(a, m, max_tiles, s);
  return launch_blend_dg<DT, 64, true>(a, m, max_tiles, s);
}

__global__ void finalize_kernel(const float* __restrict__ U, const float2* __restrict__ beta,
                                int64_t n, int D, float* __restrict__ f, float* __restrict__ wsum,
                                float* __restrict__ usum) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * D) return;
  int64_t i = e / D;
  float2 b = beta[i];
  float bs = b.x + b.y;
  float u = U[e];
  if (f) f[e] = bs > 0.0f ? u / bs : 0.0f;
  if (usum) usum[e] = u;
  if (wsum && e - i * D == 0) wsum[i] = bs;
}

}  // namespace

hipError_t launch_blend(const BlendArgs& a, lv_dtype dtype, int m, int max_tiles, hipStream_t s) {
  if (m == 0 || max_tiles == 0) return hipSuccess;
  switch (dtype) {
    case LV_F32: return launch_blend_t<LV_F32>(a, m, max_tiles, s);
    case LV_BF16: return launch_blend_t<LV_BF16>(a, m, max_tiles, s);
    case LV_FP8_E4M3: return launch_blend_t<LV_FP8_E4M3>(a, m, max_tiles, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const float* U, const float2* beta, int64_t n, int D, float* f,
                           float* wsum, float* usum, hipStream_t s) {
  int64_t total = n * (int64_t)D;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, U,
                     beta, n, D, f, wsum, usum);
  return hipGetLastError();
}

}  // namespace lv
