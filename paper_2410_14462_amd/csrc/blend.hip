// Blend-and-accumulate (Sec. 3.2, Eq. 3 / Eq. 5): for every tile of every
// view, walk the tile's depth-ordered Gaussians front to back, form the
// alpha-blending weight w_i(p) = alpha_i(p) T_i(p) of each Gaussian at each
// pixel (Eq. 1), and scatter w_i(p) F(p) and w_i(p) into the per-Gaussian
// accumulators U_i and beta_i.  W is never materialised.
//
// One workgroup = one 16x16 tile x one group of 64 channels; 4 wave64s, each
// owning an 8x8 quadrant (one pixel per lane).  Per step of 32 Gaussians:
//   A. walk: each lane evaluates the 32 Gaussians for its pixel in order
//      (records fetched with scalar loads; a wave skips a Gaussian whose
//      conservative footprint box misses its quadrant), keeping w in VGPRs;
//   B. accumulate: per Gaussian, the wave visits the lanes with w > 0 and,
//      one channel per lane, sums w * F from the LDS-staged tile; the four
//      waves' partials meet in LDS; then one global atomic per (Gaussian,
//      channel) and one compensated update of beta.
#include "lv_internal.h"

namespace lv {

namespace {

constexpr int kDG = 64;  // channels per workgroup

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

template <lv_dtype DT>
__global__ __launch_bounds__(kBlendThreads, 2) void blend_kernel(
    const Rec* __restrict__ rec, const uint32_t* __restrict__ ids, const uint2* __restrict__ ranges,
    const ViewGeom* __restrict__ geom, const void* const* __restrict__ maps,
    const float* __restrict__ fp8_scales, int view_base, int64_t n, int D, int tiles_stride,
    float* __restrict__ U, float2* __restrict__ beta, uint32_t* __restrict__ counts) {
  extern __shared__ float smem[];
  float* Fs = smem;                                    // [256][kDG]
  float* red = Fs + kBlendThreads * kDG;               // [kChunk][kDG]
  float* redb = red + kChunk * kDG;                    // [kChunk]
  uint32_t* redc = reinterpret_cast<uint32_t*>(redb + kChunk);  // [kChunk]
  uint32_t* gids = redc + kChunk;                      // [kChunk]

  const int v = blockIdx.y, tile = blockIdx.x, cg = blockIdx.z;
  const ViewGeom g = geom[v];
  if (tile >= g.TX * g.TY) return;
  const uint2 rg = ranges[(int64_t)v * tiles_stride + tile];
  if (rg.y <= rg.x) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int tx = tile % g.TX, ty = tile / g.TX;
  const int qx = tx * kTile + (w & 1) * 8, qy = ty * kTile + (w >> 1) * 8;
  const int px = qx + (lane & 7), py = qy + (lane >> 3);
  const bool inside = px < g.W && py < g.H;
  const int c0 = cg * kDG;
  const int dv = D - c0 < kDG ? D - c0 : kDG;  // valid channels in this group

  // Stage the tile's features for channels [c0, c0 + dv) in LDS.  Pixel index
  // of thread t is t (quadrant-major), matching the walk below.
  const void* map = maps[v];
  for (int e = t; e < kBlendThreads * kDG; e += kBlendThreads) {
    int p = e / kDG, c = e - p * kDG;
    int ww = p >> 6, ll = p & 63;
    int gx = tx * kTile + (ww & 1) * 8 + (ll & 7), gy = ty * kTile + (ww >> 1) * 8 + (ll >> 3);
    float val = 0.0f;
    if (c < dv && gx < g.W && gy < g.H) {
      float sc = 1.0f;
      if constexpr (DT == LV_FP8_E4M3) sc = fp8_scales[(int64_t)(view_base + v) * D + c0 + c];
      val = load_feature<DT>(map, ((int64_t)gy * g.W + gx) * D + c0 + c, sc);
    }
    Fs[e] = val;
  }
  for (int e = t; e < kChunk * kDG; e += kBlendThreads) red[e] = 0.0f;
  if (t < kChunk) {
    redb[t] = 0.0f;
    redc[t] = 0u;
  }
  __syncthreads();

  const Rec* vrec = rec + (int64_t)v * n;
  const float pxf = (float)px + 0.5f, pyf = (float)py + 0.5f;
  const float qlox = (float)qx + 0.5f, qhix = (float)qx + 7.5f;
  const float qloy = (float)qy + 0.5f, qhiy = (float)qy + 7.5f;
  float T = 1.0f;
  bool alive = inside;
  const float* fcol = Fs + (w * 64) * kDG + lane;  // this lane's channel, pixel 0 of the wave

  for (uint32_t base = rg.x; base < rg.y; base += kChunk) {
    if (!__syncthreads_or(alive)) break;
    const int cnt = (int)(rg.y - base < (uint32_t)kChunk ? rg.y - base : (uint32_t)kChunk);
    if (t < cnt) gids[t] = ids[base + t];

    // ---- A: walk
    float wv[kChunk];
    const bool wave_alive = __ballot(alive) != 0ull;
#pragma unroll
    for (int j = 0; j < kChunk; j++) {
      wv[j] = 0.0f;
      if (j < cnt && wave_alive) {
        const uint32_t gid = __builtin_amdgcn_readfirstlane(ids[base + j]);
        const float4 r0 = vrec[gid].r0;
        const float4 r1 = vrec[gid].r1;
        const bool hit = !(r0.x + r1.z < qlox || r0.x - r1.z > qhix || r0.y + r1.w < qloy ||
                           r0.y - r1.w > qhiy);
        if (hit && alive) {
          float dx = pxf - r0.x, dy = pyf - r0.y;
          float pw = (r0.w * dx) * dy;
          pw = __builtin_fmaf(r1.x * dy, dy, pw);
          pw = __builtin_fmaf(r0.z * dx, dx, pw);
          pw = fminf(pw, 0.0f);
          float al = fminf(kAlphaMax, r1.y * exp32(pw));
          if (al >= kAlphaMin) {
            float Tn = T * (1.0f - al);
            if (Tn < kTEps) {
              alive = false;
            } else {
              wv[j] = al * T;
              T = Tn;
            }
          }
        }
      }
    }
    __syncthreads();  // gids visible

    // ---- B: accumulate, one Gaussian at a time, one channel per lane
#pragma unroll
    for (int j = 0; j < kChunk; j++) {
      if (j < cnt) {
        uint64_t msk = __ballot(wv[j] > 0.0f);
        if (msk) {
          const uint32_t nc = (uint32_t)__popcll(msk);
          float acc = 0.0f, ws = 0.0f;
          const int wj = __float_as_int(wv[j]);
          while (msk) {
            const int l = (int)__builtin_ctzll(msk);
            msk &= msk - 1ull;
            const float wl = __int_as_float(__builtin_amdgcn_readlane(wj, l));
            acc = __builtin_fmaf(wl, fcol[l * kDG], acc);
            ws += wl;
          }
          atomicAdd(&red[j * kDG + lane], acc);
          if (lane == 0) {
            atomicAdd(&redb[j], ws);
            atomicAdd(&redc[j], nc);
          }
        }
      }
    }
    __syncthreads();

    // ---- flush the step: one atomic per (Gaussian, channel)
    for (int e = t; e < cnt * kDG; e += kBlendThreads) {
      int j = e / kDG, c = e - j * kDG;
      if (redc[j] != 0u && c < dv) unsafeAtomicAdd(&U[(int64_t)gids[j] * D + c0 + c], red[e]);
      red[e] = 0.0f;
    }
    __syncthreads();
    if (t < cnt) {
      if (redc[t] != 0u && cg == 0) {
        kahan_atomic_add(&beta[gids[t]], redb[t]);
        if (counts) atomicAdd(&counts[gids[t]], redc[t]);
      }
      redb[t] = 0.0f;
      redc[t] = 0u;
    }
  }
}

template <lv_dtype DT>
hipError_t launch_blend_t(const BlendArgs& a, int m, int max_tiles, hipStream_t s) {
  size_t lds = sizeof(float) * (kBlendThreads * kDG + kChunk * kDG + kChunk) +
               sizeof(uint32_t) * 2 * kChunk;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&blend_kernel<DT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  int groups = (a.D + kDG - 1) / kDG;
  hipLaunchKernelGGL(blend_kernel<DT>, dim3(max_tiles, m, groups), dim3(kBlendThreads), lds, s,
                     a.rec, a.ids, a.ranges, a.geom, a.maps, a.fp8_scales, a.view_base, a.n, a.D,
                     a.tiles_stride, a.U, a.beta, a.counts);
  return hipGetLastError();
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
