// Feature-map storage codec: FP32 -> BF16 (round to nearest even) and
// FP32 -> OCP FP8 E4M3FN with one FP32 scale per channel
// (scale = absmax / 448, 1 for an all-zero channel; code = saturating
// round-to-nearest-even of x / scale).  Decoding happens inside the blend
// kernel's tile staging.
#include <algorithm>
#include <mutex>

#include "lv_internal.h"

namespace lv {

namespace {

__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint8_t to_e4m3(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t sign = (u >> 24) & 0x80u;
  float ax = fabsf(x);
  uint32_t code;
  if (!(ax < 448.0f)) {
    code = 0x7Eu;                                   // saturate (also +inf)
  } else if (ax < 0x1.0p-6f) {
    code = (uint32_t)rintf(ax * 0x1.0p9f);          // subnormal quantum 2^-9; 8 -> min normal
  } else {
    uint32_t a = __float_as_uint(ax);
    a += 0x7FFFFu + ((a >> 20) & 1u);               // round to 3 mantissa bits, ties to even
    a &= ~0xFFFFFu;
    int e = (int)(a >> 23) - 127;
    uint32_t mt = (a >> 20) & 7u;
    if (e > 8 || (e == 8 && mt > 6u)) code = 0x7Eu;
    else code = ((uint32_t)(e + 7) << 3) | mt;
  }
  return (uint8_t)(sign | code);
}

// Elements [first, total), one per thread.
__global__ void encode_bf16_kernel(const float* __restrict__ src, int64_t first, int64_t total,
                                   uint16_t* __restrict__ dst) {
  int64_t e = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) dst[e] = to_bf16(src[e]);
}

// Groups of 8 elements (two 16-byte loads, one 16-byte store), for 16-byte
// aligned arrays; a grid-stride loop.
__global__ __launch_bounds__(256) void encode_bf16_vec_kernel(const float4* __restrict__ src,
                                                              int64_t groups,
                                                              uint4* __restrict__ dst) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < groups;
       k += (int64_t)gridDim.x * 256) {
    const float4 a = src[2 * k], b = src[2 * k + 1];
    uint4 o;
    o.x = (uint32_t)to_bf16(a.x) | ((uint32_t)to_bf16(a.y) << 16);
    o.y = (uint32_t)to_bf16(a.z) | ((uint32_t)to_bf16(a.w) << 16);
    o.z = (uint32_t)to_bf16(b.x) | ((uint32_t)to_bf16(b.y) << 16);
    o.w = (uint32_t)to_bf16(b.z) | ((uint32_t)to_bf16(b.w) << 16);
    dst[k] = o;
  }
}

// Per-channel absmax: block = 4 waves over a pixel range, lane = channel.
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ src, int64_t pixels,
                                                     int D, int rows_per_block,
                                                     uint32_t* __restrict__ amax) {
  __shared__ float part[4][64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int c = blockIdx.y * 64 + lane;
  int64_t p0 = (int64_t)blockIdx.x * rows_per_block;
  int64_t p1 = p0 + rows_per_block < pixels ? p0 + rows_per_block : pixels;
  float m = 0.0f;
  if (c < D)
    for (int64_t p = p0 + w; p < p1; p += 4) m = fmaxf(m, fabsf(src[p * D + c]));
  part[w][lane] = m;
  __syncthreads();
  if (w == 0 && c < D) {
    m = fmaxf(fmaxf(part[0][lane], part[1][lane]), fmaxf(part[2][lane], part[3][lane]));
    atomicMax(&amax[c], __float_as_uint(m));
  }
}

__global__ void zero_kernel(uint32_t* __restrict__ p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void scale_kernel(const uint32_t* __restrict__ amax, int D, float* __restrict__ scales) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= D) return;
  float a = __uint_as_float(amax[c]);
  scales[c] = a > 0.0f ? a / 448.0f : 1.0f;
}

// Elements [first, total), one per thread.
__global__ void encode_fp8_kernel(const float* __restrict__ src, int64_t first, int64_t total,
                                  int D, const float* __restrict__ scales,
                                  uint8_t* __restrict__ dst) {
  int64_t e = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) dst[e] = to_e4m3(src[e] / scales[e % D]);
}

// Groups of 8 elements (two 16-byte loads, one 8-byte store), for aligned
// arrays; the channel of element 8 k + j is (8 k + j) mod D.
__global__ __launch_bounds__(256) void encode_fp8_vec_kernel(const float4* __restrict__ src,
                                                             int64_t groups, int D,
                                                             const float* __restrict__ scales,
                                                             uint2* __restrict__ dst) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < groups;
       k += (int64_t)gridDim.x * 256) {
    const float4 a = src[2 * k], b = src[2 * k + 1];
    const float x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    const int c0 = (int)((8 * k) % D);
    uint32_t lo = 0u, hi = 0u;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const uint32_t q = to_e4m3(x[j] / scales[(c0 + j) % D]);
      if (j < 4) lo |= q << (8 * j);
      else hi |= q << (8 * (j - 4));
    }
    dst[k] = make_uint2(lo, hi);
  }
}

// Pixel-block layout: thread k writes element (block k / D, channel k % D):
// the 8 pixels of its block of an image row, read from the HWC source (for
// each pixel, consecutive threads read consecutive channels) and written as
// one contiguous run (consecutive threads, consecutive runs).  Pixels past W
// are zeros.  E: element type; scales for FP8.
template <lv_dtype E>
__global__ __launch_bounds__(256) void encode_px8_kernel(const float* __restrict__ src, int W, int D,
                                                         int64_t runs,
                                                         const float* __restrict__ scales,
                                                         void* __restrict__ dst) {
  const int W8 = (W + 7) >> 3;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < runs;
       k += (int64_t)gridDim.x * 256) {
    const int c = (int)(k % D);
    const int64_t blk = k / D;
    const int64_t y = blk / W8;
    const int x0 = (int)(blk - y * W8) * 8;
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = x0 + i < W ? src[(y * W + x0 + i) * D + c] : 0.0f;
    if constexpr (E == LV_F32) {
      float4* o = static_cast<float4*>(dst) + 2 * k;
      o[0] = make_float4(v[0], v[1], v[2], v[3]);
      o[1] = make_float4(v[4], v[5], v[6], v[7]);
    } else if constexpr (E == LV_BF16) {
      uint4 o;
      o.x = (uint32_t)to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16);
      o.y = (uint32_t)to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16);
      o.z = (uint32_t)to_bf16(v[4]) | ((uint32_t)to_bf16(v[5]) << 16);
      o.w = (uint32_t)to_bf16(v[6]) | ((uint32_t)to_bf16(v[7]) << 16);
      static_cast<uint4*>(dst)[k] = o;
    } else {
      const float sc = scales[c];
      uint32_t lo = 0u, hi = 0u;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        lo |= (uint32_t)to_e4m3(v[i] / sc) << (8 * i);
        hi |= (uint32_t)to_e4m3(v[4 + i] / sc) << (8 * i);
      }
      static_cast<uint2*>(dst)[k] = make_uint2(lo, hi);
    }
  }
}

}  // namespace

hipError_t launch_encode(const float* src, int64_t pixels, int D, lv_dtype dtype, void* dst,
                         float* scales, float* tmp_absmax, hipStream_t s, int W) {
  int64_t total = pixels * (int64_t)D;
  if (total == 0) return hipSuccess;
  if (map_px8(dtype)) {
    const lv_dtype el = map_elem(dtype);
    if (el == LV_FP8_E4M3) {
      uint32_t* amax = reinterpret_cast<uint32_t*>(tmp_absmax);
      hipLaunchKernelGGL(zero_kernel, dim3((D + 255) / 256), dim3(256), 0, s, amax, D);
      int rows = 512;
      hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)((pixels + rows - 1) / rows), (D + 63) / 64),
                         dim3(256), 0, s, src, pixels, D, rows, amax);
      hipLaunchKernelGGL(scale_kernel, dim3((D + 255) / 256), dim3(256), 0, s, amax, D, scales);
    }
    const int64_t runs = pixels / W * ((W + 7) / 8) * (int64_t)D;
    const unsigned nb = (unsigned)std::min<int64_t>((runs + 255) / 256, 65536);
    if (el == LV_F32)
      hipLaunchKernelGGL(encode_px8_kernel<LV_F32>, dim3(nb), dim3(256), 0, s, src, W, D, runs, scales, dst);
    else if (el == LV_BF16)
      hipLaunchKernelGGL(encode_px8_kernel<LV_BF16>, dim3(nb), dim3(256), 0, s, src, W, D, runs, scales, dst);
    else
      hipLaunchKernelGGL(encode_px8_kernel<LV_FP8_E4M3>, dim3(nb), dim3(256), 0, s, src, W, D, runs, scales,
                         dst);
    return hipGetLastError();
  }
  if (dtype == LV_F32) {
    return hipMemcpyAsync(dst, src, (size_t)total * sizeof(float), hipMemcpyDeviceToDevice, s);
  }
  // 8 elements per thread where source and destination allow 16-byte (BF16)
  // or 8-byte (FP8) accesses, the rest one per thread
  const bool vec = ((uintptr_t)src % 16 == 0) &&
                   ((uintptr_t)dst % (dtype == LV_BF16 ? 16 : 8) == 0);
  const int64_t groups = vec ? total / 8 : 0;
  const int64_t first = groups * 8;
  const unsigned vb = (unsigned)std::min<int64_t>((groups + 255) / 256, 32768);
  const unsigned tb = (unsigned)((total - first + 255) / 256);
  if (dtype == LV_BF16) {
    if (groups)
      hipLaunchKernelGGL(encode_bf16_vec_kernel, dim3(vb), dim3(256), 0, s,
                         reinterpret_cast<const float4*>(src), groups, static_cast<uint4*>(dst));
    if (tb)
      hipLaunchKernelGGL(encode_bf16_kernel, dim3(tb), dim3(256), 0, s, src, first, total,
                         static_cast<uint16_t*>(dst));
    return hipGetLastError();
  }
  // the per-channel absmax starts at zero (a kernel, not a memset: callers
  // may capture the launches in a graph)
  uint32_t* amax = reinterpret_cast<uint32_t*>(tmp_absmax);
  hipLaunchKernelGGL(zero_kernel, dim3((D + 255) / 256), dim3(256), 0, s, amax, D);
  int rows = 512;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)((pixels + rows - 1) / rows), (D + 63) / 64),
                     dim3(256), 0, s, src, pixels, D, rows, amax);
  hipLaunchKernelGGL(scale_kernel, dim3((D + 255) / 256), dim3(256), 0, s, amax, D, scales);
  if (groups)
    hipLaunchKernelGGL(encode_fp8_vec_kernel, dim3(vb), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(src), groups, D, scales,
                       static_cast<uint2*>(dst));
  if (tb)
    hipLaunchKernelGGL(encode_fp8_kernel, dim3(tb), dim3(256), 0, s, src, first, total, D, scales,
                       static_cast<uint8_t*>(dst));
  return hipGetLastError();
}

}  // namespace lv

// ------------------------------------------------------------ no allocation
// Scratch of lv_encode_noalloc: the per-channel absmax of an FP8 encode, in
// device memory the library never allocates (each GPU holds its own copy of
// the array until the process ends).  Host code uses the per-device address
// from hipGetSymbolAddress, never the array's name.
constexpr int kNoAllocMaxD = 4096;
static __device__ __align__(256) uint32_t scratch[kNoAllocMaxD];

namespace {
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// The current device's copy of `scratch` (looked up once per device).
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" lv_status lv_encode_noalloc(const float* src, int64_t pixels, int32_t D, lv_dtype dtype,
                                       void* dst, float* scales, void* stream) {
  if (pixels < 0) return lv::set_error(LV_ERR_INVALID_ARG, "pixels = %lld < 0", (long long)pixels);
  if (D < 1 || D > kNoAllocMaxD)
    return lv::set_error(LV_ERR_INVALID_ARG, "D = %d outside [1, %d], the size of the static scratch", D,
                         kNoAllocMaxD);
  if (pixels > 0 && (!src || !dst)) return lv::set_error(LV_ERR_INVALID_ARG, "null buffer");
  if (dtype != LV_F32 && dtype != LV_BF16 && dtype != LV_FP8_E4M3)
    return lv::set_error(LV_ERR_INVALID_ARG, "unknown dtype");
  if (dtype == LV_FP8_E4M3 && !scales) return lv::set_error(LV_ERR_INVALID_ARG, "FP8 needs scales");
  void* amax = nullptr;
  hipError_t e = scratch_ptr(&amax);
  if (e != hipSuccess) return lv::set_error(LV_ERR_DEVICE, "scratch address: %s", hipGetErrorString(e));
  e = lv::launch_encode(src, pixels, D, dtype, dst, scales, static_cast<float*>(amax),
                        static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return lv::set_error(LV_ERR_DEVICE, "encode: %s", hipGetErrorString(e));
  return LV_OK;
}
