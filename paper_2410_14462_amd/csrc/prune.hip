// Weight-based Gaussian filtering (Sec. 3.2: beta_i, the sum of a Gaussian's
// blending weights over all views and pixels, estimates its importance; the
// least important half can be dropped) and the count-normalised uplift of
// the comparison with GaussianEditor (appendix: f_i = U_i / c_i with c_i the
// number of counted (view, pixel) pairs instead of their summed weights).
//
// Filtering keeps the k Gaussians with the largest beta, ties to the lower
// index: a stable radix sort of (descending-order key, index) over all n,
// then the first k are marked.  The same order gives the anchors of a
// diffusion (appendix on diffusion for segmentation: the largest fraction
// of the positive uplifted mask values) and the reachability output h.
#include "lv_internal.h"

namespace lv {

namespace {

// Key whose ascending unsigned order is the descending IEEE order of x
// (a total order: -0 after +0, NaNs by their bits).
__device__ __forceinline__ uint32_t descending_key(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ~asc;
}

__global__ void prune_keys_kernel(const float* __restrict__ w, int64_t n, uint32_t* __restrict__ key,
                                  uint32_t* __restrict__ idx, uint8_t* __restrict__ keep,
                                  uint32_t* __restrict__ seg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    seg[0] = 0u;
    seg[1] = (uint32_t)n;
  }
  if (i >= n) return;
  key[i] = descending_key(w[i]);
  idx[i] = (uint32_t)i;
  keep[i] = 0;
}

__global__ void prune_mark_kernel(const uint32_t* __restrict__ sorted_idx, int64_t k,
                                  uint8_t* __restrict__ keep) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < k) keep[sorted_idx[r]] = 1;
}

// anchor initialisation: keys as for filtering, g0 cleared, positives counted
__global__ void anchor_keys_kernel(const float* __restrict__ g, int64_t n, uint32_t* __restrict__ key,
                                   uint32_t* __restrict__ idx, float* __restrict__ g0,
                                   uint32_t* __restrict__ seg, unsigned long long* __restrict__ npos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    seg[0] = 0u;
    seg[1] = (uint32_t)n;
  }
  const bool pos = i < n && g[i] > 0.0f;
  const uint64_t b = __ballot(pos);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(npos, (unsigned long long)__popcll(b));
  if (i >= n) return;
  key[i] = descending_key(g[i]);
  idx[i] = (uint32_t)i;
  g0[i] = 0.0f;
}

__global__ void anchor_mark_kernel(const uint32_t* __restrict__ sorted_idx, int64_t n, float fraction,
                                   const unsigned long long* __restrict__ npos,
                                   const float* __restrict__ g, float* __restrict__ g0) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = (int64_t)ceil((double)fraction * (double)npos[0]);
  if (r < k && r < n) {
    const uint32_t i = sorted_idx[r];
    g0[i] = g[i];
  }
}

__global__ void reach_unary_kernel(const float* __restrict__ gT, const float* __restrict__ unary,
                                   int64_t n, int D, float* __restrict__ h) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * D) return;
  h[e] = gT[e] > 0.0f ? unary[e / D] : 0.0f;
}

__global__ void finalize_count_kernel(const float* __restrict__ U, const uint32_t* __restrict__ cnt,
                                      int64_t n, int D, float* __restrict__ f,
                                      const uint32_t* __restrict__ perm, bool fixed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * D) return;
  const int64_t i = e / D;
  const uint32_t c = cnt[i];
  const int64_t o = perm ? (int64_t)perm[i] : i;  // the output row
  float r = 0.0f;
  if (c && fixed)  // fixed-point U (units of 2^-35)
    r = (float)((double)reinterpret_cast<const long long*>(U)[e] * (1.0 / kBetaUnit) / (double)c);
  else if (c)
    r = U[e] / (float)c;
  f[o * D + (e - i * D)] = r;
}

}  // namespace

hipError_t launch_prune(const float* wsum, int64_t n, int64_t k, uint8_t* keep, hipStream_t s) {
  if (n == 0) return hipSuccess;
  // key/index pairs double buffered, one segment, histogram rows
  const size_t words = 4 * (size_t)n + 2 + sort_hist_size(1, n);
  void* mem = nullptr;
  hipError_t e = dev_alloc(&mem, 4 * words, s, true);
  if (e != hipSuccess) return e;
  uint32_t* k0 = static_cast<uint32_t*>(mem);
  uint32_t* v0 = k0 + n;
  uint32_t* k1 = v0 + n;
  uint32_t* v1 = k1 + n;
  uint32_t* seg = v1 + n;
  uint32_t* hist = seg + 2;
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(prune_keys_kernel, dim3(nb), dim3(256), 0, s, wsum, n, k0, v0, keep, seg);
  bool second = false;
  e = radix_sort(k0, v0, k1, v1, seg, seg + 1, 1, n, 32, hist, false, &second, s);
  if (e == hipSuccess && k > 0) {
    hipLaunchKernelGGL(prune_mark_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s,
                       second ? v1 : v0, k, keep);
    e = hipGetLastError();
  }
  dev_free(mem, 4 * words, s, true);
  return e;
}

hipError_t launch_anchor_init(const float* g, int64_t n, float fraction, float* g0, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t words = 4 * (size_t)n + 2 + 2 + sort_hist_size(1, n);
  void* mem = nullptr;
  hipError_t e = dev_alloc(&mem, 4 * words, s, true);
  if (e != hipSuccess) return e;
  uint32_t* k0 = static_cast<uint32_t*>(mem);
  uint32_t* v0 = k0 + n;
  uint32_t* k1 = v0 + n;
  uint32_t* v1 = k1 + n;
  uint32_t* seg = v1 + n;
  unsigned long long* npos = reinterpret_cast<unsigned long long*>(seg + 2);  // 8-byte aligned: 4n + 2 even
  uint32_t* hist = seg + 4;
  e = hipMemsetAsync(npos, 0, 8, s);
  if (e == hipSuccess) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(anchor_keys_kernel, dim3(nb), dim3(256), 0, s, g, n, k0, v0, g0, seg, npos);
    bool second = false;
    e = radix_sort(k0, v0, k1, v1, seg, seg + 1, 1, n, 32, hist, false, &second, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(anchor_mark_kernel, dim3(nb), dim3(256), 0, s, second ? v1 : v0, n, fraction, npos,
                         g, g0);
      e = hipGetLastError();
    }
  }
  dev_free(mem, 4 * words, s, true);
  return e;
}

hipError_t launch_reach_unary(const float* gT, const float* unary, int64_t n, int D, float* h,
                              hipStream_t s) {
  const int64_t total = n * (int64_t)D;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(reach_unary_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, gT, unary,
                     n, D, h);
  return hipGetLastError();
}

hipError_t launch_finalize_count(const float* U, const uint32_t* cnt, int64_t n, int D, float* f,
                                 const uint32_t* perm, bool fixed, hipStream_t s) {
  const int64_t total = n * (int64_t)D;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_count_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     U, cnt, n, D, f, perm, fixed);
  return hipGetLastError();
}

}  // namespace lv
