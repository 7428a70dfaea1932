// Graph diffusion (Sec. 3.3, Eq. 8): g_{t+1} = A (g_t / ||g_t||_2), each
// channel normalised by its own norm.  Since the normalisation is a
// per-channel scale, step t computes y = s_t * (A g_t) with
// s_t = 1 / ||g_t|| (0 for a zero channel) and, in the same pass, the squared
// norms of y for step t+1.  CSR SpMM: a group of C lanes (C = channel width,
// power of two <= 64) owns one row; lane c handles channels c, c + C, ...
#include "lv_internal.h"

namespace lv {

namespace {

template <lv_dtype DT>
__device__ __forceinline__ float ld(const void* p, int64_t i) {
  if constexpr (DT == LV_F32) return static_cast<const float*>(p)[i];
  else return __uint_as_float((uint32_t) static_cast<const uint16_t*>(p)[i] << 16);
}

template <lv_dtype DT>
__device__ __forceinline__ void st(void* p, int64_t i, float x) {
  if constexpr (DT == LV_F32) {
    static_cast<float*>(p)[i] = x;
  } else {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    static_cast<uint16_t*>(p)[i] = (uint16_t)(u >> 16);
  }
}

// Squared column norms of g [n][D] into nrm [D] (pre-zeroed).
template <lv_dtype DT>
__global__ __launch_bounds__(256) void colnorm_kernel(const void* __restrict__ g, int64_t n, int D,
                                                      int rows_per_block, float* __restrict__ nrm) {
  __shared__ float part[4][64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int c = blockIdx.y * 64 + lane;
  int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  float s = 0.0f;
  if (c < D)
    for (int64_t r = r0 + w; r < r1; r += 4) {
      float x = ld<DT>(g, r * D + c);
      s = __builtin_fmaf(x, x, s);
    }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && c < D) atomicAdd(&nrm[c], (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]));
}

template <int C, lv_dtype GT, lv_dtype VT>
__global__ __launch_bounds__(256) void spmm_kernel(const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const void* __restrict__ val, int64_t n, int D,
                                                   const void* __restrict__ g,
                                                   const float* __restrict__ nrm_in,
                                                   void* __restrict__ y, float* __restrict__ nrm_out) {
  constexpr int R = 64 / C;                 // rows per wave
  __shared__ float sq[256];
  const int t = threadIdx.x, lane = t & 63;
  const int sub = lane / C, c = lane % C;
  const int64_t row = ((int64_t)blockIdx.x * 4 + (t >> 6)) * R + sub;
  const int cpl = (D + C - 1) / C;          // channels per lane
  for (int k = 0; k < cpl; k += 1) {
    const int ch = c + k * C;
    float out = 0.0f;
    if (row < n && ch < D) {
      float n2 = nrm_in[ch];
      float sc = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
      int32_t a = row_ptr[row], b = row_ptr[row + 1];
      float acc = 0.0f;
      for (int32_t e = a; e < b; e++) acc = __builtin_fmaf(ld<VT>(val, e), ld<GT>(g, (int64_t)col[e] * D + ch), acc);
      out = sc * acc;
      st<GT>(y, row * D + ch, out);
      if constexpr (GT == LV_BF16) out = ld<GT>(y, row * D + ch);  // norm of what is stored
    }
    // per-channel sum of squares over the block's rows: threads t, t + C, ...
    // hold the same channel (64 is a multiple of C)
    sq[t] = out * out;
    __syncthreads();
    if (t < C) {
      float acc2 = 0.0f;
      for (int q = t; q < 256; q += C) acc2 += sq[q];
      int chn = t + k * C;
      if (chn < D && acc2 != 0.0f) atomicAdd(&nrm_out[chn], acc2);
    }
    __syncthreads();
  }
}

template <lv_dtype GT>
__global__ void copy_kernel(const void* __restrict__ src, void* __restrict__ dst, int64_t total) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) st<GT>(dst, e, ld<GT>(src, e));
}

template <int C, lv_dtype GT, lv_dtype VT>
hipError_t spmm_launch(const int32_t* rp, const int32_t* col, const void* val, int64_t n, int D,
                       const void* g, const float* nin, void* y, float* nout, hipStream_t s) {
  constexpr int R = 64 / C;
  int64_t rows_per_block = 4 * R;
  unsigned blocks = (unsigned)((n + rows_per_block - 1) / rows_per_block);
  hipLaunchKernelGGL((spmm_kernel<C, GT, VT>), dim3(blocks), dim3(256), 0, s, rp, col, val, n, D, g,
                     nin, y, nout);
  return hipGetLastError();
}

template <lv_dtype GT, lv_dtype VT>
hipError_t spmm_dispatch(const int32_t* rp, const int32_t* col, const void* val, int64_t n, int D,
                         const void* g, const float* nin, void* y, float* nout, hipStream_t s) {
  if (D >= 64) return spmm_launch<64, GT, VT>(rp, col, val, n, D, g, nin, y, nout, s);
  if (D > 16) return spmm_launch<32, GT, VT>(rp, col, val, n, D, g, nin, y, nout, s);
  if (D > 4) return spmm_launch<8, GT, VT>(rp, col, val, n, D, g, nin, y, nout, s);
  return spmm_launch<1, GT, VT>(rp, col, val, n, D, g, nin, y, nout, s);
}

template <lv_dtype GT>
hipError_t diffuse_t(const int32_t* rp, const int32_t* col, const void* val, lv_dtype vt, int64_t n,
                     const void* g0, int D, int steps, void* out, void* b0, void* b1, float* norms,
                     hipStream_t s) {
  int64_t total = n * (int64_t)D;
  if (steps == 0) {
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_kernel<GT>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g0,
                       out, total);
    return hipGetLastError();
  }
  hipError_t e = hipMemsetAsync(norms, 0, sizeof(float) * (size_t)D * (size_t)(steps + 1), s);
  if (e != hipSuccess) return e;
  if (total == 0) return hipSuccess;
  int rows = 1024;
  hipLaunchKernelGGL(colnorm_kernel<GT>, dim3((unsigned)((n + rows - 1) / rows), (D + 63) / 64),
                     dim3(256), 0, s, g0, n, D, rows, norms);
  const void* cur = g0;
  for (int t = 0; t < steps; t++) {
    void* dst = (t == steps - 1) ? out : ((t & 1) ? b1 : b0);
    e = vt == LV_F32 ? spmm_dispatch<GT, LV_F32>(rp, col, val, n, D, cur, norms + (size_t)t * D, dst,
                                                 norms + (size_t)(t + 1) * D, s)
                     : spmm_dispatch<GT, LV_BF16>(rp, col, val, n, D, cur, norms + (size_t)t * D, dst,
                                                  norms + (size_t)(t + 1) * D, s);
    if (e != hipSuccess) return e;
    cur = dst;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_diffuse(const int32_t* row_ptr, const int32_t* col, const void* val,
                          lv_dtype val_dtype, int64_t n, const void* g0, lv_dtype dtype, int D,
                          int steps, void* out, float* buf0, float* buf1, float* norms,
                          hipStream_t s) {
  if (dtype == LV_F32)
    return diffuse_t<LV_F32>(row_ptr, col, val, val_dtype, n, g0, D, steps, out, buf0, buf1, norms, s);
  return diffuse_t<LV_BF16>(row_ptr, col, val, val_dtype, n, g0, D, steps, out, buf0, buf1, norms, s);
}

}  // namespace lv
