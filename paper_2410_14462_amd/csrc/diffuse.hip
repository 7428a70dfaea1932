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

// One group of C lanes per row (R = 64 / C rows per wave, 4 waves per
// block); blocks stride over the row tiles, so each block issues one atomic
// per channel for the norms of the next step instead of one per tile.  The
// row's edges are fetched C at a time, one per lane (column index and weight
// in registers), then broadcast with shuffles, so the gathers of g do not
// wait on the index loads and several are in flight at once.
template <int C, lv_dtype GT, lv_dtype VT>
__global__ __launch_bounds__(256) void spmm_kernel(const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const void* __restrict__ val, int64_t n, int D,
                                                   const void* __restrict__ g,
                                                   const float* __restrict__ nrm_in,
                                                   void* __restrict__ y, float* __restrict__ nrm_out) {
  constexpr int R = 64 / C;                 // rows per wave
  constexpr int U = C < 8 ? C : 8;          // gathers in flight per lane
  __shared__ float sq[256];
  const int t = threadIdx.x, lane = t & 63;
  const int sub = lane / C, c = lane % C, gbase = sub * C;
  const int64_t tiles = (n + 4 * R - 1) / (4 * R);
  const int cpl = (D + C - 1) / C;          // channels per lane
  for (int k = 0; k < cpl; k += 1) {
    const int ch = c + k * C;
    const int64_t chc = ch < D ? ch : 0;
    const float n2 = nrm_in[chc];
    const float scl = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
    float ss = 0.0f;  // this lane's sum of squares of channel ch
    // Workgroups go to the 8 XCDs round-robin: XCD x (= blockIdx mod 8)
    // takes the x-th eighth of the rows, so that with rows in a locality
    // order the gathered neighbours stay in that XCD's L2.
    const int64_t xcd = blockIdx.x & 7, nloc = gridDim.x >> 3;
    const int64_t t0 = tiles * xcd / 8, t1 = tiles * (xcd + 1) / 8;
    for (int64_t tile = t0 + (blockIdx.x >> 3); tile < t1; tile += nloc) {
      const int64_t row = (tile * 4 + (t >> 6)) * R + sub;
      const bool valid = row < n;
      const bool live = valid && ch < D;
      const int32_t a = valid ? row_ptr[row] : 0, b = valid ? row_ptr[row + 1] : 0;
      float acc = 0.0f;
      for (int32_t e0 = a; e0 < b; e0 += C) {
        const int32_t my = e0 + c;
        const int32_t cv = my < b ? col[my] : 0;
        const float wv = my < b ? ld<VT>(val, my) : 0.0f;
        const int cnt = b - e0 < C ? b - e0 : C;
        for (int j = 0; j < cnt; j += U) {
          // U gathers in flight; slots past the row's end read column 0 of a
          // valid row with weight 0 (lanes past the end hold col 0, w 0)
          float x[U], w[U];
#pragma unroll
          for (int u = 0; u < U; u++) {
            const int src = gbase + ((j + u) < C ? (j + u) : 0);
            const int32_t cj = __shfl(cv, src, 64);
            const float wj = __shfl(wv, src, 64);
            w[u] = (j + u) < cnt ? wj : 0.0f;
            x[u] = ld<GT>(g, (int64_t)cj * D + chc);
          }
#pragma unroll
          for (int u = 0; u < U; u++) acc = __builtin_fmaf(w[u], x[u], acc);
        }
      }
      if (live) {
        float out = scl * acc;
        st<GT>(y, row * D + ch, out);
        if constexpr (GT == LV_BF16) out = ld<GT>(y, row * D + ch);  // norm of what is stored
        ss = __builtin_fmaf(out, out, ss);
      }
    }
    // per-channel sum over the block: threads t, t + C, ... hold the same
    // channel (64 is a multiple of C)
    sq[t] = ss;
    __syncthreads();
    if (t < C) {
      float acc2 = 0.0f;
      for (int q = t; q < 256; q += C) acc2 += sq[q];
      const int chn = t + k * C;
      if (chn < D && acc2 != 0.0f) atomicAdd(&nrm_out[chn], acc2);
    }
    __syncthreads();
  }
}

// The value a signal element holds once stored (BF16 storage rounds).
template <lv_dtype DT>
__device__ __forceinline__ float stored(float x) {
  if constexpr (DT == LV_F32) {
    return x;
  } else {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
  }
}

// One channel (D = 1): one row per lane.  A row's edges go 8 at a time: the
// 8 column indices and weights are loaded together, then the 8 gathers, so
// each lane has 8 loads in flight instead of walking its edges one by one.
// Sums in edge order, as spmm_kernel.
template <lv_dtype GT, lv_dtype VT>
__global__ __launch_bounds__(256) void spmm1_kernel(const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const void* __restrict__ val, int64_t n,
                                                    const void* __restrict__ g,
                                                    const float* __restrict__ nrm_in,
                                                    void* __restrict__ y, float* __restrict__ nrm_out) {
  constexpr int U = 8;
  __shared__ float sq[4];
  const float n2 = nrm_in[0];
  const float scl = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
  float ss = 0.0f;
  // XCD x (= blockIdx mod 8) takes the x-th eighth of the rows (locality order)
  const int64_t tiles = (n + 255) / 256;
  const int64_t xcd = blockIdx.x & 7, nloc = gridDim.x >> 3;
  const int64_t t0 = tiles * xcd / 8, t1 = tiles * (xcd + 1) / 8;
  for (int64_t tile = t0 + (blockIdx.x >> 3); tile < t1; tile += nloc) {
    const int64_t row = tile * 256 + threadIdx.x;
    if (row >= n) continue;
    const int32_t a = row_ptr[row], b = row_ptr[row + 1];
    float acc = 0.0f;
    for (int32_t e = a; e < b; e += U) {
      int32_t cj[U];
      float w[U], x[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const bool ok = e + u < b;
        cj[u] = ok ? col[e + u] : 0;
        w[u] = ok ? ld<VT>(val, e + u) : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; u++) x[u] = ld<GT>(g, cj[u]);
#pragma unroll
      for (int u = 0; u < U; u++)
        if (e + u < b) acc = __builtin_fmaf(w[u], x[u], acc);
    }
    const float out = scl * acc;
    st<GT>(y, row, out);
    const float o = stored<GT>(out);  // the norm of what is stored
    ss = __builtin_fmaf(o, o, ss);
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if ((threadIdx.x & 63) == 0) sq[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float t = (sq[0] + sq[1]) + (sq[2] + sq[3]);
    if (t != 0.0f) atomicAdd(&nrm_out[0], t);
  }
}

// Four consecutive channels per lane (D = 4 L, L lanes per row, 64 / L rows
// per wave): the gathers are 16-byte (FP32) or 8-byte (BF16) loads of a
// neighbour's channels and a wave keeps several rows in flight.  A row's
// edges are fetched L at a time, one per lane, and broadcast with shuffles;
// 8 gathers in flight per lane.  Sums in edge order, as spmm_kernel.
template <int L, lv_dtype GT, lv_dtype VT>
__global__ __launch_bounds__(256) void spmm4_kernel(const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const void* __restrict__ val, int64_t n,
                                                    const void* __restrict__ g,
                                                    const float* __restrict__ nrm_in,
                                                    void* __restrict__ y, float* __restrict__ nrm_out) {
  constexpr int D = 4 * L, R = 64 / L, U = 8;
  __shared__ float sq[256 * 4];
  const int t = threadIdx.x, lane = t & 63;
  const int sub = lane / L, c4 = lane % L, gbase = sub * L;
  float scl[4], ss[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const float n2 = nrm_in[4 * c4 + k];
    scl[k] = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
  }
  const int64_t tiles = (n + 4 * R - 1) / (4 * R);
  const int64_t xcd = blockIdx.x & 7, nloc = gridDim.x >> 3;
  const int64_t t0 = tiles * xcd / 8, t1 = tiles * (xcd + 1) / 8;
  for (int64_t tile = t0 + (blockIdx.x >> 3); tile < t1; tile += nloc) {
    const int64_t row = (tile * 4 + (t >> 6)) * R + sub;
    const bool valid = row < n;
    const int32_t a = valid ? row_ptr[row] : 0, b = valid ? row_ptr[row + 1] : 0;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int32_t e0 = a; e0 < b; e0 += L) {
      const int32_t my = e0 + c4;
      const int32_t cv = my < b ? col[my] : 0;
      const float wv = my < b ? ld<VT>(val, my) : 0.0f;
      const int cnt = b - e0 < L ? b - e0 : L;
      for (int j = 0; j < cnt; j += U) {
        float w[U], x[U][4];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int src = gbase + ((j + u) < L ? (j + u) : 0);
          const int32_t cj = __shfl(cv, src, 64);
          const float wj = __shfl(wv, src, 64);
          w[u] = (j + u) < cnt ? wj : 0.0f;
          const int64_t off = (int64_t)cj * D + 4 * c4;
          if constexpr (GT == LV_F32) {
            const float4 q = *reinterpret_cast<const float4*>(static_cast<const float*>(g) + off);
            x[u][0] = q.x;
            x[u][1] = q.y;
            x[u][2] = q.z;
            x[u][3] = q.w;
          } else {
            const uint2 q = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(g) + off);
            x[u][0] = __uint_as_float(q.x << 16);
            x[u][1] = __uint_as_float(q.x & 0xFFFF0000u);
            x[u][2] = __uint_as_float(q.y << 16);
            x[u][3] = __uint_as_float(q.y & 0xFFFF0000u);
          }
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
          for (int k = 0; k < 4; k++) acc[k] = __builtin_fmaf(w[u], x[u][k], acc[k]);
      }
    }
    if (valid) {
      float o[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        o[k] = stored<GT>(scl[k] * acc[k]);
        ss[k] = __builtin_fmaf(o[k], o[k], ss[k]);
      }
      const int64_t off = row * D + 4 * c4;
      if constexpr (GT == LV_F32) {
        *reinterpret_cast<float4*>(static_cast<float*>(y) + off) = make_float4(o[0], o[1], o[2], o[3]);
      } else {
        const uint2 q = make_uint2((__float_as_uint(o[0]) >> 16) | (__float_as_uint(o[1]) & 0xFFFF0000u),
                                   (__float_as_uint(o[2]) >> 16) | (__float_as_uint(o[3]) & 0xFFFF0000u));
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(y) + off) = q;
      }
    }
  }
  // per-channel sums over the block: threads t = c4 (mod L) hold channels 4 c4 .. 4 c4 + 3
#pragma unroll
  for (int k = 0; k < 4; k++) sq[k * 256 + t] = ss[k];
  __syncthreads();
  if (t < D) {
    const int k = t & 3, cc = t >> 2;
    float s2 = 0.0f;
    for (int q = cc; q < 256; q += L) s2 += sq[k * 256 + q];
    if (s2 != 0.0f) atomicAdd(&nrm_out[t], s2);
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
  const int64_t rows_per_tile = 4 * R;
  const int64_t tiles = (n + rows_per_tile - 1) / rows_per_tile;
  // enough blocks to fill the chip several times over (a multiple of 8, one
  // share per XCD); each strides over the tiles of its XCD's share
  const int64_t want = (tiles + 7) / 8 * 8;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL((spmm_kernel<C, GT, VT>), dim3(blocks), dim3(256), 0, s, rp, col, val, n, D, g,
                     nin, y, nout);
  return hipGetLastError();
}

template <int L, lv_dtype GT, lv_dtype VT>
hipError_t spmm4_launch(const int32_t* rp, const int32_t* col, const void* val, int64_t n,
                        const void* g, const float* nin, void* y, float* nout, hipStream_t s) {
  constexpr int R = 64 / L;
  const int64_t tiles = (n + 4 * R - 1) / (4 * R);
  const int64_t want = (tiles + 7) / 8 * 8;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL((spmm4_kernel<L, GT, VT>), dim3(blocks), dim3(256), 0, s, rp, col, val, n, g, nin,
                     y, nout);
  return hipGetLastError();
}

template <lv_dtype GT, lv_dtype VT>
hipError_t spmm_dispatch(const int32_t* rp, const int32_t* col, const void* val, int64_t n, int D,
                         const void* g, const float* nin, void* y, float* nout, hipStream_t s) {
  if (D == 1) {
    const int64_t tiles = (n + 255) / 256;
    const int64_t want = (tiles + 7) / 8 * 8;
    const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL((spmm1_kernel<GT, VT>), dim3(blocks), dim3(256), 0, s, rp, col, val, n, g, nin, y,
                       nout);
    return hipGetLastError();
  }
  // four channels per lane where D = 4 L, L a power of two up to 16 and the
  // rows are 16-byte (FP32) or 8-byte (BF16) aligned
  if (((uintptr_t)g % 16 == 0) && ((uintptr_t)y % 16 == 0)) {
    if (D == 64) return spmm4_launch<16, GT, VT>(rp, col, val, n, g, nin, y, nout, s);
    if (D == 32) return spmm4_launch<8, GT, VT>(rp, col, val, n, g, nin, y, nout, s);
    if (D == 16) return spmm4_launch<4, GT, VT>(rp, col, val, n, g, nin, y, nout, s);
    if (D == 8) return spmm4_launch<2, GT, VT>(rp, col, val, n, g, nin, y, nout, s);
    if (D == 4) return spmm4_launch<1, GT, VT>(rp, col, val, n, g, nin, y, nout, s);
  }
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
  int rows = 256;
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

// ------------------------------------------------------- locality order
// Rows of A are renumbered along a Morton (Z-order) curve of the Gaussian
// centres, so that the neighbours of a row sit close in memory and the
// gathers of g hit the caches.  The renumbering is a similarity transform
// P A P^T: Eq. 8 commutes with it, and the per-channel norms are invariant.

// Order-preserving map of a float to uint32 (for atomic min / max).
__device__ __forceinline__ uint32_t ordered(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float unordered(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

__global__ void box_init_kernel(uint32_t* box) {
  if (threadIdx.x < 3) box[threadIdx.x] = 0xFFFFFFFFu;
  else if (threadIdx.x < 6) box[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void box_kernel(const float4* __restrict__ p0, int64_t n,
                                                  uint32_t* __restrict__ box) {
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float4 a = p0[i];
    const float v[3] = {a.x, a.y, a.z};
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const uint32_t o = ordered(v[k]);
      lo[k] = o < lo[k] ? o : lo[k];
      hi[k] = o > hi[k] ? o : hi[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; k++) {
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t l = __shfl_xor(lo[k], off, 64), h = __shfl_xor(hi[k], off, 64);
      lo[k] = l < lo[k] ? l : lo[k];
      hi[k] = h > hi[k] ? h : hi[k];
    }
  }
  // the block's four waves through LDS, then one atomic per bound and block
  // (few blocks: the six words would serialise thousands of wave atomics)
  __shared__ uint32_t wb[4][6];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
      wb[w][k] = lo[k];
      wb[w][3 + k] = hi[k];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    uint32_t r = wb[0][k];
    for (int q = 1; q < (int)(blockDim.x >> 6); q++) r = k < 3 ? (wb[q][k] < r ? wb[q][k] : r) : (wb[q][k] > r ? wb[q][k] : r);
    if (k < 3) atomicMin(&box[k], r);
    else atomicMax(&box[k], r);
  }
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {  // bit i -> bit 3i
  x &= 0x3FFu;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__global__ void morton_kernel(const float4* __restrict__ p0, int64_t n,
                              const uint32_t* __restrict__ box, uint32_t* __restrict__ key,
                              uint32_t* __restrict__ val, uint32_t* __restrict__ deg,
                              const int32_t* __restrict__ row_ptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 a = p0[i];
  const float v[3] = {a.x, a.y, a.z};
  uint32_t code = 0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const float lo = unordered(box[k]), hi = unordered(box[3 + k]);
    const float ext = hi - lo;
    float q = ext > 0.0f ? (v[k] - lo) / ext * 1024.0f : 0.0f;
    q = fminf(fmaxf(q, 0.0f), 1023.0f);
    code |= spread10((uint32_t)q) << k;
  }
  key[i] = code;
  val[i] = (uint32_t)i;
  if (row_ptr) deg[i] = (uint32_t)(row_ptr[i + 1] - row_ptr[i]);
}

// One sort segment covering all n items.
__global__ void seg_init_kernel(uint32_t* seg, int64_t n) {
  if (threadIdx.x == 0) {
    seg[0] = 0u;
    seg[1] = (uint32_t)n;
  }
}

// perm[r] = old index of new row r; inv[perm[r]] = r.
__global__ void invert_kernel(const uint32_t* __restrict__ perm, int64_t n, uint32_t* __restrict__ inv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) inv[perm[r]] = (uint32_t)r;
}

// New row r = old row perm[r], its columns renumbered; off[r] = new row start.
template <typename VT>
__global__ void permute_csr_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                   const VT* __restrict__ val, const uint32_t* __restrict__ perm,
                                   const uint32_t* __restrict__ inv, const uint32_t* __restrict__ off,
                                   int64_t n, int64_t nnz, int32_t* __restrict__ rp2,
                                   int32_t* __restrict__ col2, VT* __restrict__ val2) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n) return;
  if (r == n) {
    rp2[n] = (int32_t)nnz;
    return;
  }
  const int64_t o = perm[r];
  const int32_t a = rp[o], b = rp[o + 1];
  const int64_t d = off[r];
  rp2[r] = (int32_t)d;
  for (int32_t e = a; e < b; e++) {
    col2[d + (e - a)] = (int32_t)inv[col[e]];
    val2[d + (e - a)] = val[e];
  }
}

// Row gather / scatter of an [n][D] signal of `esize`-byte elements:
// dst[r] = src[perm[r]] (gather) or dst[perm[r]] = src[r] (scatter).
template <typename T>
__global__ void permute_rows_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                    const uint32_t* __restrict__ perm, int64_t n, int D,
                                    bool scatter) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * (int64_t)D) return;
  const int64_t r = e / D, c = e - r * D;
  const int64_t o = perm[r];
  if (scatter) dst[o * D + c] = src[e];
  else dst[e] = src[o * D + c];
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

namespace lv {

size_t reorder_scratch_words(int64_t n) {
  // keys/vals x2, degrees, offsets, box, seg start/len, totals, sort histogram, scan tmp
  return (size_t)n * 6 + 16 + sort_hist_size(1, n) + scan_tmp_size(n);
}

hipError_t launch_scene_box(const float4* p0, int64_t n, uint32_t* box, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(box_init_kernel, dim3(1), dim3(64), 0, s, box);
  hipLaunchKernelGGL(box_kernel, dim3(nb < 256 ? nb : 256), dim3(256), 0, s, p0, n, box);
  return hipGetLastError();
}

hipError_t launch_morton_order(const float4* p0, int64_t n, uint32_t* scratch, uint32_t* perm,
                               uint32_t* inv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t* k0 = scratch;
  uint32_t* v0 = k0 + n;
  uint32_t* k1 = v0 + n;
  uint32_t* v1 = k1 + n;
  uint32_t* box = v1 + n;  // within reorder_scratch_words(n)
  uint32_t* seg = box + 6;
  uint32_t* hist = box + 16;
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(box_init_kernel, dim3(1), dim3(64), 0, s, box);
  hipLaunchKernelGGL(box_kernel, dim3(nb < 256 ? nb : 256), dim3(256), 0, s, p0, n, box);
  hipLaunchKernelGGL(morton_kernel, dim3(nb), dim3(256), 0, s, p0, n, box, k0, v0, nullptr, nullptr);
  hipLaunchKernelGGL(seg_init_kernel, dim3(1), dim3(64), 0, s, seg, n);
  bool second = false;
  hipError_t e = radix_sort(k0, v0, k1, v1, seg, seg + 1, 1, n, 30, hist, false, &second, s);
  if (e != hipSuccess) return e;
  const uint32_t* sorted = second ? v1 : v0;
  hipLaunchKernelGGL(invert_kernel, dim3(nb), dim3(256), 0, s, sorted, n, inv);
  return hipMemcpyAsync(perm, sorted, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
}

hipError_t launch_graph_reorder(const float4* p0, int64_t n, const int32_t* rp, const int32_t* col,
                                const void* val, lv_dtype vt, int64_t nnz, uint32_t* scratch,
                                uint32_t* perm, uint32_t* inv, int32_t* rp2, int32_t* col2,
                                void* val2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t* k0 = scratch;
  uint32_t* v0 = k0 + n;
  uint32_t* k1 = v0 + n;
  uint32_t* v1 = k1 + n;
  uint32_t* deg = v1 + n;
  uint32_t* off = deg + n;
  uint32_t* box = off + n;          // 6 words
  uint32_t* seg = box + 6;          // start, len
  unsigned long long* totals = reinterpret_cast<unsigned long long*>(box + 8);  // 2 x u64, 8-aligned
  uint32_t* hist = box + 16;
  uint32_t* tmp = hist + sort_hist_size(1, n);
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(box_init_kernel, dim3(1), dim3(64), 0, s, box);
  hipLaunchKernelGGL(box_kernel, dim3(nb < 256 ? nb : 256), dim3(256), 0, s, p0, n, box);
  hipLaunchKernelGGL(morton_kernel, dim3(nb), dim3(256), 0, s, p0, n, box, k0, v0, deg, rp);
  hipLaunchKernelGGL(seg_init_kernel, dim3(1), dim3(64), 0, s, seg, n);
  bool second = false;
  hipError_t e = radix_sort(k0, v0, k1, v1, seg, seg + 1, 1, n, 30, hist, false, &second, s);
  if (e != hipSuccess) return e;
  const uint32_t* sorted = second ? v1 : v0;
  hipLaunchKernelGGL(invert_kernel, dim3(nb), dim3(256), 0, s, sorted, n, inv);
  e = hipMemcpyAsync(perm, sorted, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  // new row starts: exclusive scan of the degrees in the new order
  uint32_t* dummy = k0;  // seg_start / seg_len outputs of the scan (one view)
  e = scan_counts(deg, perm, n, 1, off, dummy, dummy + 1, totals, tmp, s);
  if (e != hipSuccess) return e;
  const unsigned nr = (unsigned)((n + 1 + 255) / 256);
  if (vt == LV_F32)
    hipLaunchKernelGGL(permute_csr_kernel<float>, dim3(nr), dim3(256), 0, s, rp, col,
                       static_cast<const float*>(val), perm, inv, off, n, nnz, rp2, col2,
                       static_cast<float*>(val2));
  else
    hipLaunchKernelGGL(permute_csr_kernel<uint16_t>, dim3(nr), dim3(256), 0, s, rp, col,
                       static_cast<const uint16_t*>(val), perm, inv, off, n, nnz, rp2, col2,
                       static_cast<uint16_t*>(val2));
  return hipGetLastError();
}

hipError_t launch_permute_rows(const void* src, void* dst, const uint32_t* perm, int64_t n, int D,
                               lv_dtype dt, bool scatter, hipStream_t s) {
  const int64_t total = n * (int64_t)D;
  if (total == 0) return hipSuccess;
  const unsigned nb = (unsigned)((total + 255) / 256);
  if (dt == LV_F32)
    hipLaunchKernelGGL(permute_rows_kernel<uint32_t>, dim3(nb), dim3(256), 0, s,
                       static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst), perm, n, D,
                       scatter);
  else
    hipLaunchKernelGGL(permute_rows_kernel<uint16_t>, dim3(nb), dim3(256), 0, s,
                       static_cast<const uint16_t*>(src), static_cast<uint16_t*>(dst), perm, n, D,
                       scatter);
  return hipGetLastError();
}

}  // namespace lv
