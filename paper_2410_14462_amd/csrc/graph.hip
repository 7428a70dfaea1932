// The diffusion graph over the Gaussian centres, built on the device
// (Sec. 3.3: diffusion runs on a weighted graph joining each Gaussian to its
// spatial neighbours; the relation is symmetrised by the union of the
// directed kNN pairs).  Weight of a pair: exp(-|x_i - x_j|^2 / sigma^2) *
// max(0, cos(f_i, f_j)), sigma the median directed kNN distance, the larger
// directed weight where both exist; rows normalised to sum 1, a row whose
// weights are all 0 gets a self-loop of weight 1.
//
// Reproducible structure: squared distances in FP64 as ((dx dx + dy dy) +
// dz dz) of the FP32 centres, neighbours ordered by (squared distance,
// index); the union pairs with a positive FP64 weight are stored, columns
// ascending; a self-loop is the only entry of its row.
//
// The paper's own weights (Eq. 7 with the feature kernel of Eq. 9, the
// appendix on diffusion for segmentation) are the other kind: A_ij =
// exp(-|g_i - g_j|^2 / (b s_f^2)) (sqrt(P_i) sqrt(P_j)) with g the
// l2-normalised features, s_f the median feature distance over the directed
// kNN pairs, b a bandwidth and P a caller-given unary term (1 if absent); no
// row normalisation, no self-loops; optionally binarised (1 where the weight
// exceeds a threshold).
//
// Steps: bounding box; uniform grid (about two centres per cell), centres
// sorted by cell; exact kNN by shells of cells around each centre until the
// k-th distance is below the distance to the next shell; sigma from the two
// middle order statistics of the n k squared distances (radix select on
// their bits); per-node feature norms and per-edge weights (one wave per
// node, lanes over channels); union rows (own k entries plus the reversed
// edges, placed with atomics, then sorted by column in each row and merged
// with max), row sums in column order, normalisation into the CSR.
#include "lv_internal.h"

namespace lv {

namespace {

constexpr int kGraphMaxK = 32;

// ---------------------------------------------------------------- grid
__global__ void bbox_partial_kernel(const float4* __restrict__ c, int64_t n, float* __restrict__ part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 p = c[i];
    lo[0] = fminf(lo[0], p.x); hi[0] = fmaxf(hi[0], p.x);
    lo[1] = fminf(lo[1], p.y); hi[1] = fmaxf(hi[1], p.y);
    lo[2] = fminf(lo[2], p.z); hi[2] = fmaxf(hi[2], p.z);
  }
  __shared__ float red[6][256];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    red[a][threadIdx.x] = lo[a];
    red[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
#pragma unroll
      for (int a = 0; a < 3; a++) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + o]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// grid parameters: gp[0..2] = box minimum, gp[3..5] = cells per unit length
// (0 for a flat axis), gp[6..8] = cell edge lengths
__global__ void grid_params_kernel(const float* __restrict__ part, int nparts, int G, float* __restrict__ gp) {
  // one wave: lanes stride over the partials, then a wave reduction
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nparts; b += 64)
    for (int a = 0; a < 3; a++) {
      lo[a] = fminf(lo[a], part[6 * b + a]);
      hi[a] = fmaxf(hi[a], part[6 * b + 3 + a]);
    }
  for (int a = 0; a < 3; a++)
    for (int o = 32; o > 0; o >>= 1) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
    }
  if (threadIdx.x != 0) return;
  for (int a = 0; a < 3; a++) {
    const float ext = hi[a] - lo[a];
    gp[a] = lo[a];
    gp[3 + a] = ext > 0.0f ? (float)G / ext : 0.0f;
    gp[6 + a] = ext > 0.0f ? ext / (float)G : 0.0f;
  }
}

__device__ __forceinline__ int cell_coord(float x, float lo, float inv, int G) {
  const int c = (int)floorf((x - lo) * inv);
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

__global__ void cell_keys_kernel(const float4* __restrict__ c, int64_t n, const float* __restrict__ gp,
                                 int G, uint32_t* __restrict__ key, uint32_t* __restrict__ id) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = c[i];
  const int cx = cell_coord(p.x, gp[0], gp[3], G), cy = cell_coord(p.y, gp[1], gp[4], G),
            cz = cell_coord(p.z, gp[2], gp[5], G);
  key[i] = ((uint32_t)cz * (uint32_t)G + (uint32_t)cy) * (uint32_t)G + (uint32_t)cx;
  id[i] = (uint32_t)i;
}

// cell ranges [start, end) from the sorted keys (cells without centres keep
// start = end = 0 from the fill)
__global__ void cell_ranges_kernel(const uint32_t* __restrict__ key, int64_t n,
                                   uint32_t* __restrict__ start, uint32_t* __restrict__ end) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = key[i];
  if (i == 0 || key[i - 1] != k) start[k] = (uint32_t)i;
  if (i + 1 == n || key[i + 1] != k) end[k] = (uint32_t)(i + 1);
}

// (d, j) < (bd, bj) in the (squared distance, index) order
__device__ __forceinline__ bool closer(double d, uint32_t j, double bd, uint32_t bj) {
  return d < bd || (d == bd && j < bj);
}

// Exact kNN of the centre at sorted position p: shells of cells at Chebyshev
// distance r = 0, 1, 2, ... around its cell; after shell r every centre not
// yet seen is at least (r - 0.001) min(cell edge) away (0.001 of a cell
// covers the rounding of the cell assignment), so the search stops once K
// candidates are held and the k-th is strictly closer than that.
template <int K>
__global__ __launch_bounds__(256) void knn_kernel(const float4* __restrict__ c, int64_t n,
                                                  const uint32_t* __restrict__ sorted_id,
                                                  const uint32_t* __restrict__ cstart,
                                                  const uint32_t* __restrict__ cend,
                                                  const float* __restrict__ gp, int G, int k,
                                                  int32_t* __restrict__ out_idx,
                                                  double* __restrict__ out_d2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t i = sorted_id[p];
  const float4 pi = c[i];
  const double xi = pi.x, yi = pi.y, zi = pi.z;
  const int cx = cell_coord(pi.x, gp[0], gp[3], G), cy = cell_coord(pi.y, gp[1], gp[4], G),
            cz = cell_coord(pi.z, gp[2], gp[5], G);
  float hmin = INFINITY;
  for (int a = 0; a < 3; a++)
    if (gp[6 + a] > 0.0f) hmin = fminf(hmin, gp[6 + a]);
  if (!(hmin < INFINITY)) hmin = 0.0f;  // all centres equal: every shell is empty but the first
  double bd[K];
  uint32_t bj[K];
#pragma unroll
  for (int t = 0; t < K; t++) {
    bd[t] = INFINITY;
    bj[t] = 0xFFFFFFFFu;
  }
  for (int r = 0; r < G; r++) {
    for (int dz = -r; dz <= r; dz++) {
      const int z = cz + dz;
      if (z < 0 || z >= G) continue;
      for (int dy = -r; dy <= r; dy++) {
        const int y = cy + dy;
        if (y < 0 || y >= G) continue;
        const bool face = dz == -r || dz == r || dy == -r || dy == r;
        const int step = face ? 1 : (2 * r > 0 ? 2 * r : 1);  // inside: only dx = +-r
        for (int dx = -r; dx <= r; dx += step) {
          const int x = cx + dx;
          if (x < 0 || x >= G) continue;
          const uint32_t cell = ((uint32_t)z * (uint32_t)G + (uint32_t)y) * (uint32_t)G + (uint32_t)x;
          const uint32_t q1 = cend[cell];
          for (uint32_t q = cstart[cell]; q < q1; q++) {
            const uint32_t j = sorted_id[q];
            if (j == i) continue;
            const float4 pj = c[j];
            const double ex = xi - (double)pj.x, ey = yi - (double)pj.y, ez = zi - (double)pj.z;
            double d = (ex * ex + ey * ey) + ez * ez;
            uint32_t jj = j;
            if (!closer(d, jj, bd[K - 1], bj[K - 1])) continue;
#pragma unroll
            for (int t = 0; t < K; t++) {  // insert, keeping the list sorted
              if (closer(d, jj, bd[t], bj[t])) {
                const double td = bd[t];
                const uint32_t tj = bj[t];
                bd[t] = d;
                bj[t] = jj;
                d = td;
                jj = tj;
              }
            }
          }
        }
      }
    }
    double kth = INFINITY;
#pragma unroll
    for (int t = 0; t < K; t++)
      if (t == k - 1) kth = bd[t];
    const double gap = (double)(r - 0.001) * (double)hmin;
    if (kth < INFINITY && r > 0 && kth < gap * gap) break;
  }
#pragma unroll
  for (int t = 0; t < K; t++)
    if (t < k) {
      out_idx[(int64_t)i * k + t] = (int32_t)bj[t];
      out_d2[(int64_t)i * k + t] = bd[t];
    }
}

// ---------------------------------------------------- median (radix select)
// Two order statistics (ranks rk[0], rk[1]) of N non-negative doubles, by
// their bits, 11 bits per round from the top.  st: prefix[2], rank[2]
// (uint64), advanced by the pick kernel after each round.
constexpr int kSelBins = 2048;

__global__ void select_hist_kernel(const double* __restrict__ v, int64_t N, int shift, int width,
                                   const unsigned long long* __restrict__ st,
                                   unsigned int* __restrict__ hist) {
  __shared__ unsigned int h[2][kSelBins];
  for (int e = threadIdx.x; e < 2 * kSelBins; e += blockDim.x) (&h[0][0])[e] = 0u;
  __syncthreads();
  const int top = shift + width;
  const unsigned long long p0 = top >= 64 ? 0ull : st[0] >> top, p1 = top >= 64 ? 0ull : st[1] >> top;
  const unsigned long long mask = (1ull << width) - 1ull;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v[e]);
    const unsigned long long hb = top >= 64 ? 0ull : b >> top;
    const unsigned int d = (unsigned int)((b >> shift) & mask);
    if (hb == p0) atomicAdd(&h[0][d], 1u);
    if (hb == p1) atomicAdd(&h[1][d], 1u);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * kSelBins; e += blockDim.x) {
    const unsigned int x = (&h[0][0])[e];
    if (x) atomicAdd(&hist[e], x);
  }
}

// one block of 1024 threads: for each target, the digit whose cumulative
// count passes the residual rank; the histogram is cleared for the next round
__global__ __launch_bounds__(1024) void select_pick_kernel(unsigned int* __restrict__ hist, int shift,
                                                           unsigned long long* __restrict__ st) {
  // thread t owns bins 2t, 2t + 1 of each target; block-wide exclusive scan
  __shared__ unsigned long long wsum[2][16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  unsigned long long rank[2], part[2], c0[2], c1[2];
#pragma unroll
  for (int g = 0; g < 2; g++) {
    rank[g] = st[2 + g];
    c0[g] = hist[g * kSelBins + 2 * t];
    c1[g] = hist[g * kSelBins + 2 * t + 1];
    unsigned long long incl = c0[g] + c1[g];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    part[g] = incl - (c0[g] + c1[g]);  // exclusive within the wave
    if (lane == 63) wsum[g][w] = incl;
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < 2; g++) {
    unsigned long long base = part[g];
    for (int q = 0; q < w; q++) base += wsum[g][q];
    // the bin whose [cum, cum + count) holds the rank (exactly one thread)
    if (rank[g] >= base && rank[g] < base + c0[g]) {
      st[g] |= (unsigned long long)(2 * t) << shift;
      st[2 + g] = rank[g] - base;
    } else if (rank[g] >= base + c0[g] && rank[g] < base + c0[g] + c1[g]) {
      st[g] |= (unsigned long long)(2 * t + 1) << shift;
      st[2 + g] = rank[g] - base - c0[g];
    }
  }
  __syncthreads();
  for (int e = t; e < 2 * kSelBins; e += blockDim.x) hist[e] = 0u;
}

__global__ void select_init_kernel(unsigned long long* st, unsigned long long r0, unsigned long long r1,
                                   unsigned int* hist) {
  if (threadIdx.x == 0) {
    st[0] = 0ull;
    st[1] = 0ull;
    st[2] = r0;
    st[3] = r1;
  }
  for (int e = threadIdx.x; e < 2 * kSelBins; e += blockDim.x) hist[e] = 0u;
}

// sig2 = (median of the roots)^2, from the two middle squared values (their
// roots averaged)
__global__ void sigma_kernel(const unsigned long long* st, double* sig2) {
  if (threadIdx.x != 0) return;
  const double a = __longlong_as_double((long long)st[0]), b = __longlong_as_double((long long)st[1]);
  const double s = (sqrt(a) + sqrt(b)) / 2.0;
  sig2[0] = s * s;
}

// ------------------------------------------------------------ edge weights
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// one wave per node: norms first (a pass of their own), then each edge's
// dot product with lanes over channels
__global__ __launch_bounds__(256) void norms_kernel(const float* __restrict__ f, int64_t n, int D,
                                                    double* __restrict__ nrm) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s = 0.0;
  for (int ch = lane; ch < D; ch += 64) {
    const double x = f[i * D + ch];
    s += x * x;
  }
  s = wave_sum_f64(s);
  if (lane == 0) nrm[i] = sqrt(s);
}

__global__ __launch_bounds__(256) void edge_weights_kernel(const float* __restrict__ f, int64_t n, int D,
                                                           int k, const int32_t* __restrict__ idx,
                                                           const double* __restrict__ d2,
                                                           const double* __restrict__ nrm,
                                                           const double* __restrict__ sig2,
                                                           double* __restrict__ w) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const double s2 = sig2[0];
  for (int t = 0; t < k; t++) {
    const int64_t j = idx[i * k + t];
    double dot = 0.0;
    for (int ch = lane; ch < D; ch += 64) dot += (double)f[i * D + ch] * (double)f[j * D + ch];
    dot = wave_sum_f64(dot);
    if (lane == 0) {
      const double den = nrm[i] * nrm[j];
      const double cs = den > 0.0 ? dot / den : 0.0;
      w[i * k + t] = exp(-d2[i * k + t] / s2) * (cs > 0.0 ? cs : 0.0);
    }
  }
}

// squared distances of the l2-normalised features of each directed pair
// (a zero feature stays zero), one wave per node
__global__ __launch_bounds__(256) void feature_d2_kernel(const float* __restrict__ f, int64_t n, int D,
                                                         int k, const int32_t* __restrict__ idx,
                                                         const double* __restrict__ nrm,
                                                         double* __restrict__ fd2) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const double ni = nrm[i];
  for (int t = 0; t < k; t++) {
    const int64_t j = idx[i * k + t];
    const double nj = nrm[j];
    double acc = 0.0;
    for (int ch = lane; ch < D; ch += 64) {
      const double a = ni > 0.0 ? (double)f[i * D + ch] / ni : 0.0;
      const double b = nj > 0.0 ? (double)f[j * D + ch] / nj : 0.0;
      acc += (a - b) * (a - b);
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) fd2[i * k + t] = acc;
  }
}

// Eq. 7 / Eq. 9 weight of each directed pair
__global__ void rbf_weights_kernel(int64_t nk, int k, const int32_t* __restrict__ idx,
                                   const double* __restrict__ fd2, const double* __restrict__ s2,
                                   double bandwidth, const float* __restrict__ unary,
                                   double* __restrict__ w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk) return;
  const int64_t i = e / k, j = idx[e];
  const double pp = unary ? sqrt((double)unary[i]) * sqrt((double)unary[j]) : 1.0;
  w[e] = exp(-fd2[e] / (bandwidth * s2[0])) * pp;
}

// ------------------------------------------------------------ union rows
__global__ void indeg_kernel(const int32_t* __restrict__ idx, int64_t nk, uint32_t* __restrict__ indeg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nk) atomicAdd(&indeg[idx[e]], 1u);
}

__global__ void row_cap_kernel(const uint32_t* __restrict__ indeg, int64_t n, int k,
                               uint32_t* __restrict__ cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cap[i] = (uint32_t)k + indeg[i] + 1u;  // own, reversed, a possible self-loop
}

// row i: its own k entries first, then the reversed edges of the nodes that
// chose i (in arrival order; sorted afterwards)
__global__ void fill_rows_kernel(const int32_t* __restrict__ idx, const double* __restrict__ w,
                                 int64_t n, int k, const uint32_t* __restrict__ start,
                                 uint32_t* __restrict__ fillpos, int32_t* __restrict__ ucol,
                                 double* __restrict__ uw) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t i = e / k;
  const int t = (int)(e - i * k);
  const int32_t j = idx[e];
  ucol[start[i] + t] = j;
  uw[start[i] + t] = w[e];
  const uint32_t slot = atomicAdd(&fillpos[j], 1u);
  ucol[start[j] + (uint32_t)k + slot] = (int32_t)i;
  uw[start[j] + (uint32_t)k + slot] = w[e];
}

// per row of more than 64 entries (the others are merged by one wave each,
// below): sort by column (ties: larger weight first), keep one entry per
// column with the larger weight if it passes, sum in column order; a row
// left empty gets the self-loop (weight 1).  len[i] = entries kept.
__global__ void merge_rows_kernel(int64_t n, int k, const uint32_t* __restrict__ start,
                                  const uint32_t* __restrict__ indeg, int32_t* __restrict__ ucol,
                                  double* __restrict__ uw, uint32_t* __restrict__ len,
                                  double* __restrict__ rsum, double thresh, bool binarize,
                                  bool self_loops) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || len[i] != 0xFFFFFFFFu) return;  // rows of more than 64 entries only
  int32_t* cl = ucol + start[i];
  double* wv = uw + start[i];
  const int m = k + (int)indeg[i];
  for (int a = 1; a < m; a++) {  // insertion sort
    const int32_t c = cl[a];
    const double x = wv[a];
    int b = a - 1;
    while (b >= 0 && (cl[b] > c || (cl[b] == c && wv[b] < x))) {
      cl[b + 1] = cl[b];
      wv[b + 1] = wv[b];
      b--;
    }
    cl[b + 1] = c;
    wv[b + 1] = x;
  }
  int u = 0;
  double s = 0.0;
  int32_t last = -1;
  for (int a = 0; a < m; a++) {
    if (cl[a] == last) continue;  // the first of a column has the larger weight
    last = cl[a];
    if (!(wv[a] > thresh)) continue;
    cl[u] = cl[a];
    wv[u] = binarize ? 1.0 : wv[a];
    s += wv[u];
    u++;
  }
  if (u == 0 && self_loops) {  // self-loop
    cl[0] = (int32_t)i;
    wv[0] = 1.0;
    u = 1;
    s = 1.0;
  }
  len[i] = (uint32_t)u;
  rsum[i] = s;
}

// The same for rows of at most 64 entries, one wave per row: a bitonic sort
// of (column ascending, weight descending) across the lanes, the first of
// each column kept if its weight passes, compaction by ballot.  Rows with
// more entries are left to merge_rows_kernel (flagged with len = ~0).
__device__ __forceinline__ bool before(int32_t c1, double x1, int32_t c2, double x2) {
  return c1 < c2 || (c1 == c2 && x1 > x2);
}

__global__ __launch_bounds__(256) void merge_rows_wave_kernel(int64_t n, int k, const uint32_t* __restrict__ start,
                                                              const uint32_t* __restrict__ indeg,
                                                              int32_t* __restrict__ ucol, double* __restrict__ uw,
                                                              uint32_t* __restrict__ len,
                                                              double* __restrict__ rsum, double thresh,
                                                              bool binarize, bool self_loops) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int m = k + (int)indeg[i];
  if (m > 64) {  // wave-uniform
    if (lane == 0) len[i] = 0xFFFFFFFFu;
    return;
  }
  int32_t* cl = ucol + start[i];
  double* wv = uw + start[i];
  int32_t c = lane < m ? cl[lane] : 0x7FFFFFFF;
  double x = lane < m ? wv[lane] : -INFINITY;
  for (int kk = 2; kk <= 64; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      const int32_t pc = __shfl_xor(c, j, 64);
      const double px = __shfl_xor(x, j, 64);
      const bool up = (lane & kk) == 0;
      const bool low = (lane & j) == 0;
      // the lower lane of an ascending pair keeps the earlier element
      const bool take = (low == up) ? before(pc, px, c, x) : before(c, x, pc, px);
      if (take) {
        c = pc;
        x = px;
      }
    }
  const int32_t prev = __shfl_up(c, 1, 64);
  const bool keep = lane < m && (lane == 0 || prev != c) && x > thresh;
  const uint64_t kb = __ballot(keep);
  const uint32_t pos = (uint32_t)__popcll(kb & (lane ? (~0ull >> (64 - lane)) : 0ull));
  const double v = keep ? (binarize ? 1.0 : x) : 0.0;
  if (keep) {
    cl[pos] = c;
    wv[pos] = v;
  }
  double sum = v;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  uint32_t u = (uint32_t)__popcll(kb);
  if (lane == 0) {
    if (u == 0 && self_loops) {  // self-loop
      cl[0] = (int32_t)i;
      wv[0] = 1.0;
      u = 1;
      sum = 1.0;
    }
    len[i] = u;
    rsum[i] = sum;
  }
}

__global__ void csr_out_kernel(int64_t n, const uint32_t* __restrict__ start,
                               const uint32_t* __restrict__ len, const uint32_t* __restrict__ rp,
                               const int32_t* __restrict__ ucol, const double* __restrict__ uw,
                               const double* __restrict__ rsum, int32_t* __restrict__ col,
                               float* __restrict__ val, int32_t* __restrict__ row_ptr, uint64_t nnz,
                               bool normalise) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t a = start[i], o = rp[i], m = len[i];
  const double s = rsum[i];
  for (uint32_t q = 0; q < m; q++) {
    col[o + q] = ucol[a + q];
    val[o + q] = normalise ? (float)(uw[a + q] / s) : (float)uw[a + q];
  }
  row_ptr[i] = (int32_t)o;
  if (i == n - 1) row_ptr[n] = (int32_t)nnz;
}

__global__ void one_segment_kernel(uint32_t* seg, int64_t n) {
  if (threadIdx.x == 0) {
    seg[0] = 0u;
    seg[1] = (uint32_t)n;
  }
}

unsigned grid1(int64_t items) { return (unsigned)((items + 255) / 256); }

}  // namespace

hipError_t build_knn_graph(const float4* centres, int64_t n, const float* feats, int D, int k,
                           const GraphWeights& gw, hipStream_t s, int32_t** row_ptr, int32_t** col,
                           float** val, int64_t* nnz_out) {
  const bool rbf = gw.kind == LV_GRAPH_FEATURE_RBF;
  *row_ptr = nullptr;
  *col = nullptr;
  *val = nullptr;
  *nnz_out = 0;
  const int64_t nk = n * (int64_t)k;
  const int64_t ucap = n * (int64_t)(2 * k + 1);  // union entries before merging
  // grid: about two centres per cell
  int G = 1;
  while ((int64_t)(G + 1) * (G + 1) * (G + 1) * 2 <= n && G < 1024) G++;
  const int64_t cells = (int64_t)G * G * G;
  int cell_bits = 0;
  while (((int64_t)1 << cell_bits) < cells) cell_bits++;
  const int nparts = (int)std::min<int64_t>(1024, (n + 255) / 256);

  // scratch layout (bytes), from the stream-ordered allocator
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
  const size_t o_part = take(4 * 6 * (size_t)nparts), o_gp = take(4 * 9);
  const size_t o_k0 = take(4 * (size_t)n), o_v0 = take(4 * (size_t)n), o_k1 = take(4 * (size_t)n),
               o_v1 = take(4 * (size_t)n), o_seg = take(8), o_hist = take(4 * sort_hist_size(1, n));
  const size_t o_cs = take(4 * (size_t)cells), o_ce = take(4 * (size_t)cells);
  const size_t o_idx = take(4 * (size_t)nk), o_d2 = take(8 * (size_t)nk), o_w = take(8 * (size_t)nk);
  const size_t o_st = take(8 * 4), o_shist = take(4 * 2 * kSelBins), o_sig = take(8),
               o_nrm = take(8 * (size_t)n);
  const size_t o_indeg = take(4 * (size_t)n), o_cap = take(4 * (size_t)n), o_start = take(4 * (size_t)n),
               o_fill = take(4 * (size_t)n), o_len = take(4 * (size_t)n), o_rp = take(4 * (size_t)n),
               o_rsum = take(8 * (size_t)n);
  const size_t o_ucol = take(4 * (size_t)ucap), o_uw = take(8 * (size_t)ucap);
  const size_t o_sseg = take(8), o_tot = take(16), o_stmp = take(4 * scan_tmp_size(n));
  char* base = nullptr;
  hipError_t e = dev_alloc((void**)&base, off, s, true);
  if (e != hipSuccess) return e;
  auto at = [&](size_t o) { return base + o; };
  float* part = (float*)at(o_part);
  float* gp = (float*)at(o_gp);
  uint32_t *k0 = (uint32_t*)at(o_k0), *v0 = (uint32_t*)at(o_v0), *k1 = (uint32_t*)at(o_k1),
           *v1 = (uint32_t*)at(o_v1), *seg = (uint32_t*)at(o_seg), *hist = (uint32_t*)at(o_hist);
  uint32_t *cs = (uint32_t*)at(o_cs), *ce = (uint32_t*)at(o_ce);
  int32_t* idx = (int32_t*)at(o_idx);
  double *d2 = (double*)at(o_d2), *w = (double*)at(o_w);
  unsigned long long* st = (unsigned long long*)at(o_st);
  unsigned int* shist = (unsigned int*)at(o_shist);
  double *sig2 = (double*)at(o_sig), *nrm = (double*)at(o_nrm);
  uint32_t *indeg = (uint32_t*)at(o_indeg), *cap = (uint32_t*)at(o_cap), *start = (uint32_t*)at(o_start),
           *fillpos = (uint32_t*)at(o_fill), *len = (uint32_t*)at(o_len), *rp = (uint32_t*)at(o_rp);
  double* rsum = (double*)at(o_rsum);
  int32_t* ucol = (int32_t*)at(o_ucol);
  double* uw = (double*)at(o_uw);
  uint32_t* sseg = (uint32_t*)at(o_sseg);
  unsigned long long* tot = (unsigned long long*)at(o_tot);
  uint32_t* stmp = (uint32_t*)at(o_stmp);
  uint64_t nnz = 0;

  do {
    // grid and centres sorted by cell
    hipLaunchKernelGGL(bbox_partial_kernel, dim3(nparts), dim3(256), 0, s, centres, n, part);
    hipLaunchKernelGGL(grid_params_kernel, dim3(1), dim3(64), 0, s, part, nparts, G, gp);
    hipLaunchKernelGGL(cell_keys_kernel, dim3(grid1(n)), dim3(256), 0, s, centres, n, gp, G, k0, v0);
    hipLaunchKernelGGL(one_segment_kernel, dim3(1), dim3(64), 0, s, seg, n);
    bool second = false;
    if ((e = radix_sort(k0, v0, k1, v1, seg, seg + 1, 1, n, cell_bits, hist, true, &second, s)) != hipSuccess) break;
    const uint32_t* skey = second ? k1 : k0;
    const uint32_t* sid = second ? v1 : v0;
    if ((e = hipMemsetAsync(cs, 0, 4 * (size_t)cells, s)) != hipSuccess) break;
    if ((e = hipMemsetAsync(ce, 0, 4 * (size_t)cells, s)) != hipSuccess) break;
    hipLaunchKernelGGL(cell_ranges_kernel, dim3(grid1(n)), dim3(256), 0, s, skey, n, cs, ce);
    // exact kNN
    if (k <= 8)
      hipLaunchKernelGGL(knn_kernel<8>, dim3(grid1(n)), dim3(256), 0, s, centres, n, sid, cs, ce, gp, G, k, idx, d2);
    else if (k <= 16)
      hipLaunchKernelGGL(knn_kernel<16>, dim3(grid1(n)), dim3(256), 0, s, centres, n, sid, cs, ce, gp, G, k, idx, d2);
    else
      hipLaunchKernelGGL(knn_kernel<32>, dim3(grid1(n)), dim3(256), 0, s, centres, n, sid, cs, ce, gp, G, k, idx, d2);
    // sigma: ranks (N - 1) / 2 and N / 2 of the squared distances
    const unsigned long long N = (unsigned long long)nk;
    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, st, (N - 1) / 2, N / 2, shist);
    const unsigned sblocks = (unsigned)std::min<int64_t>(1024, (nk + 255) / 256);
    for (int shift = 53, width = 11; ; ) {
      hipLaunchKernelGGL(select_hist_kernel, dim3(sblocks), dim3(256), 0, s, d2, nk, shift, width, st, shist);
      hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(1024), 0, s, shist, shift, st);
      if (shift == 0) break;
      width = shift >= 11 ? 11 : shift;
      shift -= width;
    }
    hipLaunchKernelGGL(sigma_kernel, dim3(1), dim3(64), 0, s, st, sig2);
    // weights
    hipLaunchKernelGGL(norms_kernel, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, s, feats, n, D, nrm);
    if (!rbf) {
      hipLaunchKernelGGL(edge_weights_kernel, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, s, feats,
                         n, D, k, idx, d2, nrm, sig2, w);
    } else {
      // s_f: median feature distance over the directed pairs (d2 is reused
      // for the feature distances; sigma above is not needed)
      hipLaunchKernelGGL(feature_d2_kernel, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, s, feats, n,
                         D, k, idx, nrm, w);
      hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, st, (N - 1) / 2, N / 2, shist);
      for (int shift = 53, width = 11; ; ) {
        hipLaunchKernelGGL(select_hist_kernel, dim3(sblocks), dim3(256), 0, s, w, nk, shift, width, st, shist);
        hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(1024), 0, s, shist, shift, st);
        if (shift == 0) break;
        width = shift >= 11 ? 11 : shift;
        shift -= width;
      }
      hipLaunchKernelGGL(sigma_kernel, dim3(1), dim3(64), 0, s, st, sig2);
      hipLaunchKernelGGL(rbf_weights_kernel, dim3(grid1(nk)), dim3(256), 0, s, nk, k, idx, w, sig2,
                         (double)gw.bandwidth, gw.unary, d2);
      double* t = w;  // the weights are in d2's buffer
      w = d2;
      d2 = t;
    }
    // union rows
    if ((e = hipMemsetAsync(indeg, 0, 4 * (size_t)n, s)) != hipSuccess) break;
    if ((e = hipMemsetAsync(fillpos, 0, 4 * (size_t)n, s)) != hipSuccess) break;
    hipLaunchKernelGGL(indeg_kernel, dim3(grid1(nk)), dim3(256), 0, s, idx, nk, indeg);
    hipLaunchKernelGGL(row_cap_kernel, dim3(grid1(n)), dim3(256), 0, s, indeg, n, k, cap);
    if ((e = scan_counts(cap, nullptr, n, 1, start, sseg, sseg + 1, tot, stmp, s)) != hipSuccess) break;
    hipLaunchKernelGGL(fill_rows_kernel, dim3(grid1(nk)), dim3(256), 0, s, idx, w, n, k, start, fillpos, ucol, uw);
    const bool bin = rbf && gw.binarize > 0.0f;
    hipLaunchKernelGGL(merge_rows_wave_kernel, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, s, n, k,
                       start, indeg, ucol, uw, len, rsum, bin ? (double)gw.binarize : 0.0, bin, !rbf);
    hipLaunchKernelGGL(merge_rows_kernel, dim3(grid1(n)), dim3(256), 0, s, n, k, start, indeg, ucol, uw, len,
                       rsum, bin ? (double)gw.binarize : 0.0, bin, !rbf);
    if ((e = scan_counts(len, nullptr, n, 1, rp, sseg, sseg + 1, tot, stmp, s)) != hipSuccess) break;
    unsigned long long th[2] = {0, 0};
    if ((e = hipMemcpyAsync(th, tot, 16, hipMemcpyDeviceToHost, s)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    nnz = th[0];
    if ((e = dev_alloc((void**)row_ptr, 4 * (size_t)(n + 1), s)) != hipSuccess) break;
    if ((e = dev_alloc((void**)col, 4 * (size_t)(nnz + 1), s)) != hipSuccess) break;
    if ((e = dev_alloc((void**)val, 4 * (size_t)(nnz + 1), s)) != hipSuccess) break;
    hipLaunchKernelGGL(csr_out_kernel, dim3(grid1(n)), dim3(256), 0, s, n, start, len, rp, ucol, uw, rsum,
                       *col, *val, *row_ptr, (uint64_t)nnz, !rbf);
    e = hipGetLastError();
  } while (false);
  dev_free(base, off, s, true);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    dev_free(*row_ptr, 4 * (size_t)(n + 1), s);
    dev_free(*col, 4 * (size_t)(nnz + 1), s);
    dev_free(*val, 4 * (size_t)(nnz + 1), s);
    *row_ptr = nullptr;
    *col = nullptr;
    *val = nullptr;
    return e;
  }
  *nnz_out = (int64_t)nnz;
  return hipSuccess;
}

}  // namespace lv
