// Per-view ordering (Sec. 3.1: each pixel blends its Gaussians in the order
// the ray meets them): depth sort of the Gaussians, tile duplication in depth
// order, stable sort of the (tile, Gaussian) pairs by tile, tile ranges.
// The result per tile is its Gaussians sorted by (depth key, index).
//
// The radix sort is a segmented, stable LSD sort with digits of up to 11 bits
// in three kernels per pass (block histograms, per-segment scan, stable
// scatter).
// Within a block, each wave ranks its items in rounds of 64 in index order;
// lanes holding the same digit are found with one wave ballot per digit bit,
// so ranking needs no atomics and keeps input order among equal digits.
#include <type_traits>

#include "lv_internal.h"

namespace lv {

namespace {

__device__ __forceinline__ uint64_t lanemask_lt() {
  uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave (among `active`) whose digit equals this lane's digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits, uint64_t active) {
  uint64_t peers = active;
  for (int b = 0; b < bits; b++) {
    uint64_t bal = __ballot((d >> b) & 1u);
    peers &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return peers;
}

constexpr int kBins = 1 << kRadixBits;        // digit values per pass
static_assert(kBins <= 2048, "the scan gives each of its 1024 threads at most two digits");
constexpr int kWaveItems = kSortItems / 4;    // contiguous items per wave
constexpr int kPerLane = kWaveItems / 64;     // items per lane, held in registers
constexpr int kPerThread = kSortItems / kSortThreads;
static_assert(kSortThreads == 256 && kWaveItems % 64 == 0, "four waves per block");

// Digit counts of one block's items (LDS atomics: the order of counting does
// not matter), written as the block's row hist[segment][block][digit].  All
// of the block's keys are loaded before any is counted.
// kB: digit values the LDS arrays hold (passes of at most 8 or 10 bits use
// smaller arrays, so more blocks fit on a CU).
template <int kB, typename K = uint32_t>
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(
    const K* __restrict__ keys, const uint32_t* __restrict__ seg_start,
    const uint32_t* __restrict__ seg_len, int shift, int bits, int nb, uint32_t* __restrict__ hist) {
  __shared__ uint32_t hs[kB];
  const int g = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
  const int nbins = 1 << bits;
  const uint32_t mask = (uint32_t)nbins - 1u;
  const uint32_t len = seg_len[g];
  const uint32_t base = (uint32_t)b * kSortItems;
  const K* k = keys + seg_start[g];
  uint32_t d[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; r++) {
    const uint32_t i = base + (uint32_t)(r * kSortThreads + t);
    d[r] = i < len ? (k[i] >> shift) & mask : ~0u;
  }
  for (int e = t; e < nbins; e += kSortThreads) hs[e] = 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPerThread; r++)
    if (d[r] != ~0u) atomicAdd(&hs[d[r]], 1u);
  __syncthreads();
  uint32_t* hb = hist + ((size_t)g * nb + b) * nbins;  // this block's row: contiguous writes
  for (int e = t; e < nbins; e += kSortThreads) hb[e] = hs[e];
}

// Exclusive scan, per segment, over (digit, block) in digit-major order, of
// counts stored block-major (hist[segment][block][digit]).  Thread t owns
// digits [k t, k t + k): it sums its columns over the blocks, the digit totals
// are scanned across the threads, and a second walk down the columns writes
// each entry's start.  Rows are read whole by the block (coalesced).
__global__ __launch_bounds__(1024) void radix_scan_kernel(uint32_t* __restrict__ hist, int nb,
                                                          int bits) {
  __shared__ uint32_t part[1024 / 64];
  const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nbins = 1 << bits;
  const int k = nbins > 1024 ? nbins / 1024 : 1;  // digits per thread (1 or 2)
  const int d0 = k * t;
  const bool own = d0 < nbins;
  uint32_t* h = hist + (size_t)g * nb * nbins;
  uint32_t tot[2] = {0u, 0u};
  if (own) {
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
      uint32_t x[8][2];
#pragma unroll
      for (int u = 0; u < 8; u++)
#pragma unroll
        for (int j = 0; j < 2; j++) x[u][j] = j < k ? h[(size_t)(b + u) * nbins + d0 + j] : 0u;
#pragma unroll
      for (int u = 0; u < 8; u++) {
        tot[0] += x[u][0];
        tot[1] += x[u][1];
      }
    }
    for (; b < nb; b++)
      for (int j = 0; j < k; j++) tot[j] += h[(size_t)b * nbins + d0 + j];
  }
  const uint32_t mine = tot[0] + tot[1];
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) part[w] = incl;
  __syncthreads();
  uint32_t run0 = incl - mine;
  for (int q = 0; q < w; q++) run0 += part[q];
  if (!own) return;
  uint32_t run[2] = {run0, run0 + tot[0]};
  int b = 0;
  for (; b + 8 <= nb; b += 8) {
    uint32_t x[8][2];
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int j = 0; j < 2; j++) x[u][j] = j < k ? h[(size_t)(b + u) * nbins + d0 + j] : 0u;
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int j = 0; j < 2; j++)
        if (j < k) {
          h[(size_t)(b + u) * nbins + d0 + j] = run[j];
          run[j] += x[u][j];
        }
  }
  for (; b < nb; b++)
    for (int j = 0; j < k; j++) {
      const uint32_t x = h[(size_t)b * nbins + d0 + j];
      h[(size_t)b * nbins + d0 + j] = run[j];
      run[j] += x;
    }
}

// The same scan split over row chunks, for segments with many blocks and at
// most 1024 digits (the scan above runs one block per segment, so a few
// segments of many rows leave the chip mostly idle).  part[segment][chunk]
// [digit] holds first the chunk's column sums, then each chunk's starting
// offset per digit.
__global__ __launch_bounds__(1024) void radix_chunk_sum_kernel(const uint32_t* __restrict__ hist,
                                                               int nb, int bits, int chunks,
                                                               uint32_t* __restrict__ part) {
  const int g = blockIdx.y, c = blockIdx.x, t = threadIdx.x;
  const int nbins = 1 << bits;
  const int r0 = (int)((int64_t)nb * c / chunks), r1 = (int)((int64_t)nb * (c + 1) / chunks);
  if (t >= nbins) return;
  const uint32_t* h = hist + (size_t)g * nb * nbins + t;
  uint32_t sum = 0u;
  for (int b = r0; b < r1; b++) sum += h[(size_t)b * nbins];
  part[((size_t)g * chunks + c) * nbins + t] = sum;
}

__global__ __launch_bounds__(1024) void radix_chunk_scan_kernel(uint32_t* __restrict__ part,
                                                                int bits, int chunks) {
  __shared__ uint32_t wsum[1024 / 64];
  const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nbins = 1 << bits;
  uint32_t* pg = part + (size_t)g * chunks * nbins;
  uint32_t tot = 0u;
  if (t < nbins)
    for (int c = 0; c < chunks; c++) tot += pg[(size_t)c * nbins + t];
  uint32_t incl = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - tot;
  for (int q = 0; q < w; q++) run += wsum[q];
  if (t >= nbins) return;
  for (int c = 0; c < chunks; c++) {
    const uint32_t x = pg[(size_t)c * nbins + t];
    pg[(size_t)c * nbins + t] = run;
    run += x;
  }
}

__global__ __launch_bounds__(1024) void radix_chunk_write_kernel(uint32_t* __restrict__ hist,
                                                                 int nb, int bits, int chunks,
                                                                 const uint32_t* __restrict__ part) {
  const int g = blockIdx.y, c = blockIdx.x, t = threadIdx.x;
  const int nbins = 1 << bits;
  const int r0 = (int)((int64_t)nb * c / chunks), r1 = (int)((int64_t)nb * (c + 1) / chunks);
  if (t >= nbins) return;
  uint32_t* h = hist + (size_t)g * nb * nbins + t;
  uint32_t run = part[((size_t)g * chunks + c) * nbins + t];
  for (int b = r0; b < r1; b++) {
    const uint32_t x = h[(size_t)b * nbins];
    h[(size_t)b * nbins] = run;
    run += x;
  }
}

// Stable scatter through LDS.  Each wave takes a contiguous quarter of the
// block's items into registers (item lo + 64 r + lane), finds for each round
// of 64 the lanes sharing its digit (kept for both uses below), and counts
// per (wave, digit).  The block then ranks its items locally in digit order
// (waves in order, rounds in order, lanes in order), places them in LDS at
// those ranks and writes the LDS contents out in order: items of one digit
// are consecutive in LDS and go to consecutive global positions.  kout may
// be NULL (keys not needed after this pass).  With a payload, each item also
// takes rect[s0 + val] (and its area, the count) to its output position.
// kKeys false: the keys are not written (kout NULL), so LDS holds each
// item's digit instead of its key (a smaller block footprint).
template <int kB, bool kKeys = true, typename K = uint32_t>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ seg_start,
    const uint32_t* __restrict__ seg_len, int shift, int bits, int nb,
    const uint32_t* __restrict__ hist, SortPayload pl) {
  constexpr int kPer = kB / kSortThreads;          // digits per thread in the scan
  __shared__ uint16_t wc[4][kB];                    // per-wave counts, then local cursors
  __shared__ uint32_t gdelta[kB];                   // global minus local position, per digit
  // LDS keeps each item's key (16-bit keys, or 32-bit ones that are written
  // out) or only its digit
  typedef typename std::conditional<kKeys && sizeof(K) == 4, uint32_t, uint16_t>::type lk_t;
  __shared__ lk_t lk[kSortItems];
  __shared__ uint32_t lval[kSortItems];
  __shared__ uint32_t wsum[kSortThreads / 64];
  const int g = blockIdx.y, b = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint32_t s0 = seg_start[g];
  const uint32_t len = seg_len[g];
  const uint32_t base = (uint32_t)b * kSortItems;
  if (base >= len) return;  // whole block idle (uniform)
  const uint32_t items = min(len - base, (uint32_t)kSortItems);
  const uint32_t lo = base + w * kWaveItems;
  const uint32_t hi = min(len, lo + kWaveItems);  // lo >= hi: the wave has no items
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t lt = lanemask_lt();

  uint32_t key[kPerLane], val[kPerLane];
#pragma unroll
  for (int r = 0; r < kPerLane; r++) {
    const uint32_t i = lo + 64u * r + lane;
    key[r] = i < hi ? kin[s0 + i] : 0u;
    val[r] = i < hi ? (vin ? vin[s0 + i] : i) : 0u;  // no vin: the item's index in its segment
  }
  for (int e = t; e < 4 * kB; e += kSortThreads) (&wc[0][0])[e] = 0;
  __syncthreads();

  // count per (wave, digit): the lowest lane of each group of equal digits
  // adds the group's size
  uint64_t peers[kPerLane];
  uint16_t* cur = wc[w];
#pragma unroll
  for (int r = 0; r < kPerLane; r++) {
    peers[r] = 0ull;
    if (lo + 64u * r < hi) {  // wave-uniform
      const bool valid = lo + 64u * r + lane < hi;
      const uint32_t d = (key[r] >> shift) & mask;
      peers[r] = match_digit(d, bits, __ballot(valid));
      if (valid && (peers[r] & lt) == 0) cur[d] = (uint16_t)(cur[d] + (uint32_t)__popcll(peers[r]));
    }
  }
  __syncthreads();

  // block-local exclusive scan over digits (thread t owns digits [kPer t, kPer t + kPer))
  const int nbins = 1 << bits;
  uint32_t tot = 0;
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const int d = kPer * t + k;
    if (d < nbins) tot += (uint32_t)wc[0][d] + wc[1][d] + wc[2][d] + wc[3][d];
  }
  uint32_t incl = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - tot;
  for (int q = 0; q < w; q++) run += wsum[q];
  const uint32_t* hrow = hist + ((size_t)g * nb + b) * nbins;
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const int d = kPer * t + k;
    if (d < nbins) {
      gdelta[d] = s0 + hrow[d] - run;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const uint32_t c = wc[q][d];
        wc[q][d] = (uint16_t)run;
        run += c;
      }
    }
  }
  __syncthreads();

  // each wave places its items at their block-local ranks
#pragma unroll
  for (int r = 0; r < kPerLane; r++) {
    if (lo + 64u * r < hi) {  // wave-uniform
      const bool valid = lo + 64u * r + lane < hi;
      const uint32_t d = (key[r] >> shift) & mask;
      const uint32_t rank = (uint32_t)__popcll(peers[r] & lt);
      if (valid) {
        const uint32_t pos = (uint32_t)cur[d] + rank;
        lk[pos] = (lk_t)(kKeys ? key[r] : d);
        lval[pos] = val[r];
      }
      __builtin_amdgcn_wave_barrier();  // every lane has read cur[d]
      if (valid && rank == 0) cur[d] = (uint16_t)(cur[d] + (uint32_t)__popcll(peers[r]));
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();

  // write out in local order: runs of one digit land on consecutive positions
  if (!pl.orect) {
    for (uint32_t p = t; p < items; p += kSortThreads) {
      const uint32_t k = lk[p];
      const uint32_t pos = gdelta[kKeys ? (k >> shift) & mask : k] + p;
      if (kKeys && kout) kout[pos] = (K)k;
      vout[pos] = lval[p];
    }
    return;
  }
  // with the payload: every rect gathered first (all in flight together),
  // then the writes; the count is the rect's area
  uint32_t pos[kPerThread], vv[kPerThread];
  uint2 rr[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; r++) {
    const uint32_t p = (uint32_t)(t + r * kSortThreads);
    pos[r] = 0u;
    vv[r] = 0u;
    rr[r] = make_uint2(0u, 0u);
    if (p < items) {
      const uint32_t k = lk[p];
      pos[r] = gdelta[kKeys ? (k >> shift) & mask : k] + p;
      vv[r] = lval[p];
      rr[r] = pl.rect[s0 + vv[r]];
      if (kKeys && kout) kout[pos[r]] = (K)k;
    }
  }
#pragma unroll
  for (int r = 0; r < kPerThread; r++) {
    if ((uint32_t)(t + r * kSortThreads) < items) {
      vout[pos[r]] = vv[r];
      pl.orect[pos[r]] = rr[r];
      pl.ocnt[pos[r]] = ((rr[r].y & 0xFFFFu) - (rr[r].x & 0xFFFFu)) * ((rr[r].y >> 16) - (rr[r].x >> 16));
    }
  }
}

// Tile ranges of a single-pass tile sort, from its scanned counts: block 0's
// row holds the start of every digit (tile) within the segment (view).
__global__ void hist_ranges_kernel(const uint32_t* __restrict__ hist,
                                   const uint32_t* __restrict__ seg_start,
                                   const uint32_t* __restrict__ seg_len, int nb, int bits,
                                   int stride, uint2* __restrict__ ranges) {
  const int g = blockIdx.y;
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= stride) return;
  const int nbins = 1 << bits;
  const uint32_t* h0 = hist + (size_t)g * nb * nbins;
  const uint32_t s0 = seg_start[g], len = seg_len[g];
  const uint32_t a = d < nbins ? h0[d] : len;
  const uint32_t e = d + 1 < nbins ? h0[d + 1] : len;
  ranges[(int64_t)g * stride + d] = make_uint2(s0 + a, s0 + e);
}

// ---- scan of per-(view, Gaussian) tile counts in depth order
constexpr int kScanItems = 4096;

__global__ __launch_bounds__(256) void count_reduce_kernel(const uint32_t* __restrict__ cnt,
                                                           const uint32_t* __restrict__ sval,
                                                           int64_t n, int64_t items,
                                                           unsigned long long* __restrict__ bsum,
                                                           unsigned long long* __restrict__ nvis) {
  __shared__ unsigned long long red[4], redv[4];
  const int64_t base = (int64_t)blockIdx.x * kScanItems;
  unsigned long long s = 0, nv = 0;
  // item i belongs to view i / n: one division, then the view start moves
  // along with i (steps of 256 may cross several views when n is small)
  int64_t i = base + threadIdx.x;
  int64_t vs = (i / n) * n;  // start of i's view
  for (int k = threadIdx.x; k < kScanItems; k += 256, i += 256) {
    while (i >= vs + n) vs += n;
    if (i < items) {
      const uint32_t c = sval ? cnt[vs + sval[i]] : cnt[i];
      s += c;
      nv += c != 0u;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_down(s, o, 64);
    nv += __shfl_down(nv, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = s;
    redv[threadIdx.x >> 6] = nv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    atomicAdd(nvis, redv[0] + redv[1] + redv[2] + redv[3]);
  }
}

// Exclusive scan of the block sums (one block); total into bsum[nblocks].
__global__ __launch_bounds__(1024) void bsum_scan_kernel(unsigned long long* __restrict__ bsum,
                                                         int64_t nblocks) {
  __shared__ unsigned long long part[16];
  __shared__ unsigned long long carry_s;
  int t = threadIdx.x, lane = t & 63, w = t >> 6;
  unsigned long long carry = 0;
  for (int64_t base = 0; base < nblocks; base += 1024) {
    int64_t i = base + t;
    unsigned long long x = i < nblocks ? bsum[i] : 0ull;
    unsigned long long incl = x;
    for (int o = 1; o < 64; o <<= 1) {
      unsigned long long y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) part[w] = incl;
    __syncthreads();
    if (t == 0) {
      unsigned long long s = 0;
      for (int q = 0; q < 16; q++) {
        unsigned long long p = part[q];
        part[q] = s;
        s += p;
      }
      carry_s = s;
    }
    __syncthreads();
    if (i < nblocks) bsum[i] = carry + part[w] + incl - x;
    carry += carry_s;
    __syncthreads();
  }
  if (t == 0) bsum[nblocks] = carry;
}

__global__ __launch_bounds__(256) void count_scan_kernel(const uint32_t* __restrict__ cnt,
                                                         const uint32_t* __restrict__ sval,
                                                         int64_t n, int64_t items,
                                                         const unsigned long long* __restrict__ bsum,
                                                         uint32_t* __restrict__ off) {
  // the block's 4096 counts go through LDS (one pad word per 16, so that a
  // thread's 16 consecutive items are read without bank conflicts): loads
  // and stores are coalesced, thread t scans items [16 t, 16 t + 16)
  __shared__ uint32_t buf[kScanItems + kScanItems / 16];
  __shared__ uint32_t part[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanItems;
  int64_t i = base + t;
  int64_t vs = (i / n) * n;  // start of i's view (one division, then moved along)
#pragma unroll
  for (int r = 0; r < kScanItems / 256; r++, i += 256) {
    while (i >= vs + n) vs += n;
    uint32_t c = 0;
    if (i < items) c = sval ? cnt[vs + sval[i]] : cnt[i];
    const int e = t + 256 * r;
    buf[e + (e >> 4)] = c;
  }
  __syncthreads();
  uint32_t x[16];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int e = 16 * t + k;
    x[k] = buf[e + (e >> 4)];
    sum += x[k];
  }
  uint32_t incl = sum;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) part[w] = incl;
  __syncthreads();
  uint32_t wo = 0;
  for (int q = 0; q < w; q++) wo += part[q];
  uint32_t run = (uint32_t)bsum[blockIdx.x] + wo + incl - sum;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int e = 16 * t + k;
    buf[e + (e >> 4)] = run;
    run += x[k];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScanItems / 256; r++) {
    const int e = t + 256 * r;
    const int64_t j = base + e;
    if (j < items) off[j] = buf[e + (e >> 4)];
  }
}

__global__ void seg_kernel(const uint32_t* __restrict__ off, int64_t n, int m,
                           const unsigned long long* __restrict__ total,
                           uint32_t* __restrict__ seg_start, uint32_t* __restrict__ seg_len,
                           unsigned long long* __restrict__ out_total) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) out_total[0] = *total;
  if (v >= m) return;
  uint32_t a = n ? off[(int64_t)v * n] : 0u;
  uint32_t b = (v + 1 < m && n) ? off[(int64_t)(v + 1) * n] : (uint32_t)*total;
  seg_start[v] = a;
  seg_len[v] = b - a;
}

// Pairs of 64 consecutive depth-sorted items of a view, written by their wave
// together: the items' pairs are consecutive in the output (off is the
// exclusive scan of the counts in this order), so the wave walks them 64 at a
// time, each lane finding the item that owns its pair by a binary search over
// the wave's inclusive count prefix.  Within an item, tiles go row by row.
// K = uint32_t: key view << 20 | tile; K = uint16_t: the tile alone (the
// sort is segmented by view, so the view is its segment)
template <typename K>
__global__ __launch_bounds__(256) void duplicate_kernel(const uint32_t* __restrict__ sval,
                                                        const uint32_t* __restrict__ off,
                                                        const uint2* __restrict__ srect,
                                                        const uint32_t* __restrict__ scnt,
                                                        const ViewGeom* __restrict__ geom, int64_t n,
                                                        K* __restrict__ pkey,
                                                        uint32_t* __restrict__ pval) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  const int lane = threadIdx.x & 63;
  if (k - lane >= n) return;  // the whole wave is past the view's end
  uint32_t gi = 0u, c = 0u, p = 0u, x0 = 0u, y0 = 0u, w = 1u;
  if (k < n) {
    const int64_t o = (int64_t)v * n + k;
    gi = sval[o];
    c = scnt[o];
    p = off[o];
    if (c) {
      const uint2 r = srect[o];
      x0 = r.x & 0xFFFFu;
      y0 = r.x >> 16;
      w = (r.y & 0xFFFFu) - x0;
    }
  }
  uint32_t incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  const uint32_t p0 = __shfl(p, 0, 64);  // lane 0 is inside the view
  const uint32_t excl = incl - c;
  const uint32_t TX = (uint32_t)geom[v].TX;
  const uint32_t hv = sizeof(K) == 4 ? (uint32_t)v << kViewShift : 0u;
  for (uint32_t j = 0; j < total; j += 64) {
    const uint32_t slot = j + lane;
    // owner: the number of lanes whose inclusive prefix is <= slot
    int pos = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (__shfl(incl, pos + step - 1, 64) <= slot) pos += step;
    const uint32_t kk = slot - __shfl(excl, pos, 64);
    const uint32_t ow = __shfl(w, pos, 64), ox = __shfl(x0, pos, 64), oy = __shfl(y0, pos, 64);
    const uint32_t og = __shfl(gi, pos, 64);
    if (slot < total) {
      const uint32_t dy = kk / ow;
      pkey[p0 + slot] = (K)(hv | ((oy + dy) * TX + ox + (kk - dy * ow)));
      pval[p0 + slot] = og;
    }
  }
}

// Four consecutive sorted keys per thread (one 16-byte load where the key
// array is 16-byte aligned): a key that differs from its predecessor starts
// its tile's range, one that differs from its successor ends it.
__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t* __restrict__ key, int64_t P,
                                                     int stride, bool aligned, uint2* __restrict__ ranges) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i0 = 4 * q;
  if (i0 >= P) return;
  uint32_t k[4];
  if (aligned && i0 + 4 <= P) {
    const uint4 v = reinterpret_cast<const uint4*>(key)[q];
    k[0] = v.x;
    k[1] = v.y;
    k[2] = v.z;
    k[3] = v.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; j++) k[j] = i0 + j < P ? key[i0 + j] : 0u;
  }
  const uint32_t before = i0 > 0 ? key[i0 - 1] : 0u;
  const uint32_t after = i0 + 4 < P ? key[i0 + 4] : 0u;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int64_t i = i0 + j;
    if (i >= P) break;
    const uint32_t v = k[j] >> kViewShift, tile = k[j] & ((1u << kViewShift) - 1u);
    uint2* r = ranges + (int64_t)v * stride + tile;
    const uint32_t prev = j > 0 ? k[j - 1] : before;
    const uint32_t next = j < 3 ? k[j + 1] : after;
    if (i == 0 || prev != k[j]) r->x = (uint32_t)i;
    if (i + 1 == P || next != k[j]) r->y = (uint32_t)(i + 1);
  }
}

// Exact depth ties of a scene stored in Morton order, back in the caller's
// index order.  Grid row blockIdx.y is a view (its n depth-sorted items);
// four consecutive items per thread (one 16-byte load where aligned).  A
// lane first finds the runs (two or more equal visible keys) that start
// among its items, at most two, then handles them together: a pair (by far
// the commonest tie) is, where the two tile rectangles overlap (else no
// tile list holds both), one compare of the two caller indices and a swap,
// with the loads of both runs in flight at once; longer runs are
// insertion-sorted by caller index.
__global__ __launch_bounds__(256) void depth_ties_kernel(const uint32_t* __restrict__ key,
                                                         uint32_t* __restrict__ val,
                                                         uint2* __restrict__ rect,
                                                         uint32_t* __restrict__ cnt, int64_t n,
                                                         bool aligned,
                                                         const uint32_t* __restrict__ perm) {
  const int64_t e0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);  // in the view
  if (e0 >= n) return;
  const int64_t base = (int64_t)blockIdx.y * n;
  const uint32_t* kv = key + base;
  uint32_t k[4];
  if (aligned && e0 + 4 <= n) {
    const uint4 v = *reinterpret_cast<const uint4*>(kv + e0);
    k[0] = v.x;
    k[1] = v.y;
    k[2] = v.z;
    k[3] = v.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; j++) k[j] = e0 + j < n ? kv[e0 + j] : 0xFFFFFFFFu;
  }
  if (k[0] == 0xFFFFFFFFu) return;  // culled items sort last: so are the lane's others
  const uint32_t before = e0 > 0 ? kv[e0 - 1] : 0xFFFFFFFFu;
  const uint32_t after = e0 + 4 < n ? kv[e0 + 4] : 0xFFFFFFFFu;
  int64_t st[2] = {0, 0};  // run starts (in the view)
  int ns = 0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int64_t e = e0 + j;
    const uint32_t kk = k[j];
    if (kk == 0xFFFFFFFFu || e + 1 >= n) continue;                     // culled, or the view's last item
    if ((j < 3 ? k[j + 1] : after) != kk) continue;                     // no tie after it
    if (e > 0 && (j > 0 ? k[j - 1] : before) == kk) continue;          // not the run's first item
    st[ns < 2 ? ns : 1] = e;  // at most two starts among four items
    ns++;
  }
  if (ns == 0) return;
  uint32_t a[2], b[2];
  uint2 ra[2], rb[2];
  bool longer[2];
#pragma unroll
  for (int t = 0; t < 2; t++) {
    const int64_t e = base + st[t];
    const bool on = t < ns;
    a[t] = on ? val[e] : 0u;
    b[t] = on ? val[e + 1] : 0u;
    ra[t] = on ? rect[e] : make_uint2(0u, 0u);
    rb[t] = on ? rect[e + 1] : make_uint2(0u, 0u);
    longer[t] = on && st[t] + 2 < n && key[e + 2] == key[e];
  }
#pragma unroll
  for (int t = 0; t < 2; t++) {
    const int64_t e = base + st[t];
    // two Gaussians whose tile rectangles [x0, x1) x [y0, y1) are disjoint
    // share no tile list: their relative order changes nothing
    const uint2 p = ra[t], q = rb[t];
    const bool overlap = (p.x & 0xFFFFu) < (q.y & 0xFFFFu) && (q.x & 0xFFFFu) < (p.y & 0xFFFFu) &&
                         (p.x >> 16) < (q.y >> 16) && (q.x >> 16) < (p.y >> 16);
    if (t < ns && !longer[t] && overlap && perm[a[t]] > perm[b[t]]) {
      const uint32_t c0 = cnt[e], c1 = cnt[e + 1];
      val[e] = b[t];
      val[e + 1] = a[t];
      rect[e] = q;
      rect[e + 1] = p;
      cnt[e] = c1;
      cnt[e + 1] = c0;
    }
  }
#pragma unroll
  for (int t = 0; t < 2; t++) {
    if (t >= ns || !longer[t]) continue;
    const int64_t e = base + st[t], end = base + n;
    const uint32_t kk = key[e];
    int64_t r = e + 3;
    while (r < end && key[r] == kk) r++;
    for (int64_t i = e + 1; i < r; i++) {
      const uint32_t v = val[i], pv = perm[v];
      const uint2 rc = rect[i];
      const uint32_t c = cnt[i];
      int64_t u = i;
      while (u > e && perm[val[u - 1]] > pv) {
        val[u] = val[u - 1];
        rect[u] = rect[u - 1];
        cnt[u] = cnt[u - 1];
        u--;
      }
      val[u] = v;
      rect[u] = rc;
      cnt[u] = c;
    }
  }
}

// Tile ranges from 16-bit sorted tile keys: grid row blockIdx.y is a view
// (its segment [s0, s0 + len) of the pairs); each thread takes eight keys
// at an absolute position that is a multiple of 8 (one aligned 16-byte
// load; keys of the neighbouring segments in it are skipped, and the key
// buffer has 16 bytes of slack past the last pair).
__global__ __launch_bounds__(256) void ranges16_kernel(const uint16_t* __restrict__ key,
                                                       const uint32_t* __restrict__ seg_start,
                                                       const uint32_t* __restrict__ seg_len, int stride,
                                                       bool aligned, uint2* __restrict__ ranges) {
  const int v = blockIdx.y;
  const int64_t s0 = seg_start[v], e = s0 + (int64_t)seg_len[v];
  const int64_t p0 = (s0 & ~(int64_t)7) + 8 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (p0 >= e) return;
  uint32_t k[8];
  if (aligned) {
    const uint4 w = *reinterpret_cast<const uint4*>(key + p0);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; j++) {
      k[2 * j] = ws[j] & 0xFFFFu;
      k[2 * j + 1] = ws[j] >> 16;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; j++) k[j] = p0 + j >= s0 && p0 + j < e ? key[p0 + j] : 0u;
  }
  const uint32_t before = p0 > s0 ? key[p0 - 1] : 0u;
  const uint32_t after = p0 + 8 < e ? key[p0 + 8] : 0u;
  uint2* rv = ranges + (int64_t)v * stride;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    const int64_t i = p0 + j;
    if (i < s0 || i >= e) continue;
    const uint32_t prev = j > 0 ? k[j - 1] : before;
    const uint32_t next = j < 7 ? k[j + 1] : after;
    if (i == s0 || prev != k[j]) rv[k[j]].x = (uint32_t)i;
    if (i + 1 == e || next != k[j]) rv[k[j]].y = (uint32_t)(i + 1);
  }
}

}  // namespace

hipError_t launch_depth_ties(const uint32_t* key, uint32_t* val, uint2* rect, uint32_t* cnt, int64_t n,
                             int mv, const uint32_t* perm, hipStream_t s) {
  if (n < 2 || mv == 0) return hipSuccess;
  const int64_t quads = (n + 3) / 4;
  const bool aligned = ((uintptr_t)key & 15) == 0 && n % 4 == 0;  // every view's start too
  hipLaunchKernelGGL(depth_ties_kernel, dim3((unsigned)((quads + 255) / 256), mv), dim3(256), 0, s, key, val,
                     rect, cnt, n, aligned, perm);
  return hipGetLastError();
}

size_t sort_hist_size(int nseg, int64_t max_len) {
  int64_t nb = (max_len + kSortItems - 1) / kSortItems;
  if (nb < 1) nb = 1;
  return (size_t)nseg * kBins * (size_t)nb;
}

namespace {
template <typename K>
hipError_t radix_sort_t(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const uint32_t* seg_start,
                        const uint32_t* seg_len, int nseg, int64_t max_len, int bits, uint32_t* hist,
                        bool keys_last, bool* in_second, hipStream_t s, SortPayload payload, int pass_bits,
                        bool iota_values) {
  *in_second = false;
  if (nseg == 0 || max_len == 0 || bits == 0) return hipSuccess;
  int nb = (int)((max_len + kSortItems - 1) / kSortItems);
  K *ki = k0, *ko = k1;
  uint32_t *vi = v0, *vo = v1;
  // fewest passes of at most kRadixBits bits, widths balanced
  pass_bits = pass_bits < 1 ? 1 : (pass_bits > kRadixBits ? kRadixBits : pass_bits);
  const int passes = radix_passes(bits, pass_bits);
  for (int p = 0, shift = 0; p < passes; p++) {
    const int pb = (bits - shift + (passes - p) - 1) / (passes - p);
    K* const kout = (p + 1 < passes || keys_last) ? ko : nullptr;
    const uint32_t* const vin = p == 0 && iota_values ? nullptr : vi;
    const SortPayload pl = p + 1 < passes ? SortPayload{} : payload;
    if (pb <= 8) {
      hipLaunchKernelGGL((radix_hist_kernel<256, K>), dim3(nb, nseg), dim3(kSortThreads), 0, s, ki,
                         seg_start, seg_len, shift, pb, nb, hist);
    } else if (pb <= 10) {
      hipLaunchKernelGGL((radix_hist_kernel<1024, K>), dim3(nb, nseg), dim3(kSortThreads), 0, s, ki,
                         seg_start, seg_len, shift, pb, nb, hist);
    } else {
      hipLaunchKernelGGL((radix_hist_kernel<kBins, K>), dim3(nb, nseg), dim3(kSortThreads), 0, s, ki,
                         seg_start, seg_len, shift, pb, nb, hist);
    }
    if (pb <= 10 && nb >= 64) {
      // chunks of rows; their sums live in the unused upper half of hist
      // (sized for kBins >= 2 x 1024 digits per row)
      const int chunks = 16;
      uint32_t* part = hist + (size_t)nseg * nb * ((size_t)1 << pb);
      hipLaunchKernelGGL(radix_chunk_sum_kernel, dim3(chunks, nseg), dim3(1024), 0, s, hist, nb, pb,
                         chunks, part);
      hipLaunchKernelGGL(radix_chunk_scan_kernel, dim3(nseg), dim3(1024), 0, s, part, pb, chunks);
      hipLaunchKernelGGL(radix_chunk_write_kernel, dim3(chunks, nseg), dim3(1024), 0, s, hist, nb,
                         pb, chunks, part);
    } else {
      hipLaunchKernelGGL(radix_scan_kernel, dim3(nseg), dim3(1024), 0, s, hist, nb, pb);
    }
    if (pb <= 8) {
      hipLaunchKernelGGL((radix_scatter_kernel<256, true, K>), dim3(nb, nseg), dim3(kSortThreads), 0, s, ki,
                         vin, kout, vo, seg_start, seg_len, shift, pb, nb, hist, pl);
    } else if (pb <= 10 && !kout) {
      hipLaunchKernelGGL((radix_scatter_kernel<1024, false, K>), dim3(nb, nseg), dim3(kSortThreads), 0,
                         s, ki, vin, kout, vo, seg_start, seg_len, shift, pb, nb, hist, pl);
    } else if (pb <= 10) {
      hipLaunchKernelGGL((radix_scatter_kernel<1024, true, K>), dim3(nb, nseg), dim3(kSortThreads), 0, s, ki,
                         vin, kout, vo, seg_start, seg_len, shift, pb, nb, hist, pl);
    } else {
      hipLaunchKernelGGL((radix_scatter_kernel<kBins, true, K>), dim3(nb, nseg), dim3(kSortThreads), 0, s, ki,
                         vin, kout, vo, seg_start, seg_len, shift, pb, nb, hist, pl);
    }
    shift += pb;
    K* tk = ki;
    ki = ko;
    ko = tk;
    uint32_t* tv = vi;
    vi = vo;
    vo = tv;
    *in_second = !*in_second;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                      const uint32_t* seg_start, const uint32_t* seg_len, int nseg,
                      int64_t max_len, int bits, uint32_t* hist, bool keys_last, bool* in_second,
                      hipStream_t s, SortPayload payload, int pass_bits, bool iota_values) {
  return radix_sort_t(k0, v0, k1, v1, seg_start, seg_len, nseg, max_len, bits, hist, keys_last, in_second, s,
                      payload, pass_bits, iota_values);
}

hipError_t radix_sort16(uint16_t* k0, uint32_t* v0, uint16_t* k1, uint32_t* v1,
                        const uint32_t* seg_start, const uint32_t* seg_len, int nseg, int64_t max_len,
                        int bits, uint32_t* hist, bool keys_last, bool* in_second, hipStream_t s) {
  return radix_sort_t(k0, v0, k1, v1, seg_start, seg_len, nseg, max_len, bits, hist, keys_last, in_second, s,
                      SortPayload{}, kRadixBits, false);
}


hipError_t launch_hist_ranges(const uint32_t* hist, const uint32_t* seg_start,
                              const uint32_t* seg_len, int nseg, int64_t max_len, int bits,
                              int tiles_stride, uint2* ranges, hipStream_t s) {
  if (nseg == 0 || tiles_stride == 0) return hipSuccess;
  const int nb = (int)((max_len + kSortItems - 1) / kSortItems);
  hipLaunchKernelGGL(hist_ranges_kernel, dim3((unsigned)((tiles_stride + 255) / 256), nseg),
                     dim3(256), 0, s, hist, seg_start, seg_len, nb, bits, tiles_stride, ranges);
  return hipGetLastError();
}

size_t scan_tmp_size(int64_t items) {
  // block sums as u64 (+1 for the total), in units of uint32
  int64_t nb = (items + kScanItems - 1) / kScanItems;
  return (size_t)(nb + 1) * 2 + 2;
}

hipError_t scan_counts(const uint32_t* cnt, const uint32_t* sorted_val, int64_t n, int m,
                       uint32_t* off, uint32_t* seg_start, uint32_t* seg_len,
                       unsigned long long* totals, uint32_t* tmp, hipStream_t s) {
  int64_t items = n * (int64_t)m;
  int64_t nb = (items + kScanItems - 1) / kScanItems;
  unsigned long long* bsum = reinterpret_cast<unsigned long long*>(tmp);
  hipError_t e = hipMemsetAsync(totals, 0, 2 * sizeof(unsigned long long), s);
  if (e != hipSuccess) return e;
  if (nb > 0) {
    hipLaunchKernelGGL(count_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, s, cnt, sorted_val, n,
                       items, bsum, totals + 1);
  }
  hipLaunchKernelGGL(bsum_scan_kernel, dim3(1), dim3(1024), 0, s, bsum, nb);
  if (nb > 0) {
    hipLaunchKernelGGL(count_scan_kernel, dim3((unsigned)nb), dim3(256), 0, s, cnt, sorted_val, n,
                       items, bsum, off);
  }
  hipLaunchKernelGGL(seg_kernel, dim3((m + 255) / 256 > 0 ? (m + 255) / 256 : 1), dim3(256), 0, s,
                     off, n, m, bsum + nb, seg_start, seg_len, totals);
  return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* sorted_val, const uint32_t* off,
                            const uint2* sorted_rect, const uint32_t* sorted_cnt,
                            const ViewGeom* geom, int64_t n, int m, uint32_t* pair_key,
                            uint32_t* pair_val, hipStream_t s) {
  if (n == 0 || m == 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_kernel<uint32_t>, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0,
                     s, sorted_val, off, sorted_rect, sorted_cnt, geom, n, pair_key, pair_val);
  return hipGetLastError();
}

hipError_t launch_duplicate16(const uint32_t* sorted_val, const uint32_t* off,
                              const uint2* sorted_rect, const uint32_t* sorted_cnt,
                              const ViewGeom* geom, int64_t n, int m, uint16_t* pair_key,
                              uint32_t* pair_val, hipStream_t s) {
  if (n == 0 || m == 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_kernel<uint16_t>, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0,
                     s, sorted_val, off, sorted_rect, sorted_cnt, geom, n, pair_key, pair_val);
  return hipGetLastError();
}

hipError_t launch_ranges16(const uint16_t* pair_key, const uint32_t* seg_start, const uint32_t* seg_len,
                           int nseg, int64_t max_len, int tiles_stride, uint2* ranges, hipStream_t s) {
  if (nseg == 0 || max_len == 0) return hipSuccess;
  const int64_t octs = (max_len + 15) / 8;  // the segment's start rounded down to a multiple of 8
  const bool aligned = ((uintptr_t)pair_key & 15) == 0;
  hipLaunchKernelGGL(ranges16_kernel, dim3((unsigned)((octs + 255) / 256), (unsigned)nseg), dim3(256), 0, s,
                     pair_key, seg_start, seg_len, tiles_stride, aligned, ranges);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* pair_key, int64_t P, int tiles_stride, uint2* ranges,
                         hipStream_t s) {
  if (P == 0) return hipSuccess;
  const int64_t quads = (P + 3) / 4;
  const bool aligned = ((uintptr_t)pair_key & 15) == 0;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0, s, pair_key, P,
                     tiles_stride, aligned, ranges);
  return hipGetLastError();
}

}  // namespace lv
