// Blend-and-accumulate (Sec. 3.2, Eq. 3 / Eq. 5): for every tile of every
// view, walk the tile's depth-ordered Gaussians front to back, form the
// alpha-blending weight w_i(p) = alpha_i(p) T_i(p) of each Gaussian at each
// pixel (Eq. 1), and add w_i(p) F(p) and w_i(p) into the per-Gaussian
// accumulators U_i and beta_i.  W is never materialised.
//
// One workgroup = one wave64 = one 8x8 quadrant of a 16x16 tile (one pixel
// per lane) for one group of up to 64 channels; with several groups, one
// wave per 16x8 half tile for all of them (blend_pair_kernel, two pixels per
// lane).  Waves never wait for each other.  Per step of 64 Gaussians of the
// tile's list:
//   0. lane j loads Gaussian j's record (vector loads, all in flight
//      together), leaves it in LDS and tests whether its alpha >= 1/255
//      region can touch the quadrant (exact minimum of the conic over the
//      quadrant, conservative slack); a ballot gives the step's hit mask;
//   A. walk: a scalar loop over the hit Gaussians in order; each lane
//      evaluates the Gaussian at its pixel (the record read from LDS at one
//      address, a broadcast), every decision in the S32 sequence;
//   B. a Gaussian with some w > 0 takes the next of 32 LDS rows (its weights
//      at the 64 pixels).  A full set of rows (and the last, partial one) is
//      flushed: U_rows += W_rows F on the matrix cores, one global atomic per
//      (Gaussian, channel); beta (the rows' sums, in exact fixed point, once
//      for all feature sets that take the same views) and the tail channels
//      (the rows' dot products with up to 4 further channels) by one lane
//      pair per row.
#include <algorithm>

#include "lv_internal.h"

namespace lv {

namespace {


template <lv_dtype DT>
__device__ __forceinline__ float load_feature(const void* map, int64_t idx, float scale) {
  if constexpr (DT == LV_F32) {
    return gptr(static_cast<const float*>(map))[idx];
  } else if constexpr (DT == LV_BF16) {
    uint32_t b = gptr(static_cast<const uint16_t*>(map))[idx];
    return __uint_as_float(b << 16);
  } else {
    // without branches: a subnormal (e = 0) is built as 2^-6 (1 + m/8) and
    // 2^-6 taken off again, which is exact; the sign bit goes on last
    const uint32_t b = gptr(static_cast<const uint8_t*>(map))[idx];
    const uint32_t e = (b >> 3) & 0xFu, mt = b & 7u, sub = e == 0u;
    const float mag = __uint_as_float(((e + 120u + sub) << 23) | (mt << 20)) - __uint_as_float(sub * 0x3C800000u);
    return __uint_as_float(__float_as_uint(mag) | ((b & 0x80u) << 24)) * scale;
  }
}

// Map of set sd for view v (NULL: the set does not take the view).
__device__ __forceinline__ const void* map_of(const SetDesc& sd, int v) { return gptr(sd.maps)[v]; }

// Can -power(d) <= tau hold for some d in the rectangle [X0,X1] x [Y0,Y1]
// (offsets from the Gaussian's centre)?  -power = (L11 dx + L12 dy)^2 +
// (L22 dy)^2 is convex with its minimum at 0, so outside the rectangle its
// minimum over the rectangle lies on an edge; along each edge it is a 1D
// quadratic with a clamped vertex.  Evaluated in the factored form, which
// stays accurate for thin Gaussians.
__device__ __forceinline__ float neg_power(float L11, float L12, float L22, float dx, float dy) {
  const float u = __builtin_fmaf(L12, dy, L11 * dx), w = L22 * dy;
  return __builtin_fmaf(u, u, w * w);
}

__device__ __forceinline__ bool region_hits(float4 r0, float4 r1, float X0, float X1, float Y0,
                                            float Y1) {
  const float tau = r1.z;
  if (!(tau >= 0.0f)) return false;
  if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return true;
  const float L11 = r0.z, L12 = r0.w, L22 = r1.x;
  const float ky = -(L11 * L12) / __builtin_fmaf(L12, L12, L22 * L22);  // edge dx = X: dy* = ky X
  const float kx = -L12 / L11;                                          // edge dy = Y: dx* = kx Y
  const float dy0 = fminf(fmaxf(ky * X0, Y0), Y1);
  const float dy1 = fminf(fmaxf(ky * X1, Y0), Y1);
  const float dx0 = fminf(fmaxf(kx * Y0, X0), X1);
  const float dx1 = fminf(fmaxf(kx * Y1, X0), X1);
  const float m0 = fminf(neg_power(L11, L12, L22, X0, dy0), neg_power(L11, L12, L22, X1, dy1));
  const float m1 = fminf(neg_power(L11, L12, L22, dx0, Y0), neg_power(L11, L12, L22, dx1, Y1));
  return fminf(m0, m1) <= tau;
}

// The quadrant a workgroup handles.  Workgroups go to the 8 XCDs
// round-robin, so the four quadrant waves of a tile get ids that are equal
// mod 8 and consecutive within the XCD: they share that XCD's L2 for the
// tile's records.
struct Quad {
  int v, tile, cg, qx, qy;
  uint2 rg;
  ViewGeom g;
};

// empty_ok: a tile without Gaussians is kept (the render writes its zeros).
__device__ __forceinline__ bool decode_quad(const uint2* __restrict__ ranges,
                                            const ViewGeom* __restrict__ geom, int tiles_stride,
                                            int nviews, int ngroups, Quad& q,
                                            bool empty_ok = false) {
  const uint32_t L = blockIdx.x;
  const uint32_t kx = L >> 3;
  const uint32_t work = ((kx >> 2) << 3) | (L & 7u);
  if (work >= (uint32_t)tiles_stride * (uint32_t)nviews * (uint32_t)ngroups) return false;
  const int quad = (int)(kx & 3u);
  q.tile = (int)(work % (uint32_t)tiles_stride);
  q.v = (int)((work / (uint32_t)tiles_stride) % (uint32_t)nviews);
  q.cg = (int)(work / ((uint32_t)tiles_stride * (uint32_t)nviews));
  q.g = geom[q.v];
  if (q.tile >= q.g.TX * q.g.TY) return false;
  q.rg = ranges[(int64_t)q.v * tiles_stride + q.tile];
  if (q.rg.y <= q.rg.x && !empty_ok) return false;
  const int tx = q.tile % q.g.TX, ty = q.tile / q.g.TX;
  q.qx = tx * kTile + (quad & 1) * 8;
  q.qy = ty * kTile + (quad >> 1) * 8;
  return q.qx < q.g.W && q.qy < q.g.H;  // else the quadrant lies outside the image
}

// Per-lane walk state.
// Coordinates are relative to the tile: pixel offsets px - ox in [0, 16) and
// centres as (ux - (ox + 0.5)) + ux_lo (see Rec).
struct Walk {
  float pxo, pyo;  // this lane's pixel, relative to the tile
  float ocx, ocy;  // first pixel centre of the tile, ox + 0.5, oy + 0.5
  float qx0, qy0;  // the quadrant's first pixel, relative to the tile
  float T;
  bool alive;
};

__device__ __forceinline__ void walk_init(const Quad& q, int lane, Walk& s) {
  const int px = q.qx + (lane & 7), py = q.qy + (lane >> 3);
  const int ox = q.qx & ~(kTile - 1), oy = q.qy & ~(kTile - 1);
  s.pxo = (float)(px - ox);
  s.pyo = (float)(py - oy);
  s.ocx = (float)ox + 0.5f;
  s.ocy = (float)oy + 0.5f;
  s.qx0 = (float)(q.qx - ox);
  s.qy0 = (float)(q.qy - oy);
  s.T = 1.0f;
  s.alive = px < q.g.W && py < q.g.H;
}

// Step 0: records of Gaussians [base, base + cnt) one per lane, centres made
// tile-relative and left in rs[lane] = {(cx, cy, L11, L12), (L22, opacity,
// tau, -)} for the walk; the hit mask (the alpha >= 1/255 region can touch
// the quadrant).
// perm (nullable): storage -> caller order; my_id is then the caller's index
// (loaded beside the records).
__device__ __forceinline__ uint64_t step_records(const Rec* __restrict__ vrec,
                                                 const uint32_t* __restrict__ ids, uint32_t base,
                                                 int cnt, int lane, const Walk& s, uint32_t& my_id,
                                                 float4 (*rs)[2],
                                                 const uint32_t* __restrict__ perm = nullptr) {
  float4 q0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float4 q1 = make_float4(0.0f, 0.0f, -1.0f, 0.0f);
  my_id = 0;
  if (lane < cnt) {
    const uint32_t id = ids[base + lane];
    my_id = perm ? perm[id] : id;
    q0 = vrec[id].r0;
    q1 = vrec[id].r1;
    // centre relative to the tile (see Rec)
    const uint32_t lo = __float_as_uint(q1.w);
    q0.x = (q0.x - s.ocx) + __uint_as_float(lo << 16);
    q0.y = (q0.y - s.ocy) + __uint_as_float(lo & 0xFFFF0000u);
  }
  rs[lane][0] = q0;
  rs[lane][1] = q1;
  const float X0 = s.qx0 - q0.x, Y0 = s.qy0 - q0.y;
  const bool hit = lane < cnt && region_hits(q0, q1, X0, X0 + 7.0f, Y0, Y0 + 7.0f);
  return __ballot(hit);
}

// One step of the walk: the Gaussian of record (a, b) = ((cx, cy, L11, L12),
// (L22, opacity, -, -)) at this lane's pixel.  take: it contributes here
// (then w = alpha T > 0).
__device__ __forceinline__ float walk_rec(const float4& a, const float4& b, Walk& s, bool& take) {
  const float dx = s.pxo - a.x, dy = s.pyo - a.y;
  const float u = __builtin_fmaf(a.w, dy, a.z * dx), w = b.x * dy;
  const float al = fminf(kAlphaMax, b.y * exp_neg(-__builtin_fmaf(u, u, w * w)));
  const bool ok = s.alive && al >= kAlphaMin;
  const float Tn = s.T * (1.0f - al);
  const bool stop = ok && Tn < kTEps;
  take = ok && !stop;
  const float wj = take ? al * s.T : 0.0f;
  s.T = take ? Tn : s.T;
  s.alive = s.alive && !stop;
  return wj;
}

// ---------------------------------------------------------------- wide kernel
// Any number of feature sets; the workgroup's channel group has up to 64
// channels made of segments of the sets plus up to 4 tail channels (summed
// per LDS row at each flush).
//
// Accumulation on the matrix cores.  The weights of 32 queued Gaussians at
// the quadrant's 64 pixels form W_s (32 x 64), and their contribution to the
// group's channels is the dense product U_s = W_s F (F: 64 pixels x 64
// channels).  It runs as 32x32x16 BF16 MFMAs
// with FP32 accumulation on split operands: x = hi + lo, hi = bf16(x) and
// lo = bf16(x - hi) (both round-to-nearest-even), so |x - hi - lo| <=
// 2^-18 |x|; U_s = W_hi F_hi + W_lo F_hi + W_hi F_lo (the dropped W_lo F_lo
// and residuals are below 2^-16 |W| |F|;
// BF16 maps are exact, F_lo = 0).  A K-step of 16 pixels is two pixel rows of
// the quadrant: steps whose rows hold no contribution are skipped.  Operand
// layouts (32x32x16): lane l holds A[l % 32][8 (l / 32) + i] and
// B[8 (l / 32) + i][l % 32], i = 0..7, and D[8 (r / 4) + 4 (l / 32) + r % 4]
// [l % 32] in accumulator r.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kWtPitch = 68;  // LDS row pitch (floats) of the transposed weights

// x = hi + lo + O(2^-18 |x|), conversions round to nearest even
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    hi[i] = (__bf16)x[i];
    lo[i] = (__bf16)(x[i] - (float)hi[i]);
  }
}

// A operand of one K-step: this lane's 8 weights (two float4 from LDS), split
__device__ __forceinline__ void load_split_w(const float* w, bf16x8& hi, bf16x8& lo) {
  const float4 wa = *reinterpret_cast<const float4*>(w);
  const float4 wb = *reinterpret_cast<const float4*>(w + 4);
  const float w8[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
  split8(w8, hi, lo);
}

// The same chunk after split_w_in_place: BF16 hi in its first 16 bytes, lo
// in the next 16.
__device__ __forceinline__ void load_w(const float* w, bf16x8& hi, bf16x8& lo) {
  hi = *reinterpret_cast<const bf16x8*>(w);
  lo = *reinterpret_cast<const bf16x8*>(w + 4);
}

__device__ __forceinline__ void split_w_in_place(float* w) {
  bf16x8 hi, lo;
  load_split_w(w, hi, lo);
  *reinterpret_cast<bf16x8*>(w) = hi;
  *reinterpret_cast<bf16x8*>(w + 4) = lo;
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Rows (8 pixels each) of a 64-pixel mask that hold a set bit.
__device__ __forceinline__ uint32_t row_bits(uint64_t m) {
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) r |= (((m >> (8 * k)) & 0xFFull) != 0ull ? 1u : 0u) << k;
  return r;
}

// This lane's channel in each 32-channel block of a group (n = l % 32):
// where its features come from and where its sums go.
struct GroupLanes {
  float* outp[2];
  int outD[2];
  const void* src[2];  // a readable map even where the lane owns no channel
  bool own[2];         // the lane owns a channel of block b
  int64_t srcc[2];
  int srcld[2];
  float srcsc[2];
};

// Fills L for group grp and view q.v; false if no segment of the group takes
// the view (wave-uniform).
template <lv_dtype DT>
__device__ __forceinline__ bool group_lanes(const ChanGroup& grp, const SetDesc* __restrict__ sets,
                                            const Quad& q, int lane, GroupLanes& L) {
  bool active = false;
#pragma unroll
  for (int b = 0; b < 2; b++) {
    L.outp[b] = nullptr;
    L.outD[b] = 0;
    L.src[b] = nullptr;
    L.own[b] = false;
    L.srcc[b] = 0;
    L.srcld[b] = 0;
    L.srcsc[b] = 1.0f;
  }
  for (int k = 0; k < grp.nseg; k++) {
    const SetDesc& sd = sets[grp.set[k]];
    const void* map = map_of(sd, q.v);
    if (!map) continue;  // this set does not take the view
    active = true;
    const int vc0 = grp.vc0[k], cnt = grp.cnt[k];
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int ch = b * 32 + (lane & 31);
      if (!L.src[b]) L.src[b] = map;  // readable, for lanes without a channel
      if (ch >= vc0 && ch < vc0 + cnt) {
        const int c = grp.c0[k] + (ch - vc0);
        L.outp[b] = u_elem(sd.U, c, sd.fixed != 0);
        L.outD[b] = sd.D;
        L.src[b] = map;
        L.own[b] = true;
        L.srcc[b] = c;
        L.srcld[b] = sd.stride;
        if constexpr (DT == LV_FP8_E4M3) L.srcsc[b] = gptr(sd.scales)[(int64_t)(sd.view_base + q.v) * sd.D + c];
      }
    }
  }
  return active;
}

// Element (y, x, channel c) of a map with pixel stride ld: HWC at
// (y W + x) ld + c; pixel-block layout (PX8) at ((y W8 + x / 8) ld + c) 8 +
// x % 8 with W8 = ceil(W / 8) (pixels past W are zeros).
template <bool PX>
__device__ __forceinline__ int64_t map_index(int y, int x, int W, int ld, int64_t c) {
  if constexpr (PX)
    return (((int64_t)y * ((W + 7) >> 3) + (x >> 3)) * ld + c) * 8 + (x & 7);
  else
    return ((int64_t)y * W + x) * ld + c;
}

// Four OCP E4M3FN codes (the bytes of w) -> their values as BF16 bits, two
// per word: the hardware FP8 -> FP32 conversion (two codes per
// instruction), then FP32 -> BF16 (exact: 3 mantissa bits).
__device__ __forceinline__ void e4m3x4_bf16(uint32_t w, uint32_t& h01, uint32_t& h23) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  const f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  h01 = __builtin_bit_cast(uint32_t, (bf16x2{(__bf16)a.x, (__bf16)a.y}));
  h23 = __builtin_bit_cast(uint32_t, (bf16x2{(__bf16)b.x, (__bf16)b.y}));
}

__device__ __forceinline__ bf16x8 bf16x8_of(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3) {
  return __builtin_bit_cast(bf16x8, (u32x4{w0, w1, w2, w3}));
}

// The B operand of one K-step for block b: this lane's channel at the 8
// pixels (gx0 .. gx0 + 7, gx0 a multiple of 8) of pixel row gy, as BF16
// (hi; lo = the FP32 remainder, FP32 maps only).  BF16 maps are exact in hi;
// FP8 codes too (their per-channel scale multiplies the products, see
// batch_scatter).  Every lane loads, from a safe index (block or pixel 0 of
// the map) where it has nothing to load.  Pixel blocks: the data is used as
// loaded -- a lane without a channel feeds only its own output column, which
// is never scattered, and a pixel outside the image has weight 0 in every
// queued row.  (A select of zeros there becomes a zero fill of the
// destination registers plus a masked load, and the fill waits for every
// memory operation in flight: a group's K-steps would load one round trip at
// a time.)  HWC: eight gathers per row, selected (zeros outside the image
// and for lanes without a channel), which keeps them from all being in
// flight at once.
template <lv_dtype DT, bool PX>
__device__ __forceinline__ void load_row8(const GroupLanes& L, int b, int gy, int gx0,
                                          const ViewGeom& g, bf16x8& fh, bf16x8& fl) {
  const bool okr = L.own[b] && gy < g.H;
  if constexpr (PX) {
    // one block of 8 pixels of one channel: 32, 16 or 8 contiguous bytes
    const int64_t blk = okr ? ((int64_t)gy * ((g.W + 7) >> 3) + (gx0 >> 3)) * L.srcld[b] + L.srcc[b] : 0;
    if constexpr (DT == LV_BF16) {
      const u32x4 q = gptr(static_cast<const u32x4*>(L.src[b]))[blk];
      fh = bf16x8_of(q.x, q.y, q.z, q.w);
    } else if constexpr (DT == LV_FP8_E4M3) {
      const u32x2 q = gptr(static_cast<const u32x2*>(L.src[b]))[blk];
      uint32_t h[4];
      e4m3x4_bf16(q.x, h[0], h[1]);
      e4m3x4_bf16(q.y, h[2], h[3]);
      fh = bf16x8_of(h[0], h[1], h[2], h[3]);
    } else {
      const f32x4 qa = gptr(static_cast<const f32x4*>(L.src[b]))[2 * blk];
      const f32x4 qb = gptr(static_cast<const f32x4*>(L.src[b]))[2 * blk + 1];
      const float v[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
      split8(v, fh, fl);
    }
  } else {
    if constexpr (DT == LV_F32) {
      float v[8];
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const bool ok = okr && gx0 + i < g.W;
        const int64_t idx = ok ? ((int64_t)gy * g.W + gx0 + i) * L.srcld[b] + L.srcc[b] : 0;
        const float x = gptr(static_cast<const float*>(L.src[b]))[idx];
        v[i] = ok ? x : 0.0f;
      }
      split8(v, fh, fl);
    } else {
      uint32_t h[8];
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const bool ok = okr && gx0 + i < g.W;
        const int64_t idx = ok ? ((int64_t)gy * g.W + gx0 + i) * L.srcld[b] + L.srcc[b] : 0;
        uint32_t x;
        if constexpr (DT == LV_BF16)
          x = gptr(static_cast<const uint16_t*>(L.src[b]))[idx];
        else
          x = gptr(static_cast<const uint8_t*>(L.src[b]))[idx];
        h[i] = ok ? x : 0u;
      }
      if constexpr (DT == LV_BF16) {
        fh = bf16x8_of(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
      } else {
        uint32_t o[4];
        e4m3x4_bf16(h[0] | (h[1] << 8) | (h[2] << 16) | (h[3] << 24), o[0], o[1]);
        e4m3x4_bf16(h[4] | (h[5] << 8) | (h[6] << 16) | (h[7] << 24), o[2], o[3]);
        fh = bf16x8_of(o[0], o[1], o[2], o[3]);
      }
    }
  }
}

// U_b = W_b F for a batch of queued rows, one or two blocks of 32 channels.
// No branch separates dependent MFMAs (the widths run in separate loops).
template <bool kSplitF>
__device__ __forceinline__ void batch_mfma(bool two, uint32_t rows, const float* wrow,
                                           const bf16x8 (&fh)[2][4], const bf16x8 (&fl)[2][4],
                                           f32x16& acc0, f32x16& acc1) {
  if (two) {
#pragma unroll
    for (int t = 0; t < 4; t++) {
      if ((rows >> (2 * t)) & 3u) {
        bf16x8 ah, al;
        load_split_w(wrow + 16 * t, ah, al);
        acc0 = mfma(ah, fh[0][t], acc0);
        acc1 = mfma(ah, fh[1][t], acc1);
        acc0 = mfma(al, fh[0][t], acc0);
        acc1 = mfma(al, fh[1][t], acc1);
        if constexpr (kSplitF) {
          acc0 = mfma(ah, fl[0][t], acc0);
          acc1 = mfma(ah, fl[1][t], acc1);
        }
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; t++) {
      if ((rows >> (2 * t)) & 3u) {
        bf16x8 ah, al;
        load_split_w(wrow + 16 * t, ah, al);
        acc0 = mfma(ah, fh[0][t], acc0);
        acc0 = mfma(al, fh[0][t], acc0);
        if constexpr (kSplitF) acc0 = mfma(ah, fl[0][t], acc0);
      }
    }
  }
}

// One atomic per (queued Gaussian, channel): D row m of the batch is ring
// row m, whose Gaussian id lane m holds.  FP8 maps: the products were formed
// on the codes, the channel's scale multiplies them here.
template <lv_dtype DT, bool FIX>
__device__ __forceinline__ void batch_scatter_t(const GroupLanes& L, bool two, int count,
                                                uint32_t ring_gid, int lane, f32x16 acc0,
                                                f32x16 acc1) {
  if constexpr (DT == LV_FP8_E4M3) {
    acc0 *= L.srcsc[0];
    acc1 *= L.srcsc[1];
  }
  const bool upper = lane >= 32;
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const int m0 = 8 * (r >> 2) + (r & 3), m1 = m0 + 4;
    if (m0 < count) {
      const uint32_t g0 = (uint32_t)__builtin_amdgcn_readlane((int)ring_gid, m0);
      const uint32_t g1 = (uint32_t)__builtin_amdgcn_readlane((int)ring_gid, m1);
      const int64_t gid = (int64_t)(upper ? g1 : g0);
      if ((upper ? m1 : m0) < count) {
        if (L.outp[0] && acc0[r] != 0.0f) u_atomic_add(L.outp[0], gid * L.outD[0], acc0[r], FIX);
        if (two && L.outp[1] && acc1[r] != 0.0f) u_atomic_add(L.outp[1], gid * L.outD[1], acc1[r], FIX);
      }
    }
  }
}

// fixed (a deterministic accumulator) is wave-uniform: one branch per
// flush, each side a straight run of atomics
template <lv_dtype DT>
__device__ __forceinline__ void batch_scatter(const GroupLanes& L, bool two, int count,
                                              uint32_t ring_gid, int lane, f32x16 acc0,
                                              f32x16 acc1, bool fixed) {
  if (fixed)
    batch_scatter_t<DT, true>(L, two, count, ring_gid, lane, acc0, acc1);
  else
    batch_scatter_t<DT, false>(L, two, count, ring_gid, lane, acc0, acc1);
}

// One channel group (at most 64 + 4 channels): one wave per (view,
// quadrant); the group's F fragments are staged once in registers.  Several
// groups run on blend_pair_kernel below.  Occupancy: waves per SIMD the
// register allocation must allow (the walk is latency-bound; more resident
// waves hide it).  BF16 maps need no low operand halves, so they fit four.
template <lv_dtype DT>
constexpr int wide_waves() {
  return DT == LV_BF16 ? 4 : 3;
}

template <lv_dtype DT, bool PX>
__global__ __launch_bounds__(64, (wide_waves<DT>())) void blend_wide_kernel(
    const Rec* __restrict__ rec, const uint32_t* __restrict__ ids, const uint2* __restrict__ ranges,
    const ViewGeom* __restrict__ geom, int64_t n, int tiles_stride, int nviews,
    const SetDesc* __restrict__ sets, const ChanGroup* __restrict__ groups, int ngroups) {
  constexpr int G = kChunk;
  constexpr bool kSplitF = DT == LV_F32;  // BF16 maps and FP8 codes are exact in one BF16 operand
  __shared__ __align__(16) float Wt[32 * kWtPitch];  // queued Gaussians: [row][pixel]
  __shared__ float4 Rs[kChunk][2];                   // the step's records
  Quad q;
  if (!decode_quad(ranges, geom, tiles_stride, nviews, ngroups, q)) return;
  const int lane = threadIdx.x;
  const bool fixedU = sets[0].fixed != 0;  // one accumulation mode per launch (wave-uniform)
  const int px = q.qx + (lane & 7), py = q.qy + (lane >> 3);
  const bool inside = px < q.g.W && py < q.g.H;

  // whether the group takes the view, sets whose beta (and counts) are added
  // here; its tail channels
  bool has_main = false;
  int bsets = 0, ssets = 0;
  {
    const ChanGroup& grp = groups[q.cg];
    for (int b = grp.beta_sets; b; b &= b - 1)
      if (map_of(sets[__builtin_ctz(b)], q.v)) bsets |= b & -b;
    for (int b = grp.stats_sets; b; b &= b - 1)
      if (map_of(sets[__builtin_ctz(b)], q.v)) ssets |= b & -b;
    for (int k = 0; k < grp.nseg; k++) has_main = has_main || map_of(sets[grp.set[k]], q.v) != nullptr;
  }
  const ChanGroup& last = groups[q.cg];
  const int ntail = last.ntail;
  // tail channels: their features per pixel in LDS (Ft[t][pixel]), summed
  // against the ring rows at each flush
  __shared__ __align__(16) float Ft[kMaxTail * 64];
  float* tout[kMaxTail];
  int tD[kMaxTail];
  bool any_tail = false;
#pragma unroll
  for (int t = 0; t < kMaxTail; t++) {
    float ft = 0.0f;
    tout[t] = nullptr;
    tD[t] = 0;
    if (t < ntail && map_of(sets[last.tset[t]], q.v)) {
      const SetDesc& sd = sets[last.tset[t]];
      const int c = last.tc[t];
      float sc = 1.0f;
      if constexpr (DT == LV_FP8_E4M3) sc = gptr(sd.scales)[(int64_t)(sd.view_base + q.v) * sd.D + c];
      const int64_t idx = inside ? map_index<PX>(py, px, q.g.W, sd.stride, c) : 0;
      const float x = load_feature<DT>(map_of(sd, q.v), idx, sc);  // no branch around the load
      ft = inside ? x : 0.0f;
      tout[t] = u_elem(sd.U, c, fixedU);
      tD[t] = sd.D;
      any_tail = true;
    }
    Ft[t * 64 + lane] = ft;
  }
  if (!has_main && !any_tail && !bsets && !ssets) return;  // wave-uniform: nothing here takes the view

  // the group's lanes and fragments once, in registers
  GroupLanes L1;
  bf16x8 fh[2][4], fl[2][4];
  bool two1 = false;
  {
    const ChanGroup& grp = groups[q.cg];
    const bool takes = group_lanes<DT>(grp, sets, q, lane, L1);
    two1 = grp.width > 32;
    if (takes) {
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int t = 0; t < 4; t++)
          load_row8<DT, PX>(L1, b, q.qy + 2 * t + (lane >> 5), q.qx, q.g, fh[b][t], fl[b][t]);
    }
    has_main = has_main && takes && __ballot(L1.outp[0] != nullptr || L1.outp[1] != nullptr) != 0ull;
  }

  // Gaussians with a contribution queue up in 32 LDS rows (row r: the
  // Gaussian's weights at the 64 pixels in Wt, its id and its number of
  // contributing pixels in Rg[r] / Rc[r], read into lane r's ring_gid /
  // ring_cnt when the rows are flushed).  When the rows are
  // full, and at the end, one flush: a batch of MFMAs (M = 32 rows) and one
  // round of atomics per group, so the matrix products run on full rows
  // whatever the number of contributing Gaussians per step of the walk; and
  // the rows' sums (beta) and dot products with the tail channels, one row
  // per lane pair, each lane summing half of the row in a fixed order.
  int queued = 0;        // rows [0, queued) hold Gaussians
  uint64_t pix = 0ull;   // pixels used by the queued rows
  __shared__ uint32_t Rg[32], Rc[32];
  uint32_t ring_gid = 0u, ring_cnt = 0u;

  auto flush = [&](int count) {
    __syncthreads();  // ring rows written (one wave per workgroup: orders LDS)
    ring_gid = Rg[lane & 31];
    ring_cnt = Rc[lane & 31];
    const uint32_t rows = row_bits(pix);
    const float* wrow = Wt + (lane & 31) * kWtPitch + 8 * (lane >> 5);
    if (has_main) {
      f32x16 acc0 = {}, acc1 = {};
      batch_mfma<kSplitF>(two1, rows, wrow, fh, fl, acc0, acc1);
      batch_scatter<DT>(L1, two1, count, ring_gid, lane, acc0, acc1, fixedU);
    }
    if (bsets || any_tail) {
      // lane l: row l % 32, pixels [32 (l / 32), 32 (l / 32) + 32)
      const float* rp = Wt + (lane & 31) * kWtPitch + 32 * (lane >> 5);
      const float* fp = Ft + 32 * (lane >> 5);
      float bs = 0.0f, ts[kMaxTail] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const float4 a = *reinterpret_cast<const float4*>(rp + 4 * k);
        bs += a.x;
        bs += a.y;
        bs += a.z;
        bs += a.w;
#pragma unroll
        for (int t = 0; t < kMaxTail; t++) {
          if (t < ntail) {  // wave-uniform
            const float4 f = *reinterpret_cast<const float4*>(fp + t * 64 + 4 * k);
            ts[t] = __builtin_fmaf(a.x, f.x, ts[t]);
            ts[t] = __builtin_fmaf(a.y, f.y, ts[t]);
            ts[t] = __builtin_fmaf(a.z, f.z, ts[t]);
            ts[t] = __builtin_fmaf(a.w, f.w, ts[t]);
          }
        }
      }
      bs += __shfl_xor(bs, 32, 64);
#pragma unroll
      for (int t = 0; t < kMaxTail; t++) ts[t] += __shfl_xor(ts[t], 32, 64);
      if (lane < count) {  // lane r < 32: row r, whose id and count it holds
        for (int b = bsets; b; b &= b - 1) {
          const SetDesc& sd = sets[__builtin_ctz(b)];
          beta_atomic_add(sd.beta + ring_gid, bs);
          if (sd.counts) gatomic_add(sd.counts + ring_gid, ring_cnt);
        }
#pragma unroll
        for (int t = 0; t < kMaxTail; t++)
          if (tout[t] && ts[t] != 0.0f) u_atomic_add(tout[t], (int64_t)ring_gid * tD[t], ts[t], fixedU);
      }
    }
    __syncthreads();  // rows read before they are written again
  };

  Walk s;
  walk_init(q, lane, s);
  uint64_t covered = 0ull;  // pixels with a contribution (statistics)
  uint32_t ncontrib = 0u;   // contributions of the quadrant (statistics)
  uint32_t nrows = 0u;      // Gaussians queued (statistics)
  const Rec* vrec = rec + (int64_t)q.v * n;
  for (uint32_t base = q.rg.x; base < q.rg.y; base += G) {
    if (__ballot(s.alive) == 0ull) break;
    const int cnt = (int)(q.rg.y - base < (uint32_t)G ? q.rg.y - base : (uint32_t)G);
    uint32_t my_id;
    const uint64_t hits = step_records(vrec, ids, base, cnt, lane, s, my_id, Rs);
    if (!hits) continue;
    __syncthreads();  // records in LDS (one wave per workgroup: orders LDS)

    // the hit Gaussians in order (a scalar loop over the set bits; each
    // record read from LDS, a broadcast, one hit ahead); each with a
    // contribution takes the next ring row, a full ring is flushed
    uint64_t h = hits;
    int j = h ? (int)__builtin_ctzll(h) : 0;
    float4 ra = Rs[j][0], rb = Rs[j][1];
    while (h) {
      h &= h - 1;
      const int jn = h ? (int)__builtin_ctzll(h) : j;
      // wj: this lane's weight (0 where it takes no part), msk: the lanes
      // with a contribution
      const float dx = s.pxo - ra.x, dy = s.pyo - ra.y;
      const float u = __builtin_fmaf(ra.w, dy, ra.z * dx), w = rb.x * dy;
      const float al = fminf(kAlphaMax, rb.y * exp_neg(-__builtin_fmaf(u, u, w * w)));
      // the next record into the same registers (no copies between hits)
      ra = Rs[jn][0];
      rb = Rs[jn][1];
      const float Tn = s.T * (1.0f - al);
      const bool ok = s.alive && al >= kAlphaMin;
      const bool stop = ok && Tn < kTEps;
      const bool take = ok && !stop;
      const uint64_t msk = __builtin_amdgcn_ballot_w64(take);
      const float wj = take ? al * s.T : 0.0f;
      s.T = take ? Tn : s.T;
      s.alive = s.alive && !stop;
      if (msk) {
        covered |= msk;
        ncontrib += (uint32_t)__popcll(msk);
        nrows++;
        Wt[queued * kWtPitch + lane] = wj;
        if (lane == j) {  // lane j holds the Gaussian's id
          Rg[queued] = my_id;
          Rc[queued] = (uint32_t)__popcll(msk);
        }
        pix |= msk;
        if (++queued == 32) {
          flush(32);
          queued = 0;
          pix = 0ull;
        }
      }
      j = jn;
    }
  }
  if (queued > 0) flush(queued);
  // statistics go to every set whose statistics this work item takes
  for (int b = ssets; b; b &= b - 1) {
    const SetDesc& sd = sets[__builtin_ctz(b)];
    if (sd.stats && lane == 0) {
      gatomic_add(&sd.stats[1], (unsigned long long)ncontrib);
      gatomic_add(&sd.stats[0], (unsigned long long)__popcll(covered));
      gatomic_add(&sd.stats[2], (unsigned long long)nrows);
    }
  }
}

// ------------------------------------------------------------- pair kernel
// Several channel groups (wide D): one wave per (view, tile, half tile), the
// two 8x8 quadrants of a 16x8 half tile, two pixels per lane (lane l covers
// pixel (l % 8, l / 8) of each quadrant).  A Gaussian that reaches both
// quadrants queues one row of 128 weights instead of two rows of 64, so a
// (Gaussian, view) adds about 0.7 times as many partial sums to U as with one
// wave per quadrant -- each partial sum is D atomic adds, the binding cost at
// large D.  The walk evaluates a Gaussian only at the quadrants its
// alpha >= 1/255 region reaches.  Pixel p of a queued row: quadrant p / 64,
// pixel p % 64 of it (row-major 8x8); K-step t of the products (16 pixels)
// is pixel rows 2 (t % 4), 2 (t % 4) + 1 of quadrant t / 4.
constexpr int kPairPitch = 132;  // LDS row pitch (floats) of the 128 queued weights

struct Pair {
  int v, tile, qx, qy;  // qx, qy: the half tile's first pixel
  uint2 rg;
  ViewGeom g;
};

// The two halves of a tile get consecutive ids on the same XCD (ids equal
// mod 8), so they share that XCD's L2 for the tile's records.
__device__ __forceinline__ bool decode_pair(const uint2* __restrict__ ranges,
                                            const ViewGeom* __restrict__ geom, int tiles_stride,
                                            int nviews, Pair& q) {
  const uint32_t L = blockIdx.x;
  const uint32_t kx = L >> 3;
  const uint32_t work = ((kx >> 1) << 3) | (L & 7u);
  if (work >= (uint32_t)tiles_stride * (uint32_t)nviews) return false;
  const int half = (int)(kx & 1u);
  q.tile = (int)(work % (uint32_t)tiles_stride);
  q.v = (int)(work / (uint32_t)tiles_stride);
  q.g = geom[q.v];
  if (q.tile >= q.g.TX * q.g.TY) return false;
  q.rg = ranges[(int64_t)q.v * tiles_stride + q.tile];
  if (q.rg.y <= q.rg.x) return false;
  const int tx = q.tile % q.g.TX, ty = q.tile / q.g.TX;
  q.qx = tx * kTile;
  q.qy = ty * kTile + half * 8;
  return q.qx < q.g.W && q.qy < q.g.H;
}

// Alpha-blending step at one pixel (offsets relative to the tile), as
// walk_rec: take = the Gaussian contributes here, w = alpha T.
__device__ __forceinline__ float blend_at(const float4& a, const float4& b, float pxo, float pyo,
                                          float& T, bool& alive, bool& take) {
  const float dx = pxo - a.x, dy = pyo - a.y;
  const float u = __builtin_fmaf(a.w, dy, a.z * dx), w = b.x * dy;
  const float al = fminf(kAlphaMax, b.y * exp_neg(-__builtin_fmaf(u, u, w * w)));
  const bool ok = alive && al >= kAlphaMin;
  const float Tn = T * (1.0f - al);
  const bool stop = ok && Tn < kTEps;
  take = ok && !stop;
  const float wj = take ? al * T : 0.0f;
  T = take ? Tn : T;
  alive = alive && !stop;
  return wj;
}

// group_lanes for a half tile (only the view matters)
template <lv_dtype DT>
__device__ __forceinline__ bool group_lanes_pair(const ChanGroup& grp, const SetDesc* __restrict__ sets,
                                                 const Pair& p, int lane, GroupLanes& L) {
  Quad q;
  q.v = p.v;
  return group_lanes<DT>(grp, sets, q, lane, L);
}

template <lv_dtype DT, bool PX>
__global__ __launch_bounds__(64, 2) void blend_pair_kernel(
    const Rec* __restrict__ rec, const uint32_t* __restrict__ ids, const uint2* __restrict__ ranges,
    const ViewGeom* __restrict__ geom, int64_t n, int tiles_stride, int nviews,
    const SetDesc* __restrict__ sets, const ChanGroup* __restrict__ groups, int ngroups) {
  constexpr int G = kChunk;
  constexpr bool kSplitF = DT == LV_F32;
  __shared__ __align__(16) float Wt[32 * kPairPitch];  // queued Gaussians: [row][128 pixels]
  __shared__ float4 Rs[kChunk][2];                     // the step's records
  // tail channels per pixel [kMaxTail][128]: dynamic, allocated only when the
  // last group has a tail (without it the workgroup's 19.2 KB of LDS lets 8
  // workgroups share a CU instead of 7)
  extern __shared__ __align__(16) float Ft[];
  __shared__ uint32_t Rg[32], Rc[32];
  Pair q;
  if (!decode_pair(ranges, geom, tiles_stride, nviews, q)) return;
  const int lane = threadIdx.x;
  const bool fixedU = sets[0].fixed != 0;  // one accumulation mode per launch (wave-uniform)
  const int ox = q.qx, oy = q.qy & ~(kTile - 1);
  const float ocx = (float)ox + 0.5f, ocy = (float)oy + 0.5f;
  const float pyo = (float)(q.qy - oy + (lane >> 3));
  const float pxo0 = (float)(lane & 7), pxo1 = pxo0 + 8.0f;
  const float qy0 = (float)(q.qy - oy);
  const int py = q.qy + (lane >> 3);
  const bool in0 = q.qx + (lane & 7) < q.g.W && py < q.g.H;
  const bool in1 = q.qx + 8 + (lane & 7) < q.g.W && py < q.g.H;

  bool has_main = false;
  int bsets = 0, ssets = 0;
  uint32_t gmask = 0u;
  for (int cg = 0; cg < ngroups; cg++) {
    const ChanGroup& grp = groups[cg];
    for (int b = grp.beta_sets; b; b &= b - 1)
      if (map_of(sets[__builtin_ctz(b)], q.v)) bsets |= b & -b;
    for (int b = grp.stats_sets; b; b &= b - 1)
      if (map_of(sets[__builtin_ctz(b)], q.v)) ssets |= b & -b;
    bool any = false;
    for (int k = 0; k < grp.nseg; k++) any = any || map_of(sets[grp.set[k]], q.v) != nullptr;
    if (any) {
      gmask |= 1u << cg;
      has_main = true;
    }
  }
  const ChanGroup& last = groups[ngroups - 1];
  const int ntail = last.ntail;
  float* tout[kMaxTail];
  int tD[kMaxTail];
  bool any_tail = false;
#pragma unroll
  for (int t = 0; t < kMaxTail; t++) {
    float ft0 = 0.0f, ft1 = 0.0f;
    tout[t] = nullptr;
    tD[t] = 0;
    if (t < ntail && map_of(sets[last.tset[t]], q.v)) {
      const SetDesc& sd = sets[last.tset[t]];
      const int c = last.tc[t];
      float sc = 1.0f;
      if constexpr (DT == LV_FP8_E4M3) sc = gptr(sd.scales)[(int64_t)(sd.view_base + q.v) * sd.D + c];
      const int64_t i0 = in0 ? map_index<PX>(py, q.qx + (lane & 7), q.g.W, sd.stride, c) : 0;
      const int64_t i1 = in1 ? map_index<PX>(py, q.qx + 8 + (lane & 7), q.g.W, sd.stride, c) : 0;
      const float x0 = load_feature<DT>(map_of(sd, q.v), i0, sc);  // no branch around the loads
      const float x1 = load_feature<DT>(map_of(sd, q.v), i1, sc);
      ft0 = in0 ? x0 : 0.0f;
      ft1 = in1 ? x1 : 0.0f;
      tout[t] = u_elem(sd.U, c, fixedU);
      tD[t] = sd.D;
      any_tail = true;
    }
    if (t < ntail) {  // wave-uniform
      Ft[t * 128 + lane] = ft0;
      Ft[t * 128 + 64 + lane] = ft1;
    }
  }
  if (!has_main && !any_tail && !bsets && !ssets) return;  // wave-uniform

  int queued = 0;
  uint64_t pix0 = 0ull, pix1 = 0ull;  // pixels of each quadrant used by the queued rows
  uint32_t ring_gid = 0u, ring_cnt = 0u;

  auto flush = [&](int count) {
    __syncthreads();  // ring rows written (one wave per workgroup: orders LDS)
    ring_gid = Rg[lane & 31];
    ring_cnt = Rc[lane & 31];
    // bit r: pixel row r % 8 of quadrant r / 8; K-step t covers bits 2t, 2t + 1
    const uint32_t rows = row_bits(pix0) | (row_bits(pix1) << 8);
    const float* wrow = Wt + (lane & 31) * kPairPitch + 8 * (lane >> 5);
    if (bsets || any_tail) {
      // lane l: row l % 32, the pixels of quadrant l / 32
      const float* rp = Wt + (lane & 31) * kPairPitch + 64 * (lane >> 5);
      const float* fp = Ft + 64 * (lane >> 5);
      float bs = 0.0f, ts[kMaxTail] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < 16; k++) {
        const float4 a = *reinterpret_cast<const float4*>(rp + 4 * k);
        bs += a.x;
        bs += a.y;
        bs += a.z;
        bs += a.w;
#pragma unroll
        for (int t = 0; t < kMaxTail; t++) {
          if (t < ntail) {  // wave-uniform
            const float4 f = *reinterpret_cast<const float4*>(fp + t * 128 + 4 * k);
            ts[t] = __builtin_fmaf(a.x, f.x, ts[t]);
            ts[t] = __builtin_fmaf(a.y, f.y, ts[t]);
            ts[t] = __builtin_fmaf(a.z, f.z, ts[t]);
            ts[t] = __builtin_fmaf(a.w, f.w, ts[t]);
          }
        }
      }
      bs += __shfl_xor(bs, 32, 64);
#pragma unroll
      for (int t = 0; t < kMaxTail; t++) ts[t] += __shfl_xor(ts[t], 32, 64);
      if (lane < count) {
        for (int b = bsets; b; b &= b - 1) {
          const SetDesc& sd = sets[__builtin_ctz(b)];
          beta_atomic_add(sd.beta + ring_gid, bs);
          if (sd.counts) gatomic_add(sd.counts + ring_gid, ring_cnt);
        }
#pragma unroll
        for (int t = 0; t < kMaxTail; t++)
          if (tout[t] && ts[t] != 0.0f) u_atomic_add(tout[t], (int64_t)ring_gid * tD[t], ts[t], fixedU);
      }
      __syncthreads();  // the FP32 weights read before they are split
    }
    // the weights of this lane's operand chunks (row l % 32, pixels
    // 16 t + 8 (l / 32) + [0, 8)) split once into BF16 hi and lo in place,
    // for all groups; each lane splits exactly the chunks it reads (the FP32
    // weights' other reader, the beta and tail sums above, is done)
#pragma unroll
    for (int t = 0; t < 8; t++)
      if ((rows >> (2 * t)) & 3u) split_w_in_place(Wt + (lane & 31) * kPairPitch + 8 * (lane >> 5) + 16 * t);
    if constexpr (!kSplitF && PX) {
      // BF16 / FP8 pixel-block maps: one operand load per K-step and block
      // (the HWC layout's eight loads per operand leave no registers for
      // this).  A group's products go out (one atomic per channel) only
      // after the next group's operand loads have been issued: the vector
      // memory counter completes in order, so waiting for those loads does
      // not wait for the atomics.
      GroupLanes Lp;  // the group whose products are pending
      bool pend = false, twop = false;
      f32x16 acc0 = {}, acc1 = {};
      for (int cg = 0; cg < ngroups; cg++) {
        GroupLanes L;
        const bool ok = ((gmask >> cg) & 1u) && group_lanes_pair<DT>(groups[cg], sets, q, lane, L);
        const bool two = groups[cg].width > 32;
        bf16x8 F[2][8];
        if (ok) {
#pragma unroll
          for (int t = 0; t < 8; t++) {
            if ((rows >> (2 * t)) & 3u) {
              bf16x8 lo;
              const int gy = q.qy + 2 * (t & 3) + (lane >> 5), gx0 = q.qx + 8 * (t >> 2);
              load_row8<DT, PX>(L, 0, gy, gx0, q.g, F[0][t], lo);
              if (two) load_row8<DT, PX>(L, 1, gy, gx0, q.g, F[1][t], lo);
            }
          }
        }
        if (pend) batch_scatter<DT>(Lp, twop, count, ring_gid, lane, acc0, acc1, fixedU);
        pend = false;
        if (!ok) continue;
        acc0 = f32x16{};
        acc1 = f32x16{};
        if (two) {
#pragma unroll
          for (int t = 0; t < 8; t++) {
            if ((rows >> (2 * t)) & 3u) {
              bf16x8 ah, al;
              load_w(wrow + 16 * t, ah, al);
              acc0 = mfma(ah, F[0][t], acc0);
              acc1 = mfma(ah, F[1][t], acc1);
              acc0 = mfma(al, F[0][t], acc0);
              acc1 = mfma(al, F[1][t], acc1);
            }
          }
        } else {
#pragma unroll
          for (int t = 0; t < 8; t++) {
            if ((rows >> (2 * t)) & 3u) {
              bf16x8 ah, al;
              load_w(wrow + 16 * t, ah, al);
              acc0 = mfma(ah, F[0][t], acc0);
              acc0 = mfma(al, F[0][t], acc0);
            }
          }
        }
        Lp = L;
        twop = two;
        pend = true;
      }
      if (pend) batch_scatter<DT>(Lp, twop, count, ring_gid, lane, acc0, acc1, fixedU);
    } else {
      for (int cg = 0; cg < ngroups; cg++) {
        if (!((gmask >> cg) & 1u)) continue;
        const ChanGroup& grp = groups[cg];
        GroupLanes L;
        if (!group_lanes_pair<DT>(grp, sets, q, lane, L)) continue;
        const bool two = grp.width > 32;
        f32x16 acc0 = {}, acc1 = {};
        if (two) {
  #pragma unroll
          for (int t = 0; t < 8; t++) {
            if ((rows >> (2 * t)) & 3u) {
              bf16x8 h0, l0, h1, l1, ah, al;
              const int gy = q.qy + 2 * (t & 3) + (lane >> 5), gx0 = q.qx + 8 * (t >> 2);
              load_row8<DT, PX>(L, 0, gy, gx0, q.g, h0, l0);
              load_row8<DT, PX>(L, 1, gy, gx0, q.g, h1, l1);
              load_w(wrow + 16 * t, ah, al);
              acc0 = mfma(ah, h0, acc0);
              acc1 = mfma(ah, h1, acc1);
              acc0 = mfma(al, h0, acc0);
              acc1 = mfma(al, h1, acc1);
              if constexpr (kSplitF) {
                acc0 = mfma(ah, l0, acc0);
                acc1 = mfma(ah, l1, acc1);
              }
            }
          }
        } else {
  #pragma unroll
          for (int t = 0; t < 8; t++) {
            if ((rows >> (2 * t)) & 3u) {
              bf16x8 h0, l0, ah, al;
              load_row8<DT, PX>(L, 0, q.qy + 2 * (t & 3) + (lane >> 5), q.qx + 8 * (t >> 2), q.g, h0, l0);
              load_w(wrow + 16 * t, ah, al);
              acc0 = mfma(ah, h0, acc0);
              acc0 = mfma(al, h0, acc0);
              if constexpr (kSplitF) acc0 = mfma(ah, l0, acc0);
            }
          }
        }
        batch_scatter<DT>(L, two, count, ring_gid, lane, acc0, acc1, fixedU);
      }
    }
    __syncthreads();  // rows read before they are written again
  };

  float T0 = 1.0f, T1 = 1.0f;
  bool alive0 = in0, alive1 = in1;
  uint64_t cov0 = 0ull, cov1 = 0ull;
  uint32_t ncontrib = 0u, nrows = 0u;
  const Rec* vrec = rec + (int64_t)q.v * n;
  for (uint32_t base = q.rg.x; base < q.rg.y; base += G) {
    if (__ballot(alive0 || alive1) == 0ull) break;
    const int cnt = (int)(q.rg.y - base < (uint32_t)G ? q.rg.y - base : (uint32_t)G);
    // lane j: record j, centre made tile-relative, left in LDS; hit masks of
    // the two quadrants
    float4 r0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 r1 = make_float4(0.0f, 0.0f, -1.0f, 0.0f);
    uint32_t my_id = 0;
    if (lane < cnt) {
      my_id = ids[base + lane];
      r0 = vrec[my_id].r0;
      r1 = vrec[my_id].r1;
      const uint32_t lo = __float_as_uint(r1.w);
      r0.x = (r0.x - ocx) + __uint_as_float(lo << 16);
      r0.y = (r0.y - ocy) + __uint_as_float(lo & 0xFFFF0000u);
    }
    Rs[lane][0] = r0;
    Rs[lane][1] = r1;
    const float X0 = -r0.x, Y0 = qy0 - r0.y;
    const bool h0 = lane < cnt && region_hits(r0, r1, X0, X0 + 7.0f, Y0, Y0 + 7.0f);
    const bool h1 = lane < cnt && region_hits(r0, r1, X0 + 8.0f, X0 + 15.0f, Y0, Y0 + 7.0f);
    const uint64_t hits0 = __ballot(h0), hits1 = __ballot(h1);
    uint64_t h = hits0 | hits1;
    if (!h) continue;
    __syncthreads();  // records in LDS
    while (h) {
      const int j = (int)__builtin_ctzll(h);
      h &= h - 1;
      const float4 a = Rs[j][0], b = Rs[j][1];
      bool t0 = false, t1 = false;
      float w0 = 0.0f, w1 = 0.0f;
      if ((hits0 >> j) & 1ull) w0 = blend_at(a, b, pxo0, pyo, T0, alive0, t0);
      if ((hits1 >> j) & 1ull) w1 = blend_at(a, b, pxo1, pyo, T1, alive1, t1);
      const uint64_t m0 = __builtin_amdgcn_ballot_w64(t0), m1 = __builtin_amdgcn_ballot_w64(t1);
      if (m0 | m1) {
        cov0 |= m0;
        cov1 |= m1;
        const uint32_t c = (uint32_t)(__popcll(m0) + __popcll(m1));
        ncontrib += c;
        nrows++;
        Wt[queued * kPairPitch + lane] = w0;
        Wt[queued * kPairPitch + 64 + lane] = w1;
        if (lane == j) {  // lane j holds the Gaussian's id
          Rg[queued] = my_id;
          Rc[queued] = c;
        }
        pix0 |= m0;
        pix1 |= m1;
        if (++queued == 32) {
          flush(32);
          queued = 0;
          pix0 = pix1 = 0ull;
        }
      }
    }
  }
  if (queued > 0) flush(queued);
  for (int b = ssets; b; b &= b - 1) {
    const SetDesc& sd = sets[__builtin_ctz(b)];
    if (sd.stats && lane == 0) {
      gatomic_add(&sd.stats[1], (unsigned long long)ncontrib);
      gatomic_add(&sd.stats[0], (unsigned long long)(__popcll(cov0) + __popcll(cov1)));
      gatomic_add(&sd.stats[2], (unsigned long long)nrows);
    }
  }
}

template <lv_dtype DT, bool PX>
hipError_t launch_blend_t(const BlendArgs& a, int m, hipStream_t s) {
  // one group: one wave per (view, quadrant, group); several: one wave per
  // (view, quadrant) for all groups, sharing the walk
  const bool multi = a.ngroups > 1;
  int64_t work = (int64_t)a.tiles_stride * m * (multi ? 1 : a.ngroups);
  int64_t blocks = (work + 7) / 8 * 32;
  if (multi) {
    // one wave per half tile: two per tile, whole rounds of 8 XCDs
    const int64_t pblocks = ((int64_t)a.tiles_stride * m + 7) / 8 * 16;
    const size_t tail_lds = a.has_tail ? sizeof(float) * kMaxTail * 128 : 0;
    hipLaunchKernelGGL((blend_pair_kernel<DT, PX>), dim3((unsigned)pblocks), dim3(64), tail_lds, s, a.rec,
                       a.ids, a.ranges, a.geom, a.n, a.tiles_stride, m, a.sets, a.groups,
                       a.ngroups);
  } else
    hipLaunchKernelGGL((blend_wide_kernel<DT, PX>), dim3((unsigned)blocks), dim3(64), 0, s,
                       a.rec, a.ids, a.ranges, a.geom, a.n, a.tiles_stride, m, a.sets, a.groups,
                       a.ngroups);
  return hipGetLastError();
}

// ------------------------------------------------------------ forward render
// Eq. (4): F^(p) = sum_i w_i(p) g_i, the adjoint of the uplift.  One wave per
// (view, quadrant, group of 32 NB channels) walks its tile's list exactly as
// the uplift does; a Gaussian with some contribution queues its weights at
// the 64 pixels in one of 32 LDS rows (its index beside it).  A full queue
// (and the last, partial one) is flushed on the matrix cores: out (64 pixels
// x 32 NB channels) += W^T (64 x 32 rows) G (32 rows x 32 NB channels), split
// BF16 operands as in the uplift, the 2 x NB 32x32 output blocks held in
// registers until the walk ends; each (pixel, channel) is then written once.
// The opacity sum_i w_i(p) goes to alpha[v] (group 0).  NB = 2 (64 channels)
// for D <= 64, else 4: the walk, repeated for every group of channels, runs
// half as often, and the 8 output blocks' 128 registers leave 2 waves per
// SIMD instead of 3.
template <int NB>
__global__ __launch_bounds__(64, (NB == 2 ? 3 : 2)) void render_kernel(
    const Rec* __restrict__ rec, const uint32_t* __restrict__ ids, const uint2* __restrict__ ranges,
    const ViewGeom* __restrict__ geom, int64_t n, int tiles_stride, int nviews, int ngroups,
    const float* __restrict__ g, int D, float* const* __restrict__ outs,
    float* const* __restrict__ alphas, const uint32_t* __restrict__ perm) {
  constexpr int G = kChunk;
  __shared__ __align__(16) float Wt[32 * kWtPitch];  // queued Gaussians: [row][pixel]
  __shared__ float4 Rs[kChunk][2];                   // the step's records
  __shared__ uint32_t Rg[32];                        // queued Gaussians' ids
  Quad q;
  // every in-image (pixel, channel) of every view is written, zeros where no
  // Gaussian reaches (a tile without Gaussians walks nothing)
  if (!decode_quad(ranges, geom, tiles_stride, nviews, ngroups, q, true)) return;
  const int lane = threadIdx.x;
  const int c0 = q.cg * 32 * NB;
  // this lane's channel in each 32-channel block (a readable one where it has none)
  int ch[NB];
  bool own[NB];
#pragma unroll
  for (int b = 0; b < NB; b++) {
    ch[b] = c0 + 32 * b + (lane & 31);
    own[b] = ch[b] < D;
    if (!own[b]) ch[b] = 0;
  }
  f32x16 acc[2][NB];  // [pixel block][channel block]
#pragma unroll
  for (int b = 0; b < NB; b++) acc[0][b] = acc[1][b] = f32x16{};
  float asum = 0.0f;
  int queued = 0;

  // K-step t: queue rows 16 t + 8 (l / 32) + i, i < 8.  Rows past count
  // have weight 0 and read the features of row 0 (in this flush), and a lane
  // without a channel feeds only its own output column, never written: the
  // loaded features are used as loaded (no select, so no zero fill that would
  // wait for every load in flight).
  auto flush = [&](int count) {
    __syncthreads();  // rows written (one wave per workgroup: orders LDS)
    for (int t = 0; t < 2 && 16 * t < count; t++) {
      float w0[8], w1[8];
      int64_t gid[8];
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const int row = 16 * t + 8 * (lane >> 5) + i;
        const bool ok = row < count;
        gid[i] = (int64_t)Rg[ok ? row : 0];
        w0[i] = ok ? Wt[row * kWtPitch + (lane & 31)] : 0.0f;
        w1[i] = ok ? Wt[row * kWtPitch + 32 + (lane & 31)] : 0.0f;
      }
      float gb[NB][8];
#pragma unroll
      for (int c = 0; c < NB; c++)
#pragma unroll
        for (int i = 0; i < 8; i++) gb[c][i] = g[gid[i] * D + ch[c]];
      bf16x8 a0h, a0l, a1h, a1l;
      split8(w0, a0h, a0l);
      split8(w1, a1h, a1l);
#pragma unroll
      for (int c = 0; c < NB; c++) {
        bf16x8 bh, bl;
        split8(gb[c], bh, bl);
        acc[0][c] = mfma(a0h, bh, acc[0][c]);
        acc[1][c] = mfma(a1h, bh, acc[1][c]);
        acc[0][c] = mfma(a0l, bh, acc[0][c]);
        acc[1][c] = mfma(a1l, bh, acc[1][c]);
        acc[0][c] = mfma(a0h, bl, acc[0][c]);
        acc[1][c] = mfma(a1h, bl, acc[1][c]);
      }
    }
    __syncthreads();  // rows read before they are written again
  };

  Walk s;
  walk_init(q, lane, s);
  const Rec* vrec = rec + (int64_t)q.v * n;
  for (uint32_t base = q.rg.x; base < q.rg.y; base += G) {
    if (__ballot(s.alive) == 0ull) break;
    const int cnt = (int)(q.rg.y - base < (uint32_t)G ? q.rg.y - base : (uint32_t)G);
    uint32_t my_id;
    const uint64_t hits = step_records(vrec, ids, base, cnt, lane, s, my_id, Rs, perm);
    if (!hits) continue;
    __syncthreads();  // records in LDS (one wave per workgroup: orders LDS)
    for (uint64_t h = hits; h; h &= h - 1) {
      const int j = (int)__builtin_ctzll(h);
      bool take;
      const float wj = walk_rec(Rs[j][0], Rs[j][1], s, take);
      if (__ballot(take)) {
        Wt[queued * kWtPitch + lane] = wj;
        if (lane == j) Rg[queued] = my_id;  // lane j holds the Gaussian's (caller) index
        asum += wj;
        if (++queued == 32) {
          flush(32);
          queued = 0;
        }
      }
    }
  }
  if (queued > 0) flush(queued);

  // D row m of a block: pixel 32 pb + 8 (r / 4) + 4 (l / 32) + r % 4, column
  // (channel) l % 32
  float* const out = outs[q.v];
#pragma unroll
  for (int pb = 0; pb < 2; pb++) {
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int m = 32 * pb + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int px = q.qx + (m & 7), py = q.qy + (m >> 3);
      if (px < q.g.W && py < q.g.H) {
        const int64_t pix = (int64_t)py * q.g.W + px;
#pragma unroll
        for (int c = 0; c < NB; c++)
          if (own[c]) gptr(out)[pix * D + ch[c]] = acc[pb][c][r];
      }
    }
  }
  const int px = q.qx + (lane & 7), py = q.qy + (lane >> 3);
  if (q.cg == 0 && alphas[q.v] && px < q.g.W && py < q.g.H)
    gptr(alphas[q.v])[(int64_t)py * q.g.W + px] = asum;
}

// D a multiple of 4, 16-byte aligned arrays: a block takes 64 Gaussians,
// each thread four channels at a time (16-byte accesses, no 64-bit division
// per element).
constexpr int kFinRows = 64;
__global__ __launch_bounds__(256) void finalize4_kernel(const float4* __restrict__ U,
                                                        const beta_t* __restrict__ beta, int64_t n,
                                                        int Q, float4* __restrict__ f,
                                                        float* __restrict__ wsum,
                                                        float4* __restrict__ usum,
                                                        const uint32_t* __restrict__ perm) {
  const int64_t r0 = (int64_t)blockIdx.x * kFinRows;
  const int rows = (int)(n - r0 < kFinRows ? n - r0 : kFinRows);
  for (int k = threadIdx.x; k < rows * Q; k += 256) {
    const int r = k / Q, q = k - r * Q;
    const int64_t i = r0 + r;
    const int64_t o = perm ? (int64_t)perm[i] : i;  // the output row
    const float bs = (float)((double)beta[i] * (1.0 / kBetaUnit));
    const float4 u = U[i * Q + q];
    const int64_t e = o * Q + q;
    if (f)
      f[e] = bs > 0.0f ? make_float4(u.x / bs, u.y / bs, u.z / bs, u.w / bs)
                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (usum) usum[e] = u;
    if (wsum && q == 0) wsum[o] = bs;
  }
}

__global__ void finalize_kernel(const float* __restrict__ U, const beta_t* __restrict__ beta,
                                int64_t n, int D, float* __restrict__ f, float* __restrict__ wsum,
                                float* __restrict__ usum, const uint32_t* __restrict__ perm) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * D) return;
  int64_t i = e / D;
  const int64_t c = e - i * D;
  const int64_t o = perm ? (int64_t)perm[i] : i;  // the output row
  const float bs = (float)((double)beta[i] * (1.0 / kBetaUnit));
  float u = U[e];
  if (f) f[o * D + c] = bs > 0.0f ? u / bs : 0.0f;
  if (usum) usum[o * D + c] = u;
  if (wsum && c == 0) wsum[o] = bs;
}

__global__ void finalize_fixed_kernel(const long long* __restrict__ U, const beta_t* __restrict__ beta,
                                      int64_t n, int D, float* __restrict__ f, float* __restrict__ wsum,
                                      float* __restrict__ usum, const uint32_t* __restrict__ perm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * D) return;
  const int64_t i = e / D, c = e - i * D;
  const int64_t o = perm ? (int64_t)perm[i] : i;  // the output row
  const double b = (double)beta[i] * (1.0 / kBetaUnit);
  const double u = (double)U[e] * (1.0 / kBetaUnit);
  if (f) f[o * D + c] = b > 0.0 ? (float)(u / b) : 0.0f;
  if (usum) usum[o * D + c] = (float)u;
  if (wsum && c == 0) wsum[o] = (float)b;
}

}  // namespace

namespace {
__global__ __launch_bounds__(256) void class_add_kernel(const beta_t* __restrict__ beta,
                                                        const uint32_t* __restrict__ counts,
                                                        ClassAdd dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const beta_t b = beta[i];
    const uint32_t c = counts ? counts[i] : 0u;
    for (int k = 0; k < dst.nd; k++) {
      if (dst.beta[k]) dst.beta[k][i] += b;
      if (dst.counts[k]) dst.counts[k][i] += c;
    }
  }
}
}  // namespace

hipError_t launch_class_add(const beta_t* beta, const uint32_t* counts, const ClassAdd& dst,
                            int64_t n, hipStream_t s) {
  if (n == 0 || dst.nd == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(class_add_kernel, dim3((unsigned)blocks), dim3(256), 0, s, beta, counts, dst, n);
  return hipGetLastError();
}

hipError_t launch_blend(const BlendArgs& a, lv_dtype dtype, int m, hipStream_t s) {
  if (m == 0 || a.tiles_stride == 0) return hipSuccess;
  switch (dtype) {
    case LV_F32: return launch_blend_t<LV_F32, false>(a, m, s);
    case LV_BF16: return launch_blend_t<LV_BF16, false>(a, m, s);
    case LV_FP8_E4M3: return launch_blend_t<LV_FP8_E4M3, false>(a, m, s);
    case LV_F32_PX8: return launch_blend_t<LV_F32, true>(a, m, s);
    case LV_BF16_PX8: return launch_blend_t<LV_BF16, true>(a, m, s);
    case LV_FP8_E4M3_PX8: return launch_blend_t<LV_FP8_E4M3, true>(a, m, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_render(const BlendArgs& a, int m, const float* g, int D, float* const* outs,
                         float* const* alphas, const uint32_t* perm, hipStream_t s) {
  if (m == 0 || a.tiles_stride == 0) return hipSuccess;
  const int ch = D > 64 ? 128 : 64;  // channels per wave
  const int ngroups = (D + ch - 1) / ch;
  const int64_t work = (int64_t)a.tiles_stride * m * ngroups;
  const int64_t blocks = (work + 7) / 8 * 32;  // 4 quadrants per tile, whole rounds of 8 XCDs
  if (ch == 128)
    hipLaunchKernelGGL(render_kernel<4>, dim3((unsigned)blocks), dim3(64), 0, s, a.rec, a.ids,
                       a.ranges, a.geom, a.n, a.tiles_stride, m, ngroups, g, D, outs, alphas, perm);
  else
    hipLaunchKernelGGL(render_kernel<2>, dim3((unsigned)blocks), dim3(64), 0, s, a.rec, a.ids,
                       a.ranges, a.geom, a.n, a.tiles_stride, m, ngroups, g, D, outs, alphas, perm);
  return hipGetLastError();
}

hipError_t launch_finalize_fixed(const long long* U, const beta_t* beta, int64_t n, int D, float* f,
                                 float* wsum, float* usum, const uint32_t* perm, hipStream_t s) {
  const int64_t total = n * (int64_t)D;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_fixed_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, U, beta,
                     n, D, f, wsum, usum, perm);
  return hipGetLastError();
}

hipError_t launch_finalize(const float* U, const beta_t* beta, int64_t n, int D, float* f,
                           float* wsum, float* usum, const uint32_t* perm, hipStream_t s) {
  int64_t total = n * (int64_t)D;
  if (total == 0) return hipSuccess;
  const auto a16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (D % 4 == 0 && a16(U) && a16(f) && a16(usum)) {
    hipLaunchKernelGGL(finalize4_kernel, dim3((unsigned)((n + kFinRows - 1) / kFinRows)), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(U), beta, n, D / 4, reinterpret_cast<float4*>(f),
                       wsum, reinterpret_cast<float4*>(usum), perm);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, U,
                     beta, n, D, f, wsum, usum, perm);
  return hipGetLastError();
}

}  // namespace lv
