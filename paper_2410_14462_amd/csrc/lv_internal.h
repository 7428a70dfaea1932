// Internal declarations of the gfx950 uplifting library.  Device code is
// compiled with -ffp-contract=off: every FP32 expression below is evaluated
// exactly as written (explicit fmaf where an FMA is meant), which keeps the
// structure and the blend decisions reproducible bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include "lv.h"

namespace lv {

// A named roctx range over a host scope (the phases of a call, the
// server's passes): visible in `rocprofv3 --marker-trace`, free without a
// tool attached.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

constexpr int kTile = 16;           // tile edge in pixels
constexpr int kChunk = 64;          // Gaussians per blend step (one per lane)
constexpr int kSortItems = 4096;    // items per radix-sort block (4 waves x 1024)
constexpr int kRadixBits = 11;      // digit bits per radix pass
constexpr int kSortThreads = 256;
constexpr int kViewShift = 20;      // pair key = view << 20 | tile

// Method constants as FP32 literals (0.99f, 1/255.f, 1e-4f, 0.3f, 1.3f).
constexpr float kAlphaMax = 0x1.fae148p-1f;
constexpr float kAlphaMin = 0x1.010102p-8f;
constexpr float kTEps = 0x1.a36e2ep-14f;
constexpr float kDilate = 0x1.333334p-2f;
constexpr float kClamp = 0x1.4cccccp+0f;

// Camera as the kernels see it (same field order as lv_camera).
struct Cam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy, znear;
  int32_t width, height, reserved;
};
static_assert(sizeof(Cam) == sizeof(lv_camera), "camera layout");

// Per (view, Gaussian) projected record, 32 bytes:
//   r0 = (ux, uy, L11, L12), r1 = (L22, opacity, tau, lo)
// The centre is (ux + ux_lo, uy + uy_lo); lo packs the upper 16 bits of
// ux_lo (low half) and of uy_lo (high half).  Offsets of a pixel from the
// centre are taken relative to the first pixel centre of the pixel's tile:
// dx = (px - ox) - ((ux - (ox + 0.5)) + ux_lo), ox = 16 floor(px / 16).
// power(d) = -((L11 dx + L12 dy)^2 + (L22 dy)^2); alpha can reach 1/255
// only where -power <= tau (conservative, used only to skip work; tau < 0:
// never).
struct Rec {
  float4 r0, r1;
};

// e^x for x <= 0 on the hardware base-2 exponential, 2^(x log2 e): the
// product is rounded once (relative error of the result about |x| 2^-24)
// and v_exp_f32 adds about one ulp, so alpha = opacity e^x is within 1e-6
// (relative) of its exact value wherever it can reach 1/255 (x >= -6).
// The skip and stop decisions therefore agree with the FP64 definition
// except where its own margin is below that.
__device__ __forceinline__ float exp_neg(float x) {
  return __builtin_amdgcn_exp2f(x * 0x1.715476p+0f);
}

// Global-memory accesses through pointers held in structures: the compiler
// cannot tell their address space and would emit FLAT instructions, which
// also count as LDS operations, so every wait for an LDS result would wait
// for them too.  These helpers make them global loads and atomics.
#define LV_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ LV_GLOBAL T* gptr(T* p) {
  return (LV_GLOBAL T*)p;
}

template <typename T>
__device__ __forceinline__ const LV_GLOBAL T* gptr(const T* p) {
  return (const LV_GLOBAL T*)p;
}

template <typename T>
__device__ __forceinline__ void gatomic_add(T* p, T v) {  // relaxed, device scope
  __hip_atomic_fetch_add(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// beta_i accumulates in 64-bit fixed point, in units of 2^-35: each weight
// sum is rounded to the nearest unit and added with an integer atomic, so the
// total is exact (the sum of the rounded terms) and independent of the order
// of the atomics, and no atomic has to return.  A counted weight is at least
// 1e-4/255 (alpha >= 1/255 at transmittance >= 1e-4), so the rounding is
// below 2^-36 / (1e-4/255) < 4e-5 of each term.  Capacity: 2^29 (5.4e8)
// units of weight per Gaussian.
typedef unsigned long long beta_t;
constexpr double kBetaUnit = 34359738368.0;  // 2^35

__device__ __forceinline__ void beta_atomic_add(beta_t* p, float w) {
  gatomic_add(p, (beta_t)__double2ull_rn((double)w * kBetaUnit));
}

// U += v at p[off]: an FP32 atomic, or, for a deterministic accumulator, v
// rounded to the nearest 2^-35 and added to a signed 64-bit fixed-point word
// (two's complement: the unsigned add wraps correctly).  Integer adds
// commute, so a deterministic U is the same bit for bit whatever the order
// of the atomics; |U| must stay below 2^28.  p points at element 0 of the
// lane's channel in either element type (fixed: the word address as float*).
__device__ __forceinline__ void u_atomic_add(float* p, int64_t off, float v, bool fixed) {
  if (fixed)
    gatomic_add(reinterpret_cast<unsigned long long*>(p) + off,
                (unsigned long long)__double2ll_rn((double)v * kBetaUnit));
  else
    gatomic_add(p + off, v);
}
// Element c of a set's U row 0 as a float* (either element type).
__device__ __forceinline__ float* u_elem(float* U, int64_t c, bool fixed) {
  return fixed ? reinterpret_cast<float*>(reinterpret_cast<long long*>(U) + c) : U + c;
}

// ------------------------------------------------------------ device memory
// Every device buffer of the library: the allocator registered with
// lv_set_allocator, else hipMalloc / hipFree, or hipMallocAsync /
// hipFreeAsync for temporary (stream-ordered) scratch.  dev_free releases
// after the work enqueued on `s` (a registered allocator gets the stream;
// hipFree itself waits for the device).
hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s, bool temp = false);
void dev_free(void* p, size_t bytes, hipStream_t s, bool temp = false);

// ---------------------------------------------------------------- launches
// All launchers enqueue on `s` and return hipGetLastError().
hipError_t launch_scene_derive(const float* means, const float* scales, const float* quats,
                               const float* opacity, int64_t n, float4* p0, float4* p1, float4* p2,
                               hipStream_t s);

struct ViewGeom {      // per view of a chunk (device array)
  int32_t W, H, TX, TY;
};

hipError_t launch_preprocess(const float4* p0, const float4* p1, const float4* p2, int64_t n,
                             const Cam* cams, const ViewGeom* geom, int m, Rec* rec,
                             uint32_t* key, uint2* rect, hipStream_t s);

// Segmented stable LSD radix sort of (key, val) pairs on key bits [0, bits),
// in radix_passes(bits) passes.  Segment g occupies [seg_start[g],
// seg_start[g] + seg_len[g]); max_len bounds seg_len.  Result ends in (k0, v0)
// if the number of passes is even, else in (k1, v1); *in_second tells which.
// keys_last false: the last pass writes only the values.  hist needs
// sort_hist_size() uint32; after the sort it holds the last pass's scanned
// counts.
// payload (optional): the last pass also writes orect[i] = rect[seg_start[g]
// + val] beside each sorted value, and ocnt[i] = that rect's area in tiles
// (rect packed as x0 | y0 << 16, x1 | y1 << 16).
struct SortPayload {
  const uint2* rect = nullptr;
  uint32_t* ocnt = nullptr;
  uint2* orect = nullptr;
};
inline int radix_passes(int bits, int pass_bits = kRadixBits) {
  return (bits + pass_bits - 1) / pass_bits;
}
size_t sort_hist_size(int nseg, int64_t max_len);
hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                      const uint32_t* seg_start, const uint32_t* seg_len, int nseg,
                      int64_t max_len, int bits, uint32_t* hist, bool keys_last, bool* in_second,
                      hipStream_t s, SortPayload payload = SortPayload{},
                      int pass_bits = kRadixBits, bool iota_values = false);
// Tile ranges (absolute [start, end) per view and tile, tiles_stride per view)
// after a one-pass radix_sort by tile over the same segments, from its hist.
hipError_t launch_hist_ranges(const uint32_t* hist, const uint32_t* seg_start,
                              const uint32_t* seg_len, int nseg, int64_t max_len, int bits,
                              int tiles_stride, uint2* ranges, hipStream_t s);

// Exclusive scan of the counts of the m*n sorted items, cnt[v*n + val[v*n+k]]
// (or cnt[v*n+k] when sorted_val is NULL: counts already in sorted order):
// off[v*n+k] (global running offset over the whole chunk).  seg_start /
// seg_len per view get the view's pair range; totals[0] = number of pairs,
// totals[1] = number of visible (view, Gaussian) items.
size_t scan_tmp_size(int64_t items);
hipError_t scan_counts(const uint32_t* cnt, const uint32_t* sorted_val, int64_t n, int m,
                       uint32_t* off, uint32_t* seg_start, uint32_t* seg_len,
                       unsigned long long* totals, uint32_t* tmp, hipStream_t s);

// (tile, Gaussian) pairs of the depth-sorted items, given their ids, pair
// offsets, rects and counts in the same sorted order.
hipError_t launch_duplicate(const uint32_t* sorted_val, const uint32_t* off,
                            const uint2* sorted_rect, const uint32_t* sorted_cnt,
                            const ViewGeom* geom, int64_t n, int m, uint32_t* pair_key,
                            uint32_t* pair_val, hipStream_t s);

// The same with 16-bit tile keys (tiles_stride <= 65536): the view of a pair
// is its sort segment.
hipError_t radix_sort16(uint16_t* k0, uint32_t* v0, uint16_t* k1, uint32_t* v1,
                        const uint32_t* seg_start, const uint32_t* seg_len, int nseg, int64_t max_len,
                        int bits, uint32_t* hist, bool keys_last, bool* in_second, hipStream_t s);
hipError_t launch_duplicate16(const uint32_t* sorted_val, const uint32_t* off,
                              const uint2* sorted_rect, const uint32_t* sorted_cnt,
                              const ViewGeom* geom, int64_t n, int m, uint16_t* pair_key,
                              uint32_t* pair_val, hipStream_t s);
hipError_t launch_ranges16(const uint16_t* pair_key, const uint32_t* seg_start, const uint32_t* seg_len,
                           int nseg, int64_t max_len, int tiles_stride, uint2* ranges, hipStream_t s);
hipError_t launch_ranges(const uint32_t* pair_key, int64_t P, int tiles_stride, uint2* ranges,
                         hipStream_t s);

constexpr int kMaxSets = 8;   // feature sets per blend launch
constexpr int kMaxSegs = 8;   // set segments per channel group (one per set at most)

// One feature set of a blend launch (device array).
struct SetDesc {
  const void* const* maps;    // [views] device pointers, HWC [H][W][stride];
                              // NULL: the set does not take that view
  const float* scales;        // FP8: [all views][D] scales, else null
  float* U;                   // [n][D] FP32, or int64 fixed point (units of 2^-35) if fixed
  int32_t fixed;              // the same for every set of a launch
  beta_t* beta;               // [n] fixed point, units of 2^-35
  uint32_t* counts;           // [n] or null
  unsigned long long* stats;  // [3] covered pixels, contributions, partial sums; or null
  int32_t D;
  int32_t stride;             // elements between consecutive pixels (>= D)
  int32_t view_base;          // index of the launch's first view in scales
};

constexpr int kMaxTail = 4;   // channels of a group kept in registers

// The channels one workgroup handles.  Main part: segments [vc0, vc0 + cnt)
// of the group's (<= 64) channels taken from set `set`, channels
// [c0, c0 + cnt), vc0 ascending from 0, one channel per lane.  Tail: up to 4
// further single channels (set tset[t], channel tc[t]) reduced across the
// wave.  beta_sets: bit s set if this group adds beta (and counts) of set
// s; stats_sets: bit s set if it adds the statistics of set s.
struct ChanGroup {
  int32_t width, nseg, ntail, beta_sets, stats_sets;
  int32_t set[kMaxSegs], c0[kMaxSegs], vc0[kMaxSegs], cnt[kMaxSegs];
  int32_t tset[kMaxTail], tc[kMaxTail];
};

struct BlendArgs {
  const Rec* rec;              // [m][n]
  const uint32_t* ids;         // sorted pair values (Gaussian ids)
  const uint2* ranges;         // [m][tiles_stride]
  const ViewGeom* geom;        // [m]
  int64_t n;
  int32_t tiles_stride;
  const SetDesc* sets;         // device
  const ChanGroup* groups;     // device (wide kernel)
  int32_t ngroups;
  int32_t max_width;           // widest group (LDS size)
  int32_t has_tail;            // the last group has tail channels
};
hipError_t launch_blend(const BlendArgs& a, lv_dtype dtype, int m, hipStream_t s);
// dst_beta[k][i] += beta[i], dst_counts[k][i] += counts[i] (entries may be
// NULL) for the k < nd members of a class of feature sets that take the same
// views (their increments are equal and are accumulated once).
struct ClassAdd {
  beta_t* beta[kMaxSets];
  uint32_t* counts[kMaxSets];
  int32_t nd;
};
hipError_t launch_class_add(const beta_t* beta, const uint32_t* counts, const ClassAdd& dst,
                            int64_t n, hipStream_t s);

// Eq. (4) forward render of g [n][D] into outs[v] [H][W][D] (device table of
// m pointers) and the accumulated opacity into alphas[v] [H][W] (entries may
// be null); every in-image pixel is written (zeros where no Gaussian
// reaches).  perm (nullable): storage -> caller order of the scene; g is in
// the caller's order.
hipError_t launch_render(const BlendArgs& a, int m, const float* g, int D, float* const* outs,
                         float* const* alphas, const uint32_t* perm, hipStream_t s);
// Keep the k Gaussians with the largest wsum (ties to the lower index):
// keep[i] = 1 for them, 0 for the others (scratch from the stream-ordered
// allocator).
hipError_t launch_prune(const float* wsum, int64_t n, int64_t k, uint8_t* keep, hipStream_t s);
// kNN diffusion graph over the centres (xyz of centres[i]) with feature
// weights (feats [n][D]); CSR arrays allocated with hipMalloc (owned by the
// caller afterwards); synchronises the stream once (to size the CSR).
// Requires k < n, 1 <= k <= 32, n (2k + 1) < 2^31.
struct GraphWeights {
  int32_t kind = LV_GRAPH_SPATIAL_COSINE;
  float bandwidth = 1.0f;        // b (feature kernel)
  const float* unary = nullptr;  // P [n] (feature kernel), NULL: 1
  float binarize = 0.0f;         // > 0 (feature kernel): 1 where the weight exceeds it
};
hipError_t build_knn_graph(const float4* centres, int64_t n, const float* feats, int D, int k,
                           const GraphWeights& gw, hipStream_t s, int32_t** row_ptr, int32_t** col,
                           float** val, int64_t* nnz);
// g0 = g on the ceil(fraction npos) largest positive entries (ties to the
// lower index), 0 elsewhere.
hipError_t launch_anchor_init(const float* g, int64_t n, float fraction, float* g0, hipStream_t s);
// h[i][c] = unary[i] where gT[i][c] > 0, else 0.
hipError_t launch_reach_unary(const float* gT, const float* unary, int64_t n, int D, float* h,
                              hipStream_t s);
// f = U / cnt per Gaussian (0 where cnt = 0).  Outputs of row i go to row
// perm[i] when perm is given (a scene stored in Morton order), else to i.
hipError_t launch_finalize_count(const float* U, const uint32_t* cnt, int64_t n, int D, float* f,
                                 const uint32_t* perm, bool fixed, hipStream_t s);
hipError_t launch_finalize(const float* U, const beta_t* beta, int64_t n, int D, float* f,
                           float* wsum, float* usum, const uint32_t* perm, hipStream_t s);
// The same for a fixed-point U (units of 2^-35): f = U / beta in FP64, rounded.
hipError_t launch_finalize_fixed(const long long* U, const beta_t* beta, int64_t n, int D, float* f,
                                 float* wsum, float* usum, const uint32_t* perm, hipStream_t s);

// Feature-map formats: valid uplift input, element type, pixel-block layout.
inline bool map_format_valid(lv_dtype d) { return d >= LV_F32 && d <= LV_FP8_E4M3_PX8; }
inline lv_dtype map_elem(lv_dtype d) { return d >= LV_F32_PX8 ? (lv_dtype)(d - LV_F32_PX8) : d; }
inline bool map_px8(lv_dtype d) { return d >= LV_F32_PX8; }

// Encode src [pixels][D] (HWC; pixels = H W) in format dtype; the pixel-block
// formats need the image width W.
hipError_t launch_encode(const float* src, int64_t pixels, int D, lv_dtype dtype, void* dst,
                         float* scales, float* tmp_absmax, hipStream_t s, int W = 0);

// One merged pass of the uplift server (see serve.hip): set k takes maps[k]
// (host array [m], NULL where the set lacks the view) and writes f and beta
// to its outputs.
struct BatchSet {
  const void* const* maps;
  const float* scales;
  int32_t stride;
  int32_t D;
  float* out_feat;
  float* out_wsum;
};
lv_status run_batch(lv_scene* sc, const lv_camera* cams, int32_t m, const BatchSet* sets,
                    int nsets, lv_dtype dtype, hipStream_t s);
// Records the formatted message as the calling thread's lv_last_error and
// returns st.
lv_status set_error(lv_status st, const char* fmt, ...);

hipError_t launch_diffuse(const int32_t* row_ptr, const int32_t* col, const void* val,
                          lv_dtype val_dtype, int64_t n, const void* g0, lv_dtype dtype, int D,
                          int steps, void* out, float* buf0, float* buf1, float* norms,
                          hipStream_t s);

// Locality order for diffusion: perm (new row -> old row) sorts the Gaussians
// by the Morton code of their centres (10 bits per axis over the bounding
// box); inv is its inverse; (rp2, col2, val2) is P A P^T.  scratch holds
// reorder_scratch_words(n) uint32.
size_t reorder_scratch_words(int64_t n);
hipError_t launch_graph_reorder(const float4* p0, int64_t n, const int32_t* rp, const int32_t* col,
                                const void* val, lv_dtype vt, int64_t nnz, uint32_t* scratch,
                                uint32_t* perm, uint32_t* inv, int32_t* rp2, int32_t* col2,
                                void* val2, hipStream_t s);
// Bounding box of the centres: box[0..2] the minima, box[3..5] the maxima,
// as order-preserving unsigned encodings of the FP32 values (sign bit
// flipped for non-negative values, all bits for negative ones).
hipError_t launch_scene_box(const float4* p0, int64_t n, uint32_t* box, hipStream_t s);
// The same Morton order without a graph: perm (position -> index) and its
// inverse; scratch holds reorder_scratch_words(n) uint32.
hipError_t launch_morton_order(const float4* p0, int64_t n, uint32_t* scratch, uint32_t* perm,
                               uint32_t* inv, hipStream_t s);
// Scene storage in that order: dst_k[i] = src_k[perm[i]] for the three
// derived arrays.
hipError_t launch_gather_scene(const float4* c0, const float4* c1, const float4* c2,
                               const uint32_t* perm, int64_t n, float4* p0, float4* p1, float4* p2,
                               hipStream_t s);
// Gaussians at exactly equal depth, stored in Morton order, back in the
// order of their caller index: within each run of equal (visible) depth keys
// of the depth-sorted views, (id, rect, count) sorted by perm[id].
hipError_t launch_depth_ties(const uint32_t* key, uint32_t* val, uint2* rect, uint32_t* cnt, int64_t n,
                             int mv, const uint32_t* perm, hipStream_t s);
// dst[r] = src[perm[r]] (gather) or dst[perm[r]] = src[r] (scatter), rows of D.
hipError_t launch_permute_rows(const void* src, void* dst, const uint32_t* perm, int64_t n, int D,
                               lv_dtype dt, bool scatter, hipStream_t s);

}  // namespace lv
