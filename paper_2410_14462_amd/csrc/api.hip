// C ABI (include/lv.h): argument checking, scratch management and the order
// of launches.  Per chunk of views the uplift runs
//   preprocess -> depth sort -> count scan -> duplicate -> tile sort ->
//   ranges -> blend-accumulate
// with a single stream synchronisation (the number of (tile, Gaussian) pairs
// sizes the pair buffers).  Scratch is cached per scene and only grows.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lv_internal.h"
#include <cmath>

using namespace lv;

namespace {

thread_local std::string g_err;

lv_status fail(lv_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      if (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)                     \
        return fail(LV_ERR_OUT_OF_MEMORY, "%s: %s", #expr, hipGetErrorString(e_));         \
      return fail(LV_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));                  \
    }                                                                                      \
  } while (0)

// The registered device allocator (lv_set_allocator) and the library's own
// account of the device memory it holds.
std::mutex g_alloc_mu;
lv_alloc_fn g_alloc_fn = nullptr;
lv_free_fn g_free_fn = nullptr;
void* g_alloc_ctx = nullptr;
std::atomic<int64_t> g_dev_bytes{0}, g_dev_allocs{0};

// Grow-only device buffer.
struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes, hipStream_t s) {
    if (bytes <= cap) return hipSuccess;
    if (p) {
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      lv::dev_free(p, cap, s);
      p = nullptr;
      cap = 0;
    }
    size_t want = bytes + bytes / 8 + 256;
    hipError_t e = lv::dev_alloc(&p, want, s);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  void release(hipStream_t s = nullptr) {
    if (p) lv::dev_free(p, cap, s);
    p = nullptr;
    cap = 0;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

struct HostBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) cap = bytes;
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Scratch of the uplift pipeline.  One workspace per (device, stream),
// created on first use and kept for the life of the process; calls on the
// same stream serialise on its mutex (they would serialise on the stream
// anyway).
struct Workspace {
  std::mutex mu;
  int64_t chunk_bytes = 0;  // scratch budget of a structure build (0: chunk_budget_bytes())
  std::mutex accmu;  // held by a one-call uplift while it uses accU/accB
  Buf accUs[kMaxSets], accBs[kMaxSets];
  const uint32_t* dkey = nullptr;  // depth-sorted keys / ids of the last structure build
  const uint32_t* dval = nullptr;
  Buf rec, key0, val0, key1, val1, rect, scnt, srect, off, scan_tmp, hist, seg, pseg, total;
  Buf pk0, pv0, pk1, pv1, hist2, ranges, cams, geom, maps;
  Buf cls;  // beta and count increments of classes of sets taking the same views
  HostBuf up, down;
};

std::mutex g_pool_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_pool;

Workspace* workspace_for(hipStream_t s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_pool_mu);
  Workspace*& w = g_pool[std::make_pair(dev, s)];
  if (!w) w = new Workspace();
  return w;
}

void workspace_free(Workspace* w, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(w->mu);
    for (int k = 0; k < kMaxSets; k++) {
      w->accUs[k].release(s);
      w->accBs[k].release(s);
    }
    Buf* bufs[] = {&w->rec, &w->key0, &w->val0, &w->key1, &w->val1, &w->rect, &w->scnt,
                   &w->srect, &w->off, &w->scan_tmp, &w->hist, &w->seg, &w->pseg, &w->total,
                   &w->pk0, &w->pv0, &w->pk1, &w->pv1, &w->hist2, &w->ranges, &w->cams,
                   &w->geom, &w->maps, &w->cls};
    for (Buf* b : bufs) b->release(s);
    w->up.release();
    w->down.release();
  }
  delete w;
}

// Blend-kernel timing (HIP events around every blend launch) for benchmarks.
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;

// Workspace bytes per (view, Gaussian) item of a structure build: record,
// two key/value buffers, rect (Gaussian and depth order), count (depth
// order), offset.
constexpr int64_t kItemBytes = sizeof(Rec) + 4 * 4 + 2 * 8 + 4 + 4;

// Digit width of the depth sort's passes (tile sort: kRadixBits).  With
// kSortItems items per block, narrower digits give longer runs of one digit
// and so better coalesced writes, at the cost of more passes.
#ifndef LV_DEPTH_PASS_BITS
#define LV_DEPTH_PASS_BITS 8
#endif
constexpr int kDepthPassBits = LV_DEPTH_PASS_BITS;

// Per-(view, Gaussian) scratch of one structure build: LV_CHUNK_BYTES, else a
// sixteenth of the device's memory clamped to [4, 16] GiB (16 GiB on a
// 288 GB MI355X: a million Gaussians over 100 views in one chunk).
int64_t chunk_budget_bytes(const Workspace* ws = nullptr) {
  if (ws && ws->chunk_bytes > 0) return ws->chunk_bytes;
  const char* e = getenv("LV_CHUNK_BYTES");
  if (e) {
    long long v = atoll(e);
    if (v > 0) return v;
  }
  size_t free_b = 0, total_b = 0;
  int64_t b = (int64_t)4 << 30;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
    b = std::max<int64_t>(b, std::min<int64_t>((int64_t)16 << 30, (int64_t)(total_b / 16)));
  return b;
}

}  // namespace

struct lv_scene {
  int64_t n = 0;
  int device = 0;
  Buf p0, p1, p2;  // derived parameters, in storage order
  // Morton storage order (unless LV_SCENE_CALLER_ORDER): perm maps a
  // storage index to the caller's index, inv the reverse; p0c is p0 in the
  // caller's order (the graph builder and the diffusion's own order read it)
  bool morton = false;
  Buf perm, inv, p0c;
  // bounding box of the centres (min x, y, z, max x, y, z), for the depth
  // keys' range
  bool has_box = false;
  double box[6] = {0, 0, 0, 0, 0, 0};
  const uint32_t* out_perm() const { return morton ? perm.as<uint32_t>() : nullptr; }
  const float4* caller_p0() const { return morton ? p0c.as<float4>() : p0.as<float4>(); }
};

struct lv_accum {
  lv_scene* scene = nullptr;
  int32_t D = 0;
  uint32_t flags = 0;
  bool fixed() const { return (flags & LV_ACCUM_DETERMINISTIC) != 0; }
  size_t u_elem_bytes() const { return fixed() ? 8 : 4; }
  Buf U, beta, counts, dstats;
  int64_t views = 0, pairs = 0, visible = 0;
};

struct lv_graph {
  int64_t n = 0, nnz = 0;
  lv_dtype val_dtype = LV_F32;
  Buf row_ptr, col, val, b0, b1, norms;
  // locality order (built on the first call that passes a scene)
  bool ordered = false;
  Buf perm, inv, rp2, col2, val2, bin, bout;
  // calls share the buffers above: each call's stream waits for the last one
  std::mutex mu;
  hipEvent_t last = nullptr;
};

namespace {

size_t dtype_size(lv_dtype d) { return d == LV_F32 ? 4 : d == LV_BF16 ? 2 : 1; }

lv_status check_cams(const lv_camera* cams, int32_t m) {
  if (m < 0) return fail(LV_ERR_INVALID_ARG, "m = %d < 0", m);
  if (m > 0 && !cams) return fail(LV_ERR_INVALID_ARG, "cams is NULL");
  for (int v = 0; v < m; v++) {
    const lv_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
      return fail(LV_ERR_INVALID_ARG, "camera %d: size %dx%d out of [1,16384]", v, c.width, c.height);
    if (c.reserved != 0) return fail(LV_ERR_INVALID_ARG, "camera %d: reserved must be 0", v);
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f))
      return fail(LV_ERR_INVALID_ARG, "camera %d: focal lengths must be > 0", v);
  }
  return LV_OK;
}

int ceil_log2(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) b++;
  return b;
}

// Structure of one chunk of views: everything up to the tile ranges.  On
// return, the sorted pair values (Gaussian ids) are in *ids, the ranges in
// ws.ranges with row stride *stride, and the pair count in *P.  If the chunk
// has more than one view and its pairs would reach 2^31 or need more than
// pair_budget bytes of pair buffers, *split is set and nothing past the pair
// count is built (the caller retries with fewer views).
// Bits of the depth keys the depth sort has to order.  A visible Gaussian's
// key is the FP32 bits of its view depth z_c > znear, which grow with z_c;
// over a chunk's views, z_c of a centre in the scene's box lies in
// [zlo, zhi] (the extremes of the box corners, in FP64), widened for the
// FP32 evaluation.  Keys whose bits above h are those of every key in that
// range sort on their h low bits; culled items (0xFFFFFFFF) still sort
// after them as long as the largest key's low h bits are not all ones.
int depth_key_bits(const lv_scene* sc, const lv_camera* cams, int mv) {
  if (!sc->has_box) return 32;
  double zlo = 1e300, zhi = -1e300, amax = 0.0;
  float znear = 3.4e38f;
  for (int v = 0; v < mv; v++) {
    const float* R = cams[v].R;
    for (int c = 0; c < 8; c++) {
      const double x = sc->box[(c & 1) ? 3 : 0], y = sc->box[(c & 2) ? 4 : 1], z = sc->box[(c & 4) ? 5 : 2];
      const double zc = (double)R[6] * x + (double)R[7] * y + (double)R[8] * z + (double)cams[v].t[2];
      zlo = std::min(zlo, zc);
      zhi = std::max(zhi, zc);
      amax = std::max(amax, std::fabs((double)R[6] * x) + std::fabs((double)R[7] * y) +
                                std::fabs((double)R[8] * z) + std::fabs((double)cams[v].t[2]));
    }
    znear = std::min(znear, cams[v].znear);
  }
  const double slack = 1e-5 * (amax + std::fabs(zlo) + std::fabs(zhi));  // far above FP32 rounding
  zlo -= slack;
  zhi += slack;
  if (!(zhi > (double)znear) || !(znear >= 0.0f) || !std::isfinite(zhi)) return 32;
  const float flo = zlo > (double)znear ? std::nextafter((float)zlo, 0.0f) : znear;
  const float fhi = std::nextafter((float)zhi, 3.4e38f);
  uint32_t klo, khi;
  memcpy(&klo, &flo, 4);
  memcpy(&khi, &fhi, 4);
  if (klo > khi) return 32;
  const uint32_t diff = klo ^ khi;
  const int h = diff ? 32 - __builtin_clz(diff) : 1;
  if (h >= 32) return 32;
  const uint32_t low = (1u << h) - 1u;
  if ((khi & low) == low) return 32;
  return h;
}


// Runs launch() (a kernel launch on s); while profiling is on (lv_profile_start)
// it is bracketed by HIP events on s.
template <typename F>
static lv_status profiled_launch(hipStream_t s, F&& launch) {
  std::lock_guard<std::mutex> pk(g_prof_mu);
  if (g_prof_on) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    HIP_TRY(launch());
    HIP_TRY(hipEventRecord(e1, s));
    g_prof_events.emplace_back(e0, e1);
  } else {
    HIP_TRY(launch());
  }
  return LV_OK;
}

lv_status build_structure(lv_scene* sc, Workspace& ws, const lv_camera* cams, int mv,
                          hipStream_t s, const uint32_t** ids, int* stride,
                          int64_t* P, int64_t* nvis, int* max_tiles_out,
                          int64_t pair_budget = INT64_MAX, bool* split = nullptr) {
  TraceRange tr("lv.structure");
  if (split) *split = false;
  const int64_t n = sc->n;
  const int64_t items = n * (int64_t)mv;
  std::vector<ViewGeom> geom(mv);
  int max_tiles = 0;
  for (int v = 0; v < mv; v++) {
    geom[v].W = cams[v].width;
    geom[v].H = cams[v].height;
    geom[v].TX = (cams[v].width + kTile - 1) / kTile;
    geom[v].TY = (cams[v].height + kTile - 1) / kTile;
    max_tiles = std::max(max_tiles, geom[v].TX * geom[v].TY);
  }
  *max_tiles_out = max_tiles;
  *stride = max_tiles;
  HIP_TRY(ws.rec.ensure(sizeof(Rec) * items, s));
  HIP_TRY(ws.key0.ensure(4 * items, s));
  HIP_TRY(ws.val0.ensure(4 * items, s));
  HIP_TRY(ws.key1.ensure(4 * items, s));
  HIP_TRY(ws.val1.ensure(4 * items, s));
  HIP_TRY(ws.rect.ensure(8 * items, s));
  HIP_TRY(ws.scnt.ensure(4 * items, s));
  HIP_TRY(ws.srect.ensure(8 * items, s));
  HIP_TRY(ws.off.ensure(4 * items, s));
  HIP_TRY(ws.scan_tmp.ensure(4 * scan_tmp_size(items), s));
  HIP_TRY(ws.hist.ensure(4 * sort_hist_size(mv, n), s));
  HIP_TRY(ws.seg.ensure(8 * (size_t)mv, s));
  HIP_TRY(ws.pseg.ensure(8 * (size_t)mv, s));
  HIP_TRY(ws.total.ensure(16, s));
  HIP_TRY(ws.cams.ensure(sizeof(Cam) * mv, s));
  HIP_TRY(ws.geom.ensure(sizeof(ViewGeom) * mv, s));
  HIP_TRY(ws.ranges.ensure(sizeof(uint2) * (size_t)mv * max_tiles, s));
  size_t up_bytes = sizeof(Cam) * mv + sizeof(ViewGeom) * mv + 8 * (size_t)mv;
  size_t down_bytes = 4 * ((size_t)mv + 8);
  // the pinned staging buffers may still feed an earlier upload on this stream
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(ws.up.ensure(up_bytes));
  HIP_TRY(ws.down.ensure(down_bytes));
  char* up = static_cast<char*>(ws.up.p);
  memcpy(up, cams, sizeof(Cam) * mv);
  memcpy(up + sizeof(Cam) * mv, geom.data(), sizeof(ViewGeom) * mv);
  uint32_t* segh = reinterpret_cast<uint32_t*>(up + sizeof(Cam) * mv + sizeof(ViewGeom) * mv);
  for (int v = 0; v < mv; v++) {
    segh[v] = (uint32_t)(v * n);
    segh[mv + v] = (uint32_t)n;
  }
  HIP_TRY(hipMemcpyAsync(ws.cams.p, up, sizeof(Cam) * mv, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws.geom.p, up + sizeof(Cam) * mv, sizeof(ViewGeom) * mv,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws.seg.p, segh, 8 * (size_t)mv, hipMemcpyHostToDevice, s));

  HIP_TRY(launch_preprocess(sc->p0.as<float4>(), sc->p1.as<float4>(), sc->p2.as<float4>(), n,
                            ws.cams.as<Cam>(), ws.geom.as<ViewGeom>(), mv, ws.rec.as<Rec>(),
                            ws.key0.as<uint32_t>(), ws.rect.as<uint2>(), s));
  bool second = false;
  const uint32_t* seg = ws.seg.as<uint32_t>();
  HIP_TRY(radix_sort(ws.key0.as<uint32_t>(), ws.val0.as<uint32_t>(), ws.key1.as<uint32_t>(),
                     ws.val1.as<uint32_t>(), seg, seg + mv, mv, n, depth_key_bits(sc, cams, mv),
                     ws.hist.as<uint32_t>(),
                     true, &second, s,
                     SortPayload{ws.rect.as<uint2>(), ws.scnt.as<uint32_t>(), ws.srect.as<uint2>()},
                     kDepthPassBits, true));
  const uint32_t* sval = second ? ws.val1.as<uint32_t>() : ws.val0.as<uint32_t>();
  ws.dkey = second ? ws.key1.as<uint32_t>() : ws.key0.as<uint32_t>();
  ws.dval = sval;
  if (sc->morton)  // equal depths blend in the caller's index order, as without the reorder
    HIP_TRY(launch_depth_ties(ws.dkey, const_cast<uint32_t*>(sval), ws.srect.as<uint2>(),
                              ws.scnt.as<uint32_t>(), n, mv, sc->perm.as<uint32_t>(), s));
  uint32_t* pseg = ws.pseg.as<uint32_t>();
  HIP_TRY(scan_counts(ws.scnt.as<uint32_t>(), nullptr, n, mv, ws.off.as<uint32_t>(), pseg, pseg + mv,
                      ws.total.as<unsigned long long>(), ws.scan_tmp.as<uint32_t>(), s));
  uint32_t* down = static_cast<uint32_t*>(ws.down.p);
  HIP_TRY(hipMemcpyAsync(down, ws.total.p, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(down + 4, pseg + mv, 4 * (size_t)mv, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const unsigned long long* tot64 = reinterpret_cast<const unsigned long long*>(down);
  uint64_t total = tot64[0];
  *nvis = (int64_t)tot64[1];
  if (split && mv > 1 && (total >= 0x80000000ull || (int64_t)total * 16 > pair_budget)) {
    *split = true;
    *P = (int64_t)total;
    return LV_OK;
  }
  if (total >= 0x80000000ull)
    return fail(LV_ERR_UNSUPPORTED, "%llu (tile, Gaussian) pairs in one view (limit 2^31)",
                (unsigned long long)total);
  int64_t max_len = 0;
  for (int v = 0; v < mv; v++) max_len = std::max<int64_t>(max_len, down[4 + v]);
  *P = (int64_t)total;
  // pair keys: the tile alone (16 bits; the sort is segmented by view) where
  // the tile ids fit, else view << 20 | tile
  const bool k16 = max_tiles <= 65536;
  const size_t kbytes = k16 ? 2 : 4;
  HIP_TRY(ws.pk0.ensure(kbytes * total + 16, s));
  HIP_TRY(ws.pv0.ensure(4 * total + 4, s));
  HIP_TRY(ws.pk1.ensure(kbytes * total + 16, s));
  HIP_TRY(ws.pv1.ensure(4 * total + 4, s));
  HIP_TRY(ws.hist2.ensure(4 * sort_hist_size(mv, max_len), s));
  if (k16)
    HIP_TRY(launch_duplicate16(sval, ws.off.as<uint32_t>(), ws.srect.as<uint2>(), ws.scnt.as<uint32_t>(),
                               ws.geom.as<ViewGeom>(), n, mv, ws.pk0.as<uint16_t>(), ws.pv0.as<uint32_t>(), s));
  else
    HIP_TRY(launch_duplicate(sval, ws.off.as<uint32_t>(), ws.srect.as<uint2>(), ws.scnt.as<uint32_t>(),
                             ws.geom.as<ViewGeom>(), n, mv, ws.pk0.as<uint32_t>(), ws.pv0.as<uint32_t>(), s));
  // one pass (up to 2048 tiles): the tile ranges come from the pass's scanned
  // counts and the sorted keys are not written; else from the sorted keys
  const int tile_bits = ceil_log2(max_tiles);
  const bool one_pass = total > 0 && radix_passes(tile_bits) == 1;
  if (k16)
    HIP_TRY(radix_sort16(ws.pk0.as<uint16_t>(), ws.pv0.as<uint32_t>(), ws.pk1.as<uint16_t>(),
                         ws.pv1.as<uint32_t>(), pseg, pseg + mv, mv, max_len, tile_bits,
                         ws.hist2.as<uint32_t>(), !one_pass, &second, s));
  else
    HIP_TRY(radix_sort(ws.pk0.as<uint32_t>(), ws.pv0.as<uint32_t>(), ws.pk1.as<uint32_t>(),
                       ws.pv1.as<uint32_t>(), pseg, pseg + mv, mv, max_len, tile_bits,
                       ws.hist2.as<uint32_t>(), !one_pass, &second, s));
  *ids = second ? ws.pv1.as<uint32_t>() : ws.pv0.as<uint32_t>();
  if (one_pass) {
    HIP_TRY(launch_hist_ranges(ws.hist2.as<uint32_t>(), pseg, pseg + mv, mv, max_len, tile_bits,
                               max_tiles, ws.ranges.as<uint2>(), s));
  } else {
    HIP_TRY(hipMemsetAsync(ws.ranges.p, 0, sizeof(uint2) * (size_t)mv * max_tiles, s));
    if (k16)
      HIP_TRY(launch_ranges16(second ? ws.pk1.as<uint16_t>() : ws.pk0.as<uint16_t>(), pseg, pseg + mv, mv,
                              max_len, max_tiles, ws.ranges.as<uint2>(), s));
    else
      HIP_TRY(launch_ranges(second ? ws.pk1.as<uint32_t>() : ws.pk0.as<uint32_t>(), (int64_t)total, max_tiles,
                            ws.ranges.as<uint2>(), s));
  }
  return LV_OK;
}

lv_status check_maps(const void* const* maps, int32_t m, lv_dtype dtype, const float* scales,
                     bool allow_null = false) {
  if (!map_format_valid(dtype)) return fail(LV_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
  if (m > 0 && !maps) return fail(LV_ERR_INVALID_ARG, "maps is NULL");
  for (int v = 0; v < m && !allow_null; v++)
    if (!maps[v]) return fail(LV_ERR_INVALID_ARG, "maps[%d] is NULL", v);
  if (map_elem(dtype) == LV_FP8_E4M3 && m > 0 && !scales)
    return fail(LV_ERR_INVALID_ARG, "FP8 maps need scales");
  if (map_px8(dtype)) {  // the blocks are read whole
    const uintptr_t align = map_elem(dtype) == LV_F32 ? 16 : map_elem(dtype) == LV_BF16 ? 16 : 8;
    for (int v = 0; v < m; v++)
      if (maps[v] && (uintptr_t)maps[v] % align)
        return fail(LV_ERR_INVALID_ARG, "maps[%d] is not %d-byte aligned", v, (int)align);
  }
  return LV_OK;
}

}  // namespace

namespace lv {

hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s, bool temp) {
  lv_alloc_fn fn;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    fn = g_alloc_fn;
    ctx = g_alloc_ctx;
  }
  hipError_t e;
  if (fn) {
    *p = fn(bytes, s, ctx);
    e = *p ? hipSuccess : hipErrorOutOfMemory;
  } else {
    e = temp ? hipMallocAsync(p, bytes, s) : hipMalloc(p, bytes);
    if (e != hipSuccess) *p = nullptr;
  }
  if (e == hipSuccess) {
    g_dev_bytes += (int64_t)bytes;
    g_dev_allocs += 1;
  }
  return e;
}

void dev_free(void* p, size_t bytes, hipStream_t s, bool temp) {
  if (!p) return;
  lv_free_fn fn;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    fn = g_free_fn;
    ctx = g_alloc_ctx;
  }
  if (fn)
    fn(p, bytes, s, ctx);
  else if (temp)
    (void)hipFreeAsync(p, s);
  else
    (void)hipFree(p);
  g_dev_bytes -= (int64_t)bytes;
  g_dev_allocs -= 1;
}

// Frees the workspace of stream s (the caller guarantees it is idle).
void release_workspace(hipStream_t s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  Workspace* w = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pool.find(std::make_pair(dev, s));
    if (it == g_pool.end()) return;
    w = it->second;
    g_pool.erase(it);
  }
  (void)hipStreamSynchronize(s);
  workspace_free(w, s);
}

// Caps the structure-build scratch of stream s's workspace (items and pairs
// each at most `bytes`).
void limit_workspace(hipStream_t s, int64_t bytes) {
  Workspace* w = workspace_for(s);
  std::lock_guard<std::mutex> lk(w->mu);
  w->chunk_bytes = bytes;
}

}  // namespace lv

namespace {
void scene_cache_clear();
}

extern "C" {

const char* lv_last_error(void) { return g_err.c_str(); }

lv_status lv_release_scratch(void* stream, int32_t all_streams) {
  if (!all_streams) {
    lv::release_workspace(static_cast<hipStream_t>(stream));
    return LV_OK;
  }
  std::vector<Workspace*> ws;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto& e : g_pool) ws.push_back(e.second);
    g_pool.clear();
  }
  HIP_TRY(hipDeviceSynchronize());
  for (Workspace* w : ws) workspace_free(w, nullptr);
  scene_cache_clear();
  return LV_OK;
}

lv_status lv_set_allocator(lv_alloc_fn alloc, lv_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(LV_ERR_INVALID_ARG, "alloc and free must both be set or both be NULL");
  lv_status st = lv_release_scratch(nullptr, 1);
  if (st != LV_OK) return st;
  if (g_dev_allocs.load() != 0)
    return fail(LV_ERR_INVALID_ARG, "%lld device allocations of live handles are outstanding",
                (long long)g_dev_allocs.load());
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc_fn = alloc;
  g_free_fn = free_fn;
  g_alloc_ctx = ctx;
  return LV_OK;
}

lv_status lv_memory_stats(int64_t* bytes, int64_t* allocations) {
  if (bytes) *bytes = g_dev_bytes.load();
  if (allocations) *allocations = g_dev_allocs.load();
  return LV_OK;
}

const char* lv_version(void) { return "lv 0.1 gfx950"; }

namespace {
// Device buffers of destroyed scenes, kept for the next scenes of a similar
// size (a scene that is created and destroyed per request then costs no
// allocation); bounded in count and bytes, buffers above kSceneCacheMaxBuf
// are freed at once.
std::mutex g_scene_cache_mu;
std::vector<std::pair<int, Buf>> g_scene_cache;
constexpr size_t kSceneCacheBufs = 12;
constexpr size_t kSceneCacheMaxBuf = (size_t)256 << 20;
constexpr size_t kSceneCacheBytes = (size_t)1 << 30;

hipError_t scene_buf(Buf& out, int dev, size_t bytes, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_scene_cache_mu);
    int best = -1;
    for (size_t i = 0; i < g_scene_cache.size(); i++) {
      const Buf& b = g_scene_cache[i].second;
      if (g_scene_cache[i].first == dev && b.cap >= bytes && b.cap <= 2 * bytes + 4096 &&
          (best < 0 || b.cap < g_scene_cache[best].second.cap))
        best = (int)i;
    }
    if (best >= 0) {
      out = g_scene_cache[best].second;
      g_scene_cache.erase(g_scene_cache.begin() + best);
      return hipSuccess;
    }
  }
  return out.ensure(bytes, s);
}

void scene_cache_clear() {
  std::lock_guard<std::mutex> lk(g_scene_cache_mu);
  for (auto& e : g_scene_cache) e.second.release();
  g_scene_cache.clear();
}

// After the device has finished with the buffer (the caller synchronised).
void scene_buf_release(int dev, Buf& b) {
  if (!b.p) return;
  if (b.cap > kSceneCacheMaxBuf) {
    b.release();
    return;
  }
  std::lock_guard<std::mutex> lk(g_scene_cache_mu);
  g_scene_cache.emplace_back(dev, b);
  b.p = nullptr;
  b.cap = 0;
  size_t total = 0;
  for (const auto& e : g_scene_cache) total += e.second.cap;
  while (!g_scene_cache.empty() && (g_scene_cache.size() > kSceneCacheBufs || total > kSceneCacheBytes)) {
    total -= g_scene_cache.front().second.cap;
    g_scene_cache.front().second.release();
    g_scene_cache.erase(g_scene_cache.begin());
  }
}
}  // namespace

lv_status lv_scene_create(const float* means, const float* scales, const float* quats,
                          const float* opacity, int64_t n, const lv_scene_opts* opts, void* stream,
                          lv_scene** out) {
  if (!out) return fail(LV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (opts) {
    // the kernels are compiled for the default constants (FP32 literals)
    const bool dflt = opts->alpha_max == kAlphaMax && opts->alpha_min == kAlphaMin &&
                      opts->t_eps == kTEps && opts->dilation == kDilate && opts->tile == kTile;
    if (!dflt)
      return fail(LV_ERR_UNSUPPORTED,
                  "scene constants other than alpha_max 0.99, alpha_min 1/255, t_eps 1e-4, "
                  "dilation 0.3, tile 16 are not supported by this build");
  }
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(LV_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n > 0 && (!means || !scales || !quats || !opacity))
    return fail(LV_ERR_INVALID_ARG, "null scene array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv_scene* sc = new (std::nothrow) lv_scene();
  if (!sc) return fail(LV_ERR_OUT_OF_MEMORY, "host allocation");
  sc->n = n;
  (void)hipGetDevice(&sc->device);
  sc->morton = n > 1 && !(opts && (opts->flags & LV_SCENE_CALLER_ORDER));
  size_t b = sizeof(float4) * (size_t)(n > 0 ? n : 1);
  hipError_t e = scene_buf(sc->p0, sc->device, b, s);
  if (e == hipSuccess) e = scene_buf(sc->p1, sc->device, b, s);
  if (e == hipSuccess) e = scene_buf(sc->p2, sc->device, b, s);
  if (e == hipSuccess && !sc->morton)
    e = launch_scene_derive(means, scales, quats, opacity, n, sc->p0.as<float4>(), sc->p1.as<float4>(),
                            sc->p2.as<float4>(), s);
  if (e == hipSuccess && sc->morton) {
    // derive in the caller's order, order by the Morton code of the
    // centres (stable: equal codes keep the caller's order), gather
    void* c12 = nullptr;
    void* scratch = nullptr;
    const size_t scratch_bytes = 4 * reorder_scratch_words(n);
    e = scene_buf(sc->p0c, sc->device, b, s);
    if (e == hipSuccess) e = scene_buf(sc->perm, sc->device, 4 * (size_t)n, s);
    if (e == hipSuccess) e = scene_buf(sc->inv, sc->device, 4 * (size_t)n, s);
    if (e == hipSuccess) e = dev_alloc(&c12, 2 * b, s, true);
    if (e == hipSuccess) e = dev_alloc(&scratch, scratch_bytes, s, true);
    float4* c1 = static_cast<float4*>(c12);
    if (e == hipSuccess)
      e = launch_scene_derive(means, scales, quats, opacity, n, sc->p0c.as<float4>(), c1, c1 + n, s);
    if (e == hipSuccess)
      e = launch_morton_order(sc->p0c.as<float4>(), n, static_cast<uint32_t*>(scratch),
                              sc->perm.as<uint32_t>(), sc->inv.as<uint32_t>(), s);
    if (e == hipSuccess)
      e = launch_gather_scene(sc->p0c.as<float4>(), c1, c1 + n, sc->perm.as<uint32_t>(), n,
                              sc->p0.as<float4>(), sc->p1.as<float4>(), sc->p2.as<float4>(), s);
    dev_free(scratch, scratch_bytes, s, true);
    dev_free(c12, 2 * b, s, true);
  }
  if (e == hipSuccess && n > 0) {
    // the box on the host (one small read back): bounds of the depth keys
    void* bx = nullptr;
    uint32_t hb[6];
    e = dev_alloc(&bx, 32, s, true);
    if (e == hipSuccess) e = launch_scene_box(sc->p0.as<float4>(), n, static_cast<uint32_t*>(bx), s);
    if (e == hipSuccess) e = hipMemcpyAsync(hb, bx, 24, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(bx, 32, s, true);
    if (e == hipSuccess) {
      for (int k = 0; k < 6; k++) {
        const uint32_t u = (hb[k] & 0x80000000u) ? (hb[k] & 0x7FFFFFFFu) : ~hb[k];
        float f;
        memcpy(&f, &u, 4);
        sc->box[k] = (double)f;
      }
      sc->has_box = std::isfinite(sc->box[0]) && std::isfinite(sc->box[1]) && std::isfinite(sc->box[2]) &&
                    std::isfinite(sc->box[3]) && std::isfinite(sc->box[4]) && std::isfinite(sc->box[5]);
    }
  }
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    sc->p0.release(); sc->p1.release(); sc->p2.release();
    sc->p0c.release(); sc->perm.release(); sc->inv.release();
    delete sc;
    return fail(e == hipErrorOutOfMemory ? LV_ERR_OUT_OF_MEMORY : LV_ERR_DEVICE, "scene: %s",
                hipGetErrorString(e));
  }
  *out = sc;
  return LV_OK;
}

lv_status lv_scene_destroy(lv_scene* sc) {
  if (!sc) return LV_OK;
  int cur = sc->device;
  (void)hipGetDevice(&cur);
  if (cur != sc->device) (void)hipSetDevice(sc->device);
  (void)hipDeviceSynchronize();
  if (cur != sc->device) (void)hipSetDevice(cur);
  scene_buf_release(sc->device, sc->p0);
  scene_buf_release(sc->device, sc->p1);
  scene_buf_release(sc->device, sc->p2);
  scene_buf_release(sc->device, sc->p0c);
  scene_buf_release(sc->device, sc->perm);
  scene_buf_release(sc->device, sc->inv);
  delete sc;
  return LV_OK;
}

int64_t lv_scene_size(const lv_scene* sc) { return sc ? sc->n : -1; }

lv_status lv_accum_create(lv_scene* sc, int32_t D, uint32_t flags, void* stream, lv_accum** out) {
  if (!out) return fail(LV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!sc) return fail(LV_ERR_INVALID_ARG, "scene is NULL");
  if (D < 1 || D > 4096) return fail(LV_ERR_INVALID_ARG, "D = %d out of [1, 4096]", D);
  if (flags & ~(LV_ACCUM_COUNTS | LV_ACCUM_DETERMINISTIC))
    return fail(LV_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv_accum* a = new (std::nothrow) lv_accum();
  if (!a) return fail(LV_ERR_OUT_OF_MEMORY, "host allocation");
  a->scene = sc;
  a->D = D;
  a->flags = flags;
  size_t n1 = (size_t)(sc->n > 0 ? sc->n : 1);
  hipError_t e = a->U.ensure(a->u_elem_bytes() * n1 * D, s);
  if (e == hipSuccess) e = a->beta.ensure(sizeof(beta_t) * n1, s);
  if (e == hipSuccess && (flags & LV_ACCUM_COUNTS)) e = a->counts.ensure(4 * n1, s);
  if (e == hipSuccess && (flags & LV_ACCUM_COUNTS)) e = a->dstats.ensure(24, s);
  if (e != hipSuccess) {
    a->U.release(); a->beta.release(); a->counts.release(); a->dstats.release();
    delete a;
    return fail(LV_ERR_OUT_OF_MEMORY, "accumulator: %s", hipGetErrorString(e));
  }
  lv_status st = lv_accum_reset(a, stream);
  if (st != LV_OK) {
    lv_accum_destroy(a);
    return st;
  }
  *out = a;
  return LV_OK;
}

lv_status lv_accum_reset(lv_accum* a, void* stream) {
  if (!a) return fail(LV_ERR_INVALID_ARG, "accumulator is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  size_t n = (size_t)a->scene->n;
  a->views = a->pairs = a->visible = 0;
  if (a->dstats.p) HIP_TRY(hipMemsetAsync(a->dstats.p, 0, 24, s));
  if (n == 0) return LV_OK;
  HIP_TRY(hipMemsetAsync(a->U.p, 0, a->u_elem_bytes() * n * a->D, s));
  HIP_TRY(hipMemsetAsync(a->beta.p, 0, sizeof(beta_t) * n, s));
  if (a->counts.p) HIP_TRY(hipMemsetAsync(a->counts.p, 0, 4 * n, s));
  return LV_OK;
}

lv_status lv_accum_destroy(lv_accum* a) {
  if (!a) return LV_OK;
  (void)hipDeviceSynchronize();
  a->U.release(); a->beta.release(); a->counts.release(); a->dstats.release();
  delete a;
  return LV_OK;
}

lv_status lv_uplift_accumulate_sets(const lv_camera* cams, int32_t m, const lv_feature_set* fsets,
                                   int32_t nsets, lv_dtype dtype, void* stream) {
  TraceRange tr("lv.uplift_accumulate");
  if (nsets < 1 || nsets > kMaxSets)
    return fail(LV_ERR_INVALID_ARG, "nsets = %d out of [1, %d]", nsets, kMaxSets);
  if (!fsets) return fail(LV_ERR_INVALID_ARG, "sets is NULL");
  lv_status st = check_cams(cams, m);
  if (st != LV_OK) return st;
  lv_scene* sc = nullptr;
  int total = 0;
  for (int k = 0; k < nsets; k++) {
    if (!fsets[k].acc) return fail(LV_ERR_INVALID_ARG, "set %d: accumulator is NULL", k);
    if (sc && fsets[k].acc->scene != sc)
      return fail(LV_ERR_INVALID_ARG, "set %d: accumulators belong to different scenes", k);
    for (int q = 0; q < k; q++)
      if (fsets[q].acc == fsets[k].acc)
        return fail(LV_ERR_INVALID_ARG, "set %d repeats the accumulator of set %d", k, q);
    if (fsets[k].acc->fixed() != fsets[0].acc->fixed())
      return fail(LV_ERR_INVALID_ARG, "set %d: deterministic and FP32 accumulators in one call", k);
    sc = fsets[k].acc->scene;
    st = check_maps(fsets[k].maps, m, dtype, fsets[k].scales, true);
    if (st != LV_OK) return st;
    if (fsets[k].stride != 0 && fsets[k].stride < fsets[k].acc->D)
      return fail(LV_ERR_INVALID_ARG, "set %d: pixel stride %d < D = %d", k, fsets[k].stride,
                  fsets[k].acc->D);
    total += fsets[k].acc->D;
  }
  const int64_t n = sc->n;
  if (n == 0 || m == 0) return LV_OK;

  // Sets that take exactly the same views receive the same weights, hence the
  // same beta and count increments: the blend adds those once per class (into
  // class accumulators, by the first member) and a small kernel adds them to
  // every member.  cls[k] = first set of k's class.
  int cls[kMaxSets], members[kMaxSets] = {0};
  for (int k = 0; k < nsets; k++) {
    cls[k] = k;
    for (int q = 0; q < k && cls[k] == k; q++) {
      if (cls[q] != q) continue;
      bool same = true;
      for (int v = 0; v < m && same; v++)
        same = (fsets[q].maps[v] == nullptr) == (fsets[k].maps[v] == nullptr);
      if (same) cls[k] = q;
    }
    members[cls[k]]++;
  }
  int slot[kMaxSets], nslots = 0;  // class accumulator slot of each shared class
  for (int k = 0; k < nsets; k++) slot[k] = (cls[k] == k && members[k] > 1) ? nslots++ : -1;

  // channel groups: the sets' channels concatenated and cut into groups of
  // 64, a last part of <= kMaxTail channels joining the previous group as its
  // tail
  std::vector<ChanGroup> groups;
  {
    // 64-channel main parts; a last part of <= 4 channels becomes the tail
    // of the previous group (or the only channels of a group without a
    // main part)
    std::vector<int> starts;
    for (int b = 0; b < total; b += 64) starts.push_back(b);
    int tail_lo = total;
    if (total - starts.back() <= kMaxTail) {
      tail_lo = starts.back();
      starts.pop_back();
      if (starts.empty()) starts.push_back(0);
    }
    for (size_t gi = 0; gi < starts.size(); gi++) {
      const bool last = gi + 1 == starts.size();
      const int lo = starts[gi], hi = last ? std::min(total, tail_lo) : starts[gi + 1];
      const int thi = last ? total : hi;  // channels [hi, thi) form the tail
      ChanGroup g;
      memset(&g, 0, sizeof(g));
      g.width = hi - lo;
      int off = 0;
      for (int k = 0; k < nsets; k++) {
        const int D = fsets[k].acc->D;
        const int a0 = std::max(lo, off), a1 = std::min(hi, off + D);
        if (a0 < a1) {
          if (g.nseg == kMaxSegs)
            return fail(LV_ERR_UNSUPPORTED, "more than %d feature sets share 64 channels", kMaxSegs);
          g.set[g.nseg] = k;
          g.c0[g.nseg] = a0 - off;
          g.vc0[g.nseg] = a0 - lo;
          g.cnt[g.nseg] = a1 - a0;
          g.nseg++;
        }
        for (int c = std::max(hi, off); c < std::min(thi, off + D); c++) {
          g.tset[g.ntail] = k;
          g.tc[g.ntail] = c - off;
          g.ntail++;
        }
        if (off >= lo && off < thi) {
          g.stats_sets |= 1 << k;
          if (cls[k] == k) g.beta_sets |= 1 << k;
        }
        off += D;
      }
      groups.push_back(g);
    }
  }
  int max_width = 0;
  for (const ChanGroup& g : groups) max_width = std::max(max_width, g.width);

  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace& ws = *workspace_for(s);
  std::lock_guard<std::mutex> lk(ws.mu);
  if (nslots) HIP_TRY(ws.cls.ensure((size_t)nslots * n * 12, s));
  const int64_t per_view = n * kItemBytes;
  const int64_t budget = chunk_budget_bytes(&ws);
  int64_t mc = std::max<int64_t>(1, std::min<int64_t>(m, budget / per_view));
  mc = std::min<int64_t>(mc, 1 << (31 - kViewShift));
  for (int v0 = 0; v0 < m;) {
    int mv = (int)std::min<int64_t>(mc, m - v0);
    const uint32_t* ids = nullptr;
    int stride = 0, max_tiles = 0;
    int64_t P = 0, nvis = 0;
    bool split = false;
    st = build_structure(sc, ws, cams + v0, mv, s, &ids, &stride, &P, &nvis, &max_tiles, budget, &split);
    if (st != LV_OK) return st;
    if (split) {  // too many pairs for the chunk: fewer views per chunk, same views again
      const double fit = (double)std::min<int64_t>(budget / 16, 0x7FFFFFFF) / (double)P;
      mc = std::max<int64_t>(1, std::min<int64_t>(mv - 1, (int64_t)(mv * fit * 0.9)));
      continue;
    }
    for (int k = 0; k < nsets; k++) {
      fsets[k].acc->views += mv;
      fsets[k].acc->pairs += P;
      fsets[k].acc->visible += nvis;
    }
    // set descriptors, channel groups and per-set map tables in one upload
    // (ws.up is idle: build_structure synchronised the stream)
    const size_t b_sets = sizeof(SetDesc) * nsets;
    const size_t b_groups = sizeof(ChanGroup) * groups.size();
    const size_t b_maps = sizeof(void*) * (size_t)mv * nsets;
    const size_t bytes = b_sets + b_groups + b_maps;
    HIP_TRY(ws.maps.ensure(bytes, s));
    HIP_TRY(ws.up.ensure(bytes));
    char* up = static_cast<char*>(ws.up.p);
    char* dev = static_cast<char*>(ws.maps.p);
    SetDesc* sd = reinterpret_cast<SetDesc*>(up);
    const void** mt = reinterpret_cast<const void**>(up + b_sets + b_groups);
    for (int k = 0; k < nsets; k++) {
      lv_accum* a = fsets[k].acc;
      memcpy(mt + (size_t)k * mv, fsets[k].maps + v0, sizeof(void*) * mv);
      sd[k].maps = reinterpret_cast<const void* const*>(dev + b_sets + b_groups) + (size_t)k * mv;
      sd[k].scales = fsets[k].scales;
      sd[k].U = a->U.as<float>();
      sd[k].fixed = a->fixed() ? 1 : 0;
      sd[k].beta = a->beta.as<beta_t>();
      sd[k].counts = a->counts.as<uint32_t>();
      sd[k].stats = a->dstats.as<unsigned long long>();
      sd[k].D = a->D;
      sd[k].stride = fsets[k].stride ? fsets[k].stride : a->D;
      sd[k].view_base = v0;
      if (slot[k] >= 0) {  // shared class: its increments go to the class accumulators
        char* c = ws.cls.as<char>() + (size_t)slot[k] * n * 12;
        sd[k].beta = reinterpret_cast<beta_t*>(c);
        bool any_counts = false;
        for (int q = 0; q < nsets; q++) any_counts = any_counts || (cls[q] == k && fsets[q].acc->counts.p);
        sd[k].counts = any_counts ? reinterpret_cast<uint32_t*>(c + (size_t)n * 8) : nullptr;
      }
    }
    if (b_groups) memcpy(up + b_sets, groups.data(), b_groups);
    HIP_TRY(hipMemcpyAsync(dev, up, bytes, hipMemcpyHostToDevice, s));
    if (nslots) HIP_TRY(hipMemsetAsync(ws.cls.p, 0, (size_t)nslots * n * 12, s));
    BlendArgs ba;
    ba.rec = ws.rec.as<Rec>();
    ba.ids = ids;
    ba.ranges = ws.ranges.as<uint2>();
    ba.geom = ws.geom.as<ViewGeom>();
    ba.n = n;
    ba.tiles_stride = stride;
    ba.sets = reinterpret_cast<const SetDesc*>(dev);
    ba.groups = reinterpret_cast<const ChanGroup*>(dev + b_sets);
    ba.ngroups = (int32_t)groups.size();
    ba.max_width = max_width;
    ba.has_tail = !groups.empty() && groups.back().ntail > 0 ? 1 : 0;
    {
      TraceRange tb("lv.blend");
      st = profiled_launch(s, [&] { return launch_blend(ba, dtype, mv, s); });
      if (st != LV_OK) return st;
    }
    for (int k = 0; k < nsets; k++) {
      if (slot[k] < 0) continue;
      ClassAdd dst;
      memset(&dst, 0, sizeof(dst));
      for (int q = 0; q < nsets; q++) {
        if (cls[q] != k) continue;
        dst.beta[dst.nd] = fsets[q].acc->beta.as<beta_t>();
        dst.counts[dst.nd] = fsets[q].acc->counts.as<uint32_t>();
        dst.nd++;
      }
      const char* c = ws.cls.as<char>() + (size_t)slot[k] * n * 12;
      HIP_TRY(launch_class_add(reinterpret_cast<const beta_t*>(c), sd[k].counts ? reinterpret_cast<const uint32_t*>(c + (size_t)n * 8) : nullptr, dst, n, s));
    }
    v0 += mv;
    if (v0 < m) HIP_TRY(hipStreamSynchronize(s));  // staging buffers are reused
  }
  return LV_OK;
}

lv_status lv_uplift_accumulate(lv_accum* a, const lv_camera* cams, int32_t m, const void* const* maps,
                               lv_dtype dtype, const float* scales, void* stream) {
  if (!a) return fail(LV_ERR_INVALID_ARG, "accumulator is NULL");
  lv_feature_set fs;
  lv_status st = check_maps(maps, m, dtype, scales);
  if (st != LV_OK) return st;
  fs.acc = a;
  fs.maps = maps;
  fs.scales = scales;
  fs.stride = 0;
  return lv_uplift_accumulate_sets(cams, m, &fs, 1, dtype, stream);
}

lv_status lv_accum_finalize(lv_accum* a, float* out_feat, float* out_wsum, float* out_sum,
                            void* stream) {
  if (!a) return fail(LV_ERR_INVALID_ARG, "accumulator is NULL");
  if (a->scene->n > 0 && !out_feat && !out_wsum && !out_sum)
    return fail(LV_ERR_INVALID_ARG, "no output requested");
  TraceRange tr("lv.finalize");
  if (a->fixed())
    HIP_TRY(launch_finalize_fixed(a->U.as<long long>(), a->beta.as<beta_t>(), a->scene->n, a->D, out_feat,
                                  out_wsum, out_sum, a->scene->out_perm(), static_cast<hipStream_t>(stream)));
  else
    HIP_TRY(launch_finalize(a->U.as<float>(), a->beta.as<beta_t>(), a->scene->n, a->D, out_feat,
                            out_wsum, out_sum, a->scene->out_perm(), static_cast<hipStream_t>(stream)));
  return LV_OK;
}

namespace {
// rows of `words` 32-bit words, storage order <-> the caller's order
hipError_t move_rows(const void* src, void* dst, int64_t n, int words, const lv_scene* sc, bool to_caller,
                     hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!sc->morton)
    return hipMemcpyAsync(dst, src, 4 * (size_t)n * words, hipMemcpyDeviceToDevice, s);
  return launch_permute_rows(src, dst, sc->perm.as<uint32_t>(), n, words, LV_F32, to_caller, s);
}
}  // namespace

lv_status lv_accum_export(lv_accum* a, void* U, uint64_t* beta, uint32_t* counts, void* stream) {
  if (!a) return fail(LV_ERR_INVALID_ARG, "accumulator is NULL");
  const int64_t n = a->scene->n;
  if (n > 0 && (!U || !beta)) return fail(LV_ERR_INVALID_ARG, "U or beta is NULL");
  if (counts && !(a->flags & LV_ACCUM_COUNTS))
    return fail(LV_ERR_INVALID_ARG, "counts requested from an accumulator without LV_ACCUM_COUNTS");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int uw = (int)(a->u_elem_bytes() / 4) * a->D;
  HIP_TRY(move_rows(a->U.p, U, n, uw, a->scene, true, s));
  HIP_TRY(move_rows(a->beta.p, beta, n, 2, a->scene, true, s));
  if (counts) HIP_TRY(move_rows(a->counts.p, counts, n, 1, a->scene, true, s));
  return LV_OK;
}

lv_status lv_accum_import(lv_accum* a, const void* U, const uint64_t* beta, const uint32_t* counts,
                          void* stream) {
  if (!a) return fail(LV_ERR_INVALID_ARG, "accumulator is NULL");
  const int64_t n = a->scene->n;
  if (n > 0 && (!U || !beta)) return fail(LV_ERR_INVALID_ARG, "U or beta is NULL");
  if (counts && !(a->flags & LV_ACCUM_COUNTS))
    return fail(LV_ERR_INVALID_ARG, "counts given to an accumulator without LV_ACCUM_COUNTS");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int uw = (int)(a->u_elem_bytes() / 4) * a->D;
  HIP_TRY(move_rows(U, a->U.p, n, uw, a->scene, false, s));
  HIP_TRY(move_rows(beta, a->beta.p, n, 2, a->scene, false, s));
  if (a->counts.p && n > 0) {
    if (counts)
      HIP_TRY(move_rows(counts, a->counts.p, n, 1, a->scene, false, s));
    else
      HIP_TRY(hipMemsetAsync(a->counts.p, 0, 4 * (size_t)n, s));
  }
  return LV_OK;
}

lv_status lv_accum_finalize_count(lv_accum* a, float* out_feat, void* stream) {
  if (!a) return fail(LV_ERR_INVALID_ARG, "accumulator is NULL");
  if (!(a->flags & LV_ACCUM_COUNTS)) return fail(LV_ERR_INVALID_ARG, "created without LV_ACCUM_COUNTS");
  if (a->scene->n > 0 && !out_feat) return fail(LV_ERR_INVALID_ARG, "out_feat is NULL");
  HIP_TRY(launch_finalize_count(a->U.as<float>(), a->counts.as<uint32_t>(), a->scene->n, a->D,
                                out_feat, a->scene->out_perm(), a->fixed(), static_cast<hipStream_t>(stream)));
  return LV_OK;
}

lv_status lv_prune_by_weight(const float* wsum, int64_t n, int64_t k, uint8_t* keep, void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(LV_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (k < 0 || k > n) return fail(LV_ERR_INVALID_ARG, "k = %lld not in [0, n = %lld]", (long long)k, (long long)n);
  if (n > 0 && (!wsum || !keep)) return fail(LV_ERR_INVALID_ARG, "null buffer");
  HIP_TRY(launch_prune(wsum, n, k, keep, static_cast<hipStream_t>(stream)));
  return LV_OK;
}

lv_status lv_anchor_init(const float* g, int64_t n, float fraction, float* g0, void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(LV_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (!(fraction > 0.0f && fraction <= 1.0f)) return fail(LV_ERR_INVALID_ARG, "fraction must be in (0, 1]");
  if (n > 0 && (!g || !g0)) return fail(LV_ERR_INVALID_ARG, "null buffer");
  HIP_TRY(launch_anchor_init(g, n, fraction, g0, static_cast<hipStream_t>(stream)));
  return LV_OK;
}

lv_status lv_reach_unary(const float* gT, const float* unary, int64_t n, int32_t D, float* h,
                         void* stream) {
  if (n < 0 || D < 1) return fail(LV_ERR_INVALID_ARG, "bad size");
  if (n > 0 && (!gT || !unary || !h)) return fail(LV_ERR_INVALID_ARG, "null buffer");
  HIP_TRY(launch_reach_unary(gT, unary, n, D, h, static_cast<hipStream_t>(stream)));
  return LV_OK;
}

lv_status lv_accum_counts(lv_accum* a, uint32_t* out, void* stream) {
  if (!a) return fail(LV_ERR_INVALID_ARG, "accumulator is NULL");
  if (!(a->flags & LV_ACCUM_COUNTS)) return fail(LV_ERR_INVALID_ARG, "created without LV_ACCUM_COUNTS");
  if (!out && a->scene->n > 0) return fail(LV_ERR_INVALID_ARG, "out is NULL");
  if (a->scene->n == 0) return LV_OK;
  if (a->scene->morton)  // back to the caller's order
    HIP_TRY(launch_permute_rows(a->counts.p, out, a->scene->perm.as<uint32_t>(), a->scene->n, 1, LV_F32,
                                true, static_cast<hipStream_t>(stream)));
  else
    HIP_TRY(hipMemcpyAsync(out, a->counts.p, 4 * (size_t)a->scene->n, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
  return LV_OK;
}

lv_status lv_accum_stats(lv_accum* a, lv_uplift_stats* out) {
  if (!a || !out) return fail(LV_ERR_INVALID_ARG, "null argument");
  out->views = a->views;
  out->pairs = a->pairs;
  out->visible = a->visible;
  out->covered_pixels = -1;
  out->contributions = -1;
  out->partial_sums = -1;
  if (a->dstats.p) {
    unsigned long long h[3];
    HIP_TRY(hipMemcpy(h, a->dstats.p, 24, hipMemcpyDeviceToHost));
    out->covered_pixels = (int64_t)h[0];
    out->contributions = (int64_t)h[1];
    out->partial_sums = (int64_t)h[2];
  }
  return LV_OK;
}

lv_status lv_profile_start(void) {
  std::lock_guard<std::mutex> pk(g_prof_mu);
  for (auto& e : g_prof_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  g_prof_events.clear();
  g_prof_on = true;
  return LV_OK;
}

lv_status lv_profile_stop(int64_t* launches, double* total_ms, double* per_launch_ms,
                          int64_t capacity) {
  std::lock_guard<std::mutex> pk(g_prof_mu);
  g_prof_on = false;
  double ms = 0.0;
  int64_t k = 0;
  for (auto& e : g_prof_events) {
    HIP_TRY(hipEventSynchronize(e.second));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, e.first, e.second));
    ms += t;
    if (per_launch_ms && k < capacity) per_launch_ms[k] = t;
    k++;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (launches) *launches = (int64_t)g_prof_events.size();
  if (total_ms) *total_ms = ms;
  g_prof_events.clear();
  return LV_OK;
}

lv_status lv_uplift_sets(lv_scene* sc, const lv_camera* cams, int32_t m, const lv_uplift_set* sets,
                         int32_t nsets, lv_dtype dtype, void* stream) {
  if (!sc) return fail(LV_ERR_INVALID_ARG, "scene is NULL");
  if (nsets < 1 || nsets > kMaxSets || !sets)
    return fail(LV_ERR_INVALID_ARG, "nsets = %d out of [1, %d]", nsets, kMaxSets);
  for (int k = 0; k < nsets; k++) {
    if (sets[k].D < 1 || sets[k].D > 4096)
      return fail(LV_ERR_INVALID_ARG, "set %d: D = %d out of [1, 4096]", k, sets[k].D);
    if (sc->n > 0 && !sets[k].out_feat) return fail(LV_ERR_INVALID_ARG, "set %d: out_feat is NULL", k);
  }
  lv_status st = check_cams(cams, m);
  if (st != LV_OK) return st;
  for (int k = 0; k < nsets; k++) {
    st = check_maps(sets[k].maps, m, dtype, sets[k].scales);
    if (st != LV_OK) return st;
  }
  // transient accumulators whose buffers live in the stream's workspace
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace& ws = *workspace_for(s);
  std::lock_guard<std::mutex> alk(ws.accmu);
  lv_accum acc[kMaxSets];
  lv_feature_set fs[kMaxSets];
  size_t n1 = (size_t)(sc->n > 0 ? sc->n : 1);
  for (int k = 0; k < nsets; k++) {
    {
      std::lock_guard<std::mutex> lk(ws.mu);
      HIP_TRY(ws.accUs[k].ensure(sizeof(float) * n1 * sets[k].D, s));
      HIP_TRY(ws.accBs[k].ensure(sizeof(beta_t) * n1, s));
    }
    acc[k].scene = sc;
    acc[k].D = sets[k].D;
    acc[k].U.p = ws.accUs[k].p;
    acc[k].beta.p = ws.accBs[k].p;
    fs[k].acc = &acc[k];
    fs[k].maps = sets[k].maps;
    fs[k].scales = sets[k].scales;
    fs[k].stride = 0;
    st = lv_accum_reset(&acc[k], stream);
    if (st != LV_OK) break;
  }
  if (st == LV_OK) st = lv_uplift_accumulate_sets(cams, m, fs, nsets, dtype, stream);
  for (int k = 0; k < nsets && st == LV_OK; k++)
    st = lv_accum_finalize(&acc[k], sets[k].out_feat, sets[k].out_wsum, nullptr, stream);
  for (int k = 0; k < nsets; k++) acc[k].U.p = acc[k].beta.p = nullptr;  // owned by the workspace
  return st;
}

lv_status lv_uplift(lv_scene* sc, const lv_camera* cams, int32_t m, const void* const* maps,
                    lv_dtype dtype, const float* scales, int32_t D, float* out_feat,
                    float* out_wsum, void* stream) {
  lv_uplift_set set;
  set.maps = maps;
  set.scales = scales;
  set.D = D;
  set.out_feat = out_feat;
  set.out_wsum = out_wsum;
  return lv_uplift_sets(sc, cams, m, &set, 1, dtype, stream);
}

namespace {
// pixels = H W; W only matters for the pixel-block formats
lv_status encode_impl(const float* src, int64_t pixels, int32_t W, int32_t D, lv_dtype dtype, void* dst,
                      float* scales, void* stream) {
  if (pixels < 0 || D < 1 || D > 4096) return fail(LV_ERR_INVALID_ARG, "bad size");
  if (!map_format_valid(dtype)) return fail(LV_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
  if (pixels > 0 && (!src || !dst)) return fail(LV_ERR_INVALID_ARG, "null buffer");
  const lv_dtype el = map_elem(dtype);
  if (el == LV_FP8_E4M3 && !scales) return fail(LV_ERR_INVALID_ARG, "FP8 needs scales");
  if (map_px8(dtype) && (uintptr_t)dst % (el == LV_FP8_E4M3 ? 8 : 16))
    return fail(LV_ERR_INVALID_ARG, "dst is not aligned to the 8-pixel blocks");
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* tmp = nullptr;  // per-channel absmax (FP8), stream-ordered scratch
  if (el == LV_FP8_E4M3) HIP_TRY(dev_alloc(&tmp, 4 * (size_t)D, s, true));
  const hipError_t e = launch_encode(src, pixels, D, dtype, dst, scales, static_cast<float*>(tmp), s, W);
  dev_free(tmp, 4 * (size_t)D, s, true);
  HIP_TRY(e);
  return LV_OK;
}
}  // namespace

lv_status lv_encode(const float* src, int64_t pixels, int32_t D, lv_dtype dtype, void* dst,
                    float* scales, void* stream) {
  if (map_px8(dtype))
    return fail(LV_ERR_INVALID_ARG, "pixel-block formats need the image width: lv_encode_map");
  return encode_impl(src, pixels, 0, D, dtype, dst, scales, stream);
}

lv_status lv_encode_map(const float* src, int32_t H, int32_t W, int32_t D, lv_dtype dtype, void* dst,
                        float* scales, void* stream) {
  if (H < 0 || W < 0 || H > 16384 || W > 16384)
    return fail(LV_ERR_INVALID_ARG, "map size %dx%d out of [0, 16384]", W, H);
  return encode_impl(src, (int64_t)H * W, W, D, dtype, dst, scales, stream);
}

lv_status lv_graph_create_csr(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                              const void* val, lv_dtype val_dtype, void* stream, lv_graph** out) {
  if (!out) return fail(LV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 0 || nnz < 0 || n >= ((int64_t)1 << 31) || nnz >= ((int64_t)1 << 31))
    return fail(LV_ERR_INVALID_ARG, "graph size out of range");
  if (val_dtype != LV_F32 && val_dtype != LV_BF16)
    return fail(LV_ERR_INVALID_ARG, "graph values must be LV_F32 or LV_BF16");
  if (!row_ptr || (nnz > 0 && (!col || !val))) return fail(LV_ERR_INVALID_ARG, "null CSR array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // validate the CSR on the host (row_ptr monotone, columns in range)
  std::vector<int32_t> rp(n + 1);
  std::vector<int32_t> cl(nnz);
  HIP_TRY(hipMemcpyAsync(rp.data(), row_ptr, 4 * (size_t)(n + 1), hipMemcpyDeviceToHost, s));
  if (nnz) HIP_TRY(hipMemcpyAsync(cl.data(), col, 4 * (size_t)nnz, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (rp[0] != 0 || rp[n] != nnz) return fail(LV_ERR_INVALID_ARG, "row_ptr must run from 0 to nnz");
  for (int64_t i = 0; i < n; i++)
    if (rp[i + 1] < rp[i]) return fail(LV_ERR_INVALID_ARG, "row_ptr decreases at row %lld", (long long)i);
  for (int64_t k = 0; k < nnz; k++)
    if (cl[k] < 0 || cl[k] >= n) return fail(LV_ERR_INVALID_ARG, "column %lld out of range", (long long)k);
  lv_graph* g = new (std::nothrow) lv_graph();
  if (!g) return fail(LV_ERR_OUT_OF_MEMORY, "host allocation");
  g->n = n;
  g->nnz = nnz;
  g->val_dtype = val_dtype;
  hipError_t e = g->row_ptr.ensure(4 * (size_t)(n + 1), s);
  if (e == hipSuccess) e = g->col.ensure(4 * (size_t)(nnz + 1), s);
  if (e == hipSuccess) e = g->val.ensure(dtype_size(val_dtype) * (size_t)(nnz + 1), s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->row_ptr.p, row_ptr, 4 * (size_t)(n + 1), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && nnz) e = hipMemcpyAsync(g->col.p, col, 4 * (size_t)nnz, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && nnz)
    e = hipMemcpyAsync(g->val.p, val, dtype_size(val_dtype) * (size_t)nnz, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    g->row_ptr.release(); g->col.release(); g->val.release();
    delete g;
    return fail(LV_ERR_DEVICE, "graph: %s", hipGetErrorString(e));
  }
  *out = g;
  return LV_OK;
}

lv_status lv_graph_build_knn(lv_scene* sc, const float* feats, int32_t D, int32_t k,
                             const lv_graph_opts* opts, void* stream, lv_graph** out) {
  TraceRange tr("lv.graph_build_knn");
  if (!out) return fail(LV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!sc || !feats) return fail(LV_ERR_INVALID_ARG, "null argument");
  if (k < 1 || k > 32) return fail(LV_ERR_INVALID_ARG, "k = %d not in [1, 32]", k);
  if (D < 1 || D > 4096) return fail(LV_ERR_INVALID_ARG, "D = %d not in [1, 4096]", D);
  const int64_t n = sc->n;
  if (n <= k) return fail(LV_ERR_INVALID_ARG, "n = %lld must exceed k = %d", (long long)n, k);
  if (n * (int64_t)(2 * k + 1) >= ((int64_t)1 << 31))
    return fail(LV_ERR_UNSUPPORTED, "n (2k + 1) = %lld >= 2^31", (long long)(n * (2 * k + 1)));
  GraphWeights gw;
  if (opts) {
    if (opts->kind != LV_GRAPH_SPATIAL_COSINE && opts->kind != LV_GRAPH_FEATURE_RBF)
      return fail(LV_ERR_INVALID_ARG, "unknown graph kind %d", opts->kind);
    gw.kind = opts->kind;
    if (gw.kind == LV_GRAPH_FEATURE_RBF) {
      if (!(opts->bandwidth > 0.0f)) return fail(LV_ERR_INVALID_ARG, "bandwidth must be > 0");
      if (!(opts->binarize >= 0.0f)) return fail(LV_ERR_INVALID_ARG, "binarize must be >= 0");
      gw.bandwidth = opts->bandwidth;
      gw.unary = opts->unary;
      gw.binarize = opts->binarize;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t *rp = nullptr, *cl = nullptr;
  float* vl = nullptr;
  int64_t nnz = 0;
  HIP_TRY(build_knn_graph(sc->caller_p0(), n, feats, D, k, gw, s, &rp, &cl, &vl, &nnz));
  lv_graph* g = new (std::nothrow) lv_graph();
  if (!g) {
    (void)hipStreamSynchronize(s);
    dev_free(rp, 4 * (size_t)(n + 1), s);
    dev_free(cl, 4 * (size_t)(nnz + 1), s);
    dev_free(vl, 4 * (size_t)(nnz + 1), s);
    return fail(LV_ERR_OUT_OF_MEMORY, "host allocation");
  }
  g->n = n;
  g->nnz = nnz;
  g->val_dtype = LV_F32;
  g->row_ptr.p = rp; g->row_ptr.cap = 4 * (size_t)(n + 1);
  g->col.p = cl; g->col.cap = 4 * (size_t)(nnz + 1);
  g->val.p = vl; g->val.cap = 4 * (size_t)(nnz + 1);
  *out = g;
  return LV_OK;
}

lv_status lv_graph_csr(const lv_graph* g, int64_t* n, int64_t* nnz, int32_t* row_ptr, int32_t* col,
                       void* val, void* stream) {
  if (!g) return fail(LV_ERR_INVALID_ARG, "graph is NULL");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (row_ptr) HIP_TRY(hipMemcpyAsync(row_ptr, g->row_ptr.p, 4 * (size_t)(g->n + 1), hipMemcpyDeviceToDevice, s));
  if (col && g->nnz) HIP_TRY(hipMemcpyAsync(col, g->col.p, 4 * (size_t)g->nnz, hipMemcpyDeviceToDevice, s));
  if (val && g->nnz)
    HIP_TRY(hipMemcpyAsync(val, g->val.p, dtype_size(g->val_dtype) * (size_t)g->nnz, hipMemcpyDeviceToDevice, s));
  return LV_OK;
}

lv_status lv_graph_destroy(lv_graph* g) {
  if (!g) return LV_OK;
  (void)hipDeviceSynchronize();
  g->row_ptr.release(); g->col.release(); g->val.release();
  g->b0.release(); g->b1.release(); g->norms.release();
  g->perm.release(); g->inv.release(); g->rp2.release(); g->col2.release(); g->val2.release();
  g->bin.release(); g->bout.release();
  if (g->last) (void)hipEventDestroy(g->last);
  delete g;
  return LV_OK;
}

lv_status lv_diffuse(const lv_scene* sc, const lv_graph* gc, const void* g0, lv_dtype dtype, int32_t D,
                     int32_t steps, void* out, void* stream) {
  TraceRange tr("lv.diffuse");
  if (!gc) return fail(LV_ERR_INVALID_ARG, "graph is NULL");
  if (sc && sc->n != gc->n) return fail(LV_ERR_INVALID_ARG, "scene and graph sizes differ");
  if (D < 1 || D > 4096 || steps < 0) return fail(LV_ERR_INVALID_ARG, "bad D or steps");
  if (dtype != LV_F32 && dtype != LV_BF16) return fail(LV_ERR_INVALID_ARG, "dtype must be F32 or BF16");
  if (gc->n > 0 && (!g0 || !out)) return fail(LV_ERR_INVALID_ARG, "null signal buffer");
  if (g0 == out && steps > 0) return fail(LV_ERR_INVALID_ARG, "out must not alias g0");
  lv_graph* g = const_cast<lv_graph*>(gc);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g->mu);
  if (g->last) HIP_TRY(hipStreamWaitEvent(s, g->last, 0));
  else HIP_TRY(hipEventCreateWithFlags(&g->last, hipEventDisableTiming));
  const bool order = sc && g->n > 0 && steps > 0;
  const size_t sig = dtype_size(dtype) * (size_t)(g->n > 0 ? g->n : 1) * D;
  HIP_TRY(g->b0.ensure(sig, s));
  HIP_TRY(g->b1.ensure(sig, s));
  HIP_TRY(g->norms.ensure(sizeof(float) * (size_t)D * (steps + 1), s));
  if (order && !g->ordered) {
    // P A P^T along the Morton order of the scene's centres; any permutation
    // gives the same result, so the order is built once per graph.
    const int64_t n = g->n, nnz = g->nnz;
    Buf scratch;
    HIP_TRY(scratch.ensure(4 * reorder_scratch_words(n), s));
    hipError_t e = g->perm.ensure(4 * (size_t)n, s);
    if (e == hipSuccess) e = g->inv.ensure(4 * (size_t)n, s);
    if (e == hipSuccess) e = g->rp2.ensure(4 * (size_t)(n + 1), s);
    if (e == hipSuccess) e = g->col2.ensure(4 * (size_t)(nnz + 1), s);
    if (e == hipSuccess) e = g->val2.ensure(dtype_size(g->val_dtype) * (size_t)(nnz + 1), s);
    if (e == hipSuccess)
      e = launch_graph_reorder(sc->caller_p0(), n, g->row_ptr.as<int32_t>(), g->col.as<int32_t>(),
                               g->val.p, g->val_dtype, nnz, scratch.as<uint32_t>(),
                               g->perm.as<uint32_t>(), g->inv.as<uint32_t>(), g->rp2.as<int32_t>(),
                               g->col2.as<int32_t>(), g->val2.p, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    scratch.release();
    if (e != hipSuccess) return fail(LV_ERR_DEVICE, "graph order: %s", hipGetErrorString(e));
    g->ordered = true;
  }
  if (order) {
    HIP_TRY(g->bin.ensure(sig, s));
    HIP_TRY(g->bout.ensure(sig, s));
    const uint32_t* perm = g->perm.as<uint32_t>();
    HIP_TRY(launch_permute_rows(g0, g->bin.p, perm, g->n, D, dtype, false, s));
    HIP_TRY(launch_diffuse(g->rp2.as<int32_t>(), g->col2.as<int32_t>(), g->val2.p, g->val_dtype, g->n,
                           g->bin.p, dtype, D, steps, g->bout.p, g->b0.as<float>(), g->b1.as<float>(),
                           g->norms.as<float>(), s));
    HIP_TRY(launch_permute_rows(g->bout.p, out, perm, g->n, D, dtype, true, s));
  } else {
    HIP_TRY(launch_diffuse(g->row_ptr.as<int32_t>(), g->col.as<int32_t>(), g->val.p, g->val_dtype, g->n,
                           g0, dtype, D, steps, out, g->b0.as<float>(), g->b1.as<float>(),
                           g->norms.as<float>(), s));
  }
  HIP_TRY(hipEventRecord(g->last, s));
  return LV_OK;
}

lv_status lv_render(lv_scene* sc, const lv_camera* cams, int32_t m, const float* g, int32_t D,
                    float* const* outs, float* const* alphas, void* stream) {
  TraceRange tr("lv.render");
  if (!sc) return fail(LV_ERR_INVALID_ARG, "scene is NULL");
  if (D < 1 || D > 4096) return fail(LV_ERR_INVALID_ARG, "D = %d out of [1, 4096]", D);
  lv_status st = check_cams(cams, m);
  if (st != LV_OK) return st;
  if (m > 0 && !outs) return fail(LV_ERR_INVALID_ARG, "outs is NULL");
  for (int v = 0; v < m; v++)
    if (!outs[v]) return fail(LV_ERR_INVALID_ARG, "outs[%d] is NULL", v);
  const int64_t n = sc->n;
  if (n > 0 && !g) return fail(LV_ERR_INVALID_ARG, "g is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {  // no Gaussian: every output is 0 (with Gaussians the kernel writes every pixel)
    for (int v = 0; v < m; v++) {
      const size_t px = (size_t)cams[v].width * cams[v].height;
      HIP_TRY(hipMemsetAsync(outs[v], 0, sizeof(float) * px * D, s));
      if (alphas && alphas[v]) HIP_TRY(hipMemsetAsync(alphas[v], 0, sizeof(float) * px, s));
    }
  }
  if (n == 0 || m == 0) return LV_OK;
  // g stays in the caller's order: the kernel reads row perm[i] for the
  // scene's storage index i
  const uint32_t* perm = sc->morton ? sc->perm.as<uint32_t>() : nullptr;
  Workspace& ws = *workspace_for(s);
  std::lock_guard<std::mutex> lk(ws.mu);
  const int64_t per_view = n * kItemBytes;
  const int64_t budget = chunk_budget_bytes(&ws);
  int64_t mc = std::max<int64_t>(1, std::min<int64_t>(m, budget / per_view));
  mc = std::min<int64_t>(mc, 1 << (31 - kViewShift));
  for (int v0 = 0; v0 < m;) {
    const int mv = (int)std::min<int64_t>(mc, m - v0);
    const uint32_t* ids = nullptr;
    int stride = 0, max_tiles = 0;
    int64_t P = 0, nvis = 0;
    bool split = false;
    st = build_structure(sc, ws, cams + v0, mv, s, &ids, &stride, &P, &nvis, &max_tiles, budget, &split);
    if (st != LV_OK) return st;
    if (split) {  // too many pairs for the chunk: fewer views per chunk, same views again
      const double fit = (double)std::min<int64_t>(budget / 16, 0x7FFFFFFF) / (double)P;
      mc = std::max<int64_t>(1, std::min<int64_t>(mv - 1, (int64_t)(mv * fit * 0.9)));
      continue;
    }
    // output tables (ws.up is idle: build_structure synchronised the stream)
    const size_t bytes = 2 * sizeof(float*) * (size_t)mv;
    HIP_TRY(ws.maps.ensure(bytes, s));
    HIP_TRY(ws.up.ensure(bytes));
    float** up = static_cast<float**>(ws.up.p);
    for (int v = 0; v < mv; v++) {
      up[v] = outs[v0 + v];
      up[mv + v] = alphas ? alphas[v0 + v] : nullptr;
    }
    HIP_TRY(hipMemcpyAsync(ws.maps.p, up, bytes, hipMemcpyHostToDevice, s));
    BlendArgs ba;
    memset(&ba, 0, sizeof(ba));
    ba.rec = ws.rec.as<Rec>();
    ba.ids = ids;
    ba.ranges = ws.ranges.as<uint2>();
    ba.geom = ws.geom.as<ViewGeom>();
    ba.n = n;
    ba.tiles_stride = stride;
    float* const* dtab = static_cast<float* const*>(ws.maps.p);
    st = profiled_launch(s, [&] { return launch_render(ba, mv, g, D, dtab, dtab + mv, perm, s); });
    if (st != LV_OK) return st;
    v0 += mv;
  }
  return LV_OK;
}

lv_status lv_debug_view(lv_scene* sc, const lv_camera* cam, lv_view_debug* out, int64_t* P_out) {
  if (!sc || !cam || !out) return fail(LV_ERR_INVALID_ARG, "null argument");
  lv_status st = check_cams(cam, 1);
  if (st != LV_OK) return st;
  const int64_t n = sc->n;
  hipStream_t s = nullptr;
  if (n == 0) {
    if (P_out) *P_out = 0;
    return LV_OK;
  }
  const uint32_t* ids = nullptr;
  int stride = 0, max_tiles = 0;
  int64_t P = 0, nvis = 0;
  Workspace& ws = *workspace_for(s);
  std::lock_guard<std::mutex> lk(ws.mu);
  st = build_structure(sc, ws, cam, 1, s, &ids, &stride, &P, &nvis, &max_tiles);
  if (st != LV_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  if (P_out) *P_out = P;
  std::vector<uint32_t> key(n);
  std::vector<Rec> rec(n);
  std::vector<uint2> rect(n);
  HIP_TRY(hipMemcpy(rec.data(), ws.rec.p, sizeof(Rec) * n, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(rect.data(), ws.rect.p, 8 * n, hipMemcpyDeviceToHost));
  // depth keys in Gaussian order: scatter the depth-sorted (key, id) pairs
  // back by id
  std::vector<uint32_t> sk(n), sv(n);
  HIP_TRY(hipMemcpy(sk.data(), ws.dkey, 4 * n, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(sv.data(), ws.dval, 4 * n, hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < n; k++) key[sv[k]] = sk[k];
  // storage index -> the caller's index (the identity without the Morton order)
  std::vector<uint32_t> perm(n);
  if (sc->morton)
    HIP_TRY(hipMemcpy(perm.data(), sc->perm.p, 4 * n, hipMemcpyDeviceToHost));
  else
    for (int64_t i = 0; i < n; i++) perm[i] = (uint32_t)i;
  for (int64_t si = 0; si < n; si++) {
    const int64_t i = perm[si];  // outputs at the caller's index
    const Rec& rc = rec[si];
    const uint2& rt = rect[si];
    // visible: a non-empty tile rectangle (culled items keep the empty one)
    const bool vis = (rt.y & 0xFFFFu) > (rt.x & 0xFFFFu) && (rt.y >> 16) > (rt.x >> 16);
    if (out->visible) out->visible[i] = vis ? 1 : 0;
    if (out->depth) out->depth[i] = key[si];
    if (out->rect) {
      out->rect[4 * i] = (int32_t)(rt.x & 0xFFFF);
      out->rect[4 * i + 1] = (int32_t)(rt.x >> 16);
      out->rect[4 * i + 2] = (int32_t)(rt.y & 0xFFFF);
      out->rect[4 * i + 3] = (int32_t)(rt.y >> 16);
    }
    if (out->rec) {
      float* r = out->rec + 8 * i;
      uint32_t lo;
      memcpy(&lo, &rc.r1.w, 4);
      const uint32_t lx = lo << 16, ly = lo & 0xFFFF0000u;
      r[0] = rc.r0.x; r[1] = rc.r0.y;
      memcpy(&r[2], &lx, 4);
      memcpy(&r[3], &ly, 4);
      r[4] = rc.r0.z; r[5] = rc.r0.w; r[6] = rc.r1.x; r[7] = rc.r1.y;
    }
  }
  if (out->tile_start) {
    std::vector<uint2> rg(max_tiles);
    HIP_TRY(hipMemcpy(rg.data(), ws.ranges.p, sizeof(uint2) * max_tiles, hipMemcpyDeviceToHost));
    int64_t run = 0;
    for (int t = 0; t < max_tiles; t++) {
      out->tile_start[t] = run;
      if (rg[t].y > rg[t].x) run += rg[t].y - rg[t].x;
    }
    out->tile_start[max_tiles] = run;
  }
  if (out->ids && out->ids_capacity >= P && P > 0) {
    HIP_TRY(hipMemcpy(out->ids, ids, 4 * (size_t)P, hipMemcpyDeviceToHost));
    if (sc->morton)
      for (int64_t k = 0; k < P; k++) out->ids[k] = perm[out->ids[k]];
  }
  return LV_OK;
}

}  // extern "C"

namespace lv {

lv_status set_error(lv_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return fail(st, "%s", buf);
}

// One pass of the server: per-set accumulators from the stream-ordered
// allocator (no device-wide synchronisation), lv_uplift_accumulate_sets over
// the union of the sets' views, finalize into each set's outputs, accumulators
// returned to the allocator on the same stream.
lv_status run_batch(lv_scene* sc, const lv_camera* cams, int32_t m, const BatchSet* sets,
                    int nsets, lv_dtype dtype, hipStream_t s) {
  if (!sc || nsets < 1 || nsets > kMaxSets) return fail(LV_ERR_INVALID_ARG, "bad batch");
  lv_accum acc[kMaxSets];
  lv_feature_set fs[kMaxSets];
  const size_t n1 = (size_t)(sc->n > 0 ? sc->n : 1);
  lv_status st = LV_OK;
  int made = 0;
  for (int k = 0; k < nsets; k++) {
    void* U = nullptr;
    void* B = nullptr;
    hipError_t e = dev_alloc(&U, sizeof(float) * n1 * sets[k].D, s, true);
    if (e == hipSuccess) e = dev_alloc(&B, sizeof(beta_t) * n1, s, true);
    if (e != hipSuccess) {
      dev_free(U, sizeof(float) * n1 * sets[k].D, s, true);
      st = fail(LV_ERR_OUT_OF_MEMORY, "server accumulator: %s", hipGetErrorString(e));
      break;
    }
    acc[k].scene = sc;
    acc[k].D = sets[k].D;
    acc[k].U.p = U;
    acc[k].beta.p = B;
    fs[k].acc = &acc[k];
    fs[k].maps = sets[k].maps;
    fs[k].scales = sets[k].scales;
    fs[k].stride = sets[k].stride;
    made = k + 1;
    st = lv_accum_reset(&acc[k], s);
    if (st != LV_OK) break;
  }
  if (st == LV_OK) st = lv_uplift_accumulate_sets(cams, m, fs, nsets, dtype, s);
  for (int k = 0; k < nsets && st == LV_OK; k++)
    st = lv_accum_finalize(&acc[k], sets[k].out_feat, sets[k].out_wsum, nullptr, s);
  for (int k = 0; k < made; k++) {
    dev_free(acc[k].U.p, sizeof(float) * n1 * sets[k].D, s, true);
    dev_free(acc[k].beta.p, sizeof(beta_t) * n1, s, true);
    acc[k].U.p = acc[k].beta.p = nullptr;
  }
  return st;
}

}  // namespace lv
