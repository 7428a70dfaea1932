// Uplift request server: admission by memory budget, same-scene merging into
// one wide pass, several passes in flight on their own streams (host code;
// the passes run the library's kernels through run_batch).
#include <chrono>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lv_internal.h"
#include "serve_sched.h"

struct lv_scene;

namespace lv {
void release_workspace(hipStream_t s);
void limit_workspace(hipStream_t s, int64_t bytes);
}  // namespace lv

namespace {

struct ServeReq {
  // scheduler fields
  int64_t bytes = 0;
  int32_t D = 0;
  uint64_t key = 0;
  // the request
  lv_scene* scene = nullptr;
  std::vector<lv_camera> cams;
  std::vector<const void*> maps;
  int32_t stride = 0;
  lv_dtype dtype = LV_F32;
  const float* scales = nullptr;
  float* out_feat = nullptr;
  float* out_wsum = nullptr;
  uint64_t tag = 0;
  int64_t t_submit = 0, t_admit = 0;
  hipEvent_t ready = nullptr;  // inputs produced (recorded on the caller's stream)
};

int64_t now_ns(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0)
      .count();
}

// dst[u][c] = src[idx[u]][c] (0 where idx[u] < 0): a request's FP8 scales
// rearranged to the views of a merged pass.
__global__ __launch_bounds__(256) void gather_scale_rows(const float* __restrict__ src,
                                                         const int32_t* __restrict__ idx,
                                                         float* __restrict__ dst, int rows, int D) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * D) return;
  const int u = (int)(e / D), c = (int)(e - (int64_t)u * D);
  const int r = idx[u];
  dst[e] = r >= 0 ? src[(int64_t)r * D + c] : 0.0f;
}

}  // namespace

struct lv_server {
  lv::Scheduler<ServeReq> sched;
  std::vector<std::thread> workers;
  std::mutex mu;  // completions and counters
  std::deque<lv_completion> done;
  int64_t submitted = 0, completed = 0, passes = 0, budget = 0, cancelled = 0;
  int64_t scratch = 0;                      // per worker
  int64_t mem_base = 0, peak_device = 0;    // device memory in use at creation, peak above it
  uint64_t next_id = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  lv_server(int64_t b, int max_sets, int max_channels)
      : sched(b, max_sets, max_channels, [this](ServeReq& r) { r.t_admit = now_ns(t0); }), budget(b) {}

  void run_worker();
  void execute(std::vector<ServeReq>& batch, hipStream_t s);
  lv_status run_pass(std::vector<ServeReq*>& reqs, hipStream_t s);
  void sample_memory();
  void finish(const ServeReq& r, int32_t status, int32_t nb, int64_t t_start, int64_t t_end);
};

void lv_server::sample_memory() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return;
  const int64_t used = (int64_t)(tot - fr) - mem_base;
  std::lock_guard<std::mutex> lk(mu);
  if (used > peak_device) peak_device = used;
}

void lv_server::finish(const ServeReq& r, int32_t status, int32_t nb, int64_t t_start, int64_t t_end) {
  lv_completion c;
  c.tag = r.tag;
  c.status = status;
  c.batch_size = nb;
  c.t_submit = r.t_submit;
  c.t_start = t_start;
  c.t_end = t_end;
  c.t_admit = r.t_admit;
  c.bytes = r.bytes;
  c.D = r.D;
  c.views = (int32_t)r.cams.size();
  std::lock_guard<std::mutex> lk(mu);
  done.push_back(c);
  completed += 1;
}

// One pass over requests `reqs` (same scene and dtype): the union of their
// views (cameras compared bytewise; a camera listed twice by one request is
// two views), per request a table over the union with NULL where it lacks
// the view, and for FP8 its scales rearranged to the union's views.
lv_status lv_server::run_pass(std::vector<ServeReq*>& reqs, hipStream_t s) {
  const int nb = (int)reqs.size();
  std::vector<lv_camera> ucams;
  std::vector<std::vector<const void*>> tabs(nb);
  std::vector<std::vector<int32_t>> uses(nb);  // union view of each request view
  {
    std::unordered_map<std::string, std::vector<int>> where;  // camera bytes -> union views
    for (int k = 0; k < nb; k++) {
      std::unordered_map<std::string, int> seen;               // occurrences within request k
      for (const lv_camera& c : reqs[k]->cams) {
        std::string b(reinterpret_cast<const char*>(&c), sizeof(lv_camera));
        const int occ = seen[b]++;
        std::vector<int>& lst = where[b];
        if ((int)lst.size() <= occ) {
          lst.push_back((int)ucams.size());
          ucams.push_back(c);
        }
        uses[k].push_back(lst[occ]);
      }
    }
    for (int k = 0; k < nb; k++) {
      tabs[k].assign(ucams.size(), nullptr);
      for (size_t v = 0; v < uses[k].size(); v++) tabs[k][uses[k][v]] = reqs[k]->maps[v];
    }
  }
  const int um = (int)ucams.size();
  const bool fp8 = lv::map_elem(reqs[0]->dtype) == LV_FP8_E4M3;
  std::vector<void*> scl(nb, nullptr);
  std::vector<size_t> scl_bytes(nb, 0);
  lv_status st = LV_OK;
  if (fp8 && um > 0) {
    for (int k = 0; k < nb && st == LV_OK; k++) {
      const int D = reqs[k]->D;
      std::vector<int32_t> idx(um, -1);
      for (size_t v = 0; v < uses[k].size(); v++) idx[uses[k][v]] = (int32_t)v;
      scl_bytes[k] = 4 * ((size_t)um * D + (size_t)um);
      if (lv::dev_alloc(&scl[k], scl_bytes[k], s, true) != hipSuccess) {
        st = lv::set_error(LV_ERR_OUT_OF_MEMORY, "server: FP8 scale table");
        break;
      }
      int32_t* didx = reinterpret_cast<int32_t*>(static_cast<float*>(scl[k]) + (size_t)um * D);
      if (hipMemcpyAsync(didx, idx.data(), 4 * (size_t)um, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        st = lv::set_error(LV_ERR_DEVICE, "server: FP8 scale table upload");
        break;
      }
      const int64_t total = (int64_t)um * D;
      hipLaunchKernelGGL(gather_scale_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                         reqs[k]->scales, didx, static_cast<float*>(scl[k]), um, D);
      if (hipGetLastError() != hipSuccess) st = lv::set_error(LV_ERR_DEVICE, "server: FP8 scale gather");
    }
  }
  if (st == LV_OK) {
    std::vector<lv::BatchSet> sets(nb);
    for (int k = 0; k < nb; k++) {
      sets[k].maps = tabs[k].data();
      sets[k].scales = fp8 ? static_cast<const float*>(scl[k]) : reqs[k]->scales;
      sets[k].stride = reqs[k]->stride;
      sets[k].D = reqs[k]->D;
      sets[k].out_feat = reqs[k]->out_feat;
      sets[k].out_wsum = reqs[k]->out_wsum;
    }
    lv::TraceRange tr("lv.server_pass");
    st = lv::run_batch(reqs[0]->scene, ucams.data(), (int32_t)um, sets.data(), nb, reqs[0]->dtype, s);
  }
  for (int k = 0; k < nb; k++) lv::dev_free(scl[k], scl_bytes[k], s, true);
  if (hipStreamSynchronize(s) != hipSuccess && st == LV_OK)
    st = lv::set_error(LV_ERR_DEVICE, "server: pass failed on the device");
  return st;
}

void lv_server::execute(std::vector<ServeReq>& batch, hipStream_t s) {
  const int nb = (int)batch.size();
  // the pass waits for the work that produced each request's inputs
  for (ServeReq& r : batch)
    if (r.ready) (void)hipStreamWaitEvent(s, r.ready, 0);
  sample_memory();
  const int64_t t_start = now_ns(t0);
  int npass = 0;
  const std::vector<int> status = lv::run_isolated((size_t)nb, (int)LV_ERR_DEVICE, [&](const std::vector<size_t>& idx) {
    std::vector<ServeReq*> reqs;
    for (size_t k : idx) reqs.push_back(&batch[k]);
    npass++;
    return (int)run_pass(reqs, s);
  });
  sample_memory();
  const int64_t t_end = now_ns(t0);
  for (int k = 0; k < nb; k++) {
    finish(batch[k], status[k], nb, t_start, t_end);
    if (batch[k].ready) (void)hipEventDestroy(batch[k].ready);
    batch[k].ready = nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  passes += npass;
}

void lv_server::run_worker() {
  (void)hipSetDevice(device);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  // this worker's structure scratch: items and pairs at most 2/5 of its share each
  if (s) lv::limit_workspace(s, scratch * 2 / 5);
  std::vector<ServeReq> batch;
  while (sched.next_batch(batch)) {
    if (s) {
      execute(batch, s);
    } else {
      for (ServeReq& r : batch) {
        finish(r, (int32_t)LV_ERR_DEVICE, (int32_t)batch.size(), 0, 0);
        if (r.ready) (void)hipEventDestroy(r.ready);
      }
    }
    sched.complete(batch);
  }
  if (s) {
    lv::release_workspace(s);  // the worker's scratch goes with its stream
    (void)hipStreamDestroy(s);
  }
}

extern "C" {

lv_status lv_server_create(const lv_server_opts* opts, lv_server** out) {
  if (!out) return lv::set_error(LV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  lv_server_opts o;
  memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (o.workers == 0) o.workers = 2;
  if (o.max_sets == 0) o.max_sets = 8;
  if (o.max_channels == 0) o.max_channels = 1024;
  if (o.scratch_bytes <= 0) o.scratch_bytes = (int64_t)4 << 30;
  if (o.workers < 1 || o.workers > 8 || o.max_sets < 1 || o.max_sets > 8 || o.max_channels < 1 ||
      o.reserved != 0)
    return lv::set_error(LV_ERR_INVALID_ARG, "server options out of range");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return lv::set_error(LV_ERR_DEVICE, "no device");
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return lv::set_error(LV_ERR_DEVICE, "hipMemGetInfo");
  if (o.hbm_budget <= 0) o.hbm_budget = (int64_t)(fr / 2);
  const int64_t for_requests = o.hbm_budget - (int64_t)o.workers * o.scratch_bytes;
  if (for_requests <= 0)
    return lv::set_error(LV_ERR_INVALID_ARG, "budget %lld leaves nothing beyond %d x %lld bytes of scratch",
                         (long long)o.hbm_budget, o.workers, (long long)o.scratch_bytes);
  lv_server* srv = new (std::nothrow) lv_server(for_requests, o.max_sets, o.max_channels);
  if (!srv) return lv::set_error(LV_ERR_OUT_OF_MEMORY, "host allocation");
  srv->device = dev;
  srv->scratch = o.scratch_bytes;
  srv->mem_base = (int64_t)(tot - fr);
  for (int w = 0; w < o.workers; w++) srv->workers.emplace_back([srv] { srv->run_worker(); });
  *out = srv;
  return LV_OK;
}

lv_status lv_server_submit(lv_server* srv, const lv_request* q) {
  const lv_status bad = LV_ERR_INVALID_ARG;
  if (!srv || !q || !q->scene) return lv::set_error(bad, "server, request or scene is NULL");
  if (q->D < 1 || q->D > 4096 || q->m < 0) return lv::set_error(bad, "D or m out of range");
  if (!lv::map_format_valid(q->dtype))
    return lv::set_error(bad, "unknown dtype");
  if (q->m > 0 && (!q->cams || !q->maps)) return lv::set_error(bad, "cams or maps is NULL");
  if (lv::map_elem(q->dtype) == LV_FP8_E4M3 && q->m > 0 && !q->scales)
    return lv::set_error(bad, "FP8 maps need scales");
  if (q->stride != 0 && q->stride < q->D) return lv::set_error(bad, "pixel stride < D");
  const int64_t n = lv_scene_size(q->scene);
  if (n > 0 && !q->out_feat) return lv::set_error(bad, "out_feat is NULL");
  for (int v = 0; v < q->m; v++) {
    const lv_camera& c = q->cams[v];
    if (!q->maps[v] || c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384 ||
        c.reserved != 0 || !(c.fx > 0.0f) || !(c.fy > 0.0f))
      return lv::set_error(bad, "a map is NULL or a camera is invalid");
  }
  ServeReq r;
  r.D = q->D;
  r.bytes = (n > 0 ? n : 1) * ((int64_t)q->D + 2) * 4;
  r.scene = q->scene;
  r.cams.assign(q->cams, q->cams + q->m);
  r.maps.assign(q->maps, q->maps + q->m);
  r.stride = q->stride;
  r.dtype = q->dtype;
  r.scales = q->scales;
  r.out_feat = q->out_feat;
  r.out_wsum = q->out_wsum;
  r.tag = q->tag;
  // the pass runs on a worker's stream: order it after the work the caller
  // enqueued so far on its stream (the producer of the maps, the scene)
  if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
    return lv::set_error(LV_ERR_DEVICE, "event");
  if (hipEventRecord(r.ready, static_cast<hipStream_t>(q->stream)) != hipSuccess) {
    (void)hipEventDestroy(r.ready);
    return lv::set_error(LV_ERR_DEVICE, "event record on the request's stream");
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->next_id++;
    // batch key: scene and dtype
    r.key = ((uint64_t)reinterpret_cast<uintptr_t>(q->scene) << 2) | (uint64_t)q->dtype;
    r.t_submit = now_ns(srv->t0);
    srv->submitted++;
  }
  hipEvent_t ev = r.ready;
  if (!srv->sched.submit(std::move(r))) {
    (void)hipEventDestroy(ev);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->submitted--;
    return lv::set_error(LV_ERR_OUT_OF_MEMORY, "request needs more memory than the server budget");
  }
  return LV_OK;
}

lv_status lv_server_cancel(lv_server* srv, uint64_t tag) {
  if (!srv) return lv::set_error(LV_ERR_INVALID_ARG, "server is NULL");
  ServeReq r;
  if (!srv->sched.cancel([tag](const ServeReq& q) { return q.tag == tag; }, &r))
    return lv::set_error(LV_ERR_INVALID_ARG, "no waiting request with tag %llu", (unsigned long long)tag);
  if (r.ready) (void)hipEventDestroy(r.ready);
  const int64_t t = now_ns(srv->t0);
  srv->finish(r, (int32_t)LV_ERR_CANCELLED, 0, t, t);
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->cancelled++;
  return LV_OK;
}

lv_status lv_server_poll(lv_server* srv, lv_completion* out, int32_t cap, int32_t* n) {
  if (!srv || !n || (cap > 0 && !out) || cap < 0) return LV_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  int32_t k = 0;
  while (k < cap && !srv->done.empty()) {
    out[k++] = srv->done.front();
    srv->done.pop_front();
  }
  *n = k;
  return LV_OK;
}

lv_status lv_server_drain(lv_server* srv) {
  if (!srv) return LV_ERR_INVALID_ARG;
  srv->sched.drain();
  return LV_OK;
}

lv_status lv_server_stats_get(lv_server* srv, lv_server_stats* out) {
  if (!srv || !out) return LV_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->passes = srv->passes;
  out->peak_bytes = srv->sched.peak_used();
  out->budget = srv->budget;
  out->cancelled = srv->cancelled;
  out->peak_device_bytes = srv->peak_device;
  return LV_OK;
}

lv_status lv_server_destroy(lv_server* srv) {
  if (!srv) return LV_OK;
  srv->sched.drain();
  srv->sched.shutdown();
  for (std::thread& t : srv->workers) t.join();
  delete srv;
  return LV_OK;
}

}  // extern "C"
