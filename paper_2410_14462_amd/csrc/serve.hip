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
  int64_t t_submit = 0;
};

int64_t now_ns(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0)
      .count();
}

}  // namespace

struct lv_server {
  lv::Scheduler<ServeReq> sched;
  std::vector<std::thread> workers;
  std::mutex mu;  // completions and counters
  std::deque<lv_completion> done;
  int64_t submitted = 0, completed = 0, passes = 0, budget = 0;
  uint64_t next_id = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  lv_server(int64_t b, int max_sets, int max_channels) : sched(b, max_sets, max_channels), budget(b) {}

  void run_worker();
  void execute(std::vector<ServeReq>& batch, hipStream_t s);
};

// Union of the batch's views (cameras compared bytewise; a camera listed
// twice by one request is two views), per request a table over the union
// with NULL where the request lacks the view.
void lv_server::execute(std::vector<ServeReq>& batch, hipStream_t s) {
  const int nb = (int)batch.size();
  std::vector<lv_camera> ucams;
  std::vector<std::vector<const void*>> tabs(nb);
  if (nb == 1) {
    ucams = batch[0].cams;
    tabs[0] = batch[0].maps;
  } else {
    std::unordered_map<std::string, std::vector<int>> where;  // camera bytes -> union views
    std::vector<std::vector<int>> uses(nb);                    // union view of each request view
    for (int k = 0; k < nb; k++) {
      std::unordered_map<std::string, int> seen;               // occurrences within request k
      for (const lv_camera& c : batch[k].cams) {
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
      for (size_t v = 0; v < uses[k].size(); v++) tabs[k][uses[k][v]] = batch[k].maps[v];
    }
  }
  std::vector<lv::BatchSet> sets(nb);
  for (int k = 0; k < nb; k++) {
    sets[k].maps = tabs[k].data();
    sets[k].scales = batch[k].scales;
    sets[k].stride = batch[k].stride;
    sets[k].D = batch[k].D;
    sets[k].out_feat = batch[k].out_feat;
    sets[k].out_wsum = batch[k].out_wsum;
  }
  const int64_t t_start = now_ns(t0);
  lv_status st = lv::run_batch(batch[0].scene, ucams.data(), (int32_t)ucams.size(), sets.data(), nb,
                               batch[0].dtype, s);
  if (st == LV_OK && hipStreamSynchronize(s) != hipSuccess) st = LV_ERR_DEVICE;
  const int64_t t_end = now_ns(t0);
  {
    std::lock_guard<std::mutex> lk(mu);
    for (const ServeReq& r : batch) {
      lv_completion c;
      c.tag = r.tag;
      c.status = (int32_t)st;
      c.batch_size = nb;
      c.t_submit = r.t_submit;
      c.t_start = t_start;
      c.t_end = t_end;
      done.push_back(c);
    }
    completed += nb;
    passes += 1;
  }
}

void lv_server::run_worker() {
  (void)hipSetDevice(device);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  std::vector<ServeReq> batch;
  while (sched.next_batch(batch)) {
    if (s) {
      execute(batch, s);
    } else {
      std::lock_guard<std::mutex> lk(mu);
      for (const ServeReq& r : batch) {
        lv_completion c = {r.tag, (int32_t)LV_ERR_DEVICE, (int32_t)batch.size(), r.t_submit, 0, 0};
        done.push_back(c);
      }
      completed += (int64_t)batch.size();
    }
    sched.complete(batch);
  }
  if (s) (void)hipStreamDestroy(s);
}

extern "C" {

lv_status lv_server_create(const lv_server_opts* opts, lv_server** out) {
  if (!out) return lv::set_error(LV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  lv_server_opts o = {0, 0, 0, 0};
  if (opts) o = *opts;
  if (o.workers == 0) o.workers = 2;
  if (o.max_sets == 0) o.max_sets = 8;
  if (o.max_channels == 0) o.max_channels = 1024;
  if (o.workers < 1 || o.workers > 8 || o.max_sets < 1 || o.max_sets > 8 || o.max_channels < 1)
    return lv::set_error(LV_ERR_INVALID_ARG, "server options out of range");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LV_ERR_DEVICE;
  if (o.hbm_budget <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return LV_ERR_DEVICE;
    o.hbm_budget = (int64_t)(fr / 2);
  }
  lv_server* srv = new (std::nothrow) lv_server(o.hbm_budget, o.max_sets, o.max_channels);
  if (!srv) return LV_ERR_OUT_OF_MEMORY;
  srv->device = dev;
  for (int w = 0; w < o.workers; w++) srv->workers.emplace_back([srv] { srv->run_worker(); });
  *out = srv;
  return LV_OK;
}

lv_status lv_server_submit(lv_server* srv, const lv_request* q) {
  const lv_status bad = LV_ERR_INVALID_ARG;
  if (!srv || !q || !q->scene) return lv::set_error(bad, "server, request or scene is NULL");
  if (q->D < 1 || q->D > 4096 || q->m < 0) return lv::set_error(bad, "D or m out of range");
  if (q->dtype != LV_F32 && q->dtype != LV_BF16 && q->dtype != LV_FP8_E4M3)
    return lv::set_error(bad, "unknown dtype");
  if (q->m > 0 && (!q->cams || !q->maps)) return lv::set_error(bad, "cams or maps is NULL");
  if (q->dtype == LV_FP8_E4M3 && q->m > 0 && !q->scales) return lv::set_error(bad, "FP8 maps need scales");
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
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    const uint64_t id = srv->next_id++;
    // batch key: scene and dtype; FP8 requests get a key of their own
    r.key = q->dtype == LV_FP8_E4M3 ? ((1ull << 63) | id)
                                    : ((uint64_t)reinterpret_cast<uintptr_t>(q->scene) << 2) |
                                          (uint64_t)q->dtype;
    r.t_submit = now_ns(srv->t0);
    srv->submitted++;
  }
  if (!srv->sched.submit(std::move(r))) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->submitted--;
    return lv::set_error(LV_ERR_OUT_OF_MEMORY, "request needs more memory than the server budget");
  }
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
