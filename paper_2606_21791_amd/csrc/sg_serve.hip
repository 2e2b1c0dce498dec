// The libsg server: resident scenes and their prepared views, a request
// queue, and worker threads that each own a context and a HIP stream and run
// batched injection launches (continuous batching through serve_core.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sg.h"
#include "serve_core.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int n_comp(int f, int deg) {
  static const int base[5] = {3, 3, 4, 1, 3};
  return f < 5 ? base[f] : 3 * ((deg + 1) * (deg + 1) - 1);
}

struct Scene {
  sg_scene s;                 // component-major copy owned by the server
  void* mem = nullptr;
  sg_box box;
  void* box_mem = nullptr;
  uint32_t box_mask = 0;
  size_t bytes = 0;
};

struct View {
  int scene;
  sg_prep* prep;
  int W, H, n_tiles;
  int64_t instances;
};

struct Ticket {
  int kind;
  int view;
  std::vector<sg_site> sites;
  sg_metrics_t* out;
  int64_t arrival_ns;
  bool done = false;
  sg_result res{};
};

}  // namespace

struct sg_server {
  sg_serve_config cfg;
  int device = 0;
  sg_ctx* main = nullptr;
  std::vector<Scene> scenes;
  std::vector<View> views;
  std::unique_ptr<sgserve::Scheduler> sched;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
  uint64_t next_ticket = 1;
  std::vector<std::thread> workers;
  bool stop = false;
  bool started = false;
  std::string err;
};

namespace {

sg_status fail(sg_server* s, sg_status code, const std::string& m) {
  if (s) s->err = m;
  return code;
}

// Device bytes a launch of `nv` variants on view v may need beyond the
// resident state: batch workspaces, plus a working copy and full-render
// buffers for a guarded render that takes the full path.
size_t launch_bytes(const sg_server* s, const View& v, int kind, int nv, int n_sites) {
  size_t b = (size_t)nv * ((size_t)v.n_tiles * (8 + 32) + 8 * 48 + 512) + (size_t)n_sites * 8 + 4096;
  if (kind == sgserve::kGuardedRender && n_sites > 8) {
    const Scene& sc = s->scenes[v.scene];
    b += sc.bytes + (size_t)sc.s.n * 64 + (size_t)v.instances * 24;
  }
  return b;
}

void worker_main(sg_server* S, int idx) {
  (void)hipSetDevice(S->device);
  sg_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  sg_metrics_t* dmet = nullptr;
  sg_metrics_t* hmet = nullptr;
  const int cap = S->cfg.max_batch > 0 ? S->cfg.max_batch : 64;
  size_t met_cap = 0;
  if (sg_ctx_create(S->device, 0, &ctx) != SG_OK || hipStreamCreate(&st) != hipSuccess) {
    std::lock_guard<std::mutex> g(S->mu);
    S->err = "worker " + std::to_string(idx) + ": context or stream creation failed";
    return;
  }
  (void)cap;
  std::vector<sg_site> sites;
  std::vector<sg_variant> vars;
  for (;;) {
    sgserve::Batch b;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || S->sched->pending() > 0; });
      if (S->stop && S->sched->pending() == 0) break;
      if (!S->sched->next(&b)) {
        // memory is held by running work; wait for a launch to finish
        S->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
    }
    const View& v = S->views[b.view];
    const Scene& sc = S->scenes[v.scene];
    sg_status rc = SG_OK;
    if (b.rejected) {
      rc = SG_E_NOMEM;
    } else {
      sites.clear();
      vars.clear();
      std::vector<Ticket*> ts;
      {
        std::lock_guard<std::mutex> g(S->mu);
        for (const auto& r : b.reqs) ts.push_back(S->tickets[r.ticket].get());
      }
      for (Ticket* t : ts) {
        if (t->kind == sgserve::kCampaign) {
          for (const sg_site& x : t->sites) {
            vars.push_back({(uint32_t)sites.size(), 1u, 0u, 0u});
            sites.push_back(x);
          }
        } else {
          vars.push_back({(uint32_t)sites.size(), (uint32_t)t->sites.size(), sc.box_mask ? 1u : 0u, 0u});
          sites.insert(sites.end(), t->sites.begin(), t->sites.end());
        }
      }
      const int B = (int)vars.size();
      if ((size_t)B > met_cap) {
        if (dmet) (void)hipFree(dmet);
        if (hmet) (void)hipHostFree(hmet);
        met_cap = (size_t)B;
        if (hipMalloc((void**)&dmet, met_cap * sizeof(sg_metrics_t)) != hipSuccess ||
            hipHostMalloc((void**)&hmet, met_cap * sizeof(sg_metrics_t), hipHostMallocDefault) != hipSuccess)
          rc = SG_E_NOMEM;
      }
      if (rc == SG_OK && B > 0) {
        const int mode = S->cfg.plain ? SG_FULL : SG_INCREMENTAL;
        rc = sg_render_batch(ctx, v.prep, sites.data(), (int32_t)sites.size(), vars.data(), B,
                             sc.box_mask ? &sc.box : nullptr, sc.box_mask, nullptr, dmet, mode, st);
        if (rc == SG_OK &&
            (hipMemcpyAsync(hmet, dmet, (size_t)B * sizeof(sg_metrics_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
             hipStreamSynchronize(st) != hipSuccess))
          rc = SG_E_DEVICE;
      }
      if (rc == SG_OK) {
        size_t k = 0;
        for (Ticket* t : ts) {
          const size_t n = t->kind == sgserve::kCampaign ? t->sites.size() : 1;
          uint64_t cl = 0;
          for (size_t j = 0; j < n; ++j) cl += hmet[k + j].clamps;
          if (t->out) std::memcpy(t->out, hmet + k, n * sizeof(sg_metrics_t));
          t->res.clamps = cl;
          k += n;
        }
      } else {
        std::lock_guard<std::mutex> g(S->mu);
        S->err = std::string("launch failed: ") + sg_last_error();
      }
    }
    const int64_t done = now_ns();
    {
      std::lock_guard<std::mutex> g(S->mu);
      for (const auto& r : b.reqs) {
        Ticket* t = S->tickets[r.ticket].get();
        t->res.status = rc;
        t->res.done_ns = done;
        t->res.latency_ns = done - t->arrival_ns;
        t->done = true;
      }
      S->sched->finish(b, done);
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  if (dmet) (void)hipFree(dmet);
  if (hmet) (void)hipHostFree(hmet);
  (void)hipStreamDestroy(st);
  sg_ctx_destroy(ctx);
}

void start_workers(sg_server* S) {
  if (S->started) return;
  S->started = true;
  const int n = S->cfg.plain ? 1 : (S->cfg.max_slots > 0 ? S->cfg.max_slots : 4);
  for (int i = 0; i < n; ++i) S->workers.emplace_back(worker_main, S, i);
}

}  // namespace

extern "C" {

sg_status sg_serve_create(int32_t device, const sg_serve_config* cfg, sg_server** out) {
  if (!cfg || !out) return SG_E_INVAL;
  *out = nullptr;
  if (cfg->max_slots < 0 || cfg->max_batch < 0 || cfg->max_batch > SG_MAX_BATCH || cfg->queue_depth < 0)
    return SG_E_INVAL;
  sg_server* S = new sg_server();
  S->cfg = *cfg;
  if (S->cfg.max_batch == 0) S->cfg.max_batch = 64;
  if (S->cfg.queue_depth == 0) S->cfg.queue_depth = 1 << 20;
  S->device = device;
  sg_status rc = sg_ctx_create(device, 0, &S->main);
  if (rc != SG_OK) {
    delete S;
    return rc;
  }
  S->sched.reset(new sgserve::Scheduler(cfg->hbm_budget_bytes, 0, S->cfg.max_batch, S->cfg.queue_depth, !cfg->plain));
  *out = S;
  return SG_OK;
}

sg_status sg_serve_add_scene(sg_server* S, const sg_scene* scene, const sg_box* box, uint32_t box_mask,
                             int32_t* scene_id) {
  if (!S || !scene || !scene_id) return SG_E_INVAL;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->started) return fail(S, SG_E_INVAL, "scenes must be added before the first request");
  if (scene->n < 1 || scene->sh_degree < 0 || scene->sh_degree > 3 || scene->dtype < SG_F32 || scene->dtype > SG_BF16)
    return fail(S, SG_E_INVAL, "bad scene");
  if (box && box_mask && box->dtype != scene->dtype) return fail(S, SG_E_INVAL, "box dtype differs");
  (void)hipSetDevice(S->device);
  Scene sc;
  const size_t wb = scene->dtype == SG_F32 ? 4 : 2;
  const int64_t n = scene->n;
  size_t total = 0;
  size_t off[6];
  for (int f = 0; f < 6; ++f) {
    off[f] = total;
    total += ((size_t)n_comp(f, scene->sh_degree) * n * wb + 255) / 256 * 256;
  }
  if (hipMalloc(&sc.mem, std::max<size_t>(total, 256)) != hipSuccess) return fail(S, SG_E_NOMEM, "scene allocation");
  sc.s = *scene;
  for (int f = 0; f < 6; ++f) {
    const int C = n_comp(f, scene->sh_degree);
    sc.s.ptr[f] = static_cast<char*>(sc.mem) + off[f];
    sc.s.prim_stride[f] = 1;
    sc.s.comp_stride[f] = n;
    if (!C) continue;
    if (scene->prim_stride[f] == 1 && scene->comp_stride[f] == n) {
      if (hipMemcpy(sc.s.ptr[f], scene->ptr[f], (size_t)C * n * wb, hipMemcpyDefault) != hipSuccess)
        return fail(S, SG_E_DEVICE, "scene copy");
    } else {
      for (int c = 0; c < C; ++c)
        if (hipMemcpy2D(static_cast<char*>(sc.s.ptr[f]) + (size_t)c * n * wb, wb,
                        static_cast<const char*>(scene->ptr[f]) + (size_t)c * scene->comp_stride[f] * wb,
                        (size_t)scene->prim_stride[f] * wb, wb, (size_t)n, hipMemcpyDefault) != hipSuccess)
          return fail(S, SG_E_DEVICE, "strided scene copy");
    }
  }
  sc.bytes = total;
  std::memset(&sc.box, 0, sizeof(sc.box));
  if (box && box_mask) {
    size_t bt = 0;
    size_t boff[6][2];
    for (int f = 0; f < 6; ++f) {
      if (!((box_mask >> f) & 1u) || !n_comp(f, scene->sh_degree)) continue;
      const size_t cnt = (size_t)n_comp(f, scene->sh_degree) * (box->mode == SG_BOX_GLOBAL ? 1 : n);
      boff[f][0] = bt;
      bt += (cnt * wb + 255) / 256 * 256;
      boff[f][1] = bt;
      bt += (cnt * wb + 255) / 256 * 256;
    }
    if (hipMalloc(&sc.box_mem, std::max<size_t>(bt, 256)) != hipSuccess) return fail(S, SG_E_NOMEM, "box allocation");
    sc.box.mode = box->mode;
    sc.box.dtype = box->dtype;
    for (int f = 0; f < 6; ++f) {
      if (!((box_mask >> f) & 1u) || !n_comp(f, scene->sh_degree)) continue;
      const size_t cnt = (size_t)n_comp(f, scene->sh_degree) * (box->mode == SG_BOX_GLOBAL ? 1 : n);
      sc.box.lo[f] = static_cast<char*>(sc.box_mem) + boff[f][0];
      sc.box.hi[f] = static_cast<char*>(sc.box_mem) + boff[f][1];
      if (hipMemcpy(sc.box.lo[f], box->lo[f], cnt * wb, hipMemcpyDefault) != hipSuccess ||
          hipMemcpy(sc.box.hi[f], box->hi[f], cnt * wb, hipMemcpyDefault) != hipSuccess)
        return fail(S, SG_E_DEVICE, "box copy");
      sc.box_mask |= 1u << f;
    }
    sc.bytes += bt;
  }
  S->sched->add_resident(sc.bytes);
  S->scenes.push_back(sc);
  *scene_id = (int32_t)S->scenes.size() - 1;
  return SG_OK;
}

sg_status sg_serve_add_view(sg_server* S, int32_t scene_id, const sg_camera* cam, const sg_raster* raster,
                            int32_t* view_id) {
  if (!S || !cam || !view_id) return SG_E_INVAL;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->started) return fail(S, SG_E_INVAL, "views must be added before the first request");
  if (scene_id < 0 || scene_id >= (int)S->scenes.size()) return fail(S, SG_E_INVAL, "bad scene id");
  (void)hipSetDevice(S->device);
  const size_t before = sg_ctx_bytes(S->main);
  const size_t budget = S->cfg.hbm_budget_bytes;
  sg_prep* p = nullptr;
  sg_status rc = sg_prepare(S->main, &S->scenes[scene_id].s, cam, raster, &p, nullptr);
  if (rc != SG_OK) return fail(S, rc, std::string("prepare: ") + sg_last_error());
  if (hipDeviceSynchronize() != hipSuccess) return fail(S, SG_E_DEVICE, "prepare");
  const size_t bytes = sg_ctx_bytes(S->main) - before;
  if (budget && S->sched->resident_bytes() + bytes > budget) {
    sg_prep_destroy(p);
    return fail(S, SG_E_NOMEM, "view does not fit the device budget");
  }
  S->sched->add_resident(bytes);
  const int tile = raster && raster->tile ? raster->tile : 16;
  View v{scene_id, p, cam->width, cam->height, ((cam->width + tile - 1) / tile) * ((cam->height + tile - 1) / tile),
         sg_prep_instances(p)};
  S->views.push_back(v);
  *view_id = (int32_t)S->views.size() - 1;
  return SG_OK;
}

sg_status sg_serve_submit(sg_server* S, const sg_request* req, uint64_t* ticket) {
  if (!S || !req || !ticket) return SG_E_INVAL;
  if (req->kind != SG_REQ_CAMPAIGN && req->kind != SG_REQ_GUARDED_RENDER) return fail(S, SG_E_INVAL, "bad kind");
  if (req->n_sites < 0 || (req->n_sites > 0 && !req->sites)) return fail(S, SG_E_INVAL, "bad sites");
  if (req->kind == SG_REQ_CAMPAIGN && req->n_sites < 1) return fail(S, SG_E_INVAL, "empty campaign");
  std::unique_lock<std::mutex> lk(S->mu);
  if (req->view_id < 0 || req->view_id >= (int)S->views.size()) return fail(S, SG_E_INVAL, "bad view id");
  const View& v = S->views[req->view_id];
  const Scene& sc = S->scenes[v.scene];
  const int width = sc.s.dtype == SG_F32 ? 32 : 16;
  for (int k = 0; k < req->n_sites; ++k) {
    const sg_site& x = req->sites[k];
    if (x.field > 5 || x.comp >= n_comp(x.field, sc.s.sh_degree) || x.prim >= (uint32_t)sc.s.n || x.bit >= width)
      return fail(S, SG_E_INVAL, "site " + std::to_string(k) + " out of range");
  }
  if (req->kind == SG_REQ_CAMPAIGN && req->n_sites > S->cfg.max_batch)
    return fail(S, SG_E_INVAL, "campaign larger than max_batch");
  start_workers(S);
  auto t = std::make_unique<Ticket>();
  t->kind = req->kind;
  t->view = req->view_id;
  t->sites.assign(req->sites, req->sites + req->n_sites);
  t->out = req->per_variant;
  t->arrival_ns = req->arrival_ns ? req->arrival_ns : now_ns();
  sgserve::Request r;
  r.ticket = S->next_ticket++;
  r.kind = req->kind;
  r.view = req->view_id;
  r.n_variants = req->kind == SG_REQ_CAMPAIGN ? req->n_sites : 1;
  r.arrival_ns = t->arrival_ns;
  r.bytes = launch_bytes(S, v, req->kind, r.n_variants, req->n_sites);
  const int q = S->sched->submit(r);
  if (q == -1) return fail(S, SG_E_BUSY, "queue full");
  if (q == -2) return fail(S, SG_E_NOMEM, "request does not fit the device budget");
  S->tickets[r.ticket] = std::move(t);
  *ticket = r.ticket;
  lk.unlock();
  S->cv_work.notify_one();
  return SG_OK;
}

sg_status sg_serve_poll(sg_server* S, uint64_t ticket, sg_result* out) {
  if (!S || !out) return SG_E_INVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return fail(S, SG_E_INVAL, "unknown ticket");
  if (!it->second->done) return SG_E_PENDING;
  *out = it->second->res;
  S->tickets.erase(it);
  return SG_OK;
}

sg_status sg_serve_wait(sg_server* S, uint64_t ticket, sg_result* out, int64_t timeout_us) {
  if (!S || !out) return SG_E_INVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return fail(S, SG_E_INVAL, "unknown ticket");
  Ticket* t = it->second.get();
  const bool ok = S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us < 0 ? 0 : timeout_us),
                                      [&] { return t->done; });
  if (!ok) return SG_E_PENDING;
  *out = t->res;
  S->tickets.erase(ticket);
  return SG_OK;
}

sg_status sg_serve_stats(sg_server* S, sg_serve_stats_t* out) {
  if (!S || !out) return SG_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  const sgserve::Scheduler::Counters c = S->sched->counters();
  out->submitted = c.submitted;
  out->completed = c.completed;
  out->rejected = c.rejected;
  out->launches = c.launches;
  out->variants = c.variants_done;
  const double span = (double)(c.last_done_ns - c.first_arrival_ns) / 1e9;
  out->inj_per_s = span > 0 ? (double)c.variants_done / span : 0.0;
  out->req_per_s = span > 0 ? (double)c.completed / span : 0.0;
  for (int k = 0; k < 2; ++k) {
    const sgserve::Percentiles p = S->sched->latency(k);
    out->p50_us[k] = p.p50;
    out->p99_us[k] = p.p99;
    out->mean_us[k] = p.mean;
    out->n[k] = p.n;
  }
  out->resident_bytes = S->sched->resident_bytes();
  return SG_OK;
}

const char* sg_serve_last_error(const sg_server* S) { return S ? S->err.c_str() : ""; }

void sg_serve_destroy(sg_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  (void)hipSetDevice(S->device);
  (void)hipDeviceSynchronize();
  for (View& v : S->views) sg_prep_destroy(v.prep);
  for (Scene& s : S->scenes) {
    if (s.mem) (void)hipFree(s.mem);
    if (s.box_mem) (void)hipFree(s.box_mem);
  }
  sg_ctx_destroy(S->main);
  delete S;
}

}  // extern "C"
