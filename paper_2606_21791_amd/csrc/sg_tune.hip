// Autotuner of campaign launch configurations (sg_autotune in sg.h): a
// coordinate search over measured campaign rates, with a JSON-lines cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "sg_settings.h"
#include "tune_cache.h"

namespace {

using sgtune::Cfg;

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  return arch;
}

}  // namespace

extern "C" sg_status sg_autotune(sg_ctx* ctx, const sg_scene* scene, const sg_camera* cam, const sg_raster* raster,
                                 const sg_site* sites, int32_t n_sites, int32_t fixed_batch, int32_t max_batch,
                                 const char* cache_path, sg_tune_t* out, void* stream) {
  if (!ctx || !scene || !cam || !sites || !out) return sg_fail(SG_E_INVAL, "ctx/scene/cam/sites/out is NULL");
  if (n_sites < 64) return sg_fail(SG_E_INVAL, "the autotuner needs at least 64 sample sites");
  if (fixed_batch < 0 || max_batch < 0 || fixed_batch > 65536 || max_batch > 65536)
    return sg_fail(SG_E_INVAL, "fixed_batch/max_batch out of range");
  if (max_batch == 0) max_batch = 512;
  if (fixed_batch > 2048 || max_batch > 2048) return sg_fail(SG_E_INVAL, "B is at most 2048 per launch");
  std::memset(out, 0, sizeof(*out));
  const SgSettings saved = sg_settings_get(ctx);
  const std::string key = sgtune::make_key(device_arch(saved.device), scene->n, cam->width, cam->height,
                                           scene->dtype, scene->sh_degree, fixed_batch, max_batch);
  Cfg best;
  double best_rate = 0.0;
  if (cache_path && sgtune::lookup(cache_path, key, &best, &best_rate)) {
    *out = {best.tile, best.batch, best.streams, best.threads, best.wgs, best.resume, best.graphs, 1,
            best_rate, 0, best.grid};
    return SG_OK;
  }
  sg_raster base = raster ? *raster : sg_raster{16, 0.99f, 1.0f / 255.0f, 1e-4f, 9.0f, 0.3f, {1.f, 1.f, 1.f}};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  // single-site variants cycling over the sample: a timed campaign has at
  // least 8 batches per stream (each stream's pipeline fills and drains once
  // per campaign) and at least the whole sample
  constexpr int kMaxVars = 1 << 17;
  std::vector<sg_variant> vars(std::max(n_sites, kMaxVars));
  for (size_t i = 0; i < vars.size(); ++i) vars[i] = {(uint32_t)(i % (size_t)n_sites), 1u, 0u, 0u};
  sg_metrics_t* met = nullptr;
  if (hipMalloc(&met, vars.size() * sizeof(sg_metrics_t)) != hipSuccess)
    return sg_fail(SG_E_NOMEM, "hipMalloc of the tuning records failed");

  std::map<std::pair<int, int>, sg_prep*> preps;   // (tile, resume) -> prepared scene
  sg_status rc = SG_OK;
  int trials = 0;
  auto prep_for = [&](const Cfg& c) -> sg_prep* {
    auto it = preps.find({c.tile, c.resume});
    if (it != preps.end()) return it->second;
    SgSettings s = saved;
    s.resume_spacing = c.resume;
    sg_settings_set(ctx, s);
    sg_raster r = base;
    r.tile = c.tile;
    sg_prep* p = nullptr;
    rc = sg_prepare(ctx, scene, cam, &r, &p, stream);
    if (rc != SG_OK) return nullptr;
    preps[{c.tile, c.resume}] = p;
    return p;
  };
  auto measure = [&](const Cfg& c) -> double {
    sg_prep* p = prep_for(c);
    if (!p) return -1.0;
    SgSettings s = saved;
    s.wgs_per_cu = c.wgs;
    s.grid = c.grid;
    s.resume_spacing = c.resume;
    s.graphs = c.graphs;
    sg_settings_set(ctx, s);
    sg_campaign_cfg cc{c.batch, c.streams, c.threads, 0};
    // campaigns of one size for every stream count (so that a fixed per-call
    // cost weighs the same on each), long enough for each stream's pipeline
    // to run 16 batches
    const int want = std::min(kMaxVars, std::max(n_sites, std::max(16 * c.streams * c.batch, 32768)));
    const int use = std::max(c.batch, (want / c.batch) * c.batch);
    // one untimed campaign warms the workspaces; then campaigns are
    // timed until at least 100 ms (and two campaigns) have elapsed
    double total = 0.0;
    int64_t done = 0;
    for (int rep = 0; rep < 200 && (rep < 3 || total < 0.1); ++rep) {
      if (hipStreamSynchronize(st) != hipSuccess) { rc = sg_fail(SG_E_DEVICE, "stream synchronize failed"); return -1.0; }
      const auto t0 = std::chrono::steady_clock::now();
      rc = sg_campaign(ctx, p, sites, n_sites, vars.data(), use, nullptr, 0, &cc, met, stream);
      if (rc != SG_OK) return -1.0;
      if (hipStreamSynchronize(st) != hipSuccess) { rc = sg_fail(SG_E_DEVICE, "stream synchronize failed"); return -1.0; }
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (rep > 0) { total += dt; done += use; }
    }
    ++trials;
    return (double)done / total;
  };

  Cfg cur;
  cur.batch = fixed_batch > 0 ? fixed_batch : std::min(32, max_batch);
  double cur_rate = measure(cur);
  const std::vector<int> tiles = {8, 16, 32}, resumes = {16, 32, 64, 128, 256}, wgss = {1, 2, 4, 8}, grids = {0, 64, 128},
                         streams = {4, 8, 16, 24, 32, 48, 64}, threads = {1, 2, 4};
  std::vector<int> batches;
  if (fixed_batch > 0) batches = {fixed_batch};
  else
    for (int b = 32; b <= max_batch; b *= 2) batches.push_back(b);
  for (int sweep = 0; sweep < 2 && rc == SG_OK; ++sweep) {
    bool moved = false;
    auto try_axis = [&](int Cfg::*field, const std::vector<int>& vals) {
      for (int v : vals) {
        if (rc != SG_OK) return;
        if (cur.*field == v) continue;
        Cfg c = cur;
        c.*field = v;
        if (c.threads > c.streams) continue;
        const double r = measure(c);
        if (r > cur_rate * 1.02) {   // move only on a clear gain
          cur = c;
          cur_rate = r;
          moved = true;
        }
      }
    };
    try_axis(&Cfg::batch, batches);
    try_axis(&Cfg::tile, tiles);
    try_axis(&Cfg::resume, resumes);
    try_axis(&Cfg::wgs, wgss);
    try_axis(&Cfg::grid, grids);
    try_axis(&Cfg::streams, streams);
    try_axis(&Cfg::threads, threads);
    if (!moved) break;
  }
  for (auto& kv : preps) sg_prep_destroy(kv.second);
  (void)hipFree(met);
  sg_settings_set(ctx, saved);
  if (rc != SG_OK) return rc;
  if (cache_path) (void)sgtune::append(cache_path, key, cur, cur_rate);
  *out = {cur.tile, cur.batch, cur.streams, cur.threads, cur.wgs, cur.resume, cur.graphs, 0, cur_rate, trials, cur.grid};
  return SG_OK;
}
