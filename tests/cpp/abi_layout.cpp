// Prints the size and field offsets of the ABI structures as the C compiler
// lays them out, for comparison with the Python binding.
#include <cstddef>
#include <cstdio>

#include "../../include/sg.h"

#define F(S, m) std::printf("%s.%s %zu\n", #S, #m, offsetof(S, m))
#define Z(S) std::printf("%s %zu\n", #S, sizeof(S))

int main() {
  Z(sg_scene); F(sg_scene, ptr); F(sg_scene, prim_stride); F(sg_scene, comp_stride); F(sg_scene, n);
  F(sg_scene, sh_degree); F(sg_scene, dtype);
  Z(sg_site); F(sg_site, field); F(sg_site, bit); F(sg_site, comp); F(sg_site, prim);
  Z(sg_camera); F(sg_camera, R); F(sg_camera, t); F(sg_camera, fx); F(sg_camera, near_z); F(sg_camera, width);
  F(sg_camera, height);
  Z(sg_raster); F(sg_raster, tile); F(sg_raster, alpha_max); F(sg_raster, bg);
  Z(sg_box); F(sg_box, mode); F(sg_box, dtype); F(sg_box, lo); F(sg_box, hi);
  Z(sg_variant); F(sg_variant, site_off); F(sg_variant, n_sites); F(sg_variant, guard); F(sg_variant, protect);
  Z(sg_metrics_t); F(sg_metrics_t, sse); F(sg_metrics_t, mse); F(sg_metrics_t, psnr); F(sg_metrics_t, footprint);
  F(sg_metrics_t, max_abs); F(sg_metrics_t, nonfinite); F(sg_metrics_t, catastrophic); F(sg_metrics_t, changed_px);
  F(sg_metrics_t, dirty_tiles); F(sg_metrics_t, clamps); F(sg_metrics_t, n_pixels); F(sg_metrics_t, path);
  F(sg_metrics_t, evals); F(sg_metrics_t, predicted_regions); F(sg_metrics_t, rendered_regions);
  Z(sg_campaign_cfg); F(sg_campaign_cfg, batch); F(sg_campaign_cfg, streams); F(sg_campaign_cfg, threads);
  Z(sg_tune_t); F(sg_tune_t, tile); F(sg_tune_t, from_cache); F(sg_tune_t, inj_per_s); F(sg_tune_t, trials); F(sg_tune_t, grid);
  Z(sg_serve_config); F(sg_serve_config, hbm_budget_bytes); F(sg_serve_config, max_slots);
  F(sg_serve_config, plain);
  Z(sg_request); F(sg_request, kind); F(sg_request, sites); F(sg_request, n_sites); F(sg_request, arrival_ns);
  F(sg_request, per_variant);
  Z(sg_result); F(sg_result, status); F(sg_result, done_ns); F(sg_result, latency_ns); F(sg_result, clamps);
  Z(sg_serve_stats_t); F(sg_serve_stats_t, launches); F(sg_serve_stats_t, inj_per_s); F(sg_serve_stats_t, p50_us);
  F(sg_serve_stats_t, resident_bytes);
  return 0;
}
