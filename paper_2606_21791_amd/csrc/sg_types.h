// Plain-old-data descriptors passed by value to the libsg kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sg.h"

namespace sg {

struct DevScene {
  const void* ptr[6];
  int64_t ps[6];   // primitive stride (elements)
  int64_t cs[6];   // component stride (elements)
  int32_t ncomp[6];
  int32_t n;
  int32_t sh_degree;
  int32_t dtype;
};

struct DevBox {
  const void* lo[6];
  const void* hi[6];
  int32_t mode;    // SG_BOX_GLOBAL / SG_BOX_PER_PRIM
  int32_t dtype;
  uint32_t mask;   // fields clamped (bit f); 0 = no guard
};

struct DevCam {
  double R[9];
  double t[3];
  double fx, fy, cx, cy, nearz, farz;
  double campos[3];
  double limx, limy;   // tangent clamp of the EWA Jacobian: 1.3 * half-extent / focal
  int32_t W, H;
};

struct DevRaster {
  int32_t tile, tiles_x, tiles_y, n_tiles;
  float amax, amin, tmin, cutq, dil;
  float bg[3];
  float qcut2;         // cutq * log2(e) / 2: the cut on the scaled form evaluated per pixel
};

// Projected record of one primitive (see sg_device.h for its fields).
struct Rec {
  float4 r0, r1, r2;
};

// Per-item (tile or (variant, tile)) metric partials, reduced in a fixed order.
struct Partial {
  double sse;
  unsigned long long evals;
  uint32_t changed;
  float max_abs;
  uint32_t nonfinite;
  uint32_t _pad;
};

// A corrupted primitive of a variant in the incremental path.
struct Touch {
  uint32_t prim;
  uint32_t old_depth;   // clean key depth bits (valid if old_vis)
  uint32_t new_depth;
  uint32_t old_rect0, old_rect1;
  uint32_t new_rect0, new_rect1;
  uint32_t flags;       // bit0 old visible, bit1 new visible, bit2 unchanged (record and rect identical)
};

constexpr int kMaxTouch = 8;
// Records staged per variant: slot j holds touch j's corrupted record, slot
// kMaxTouch + j its clean record (when the clean primitive is visible).
constexpr int kRecSlots = 2 * kMaxTouch;
constexpr int kMaxBatch = 2048;   // variants per sg_render_batch launch

struct VariantState {
  uint32_t n_touch;
  uint32_t full;        // 1: needs the full-render path
  uint32_t nonfinite;   // a corrupted stored component is Inf/NaN after the guard
  uint32_t n_dirty;     // dirty tiles
  uint64_t clamps;
  uint32_t _pad0;
  uint32_t _pad;
  uint64_t pred_regions;   // regions of the dirty tiles (sg_metrics_t::predicted_regions)
  uint64_t rend_regions;   // regions with a changed pixel
  Touch touch[kMaxTouch];
};

// Region bit of tile (tx, ty) in the 8 x 8 partition of the frame's tiles.
__host__ __device__ inline uint64_t region_bit(int tx, int ty, int tiles_x, int tiles_y) {
  return 1ull << ((ty * 8 / tiles_y) * 8 + (tx * 8 / tiles_x));
}

}  // namespace sg
