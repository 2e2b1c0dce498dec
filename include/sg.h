/*
 * sg.h -- C ABI of libsg: single-bit-upset injection into stored 3D Gaussian
 * splatting parameters, batched forward rendering of the corrupted variants,
 * per-variant image metrics, and the per-primitive support guard.
 *
 * Paper: "Single-Event Upsets in 3D Gaussian Splatting Rendering: Bit-Level
 * Criticality, Spatial Extent, and a Parallel Support Guard".  Each entry
 * point cites the passage that defines the operation it performs.
 *
 * Conventions shared by every call
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - The caller owns every array it passes (scenes, sites, boxes, images,
 *     metrics).  A context owns its workspaces; a prepared scene (sg_prep)
 *     owns its resident clean state; a server owns its resident copies.
 *   - Every call is asynchronous on the given HIP stream (hipStream_t passed
 *     as void*; NULL is the null stream).  Outputs are valid once the stream
 *     has been synchronised.  Calls that must size data-dependent buffers
 *     (sg_render, sg_prepare, and the multi-upset fallback of
 *     sg_render_batch) synchronise the stream once internally.
 *   - Errors are status codes; nothing throws across the boundary.  Argument
 *     validation runs before any device work, so a call that returns
 *     SG_E_INVAL has modified nothing.  A failing HIP call returns
 *     SG_E_DEVICE; sg_last_error() gives the text (thread-local).
 *   - A context and the objects made from it are single-threaded: one host
 *     thread at a time.  The server API is thread-safe.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sg_status;
enum {
  SG_OK = 0,
  SG_E_INVAL = -1,        /* bad argument; nothing was modified */
  SG_E_NOMEM = -2,        /* device allocation failed or budget exceeded */
  SG_E_DEVICE = -3,       /* a HIP call failed (see sg_last_error) */
  SG_E_BUSY = -4,         /* server queue full */
  SG_E_PENDING = -5,      /* server request not finished yet */
  SG_E_UNSUPPORTED = -6
};

/* Storage formats (Sec. 3, "Single-bit upset model"): fp32 1|8|23, fp16 1|5|10, bf16 1|8|7. */
enum { SG_F32 = 0, SG_F16 = 1, SG_BF16 = 2 };
/* Rounding of sg_cast: nearest-even, toward -Inf, toward +Inf. */
enum { SG_RNE = 0, SG_RD = 1, SG_RU = 2 };

/* The six stored fields of a primitive (Sec. 3, "Parameter layout"):
 * mean (3), log-scale (3), quaternion w,x,y,z (4), opacity logit (1),
 * degree-0 SH colour (3), higher-order SH (3*((L+1)^2-1), component
 * c = 3*k + channel for coefficient k = 1..(L+1)^2-1). */
enum { SG_MEANS = 0, SG_LOG_SCALES = 1, SG_QUATS = 2, SG_OPACITY = 3, SG_SH_DC = 4, SG_SH_REST = 5 };
#define SG_FIELD_MASK_GUARD 0x1Fu   /* fields 0..4: the 14 components the guard covers (Sec. 5.12) */

/* A scene in storage format: field f, primitive i, component c lives at
 * ptr[f] + (i * prim_stride[f] + c * comp_stride[f]) elements of the
 * format's width (4 bytes for fp32, 2 for fp16/bf16).  Component-major
 * (prim_stride = 1, comp_stride = n) is the fast layout.  16-bit fields must
 * start on a 4-byte boundary and their allocation must extend to a 4-byte
 * boundary (true of hipMalloc and torch allocations): sg_inject flips a 16-bit
 * word through its aligned 32-bit container.  Caller-owned device memory. */
typedef struct {
  void* ptr[6];
  int64_t prim_stride[6];
  int64_t comp_stride[6];
  int32_t n;           /* primitives, >= 1 */
  int32_t sh_degree;   /* 0..3 */
  int32_t dtype;       /* SG_F32 / SG_F16 / SG_BF16 */
  int32_t _pad;
} sg_scene;

/* A fault site (field, primitive, component, bit) (Sec. 3). bit < format width. */
typedef struct {
  uint8_t field;
  uint8_t bit;
  uint16_t comp;
  uint32_t prim;
} sg_site;

/* Pinhole camera, OpenCV axes: a world point X maps to camera point R X + t,
 * pixel (u, v) = (fx x/z + cx, fy y/z + cy); pixel (i, j) has its centre at
 * (i + 0.5, j + 0.5).  Primitives with z <= near_z or z > far_z are culled. */
typedef struct {
  double R[9];         /* row-major */
  double t[3];
  double fx, fy, cx, cy, near_z, far_z;
  int32_t width, height;
} sg_camera;

/* Compositing constants (3DGS rasterizer; 0.99 and 1e-4 as configured for
 * the paper's workloads).  Pass NULL for the defaults shown. */
typedef struct {
  int32_t tile;        /* 8, 16 or 32 pixels; 0 = tuned default (16) */
  float alpha_max;     /* 0.99 */
  float alpha_min;     /* 1/255 */
  float t_min;         /* 1e-4 */
  float cut_q;         /* 9 (3-sigma ellipse) */
  float dilation;      /* 0.3 */
  float bg[3];         /* 1, 1, 1 (white, Sec. 3 "Metrics") */
} sg_raster;

/* Support box (Alg. 1; Thm. 1).  mode SG_BOX_GLOBAL: lo[f], hi[f] hold C_f
 * words each (per field and component).  mode SG_BOX_PER_PRIM: lo[f], hi[f]
 * hold C_f * n words, component-major (component c of primitive i at
 * c * n + i).  Words are in the scene's storage format. */
enum { SG_BOX_GLOBAL = 0, SG_BOX_PER_PRIM = 1 };
typedef struct {
  int32_t mode;
  int32_t dtype;
  void* lo[6];
  void* hi[6];
} sg_box;

/* One corrupted variant of a prepared scene: sites[site_off .. site_off+n_sites)
 * of the batch's site array are applied together; guard != 0 clamps the
 * variant into the batch's box before it is rendered.
 *
 * protect emulates the alternative defenses of Table 3 on the same fault
 * grid: SG_PROTECT_SIGN_EXP, a code over the sign and exponent bits of every
 * stored word (fp32 bits 23-31, fp16 bits 10-15, bf16 bits 7-15), corrects
 * the sites on those bits and lets the others through; SG_PROTECT_VOTE,
 * three copies with a majority vote, corrects every site (each upset hits
 * one copy). */
enum { SG_PROTECT_NONE = 0, SG_PROTECT_SIGN_EXP = 1, SG_PROTECT_VOTE = 2 };
typedef struct {
  uint32_t site_off;
  uint32_t n_sites;
  uint32_t guard;
  uint32_t protect;
} sg_variant;

/* Per-variant result (Sec. 3 "Metrics"; Def. 1; Def. 2).  footprint is the
 * fraction of pixels with max over RGB |delta| > 1/255; catastrophic is
 * nonfinite || footprint > 0.01; psnr is +Inf when mse == 0.
 *
 * Contamination of a sort-first partition (Sec. 5.10): the frame's tiles are
 * grouped into an 8 x 8 grid of regions, tile (tx, ty) belonging to region
 * (8 tx / tiles_x, 8 ty / tiles_y), bit 8 ry + rx.  predicted_regions holds
 * the regions of the variant's dirty tiles (the old and new footprints of its
 * corrupted primitives: the nodes whose primitive sets change), and
 * rendered_regions the regions holding a tile with a changed pixel.  Coarser
 * partitions (4 x 4, 2 x 2) are unions of 2 x 2 or 4 x 4 bit blocks.  A
 * variant on the full-render path reports every region as predicted; K-view
 * records hold the union over the views; sg_metrics leaves both at 0. */
typedef struct {
  double sse;
  double mse;
  double psnr;
  float footprint;
  float max_abs;
  uint32_t nonfinite;
  uint32_t catastrophic;
  uint32_t changed_px;
  uint32_t dirty_tiles;   /* tiles of the corrupted primitives' old and new footprint
                             rectangles (the incremental path re-composites those of
                             them that a changed record reaches) */
  uint64_t clamps;        /* guard clamps applied to this variant */
  uint32_t n_pixels;      /* K * H * W compared */
  uint32_t path;          /* 0 incremental, 1 full render */
  uint64_t evals;         /* pixel-primitive evaluations of the front-to-back loop
                             (per pixel: list entries up to and including the one
                             that stops it) over the pixels walked */
  uint64_t predicted_regions;
  uint64_t rendered_regions;
} sg_metrics_t;

typedef struct sg_ctx sg_ctx;
typedef struct sg_prep sg_prep;

/* Context on HIP device `device`.  hbm_budget_bytes caps the context's own
 * workspaces (0 = no cap).  Returns SG_E_DEVICE if the device is absent. */
sg_status sg_ctx_create(int32_t device, size_t hbm_budget_bytes, sg_ctx** out);
void sg_ctx_destroy(sg_ctx* ctx);
const char* sg_last_error(void);
/* Bytes of device memory the context and its prepared scenes hold. */
size_t sg_ctx_bytes(const sg_ctx* ctx);

/* Cast n fp32 values into `dtype` words with rounding mode `rounding`
 * (Sec. 3: reduced precisions hold the clean fp32 parameter cast to the
 * format).  Subnormals are kept; RNE overflows to Inf.  dst holds n words. */
sg_status sg_cast(sg_ctx* ctx, const float* src, void* dst, int64_t n, int32_t dtype, int32_t rounding,
                  void* stream);

/* Flip sites[k].bit of each addressed stored word in place (Sec. 3: the word
 * is XORed with 1 << bit).  sites is a HOST array of n entries; it is
 * validated (field present, comp < C_f, prim < n, bit < width) before any
 * device work.  saved (nullable, n words) receives each word's value before
 * its own flip.  Flipping the same sites again restores the scene (sg_restore). */
sg_status sg_inject(sg_ctx* ctx, const sg_scene* scene, const sg_site* sites, int32_t n, uint32_t* saved,
                    void* stream);
/* Undo sg_inject by flipping the same sites again (the paper restores the
 * working copy after each injection, Sec. 3 "Parallel injection engine").
 * saved is accepted for symmetry and may be NULL. */
sg_status sg_restore(sg_ctx* ctx, const sg_scene* scene, const sg_site* sites, int32_t n,
                     const uint32_t* saved, void* stream);

/* Precompute the support box of a clean scene (Alg. 1, first loop): for each
 * field in field_mask and each component, lo = minimum and hi = maximum of
 * the stored values over all primitives (IEEE order; a -0/+0 tie gives -0 for
 * lo and +0 for hi).  out->mode must be SG_BOX_GLOBAL and out->lo[f],
 * out->hi[f] must point to C_f words each for every field in the mask.  The
 * clean scene must be finite. */
sg_status sg_guard_box(sg_ctx* ctx, const sg_scene* clean, uint32_t field_mask, sg_box* out, void* stream);

/* Clamp every component of every primitive of the fields in field_mask into
 * the box, in place (Alg. 1, per-frame loop; Thm. 1): NaN -> lo, x < lo ->
 * lo, x > hi -> hi, otherwise the word is untouched.  clamp_count (device,
 * one uint64) receives the number of clamped components; health_alert
 * (device uint32, nullable) receives clamp_count > health_threshold. */
sg_status sg_guard(sg_ctx* ctx, const sg_scene* scene, const sg_box* box, uint32_t field_mask,
                   uint64_t health_threshold, uint64_t* clamp_count, uint32_t* health_alert, void* stream);

/* Full render of `scene` as it is in memory: projection, tile binning,
 * depth sort and front-to-back compositing over raster->bg (Sec. 2 "Gaussian
 * splatting"; Sec. 3 "Metrics").  box (nullable) clamps every guarded
 * component while it is loaded (the guard applied without writing the
 * scene).  image_out (nullable) receives height*width*3 floats, row-major
 * RGB.  If clean_frame (nullable) is given, metrics_out (device, one entry)
 * receives the metrics of this render against it.  This is the plain
 * one-render-per-injection path.  Synchronises the stream once. */
sg_status sg_render(sg_ctx* ctx, const sg_scene* scene, const sg_camera* cam, const sg_raster* raster,
                    const sg_box* box, uint32_t box_field_mask, float* image_out, const float* clean_frame,
                    sg_metrics_t* metrics_out, void* stream);

/* Make a scene resident for batched injection: project it, bin and sort its
 * tiles and render its clean frame once, and keep all of it on the device
 * (Sec. 3: the clean parameters stay resident).  The scene's memory must stay
 * valid and unmodified while the sg_prep is alive.  Synchronises once. */
sg_status sg_prepare(sg_ctx* ctx, const sg_scene* clean, const sg_camera* cam, const sg_raster* raster,
                     sg_prep** out, void* stream);
void sg_prep_destroy(sg_prep* prep);
/* Device pointer to the prepared clean frame (height*width*3 floats). */
const float* sg_prep_frame(const sg_prep* prep);
/* Instances (primitive-tile pairs) in the prepared tile lists. */
int64_t sg_prep_instances(const sg_prep* prep);
/* Copy the prepared clean frame into dst (device, height*width*3 floats). */
sg_status sg_prep_copy_frame(const sg_prep* prep, float* dst, void* stream);

/* A prepared scene is read-only once made: contexts on the same device (for
 * example one per host thread) may render batches of it concurrently. */

/* Render B corrupted variants of a prepared scene and score each against the
 * clean frame (Sec. 5.12: many independently corrupted variants per launch;
 * Sec. 3 "Metrics"; Def. 1; Def. 2).  sites: HOST array of n_sites;
 * variants: HOST array of B.  box (nullable) is used by variants with
 * guard != 0 and must contain the clean scene (Thm. 1 (i)); box_field_mask
 * selects the guarded fields.  mode SG_INCREMENTAL re-composites only the
 * tiles covered by the old or new footprint of each corrupted primitive
 * (bit-identical to a full render); variants touching more than 8 primitives
 * take the full-render path.  mode SG_FULL renders every variant in full.
 * images_out (nullable) receives B*height*width*3 floats; metrics_out
 * (device) receives B entries.  The scene is never modified. */
enum { SG_INCREMENTAL = 0, SG_FULL = 1 };
#define SG_MAX_BATCH 2048   /* variants per sg_render_batch call */
sg_status sg_render_batch(sg_ctx* ctx, sg_prep* prep, const sg_site* sites, int32_t n_sites,
                          const sg_variant* variants, int32_t B, const sg_box* box, uint32_t box_field_mask,
                          float* images_out, sg_metrics_t* metrics_out, int32_t mode, void* stream);

/* K views per injection (Def. 1 averages the footprint over the K views;
 * Sec. 3, "Parallel injection engine", renders them per injection).  preps[k]
 * are views of one scene (prepared from the same sg_scene).  Every variant
 * is rendered in each view as by sg_render_batch; per_view_out (nullable,
 * device, K x B records, view-major) receives the per-view records and
 * metrics_out (device, B records) the pooled ones: SSE, changed pixels,
 * evaluations, dirty tiles and pixels summed over the views, the largest
 * delta, the non-finite flag of any view, the footprint as the mean of the
 * per-view footprints, PSNR from the pooled MSE and the catastrophe rule on
 * the pooled footprint.  1 <= K <= 64. */
sg_status sg_render_batch_views(sg_ctx* ctx, sg_prep* const* preps, int32_t K, const sg_site* sites, int32_t n_sites,
                                const sg_variant* variants, int32_t B, const sg_box* box, uint32_t box_field_mask,
                                sg_metrics_t* metrics_out, sg_metrics_t* per_view_out, int32_t mode, void* stream);

/* A campaign: n_variants variants of one prepared scene, rendered as
 * consecutive batches of cfg->batch variants (the launch size B of
 * sg_render_batch), the batches spread round-robin over cfg->streams device
 * streams of the context, which cfg->threads host threads enqueue
 * concurrently (the parallel injection engine of Sec. 3 run as one call).
 * metrics_out (device, n_variants records) receives the same records as
 * sg_render_batch on each batch in turn; no images.  sites and variants are
 * host arrays as in sg_render_batch (offsets index `sites`).  The launches
 * are ordered after earlier work on `stream`, and later work on `stream` is
 * ordered after them; the call returns once everything is enqueued.  cfg may
 * be NULL (batch 32, 8 streams, 2 threads).  Errors of any batch stop the
 * campaign and are reported with the batch index.
 *
 * When every variant is incremental (at most 8 distinct primitives), the
 * campaign copies sites and variants to device memory once, stages and
 * projects the corrupted primitives of up to 524,288 variants in one
 * pre-pass launch per view, and then enqueues one launch per batch on its
 * stream: launch i lists the work items of the stream's batch i, composites
 * batch i - 1 and reduces the metrics of batch i - 2 (two more launches per
 * stream drain the pipeline).  With K views of one resolution, raster and
 * checkpoint spacing, each launch renders its batch in all K views when
 * B * K <= SG_MAX_BATCH and the streams' work-item buffers (room for every
 * tile of every variant-view: 3 * streams * B * K * tiles * 40 bytes) stay
 * within 16 GiB; other view sets run view after view.  The per-view records
 * are then pooled.  Campaigns on one
 * context run one at a time (a second call waits until the first one's
 * device buffers are no longer read).
 *
 * SG_ENGINE_PERSISTENT renders the campaign in chunks of `batch` variants
 * (0: as many as fit: a chunk bounds its variant-views so that each may
 * dirty every tile of its view, within 2^25 work items and 2^18
 * variant-views) with four launches per chunk on one of two internal
 * streams: the pre-pass (one per view or scene), one listing every
 * variant's work items compactly, one persistent launch compositing all of
 * them and one reducing the records (plus the pooling of K views).  It
 * needs neither many streams nor many hardware queues; its buffers take up
 * to 3.3 GB.  Its records equal the pipelined engine's.
 *
 * Throughput of the pipelined engine comes from many streams' launches
 * running at once.  The HIP
 * runtime maps streams onto GPU_MAX_HW_QUEUES hardware queues (4 unless the
 * environment sets it before the runtime starts), and each queue runs its
 * launches one after another: on the MI355X the campaign rate rises with the
 * queue count up to 23 queues and collapses at 24.  Eighteen queues with 64
 * streams is the measured configuration; the pipelined engine returns
 * SG_E_UNSUPPORTED when GPU_MAX_HW_QUEUES is above 23. */
typedef enum { SG_ENGINE_PIPELINED = 0, SG_ENGINE_PERSISTENT = 1 } sg_engine;
typedef struct {
  int32_t batch;     /* variants per launch.  Pipelined: 0 = 32, at most SG_MAX_BATCH.
                        Persistent: 0 = as many as the work-item buffers hold */
  int32_t streams;   /* pipelined: device streams; 0 = 8 (at most 64) */
  int32_t threads;   /* pipelined: host threads; 0 = 2 (at most streams) */
  int32_t engine;    /* SG_ENGINE_PIPELINED (0) or SG_ENGINE_PERSISTENT */
} sg_campaign_cfg;
sg_status sg_campaign(sg_ctx* ctx, sg_prep* prep, const sg_site* sites, int32_t n_sites, const sg_variant* variants,
                      int32_t n_variants, const sg_box* box, uint32_t box_field_mask, const sg_campaign_cfg* cfg,
                      sg_metrics_t* metrics_out, void* stream);
/* The same over K views of one scene: each batch is rendered in every view
 * as by sg_render_batch_views and metrics_out receives the pooled records. */
sg_status sg_campaign_views(sg_ctx* ctx, sg_prep* const* preps, int32_t K, const sg_site* sites, int32_t n_sites,
                            const sg_variant* variants, int32_t n_variants, const sg_box* box, uint32_t box_field_mask,
                            const sg_campaign_cfg* cfg, sg_metrics_t* metrics_out, void* stream);
/* A campaign over several prepared scenes of uneven size (Sec. 5.12: many
 * independently corrupted variants per launch): variant v is a variant of
 * preps[scene_of[v]] and is rendered there only; the batches mix the scenes,
 * and each launch composites the (variant, tile) work items of all of them.
 * preps: n_preps (1..64) prepared scenes or views on this device, any sizes
 * and formats, one tile size.  scene_of: HOST array of n_variants indices
 * into preps.  sites, variants: host arrays as in sg_campaign; a variant's
 * sites address its own scene and are validated against it.  boxes
 * (nullable; entries nullable): the guard box of each scene, used by
 * variants with guard != 0.  Every variant must touch at most 8 distinct
 * primitives (SG_E_UNSUPPORTED otherwise).  metrics_out (device, n_variants
 * records) receives what sg_render_batch gives on each variant's own scene.
 * Ordering, streams and threads as in sg_campaign. */
sg_status sg_campaign_scenes(sg_ctx* ctx, sg_prep* const* preps, int32_t n_preps, const sg_site* sites, int32_t n_sites,
                             const sg_variant* variants, const uint16_t* scene_of, int32_t n_variants,
                             const sg_box* const* boxes, uint32_t box_field_mask, const sg_campaign_cfg* cfg,
                             sg_metrics_t* metrics_out, void* stream);

/* Autotuner.  Picks the launch configuration of injection campaigns on one
 * scene and camera by measurement: tile size, variants per launch B,
 * campaign streams and host threads, persistent compositing workgroups per
 * CU (or a total grid) and checkpoint spacing.  It prepares the scene at each
 * candidate tile size and spacing, times campaigns of single-site variants
 * over `sites` (host, at least 64; the sample should follow the campaign's
 * site distribution) and moves one parameter at a time to its best value
 * until none improves (two sweeps at most).  fixed_batch > 0 keeps B at that
 * value; otherwise B is tuned up to max_batch (0 = 512; at most SG_MAX_BATCH).  The rendered
 * results never depend on the choice: every configuration is bit-identical.
 *
 * cache_path (nullable) names a text file of one JSON object per line, keyed
 * by device architecture, primitive-count bucket (ceil log2 N), frame size,
 * storage format, SH degree, fixed_batch and max_batch.  A hit fills *out
 * with from_cache = 1 and touches no device; a miss measures, appends the
 * result and sets from_cache = 0.  The context's settings are restored
 * before returning; the caller applies the result (sg_ctx_set_persistent,
 * sg_ctx_set_persistent_grid, sg_ctx_set_resume before sg_prepare with the
 * tile size, and batch/streams/threads in sg_campaign).  graphs is 0:
 * campaigns do not replay graphs. */
typedef struct {
  int32_t tile, batch, streams, threads, wgs_per_cu, resume, graphs, from_cache;
  double inj_per_s;   /* measured rate of the chosen configuration */
  int32_t trials;     /* configurations measured */
  int32_t grid;       /* total persistent workgroups (0: wgs_per_cu per CU) */
} sg_tune_t;
sg_status sg_autotune(sg_ctx* ctx, const sg_scene* scene, const sg_camera* cam, const sg_raster* raster,
                      const sg_site* sites, int32_t n_sites, int32_t fixed_batch, int32_t max_batch,
                      const char* cache_path, sg_tune_t* out, void* stream);

/* Workgroups per compute unit of the persistent incremental compositing
 * launch (0 = default for the tile size).  Fewer leave room for batches on
 * other streams to run concurrently; this is one of the tuned parameters. */
sg_status sg_ctx_set_persistent(sg_ctx* ctx, int32_t wgs_per_cu);
/* Total workgroups of that launch, overriding the per-CU count (0 = use the
 * per-CU count; at most 65536).  A grid smaller than the device lets more
 * launches from other streams be resident at once. */
sg_status sg_ctx_set_persistent_grid(sg_ctx* ctx, int32_t total_wgs);

/* Spacing, in tile-list entries, of the compositing checkpoints that
 * sg_prepare keeps with a prepared scene (default 64; 0 = none).  With a
 * spacing g, sg_prepare stores for every pixel the list index at which its
 * clean walk stopped, and for every tile the exact (colour, transmittance)
 * state of each pixel after every g entries: H*W*4 bytes plus
 * sum over tiles of floor(count / g) * tile^2 * 16 bytes of device memory.
 * The incremental path of sg_render_batch then skips pixels that stopped
 * before the first list entry a variant changes and resumes the others from
 * the nearest checkpoint; results are bit-identical either way.  Applies to
 * scenes prepared after the call; g must be 0 or in [16, 65536]. */
sg_status sg_ctx_set_resume(sg_ctx* ctx, int32_t spacing);

/* Replay the incremental part of sg_render_batch as a captured HIP graph
 * (default on).  A graph is used when every variant is incremental, no
 * images are requested, timing is off and the stream is not the null stream;
 * one graph is kept per batch shape and buffer set. */
sg_status sg_ctx_set_graphs(sg_ctx* ctx, int32_t enable);

/* Work issued on different HIP streams uses different workspaces of the
 * context, so batches on different streams may overlap on the device (the
 * host calls themselves stay single-threaded). */

/* Per-pass device timing, for profiling.  While enabled, calls record HIP
 * events on their stream around each pass; sg_ctx_pass_times waits for the
 * recorded events, adds the elapsed milliseconds per pass into ms[SG_N_PASSES]
 * and the number of timed launches into launches[SG_N_PASSES] (both host),
 * and clears the record. */
enum {
  SG_PASS_VARIANT_PREP = 0,     /* corrupted-primitive projection and dirty-tile planning
                                   (a campaign: its pre-pass over all variants) */
  SG_PASS_COMPOSITE_ITEMS = 1,  /* persistent incremental compositing (a campaign: each fused
                                   per-batch step launch with a compositing role, which also
                                   plans the next batch and reduces the previous one) */
  SG_PASS_REDUCE = 2,           /* per-variant metric reduction (a campaign: the pipeline's fill
                                   and drain step launches, which have no compositing role) */
  SG_PASS_PROJECT = 3,          /* full projection */
  SG_PASS_BIN = 4,              /* tile counts, offsets and instance scatter */
  SG_PASS_SORT = 5,             /* per-tile depth sort */
  SG_PASS_COMPOSITE_FULL = 6,   /* full-frame compositing */
  SG_PASS_GUARD = 7,            /* guard clamp pass (sg_guard) */
  SG_N_PASSES = 8
};
sg_status sg_ctx_timing(sg_ctx* ctx, int32_t enable);
sg_status sg_ctx_pass_times(sg_ctx* ctx, double* ms, int64_t* launches);

/* Structural similarity (Sec. 3 "Metrics", after Wang et al. 2004) of B
 * frames `images` (device, B x H x W x 3 fp32 in [0, 1]) against `clean`
 * (device, H x W x 3): 11 x 11 Gaussian window of standard deviation 1.5,
 * C1 = 0.01^2, C2 = 0.03^2, biased local variance and covariance, the index
 * at every window position wholly inside the frame, averaged over positions
 * and channels, computed in fp64.  out (device) receives B doubles.  H and W
 * must be at least 11. */
sg_status sg_ssim(sg_ctx* ctx, const float* images, const float* clean, int32_t B, int32_t H, int32_t W, double* out,
                  void* stream);

/* Metrics of B*K frames against K clean frames (Sec. 3; Def. 1; Def. 2):
 * images is [B][K][H][W][3], clean is [K][H][W][3]; MSE and the footprint are
 * pooled over the K views of a variant.  nonfinite is set for a variant with
 * any non-finite value in its frames.  out: B entries (device). */
sg_status sg_metrics(sg_ctx* ctx, const float* images, const float* clean, int32_t B, int32_t K, int32_t H,
                     int32_t W, sg_metrics_t* out, void* stream);

/* sg_metrics without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and records as sg_metrics.  Its
 * partials live in a fixed 4 MiB scratch array in device memory, one per
 * device, held until the process ends: B * min(256, ceil(K*H*W / 1024))
 * partials of 32 bytes must fit (131,072 of them), otherwise SG_E_INVAL with
 * the limit in sg_last_error() and nothing is launched.  The scratch address
 * of a device is recorded by sg_ctx_create.  Every call on one device shares
 * that device's scratch and overwrites it entirely before reading it, so
 * calls that overlap on one device (different streams or threads without
 * ordering between them) race; calls ordered on one stream do not. */
sg_status sg_metrics_noalloc(sg_ctx* ctx, const float* images, const float* clean, int32_t B, int32_t K, int32_t H,
                             int32_t W, sg_metrics_t* out, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop over resident scenes.  Scenes (and their guard
 * boxes) are copied to the device once; each (scene, camera) view is
 * prepared once, keeping its clean frame and tile lists resident.  Worker
 * threads, each with its own context and HIP stream, take queued requests
 * in arrival order; pending injection campaigns on the same view are merged
 * into one batched launch (continuous batching), and launches of different
 * workers run concurrently on the device.  A request is admitted only while
 * the resident state plus the memory of running launches stays within the
 * device budget.  Latencies are measured from each request's arrival time to
 * the completion of its launch, on the host's monotonic clock. */
typedef struct sg_server sg_server;
typedef struct {
  size_t hbm_budget_bytes;   /* device bytes for resident state + running launches; 0 = no cap */
  int32_t max_slots;         /* worker threads / concurrent launches (0 = 4) */
  int32_t max_batch;         /* variants per launch (0 = 64) */
  int32_t queue_depth;       /* pending requests before submit returns SG_E_BUSY (0 = unbounded) */
  int32_t plain;             /* 1: reference FIFO path: one worker, no merging, a full render per variant */
} sg_serve_config;

/* An injection campaign scores each site as its own single-upset variant
 * (per_variant receives n_sites records); a guarded render applies all sites
 * together, clamps the result into the scene's box (Alg. 1) and scores the
 * frame (per_variant receives one record).  sites and per_variant are host
 * arrays; sites are copied at submit, per_variant must stay valid until the
 * request is done.  arrival_ns is a CLOCK_MONOTONIC time (0 = now). */
enum { SG_REQ_CAMPAIGN = 0, SG_REQ_GUARDED_RENDER = 1 };
typedef struct {
  int32_t kind;
  int32_t view_id;
  const sg_site* sites;
  int32_t n_sites;
  int32_t _pad;
  int64_t arrival_ns;
  sg_metrics_t* per_variant;
} sg_request;

typedef struct {
  sg_status status;         /* SG_OK, SG_E_NOMEM (no longer fits), SG_E_DEVICE */
  int32_t _pad;
  int64_t done_ns;
  int64_t latency_ns;       /* done_ns - arrival_ns */
  uint64_t clamps;
} sg_result;

typedef struct {
  uint64_t submitted, completed, rejected, launches, variants;
  double inj_per_s, req_per_s;             /* over first arrival .. last completion */
  double p50_us[2], p99_us[2], mean_us[2]; /* per request kind */
  uint64_t n[2];
  size_t resident_bytes;
} sg_serve_stats_t;

sg_status sg_serve_create(int32_t device, const sg_serve_config* cfg, sg_server** out);
/* Copy a scene (device or host memory, any strides) and optionally its box
 * into the server.  Must precede the first submit. */
sg_status sg_serve_add_scene(sg_server* srv, const sg_scene* scene, const sg_box* box, uint32_t box_mask,
                             int32_t* scene_id);
/* Prepare a scene for one camera (resident clean frame and tile lists).
 * Returns SG_E_NOMEM if the view does not fit the budget. */
sg_status sg_serve_add_view(sg_server* srv, int32_t scene_id, const sg_camera* cam, const sg_raster* raster,
                            int32_t* view_id);
/* Non-blocking.  SG_E_BUSY when the queue is full, SG_E_NOMEM when the
 * request could never fit the budget.  Thread-safe. */
sg_status sg_serve_submit(sg_server* srv, const sg_request* req, uint64_t* ticket);
/* SG_E_PENDING until the request is done; then fills out and forgets the ticket. */
sg_status sg_serve_poll(sg_server* srv, uint64_t ticket, sg_result* out);
sg_status sg_serve_wait(sg_server* srv, uint64_t ticket, sg_result* out, int64_t timeout_us);
sg_status sg_serve_stats(sg_server* srv, sg_serve_stats_t* out);
const char* sg_serve_last_error(const sg_server* srv);
/* Finishes queued work, then releases everything the server holds. */
void sg_serve_destroy(sg_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* SG_H */
