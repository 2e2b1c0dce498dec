"""ctypes binding of libsg (include/sg.h): argument marshalling only.

Every step of the injection path runs in the HIP kernels of libsg.so; this
module turns torch device tensors, numpy site arrays and camera objects into
the C structures of the ABI and checks status codes.  PyTorch supplies device
memory and the current HIP stream.  If libsg.so is missing the import fails
loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsg.so")

SG_OK, SG_E_INVAL, SG_E_NOMEM, SG_E_DEVICE, SG_E_BUSY, SG_E_PENDING, SG_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SG_F32, SG_F16, SG_BF16 = 0, 1, 2
SG_RNE, SG_RD, SG_RU = 0, 1, 2
SG_BOX_GLOBAL, SG_BOX_PER_PRIM = 0, 1
SG_INCREMENTAL, SG_FULL = 0, 1
SG_ENGINE_PIPELINED, SG_ENGINE_PERSISTENT = 0, 1
SG_FIELD_MASK_GUARD = 0x1F
DTYPES = {"f32": SG_F32, "f16": SG_F16, "bf16": SG_BF16}

SITE_DTYPE = np.dtype([("field", "u1"), ("bit", "u1"), ("comp", "<u2"), ("prim", "<u4")])
VARIANT_DTYPE = np.dtype([("site_off", "<u4"), ("n_sites", "<u4"), ("guard", "<u4"), ("protect", "<u4")])
SG_PROTECT_NONE, SG_PROTECT_SIGN_EXP, SG_PROTECT_VOTE = 0, 1, 2
METRICS_DTYPE = np.dtype([("sse", "<f8"), ("mse", "<f8"), ("psnr", "<f8"), ("footprint", "<f4"),
                          ("max_abs", "<f4"), ("nonfinite", "<u4"), ("catastrophic", "<u4"),
                          ("changed_px", "<u4"), ("dirty_tiles", "<u4"), ("clamps", "<u8"),
                          ("n_pixels", "<u4"), ("path", "<u4"), ("evals", "<u8"),
                          ("predicted_regions", "<u8"), ("rendered_regions", "<u8")])
assert SITE_DTYPE.itemsize == 8 and VARIANT_DTYPE.itemsize == 16 and METRICS_DTYPE.itemsize == 88
PASSES = ("variant_prep", "composite_items", "reduce", "project", "bin", "sort", "composite_full", "guard")


class SgScene(C.Structure):
    _fields_ = [("ptr", C.c_void_p * 6), ("prim_stride", C.c_int64 * 6), ("comp_stride", C.c_int64 * 6),
                ("n", C.c_int32), ("sh_degree", C.c_int32), ("dtype", C.c_int32), ("_pad", C.c_int32)]


class SgCamera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("near_z", C.c_double), ("far_z", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class SgRaster(C.Structure):
    _fields_ = [("tile", C.c_int32), ("alpha_max", C.c_float), ("alpha_min", C.c_float), ("t_min", C.c_float),
                ("cut_q", C.c_float), ("dilation", C.c_float), ("bg", C.c_float * 3)]


class SgBox(C.Structure):
    _fields_ = [("mode", C.c_int32), ("dtype", C.c_int32), ("lo", C.c_void_p * 6), ("hi", C.c_void_p * 6)]


class SgCampaignCfg(C.Structure):
    _fields_ = [("batch", C.c_int32), ("streams", C.c_int32), ("threads", C.c_int32), ("engine", C.c_int32)]


class SgTune(C.Structure):
    _fields_ = [("tile", C.c_int32), ("batch", C.c_int32), ("streams", C.c_int32), ("threads", C.c_int32),
                ("wgs_per_cu", C.c_int32), ("resume", C.c_int32), ("graphs", C.c_int32), ("from_cache", C.c_int32),
                ("inj_per_s", C.c_double), ("trials", C.c_int32), ("grid", C.c_int32)]


class SgServeConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32), ("max_batch", C.c_int32),
                ("queue_depth", C.c_int32), ("plain", C.c_int32)]


class SgRequest(C.Structure):
    _fields_ = [("kind", C.c_int32), ("view_id", C.c_int32), ("sites", C.c_void_p), ("n_sites", C.c_int32),
                ("_pad", C.c_int32), ("arrival_ns", C.c_int64), ("per_variant", C.c_void_p)]


class SgResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("_pad", C.c_int32), ("done_ns", C.c_int64), ("latency_ns", C.c_int64),
                ("clamps", C.c_uint64)]


class SgServeStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("launches", C.c_uint64), ("variants", C.c_uint64), ("inj_per_s", C.c_double),
                ("req_per_s", C.c_double), ("p50_us", C.c_double * 2), ("p99_us", C.c_double * 2),
                ("mean_us", C.c_double * 2), ("n", C.c_uint64 * 2), ("resident_bytes", C.c_size_t)]


SG_REQ_CAMPAIGN, SG_REQ_GUARDED_RENDER = 0, 1


class SgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsg status {code}: {msg}")
        self.code = code


def _load():
    # torch ships its own HIP runtime under the same soname as ROCm's; loading
    # torch first makes libsg resolve to that one copy, so device pointers,
    # streams and the runtime state are shared by both.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_size_t
    P = C.POINTER
    sig = {
        "sg_ctx_create": (i32, [i32, sz, P(vp)]),
        "sg_ctx_destroy": (None, [vp]),
        "sg_last_error": (C.c_char_p, []),
        "sg_ctx_bytes": (sz, [vp]),
        "sg_cast": (i32, [vp, vp, vp, i64, i32, i32, vp]),
        "sg_inject": (i32, [vp, P(SgScene), vp, i32, vp, vp]),
        "sg_restore": (i32, [vp, P(SgScene), vp, i32, vp, vp]),
        "sg_guard_box": (i32, [vp, P(SgScene), u32, P(SgBox), vp]),
        "sg_guard": (i32, [vp, P(SgScene), P(SgBox), u32, u64, vp, vp, vp]),
        "sg_render": (i32, [vp, P(SgScene), P(SgCamera), P(SgRaster), P(SgBox), u32, vp, vp, vp, vp]),
        "sg_prepare": (i32, [vp, P(SgScene), P(SgCamera), P(SgRaster), P(vp), vp]),
        "sg_prep_destroy": (None, [vp]),
        "sg_prep_frame": (vp, [vp]),
        "sg_prep_instances": (i64, [vp]),
        "sg_prep_copy_frame": (i32, [vp, vp, vp]),
        "sg_render_batch": (i32, [vp, vp, vp, i32, vp, i32, P(SgBox), u32, vp, vp, i32, vp]),
        "sg_campaign": (i32, [vp, vp, vp, i32, vp, i32, P(SgBox), u32, P(SgCampaignCfg), vp, vp]),
        "sg_campaign_views": (i32, [vp, vp, i32, vp, i32, vp, i32, P(SgBox), u32, P(SgCampaignCfg), vp, vp]),
        "sg_campaign_scenes": (i32, [vp, vp, i32, vp, i32, vp, vp, i32, vp, u32, P(SgCampaignCfg), vp, vp]),
        "sg_render_batch_views": (i32, [vp, vp, i32, vp, i32, vp, i32, P(SgBox), u32, vp, vp, i32, vp]),
        "sg_metrics": (i32, [vp, vp, vp, i32, i32, i32, i32, vp, vp]),
        "sg_metrics_noalloc": (i32, [vp, vp, vp, i32, i32, i32, i32, vp, vp]),
        "sg_ssim": (i32, [vp, vp, vp, i32, i32, i32, vp, vp]),
        "sg_autotune": (i32, [vp, P(SgScene), P(SgCamera), P(SgRaster), vp, i32, i32, i32, C.c_char_p, P(SgTune), vp]),
        "sg_ctx_timing": (i32, [vp, i32]),
        "sg_serve_create": (i32, [i32, P(SgServeConfig), P(vp)]),
        "sg_serve_add_scene": (i32, [vp, P(SgScene), P(SgBox), u32, P(i32)]),
        "sg_serve_add_view": (i32, [vp, i32, P(SgCamera), P(SgRaster), P(i32)]),
        "sg_serve_submit": (i32, [vp, P(SgRequest), P(u64)]),
        "sg_serve_poll": (i32, [vp, u64, P(SgResult)]),
        "sg_serve_wait": (i32, [vp, u64, P(SgResult), i64]),
        "sg_serve_stats": (i32, [vp, P(SgServeStats)]),
        "sg_serve_last_error": (C.c_char_p, [vp]),
        "sg_serve_destroy": (None, [vp]),
        "sg_ctx_set_persistent": (i32, [vp, i32]),
        "sg_ctx_set_persistent_grid": (i32, [vp, i32]),
        "sg_ctx_set_resume": (i32, [vp, i32]),
        "sg_ctx_set_graphs": (i32, [vp, i32]),
        "sg_ctx_pass_times": (i32, [vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
EXPORTED = ("sg_ctx_create", "sg_ctx_destroy", "sg_last_error", "sg_ctx_bytes", "sg_cast", "sg_inject",
            "sg_restore", "sg_guard_box", "sg_guard", "sg_render", "sg_prepare", "sg_prep_destroy",
            "sg_prep_frame", "sg_prep_instances", "sg_prep_copy_frame", "sg_render_batch", "sg_render_batch_views", "sg_campaign",
            "sg_campaign_views", "sg_campaign_scenes", "sg_autotune", "sg_metrics", "sg_metrics_noalloc", "sg_ssim",
            "sg_ctx_timing", "sg_ctx_pass_times", "sg_ctx_set_persistent", "sg_ctx_set_persistent_grid", "sg_ctx_set_resume", "sg_ctx_set_graphs",
            "sg_serve_create",
            "sg_serve_add_scene", "sg_serve_add_view", "sg_serve_submit", "sg_serve_poll", "sg_serve_wait",
            "sg_serve_stats", "sg_serve_last_error", "sg_serve_destroy")


def check(code):
    if code != SG_OK:
        raise SgError(code, LIB.sg_last_error().decode(errors="replace"))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def camera_struct(cam) -> SgCamera:
    c = SgCamera()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float64).reshape(-1)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float64)]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.near_z, c.far_z = float(cam.near), float(cam.far)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def raster_struct(tile=16, alpha_max=0.99, alpha_min=1.0 / 255.0, t_min=1e-4, cut_q=9.0, dilation=0.3,
                  bg=(1.0, 1.0, 1.0)) -> SgRaster:
    r = SgRaster()
    r.tile, r.alpha_max, r.alpha_min, r.t_min, r.cut_q, r.dilation = tile, alpha_max, alpha_min, t_min, cut_q, dilation
    r.bg[:] = list(bg)
    return r


def sites_array(field, comp, prim, bit) -> np.ndarray:
    a = np.zeros(len(field), SITE_DTYPE)
    a["field"], a["comp"], a["prim"], a["bit"] = field, comp, prim, bit
    return a


def variants_array(site_off, n_sites, guard=0, protect=0) -> np.ndarray:
    a = np.zeros(len(site_off), VARIANT_DTYPE)
    a["site_off"], a["n_sites"], a["guard"], a["protect"] = site_off, n_sites, guard, protect
    return a


class Context:
    """An sg_ctx on a HIP device."""

    def __init__(self, device: int = 0, budget: int = 0):
        h = C.c_void_p()
        check(LIB.sg_ctx_create(device, budget, C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            LIB.sg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bytes(self) -> int:
        return int(LIB.sg_ctx_bytes(self.h))

    def set_persistent(self, wgs_per_cu: int):
        check(LIB.sg_ctx_set_persistent(self.h, int(wgs_per_cu)))

    def set_persistent_grid(self, total_wgs: int):
        check(LIB.sg_ctx_set_persistent_grid(self.h, int(total_wgs)))

    def set_resume(self, spacing: int):
        """Checkpoint spacing of scenes prepared from now on (0 = no resume state)."""
        check(LIB.sg_ctx_set_resume(self.h, int(spacing)))

    def set_graphs(self, enable: bool):
        check(LIB.sg_ctx_set_graphs(self.h, 1 if enable else 0))

    def timing(self, enable: bool):
        check(LIB.sg_ctx_timing(self.h, 1 if enable else 0))

    def pass_times(self) -> dict:
        ms = np.zeros(len(PASSES), np.float64)
        n = np.zeros(len(PASSES), np.int64)
        check(LIB.sg_ctx_pass_times(self.h, ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PASSES)}

    # -- storage --------------------------------------------------------------
    def cast(self, src_f32, dtype: int, rounding: int = SG_RNE):
        import torch
        src = src_f32.contiguous()
        out = torch.empty(src.shape, dtype=torch.int32 if dtype == SG_F32 else torch.int16, device=src.device)
        check(LIB.sg_cast(self.h, _ptr(src), _ptr(out), src.numel(), dtype, rounding, _stream()))
        return out

    def inject(self, scene, sites: np.ndarray, saved=None):
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        check(LIB.sg_inject(self.h, C.byref(scene.st), s.ctypes.data_as(C.c_void_p), len(s), _ptr(saved), _stream()))

    def restore(self, scene, sites: np.ndarray):
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        check(LIB.sg_restore(self.h, C.byref(scene.st), s.ctypes.data_as(C.c_void_p), len(s), None, _stream()))

    # -- guard ----------------------------------------------------------------
    def guard_box(self, scene, field_mask: int = SG_FIELD_MASK_GUARD):
        import torch
        box = Box(scene.dtype, SG_BOX_GLOBAL)
        for f in range(6):
            if (field_mask >> f) & 1 and scene.ncomp[f]:
                box.set(f, torch.empty(scene.ncomp[f], dtype=scene.words[f].dtype, device=scene.words[f].device),
                        torch.empty(scene.ncomp[f], dtype=scene.words[f].dtype, device=scene.words[f].device))
        check(LIB.sg_guard_box(self.h, C.byref(scene.st), field_mask, C.byref(box.st), _stream()))
        return box

    def guard(self, scene, box, field_mask: int = SG_FIELD_MASK_GUARD, threshold: int = 0):
        import torch
        cnt = torch.zeros(2, dtype=torch.int64, device=scene.words[0].device)
        alert = torch.zeros(1, dtype=torch.int32, device=scene.words[0].device)
        check(LIB.sg_guard(self.h, C.byref(scene.st), C.byref(box.st), field_mask, threshold, _ptr(cnt), _ptr(alert),
                           _stream()))
        return cnt, alert

    # -- rendering -------------------------------------------------------------
    def render(self, scene, cam, raster=None, box=None, box_mask: int = SG_FIELD_MASK_GUARD, image=None,
               clean=None, metrics=None):
        camst = camera_struct(cam)
        r = raster if raster is not None else raster_struct()
        check(LIB.sg_render(self.h, C.byref(scene.st), C.byref(camst), C.byref(r),
                            C.byref(box.st) if box is not None else None, box_mask if box is not None else 0,
                            _ptr(image), _ptr(clean), _ptr(metrics), _stream()))

    def prepare(self, scene, cam, raster=None):
        return Prep(self, scene, cam, raster)

    def render_batch(self, prep, sites: np.ndarray, variants: np.ndarray, box=None, box_mask: int = SG_FIELD_MASK_GUARD,
                     images=None, metrics=None, mode: int = SG_INCREMENTAL):
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        v = np.ascontiguousarray(variants, VARIANT_DTYPE)
        check(LIB.sg_render_batch(self.h, prep.h, s.ctypes.data_as(C.c_void_p), len(s), v.ctypes.data_as(C.c_void_p),
                                  len(v), C.byref(box.st) if box is not None else None,
                                  box_mask if box is not None else 0, _ptr(images), _ptr(metrics), mode, _stream()))

    def campaign(self, prep, sites: np.ndarray, variants: np.ndarray, metrics, box=None,
                 box_mask: int = SG_FIELD_MASK_GUARD, batch: int | None = None, streams: int = 8, threads: int = 2,
                 engine: int = SG_ENGINE_PIPELINED):
        """All variants of a campaign in batches of `batch` (default 32), over
        `streams` device streams enqueued by `threads` host threads (pipelined
        engine), or in persistent chunks of `batch` variants (default: as many
        as fit); records into `metrics`.  `prep` may be a list of views of one
        scene (pooled records)."""
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        v = np.ascontiguousarray(variants, VARIANT_DTYPE)
        if batch is None:
            batch = 0 if engine == SG_ENGINE_PERSISTENT else 32
        cfg = SgCampaignCfg(int(batch), int(streams), int(threads), int(engine))
        bx = C.byref(box.st) if box is not None else None
        mask = box_mask if box is not None else 0
        if isinstance(prep, (list, tuple)):
            hs = (C.c_void_p * len(prep))(*[p.h for p in prep])
            check(LIB.sg_campaign_views(self.h, hs, len(prep), s.ctypes.data_as(C.c_void_p), len(s),
                                        v.ctypes.data_as(C.c_void_p), len(v), bx, mask, C.byref(cfg), _ptr(metrics),
                                        _stream()))
        else:
            check(LIB.sg_campaign(self.h, prep.h, s.ctypes.data_as(C.c_void_p), len(s), v.ctypes.data_as(C.c_void_p),
                                  len(v), bx, mask, C.byref(cfg), _ptr(metrics), _stream()))

    def campaign_scenes(self, preps, sites: np.ndarray, variants: np.ndarray, scene_of, metrics, boxes=None,
                        box_mask: int = SG_FIELD_MASK_GUARD, batch: int | None = None, streams: int = 8,
                        threads: int = 2, engine: int = SG_ENGINE_PIPELINED):
        """Variants of several prepared scenes in one campaign: variant j belongs
        to preps[scene_of[j]]; boxes (optional) lists each scene's box or None."""
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        v = np.ascontiguousarray(variants, VARIANT_DTYPE)
        sc = np.ascontiguousarray(scene_of, np.uint16)
        assert sc.shape == (len(v),)
        if batch is None:
            batch = 0 if engine == SG_ENGINE_PERSISTENT else 32
        cfg = SgCampaignCfg(int(batch), int(streams), int(threads), int(engine))
        hs = (C.c_void_p * len(preps))(*[p.h for p in preps])
        bxs = None
        if boxes is not None:
            bxs = (C.c_void_p * len(preps))(*[C.cast(C.pointer(b.st), C.c_void_p) if b is not None else None
                                              for b in boxes])
        check(LIB.sg_campaign_scenes(self.h, hs, len(preps), s.ctypes.data_as(C.c_void_p), len(s),
                                     v.ctypes.data_as(C.c_void_p), sc.ctypes.data_as(C.c_void_p), len(v), bxs,
                                     box_mask if boxes is not None else 0, C.byref(cfg), _ptr(metrics), _stream()))

    def render_batch_views(self, preps, sites: np.ndarray, variants: np.ndarray, metrics, per_view=None, box=None,
                           box_mask: int = SG_FIELD_MASK_GUARD, mode: int = SG_INCREMENTAL):
        """Every variant in each of the K views `preps`; pooled records into
        `metrics` (B), per-view records into `per_view` (K x B) when given."""
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        v = np.ascontiguousarray(variants, VARIANT_DTYPE)
        hs = (C.c_void_p * len(preps))(*[p.h for p in preps])
        check(LIB.sg_render_batch_views(self.h, hs, len(preps), s.ctypes.data_as(C.c_void_p), len(s),
                                        v.ctypes.data_as(C.c_void_p), len(v),
                                        C.byref(box.st) if box is not None else None,
                                        box_mask if box is not None else 0, _ptr(metrics), _ptr(per_view), mode,
                                        _stream()))

    def autotune(self, scene, cam, sites: np.ndarray, raster=None, fixed_batch: int = 0, max_batch: int = 0,
                 cache: str | None = None) -> dict:
        """Measured launch configuration for campaigns on this scene and camera
        (see sg_autotune); the context's own settings are left unchanged."""
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        out = SgTune()
        check(LIB.sg_autotune(self.h, C.byref(scene.st), C.byref(camera_struct(cam)),
                              C.byref(raster) if raster is not None else None, s.ctypes.data_as(C.c_void_p), len(s),
                              int(fixed_batch), int(max_batch), cache.encode() if cache else None, C.byref(out),
                              _stream()))
        return {k: getattr(out, k) for k, _ in SgTune._fields_ if not k.startswith("_")}

    def apply_tune(self, t: dict):
        """Context settings of a tuned configuration (prepare with tile=t["tile"] afterwards)."""
        self.set_persistent(t["wgs_per_cu"])
        self.set_persistent_grid(t.get("grid", 0))
        self.set_resume(t["resume"])
        self.set_graphs(bool(t["graphs"]))

    def ssim(self, images, clean, out=None):
        """SSIM of each frame of `images` (B, H, W, 3) against `clean` (H, W, 3);
        returns a float64 device tensor of B values."""
        import torch
        B, H, W = images.shape[0], images.shape[1], images.shape[2]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=images.device)
        check(LIB.sg_ssim(self.h, _ptr(images), _ptr(clean), B, H, W, _ptr(out), _stream()))
        return out

    def metrics(self, images, clean, B, K, H, W, out):
        check(LIB.sg_metrics(self.h, _ptr(images), _ptr(clean), B, K, H, W, _ptr(out), _stream()))

    def metrics_noalloc(self, images, clean, B, K, H, W, out):
        """sg_metrics_noalloc: the same records with no device allocation."""
        check(LIB.sg_metrics_noalloc(self.h, _ptr(images), _ptr(clean), B, K, H, W, _ptr(out), _stream()))


class DeviceScene:
    """Stored words of a scene on the device (component-major (C_f, N) tensors)."""

    def __init__(self, words, n: int, sh_degree: int, dtype: int):
        self.words = words
        self.n, self.sh_degree, self.dtype = n, sh_degree, dtype
        self.ncomp = [3, 3, 4, 1, 3, 3 * ((sh_degree + 1) ** 2 - 1)]
        st = SgScene()
        for f in range(6):
            w = words[f]
            st.ptr[f] = w.data_ptr() if w.numel() else None
            st.prim_stride[f] = 1
            st.comp_stride[f] = n
        st.n, st.sh_degree, st.dtype = n, sh_degree, dtype
        self.st = st

    @staticmethod
    def upload(ctx: Context, scene, fmt: str, device="cuda"):
        """Cast a synthetic fp32 scene into its storage format on the device."""
        import torch
        dt = DTYPES[fmt]
        words = []
        for f in scene.fields:
            src = torch.from_numpy(np.ascontiguousarray(f, np.float32)).to(device)
            words.append(ctx.cast(src, dt) if src.numel() else
                         torch.empty(src.shape, dtype=torch.int32 if dt == SG_F32 else torch.int16, device=device))
        return DeviceScene(words, scene.n, scene.sh_degree, dt)

    def clone(self):
        return DeviceScene([w.clone() for w in self.words], self.n, self.sh_degree, self.dtype)

    def host_words(self):
        """Stored words as unsigned numpy arrays (uint32 / uint16)."""
        out = []
        for w in self.words:
            a = w.cpu().numpy()
            out.append(a.view(np.uint32) if self.dtype == SG_F32 else a.view(np.uint16))
        return out


class Box:
    def __init__(self, dtype: int, mode: int):
        self.st = SgBox()
        self.st.mode, self.st.dtype = mode, dtype
        self.lo, self.hi = [None] * 6, [None] * 6

    def set(self, f, lo, hi):
        self.lo[f], self.hi[f] = lo, hi
        self.st.lo[f] = lo.data_ptr()
        self.st.hi[f] = hi.data_ptr()

    @staticmethod
    def per_prim(ctx: Context, lo_f32, hi_f32, fmt: str, device="cuda"):
        """Per-primitive box from fp32 bounds (lists by field), cast outward
        (lo toward -Inf, hi toward +Inf) into the storage format."""
        import torch
        dt = DTYPES[fmt]
        b = Box(dt, SG_BOX_PER_PRIM)
        for f in range(6):
            if lo_f32[f] is None:
                continue
            lo = torch.from_numpy(np.ascontiguousarray(lo_f32[f], np.float32)).to(device)
            hi = torch.from_numpy(np.ascontiguousarray(hi_f32[f], np.float32)).to(device)
            b.set(f, ctx.cast(lo, dt, SG_RD), ctx.cast(hi, dt, SG_RU))
        return b

    def host_words(self, f):
        a, b = self.lo[f].cpu().numpy(), self.hi[f].cpu().numpy()
        if self.st.dtype == SG_F32:
            return a.view(np.uint32), b.view(np.uint32)
        return a.view(np.uint16), b.view(np.uint16)


class Prep:
    """A prepared (resident) clean scene: sg_prepare / sg_prep_destroy."""

    def __init__(self, ctx: Context, scene: DeviceScene, cam, raster=None):
        self.ctx, self.scene, self.cam = ctx, scene, cam
        self.camst = camera_struct(cam)
        self.raster = raster if raster is not None else raster_struct()
        h = C.c_void_p()
        check(LIB.sg_prepare(ctx.h, C.byref(scene.st), C.byref(self.camst), C.byref(self.raster), C.byref(h),
                             _stream()))
        self.h = h

    def frame_ptr(self) -> int:
        return int(LIB.sg_prep_frame(self.h))

    def frame(self):
        """The clean frame as a (H, W, 3) device tensor (a copy)."""
        import torch
        out = torch.empty((self.cam.height, self.cam.width, 3), dtype=torch.float32, device="cuda")
        check(LIB.sg_prep_copy_frame(self.h, _ptr(out), _stream()))
        return out

    def instances(self) -> int:
        return int(LIB.sg_prep_instances(self.h))

    def close(self):
        if getattr(self, "h", None):
            LIB.sg_prep_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def metrics_tensor(B: int):
    import torch
    return torch.zeros(B * METRICS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")


def read_metrics(t) -> np.ndarray:
    return t.cpu().numpy().view(METRICS_DTYPE)


class Server:
    """sg_server: resident scenes and views, a request queue and worker threads."""

    def __init__(self, device: int = 0, budget: int = 0, max_slots: int = 4, max_batch: int = 64,
                 queue_depth: int = 0, plain: bool = False):
        cfg = SgServeConfig(budget, max_slots, max_batch, queue_depth, 1 if plain else 0)
        h = C.c_void_p()
        check(LIB.sg_serve_create(device, C.byref(cfg), C.byref(h)))
        self.h = h
        self._live = {}

    def _check(self, code):
        if code != SG_OK:
            raise SgError(code, LIB.sg_serve_last_error(self.h).decode(errors="replace"))

    def add_scene(self, scene: "DeviceScene", box: "Box" = None, box_mask: int = SG_FIELD_MASK_GUARD) -> int:
        sid = C.c_int32()
        self._check(LIB.sg_serve_add_scene(self.h, C.byref(scene.st), C.byref(box.st) if box is not None else None,
                                           box_mask if box is not None else 0, C.byref(sid)))
        return sid.value

    def add_view(self, scene_id: int, cam, raster=None) -> int:
        vid = C.c_int32()
        camst = camera_struct(cam)
        self._check(LIB.sg_serve_add_view(self.h, scene_id, C.byref(camst),
                                          C.byref(raster) if raster is not None else None, C.byref(vid)))
        return vid.value

    def submit(self, kind: int, view: int, sites: np.ndarray, arrival_ns: int = 0) -> int:
        s = np.ascontiguousarray(sites, SITE_DTYPE)
        out = np.zeros(len(s) if kind == SG_REQ_CAMPAIGN else 1, METRICS_DTYPE)
        req = SgRequest(kind, view, s.ctypes.data_as(C.c_void_p), len(s), 0, int(arrival_ns),
                        out.ctypes.data_as(C.c_void_p))
        t = C.c_uint64()
        self._check(LIB.sg_serve_submit(self.h, C.byref(req), C.byref(t)))
        self._live[t.value] = (s, out)
        return t.value

    def wait(self, ticket: int, timeout_s: float = 60.0):
        """(result dict, per-variant records) once the request is done."""
        r = SgResult()
        code = LIB.sg_serve_wait(self.h, ticket, C.byref(r), int(timeout_s * 1e6))
        if code == SG_E_PENDING:
            raise TimeoutError(f"request {ticket} not done after {timeout_s} s")
        self._check(code)
        _, out = self._live.pop(ticket)
        return {"status": r.status, "latency_ns": r.latency_ns, "done_ns": r.done_ns, "clamps": r.clamps}, out

    def poll(self, ticket: int):
        r = SgResult()
        code = LIB.sg_serve_poll(self.h, ticket, C.byref(r))
        if code == SG_E_PENDING:
            return None
        self._check(code)
        _, out = self._live.pop(ticket)
        return {"status": r.status, "latency_ns": r.latency_ns, "done_ns": r.done_ns, "clamps": r.clamps}, out

    def stats(self) -> dict:
        st = SgServeStats()
        self._check(LIB.sg_serve_stats(self.h, C.byref(st)))
        return {"submitted": st.submitted, "completed": st.completed, "rejected": st.rejected,
                "launches": st.launches, "variants": st.variants, "inj_per_s": st.inj_per_s,
                "req_per_s": st.req_per_s,
                "campaign": {"p50_us": st.p50_us[0], "p99_us": st.p99_us[0], "mean_us": st.mean_us[0], "n": st.n[0]},
                "guarded_render": {"p50_us": st.p50_us[1], "p99_us": st.p99_us[1], "mean_us": st.mean_us[1],
                                   "n": st.n[1]},
                "resident_bytes": st.resident_bytes}

    def close(self):
        if getattr(self, "h", None):
            LIB.sg_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
