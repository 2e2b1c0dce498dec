"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no format casts, bit flips, clamps, projection or
compositing).  Both sides receive the same fp32 arrays and do every step of
the method themselves.

Scenes stand in for the trained 3DGS models of the paper (Sec. 3, "Scenes and
models", Table 1), which are not available: the primitive counts follow the
paper (134,826 for the chair model, a 5% subsample of 6,741, the 2,056,645
primitives of the real scene in Sec. 5.6).  The value distributions are the
ones `make_scene` states: uniform or clustered means, log-scales around -4,
uniform quaternion directions, opacity logits around 0, uniform base colours
and small higher-order coefficients.

Layout: every field is a C-contiguous float32 array of shape (C_f, N)
(component-major, "SoA"), which is what the device kernels read coalesced.
Fields, in storage order (Sec. 3, "Parameter layout"):
    0 means (3), 1 log_scales (3), 2 quats (4, w x y z), 3 opacity logit (1),
    4 sh_dc (3), 5 sh_rest (3 * ((L+1)^2 - 1), coefficient-major: component
    c = 3 * k + channel for coefficient k = 1 .. (L+1)^2 - 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FIELD_NAMES = ("means", "log_scales", "quats", "opacity", "sh_dc", "sh_rest")
MEANS, LOG_SCALES, QUATS, OPACITY, SH_DC, SH_REST = range(6)


def field_components(sh_degree: int) -> tuple[int, ...]:
    """Number of stored components per field for a given SH degree."""
    return (3, 3, 4, 1, 3, 3 * ((sh_degree + 1) ** 2 - 1))


@dataclass
class Scene:
    """A synthetic scene: six fp32 SoA fields of shape (C_f, N)."""
    fields: list            # list of 6 np.ndarray float32 (C_f, N); sh_rest may be (0, N)
    sh_degree: int
    seed: int

    @property
    def n(self) -> int:
        return int(self.fields[0].shape[1])

    def subset(self, n: int) -> "Scene":
        """The first n primitives (the paper subsamples trained models, Sec. 5.6)."""
        return Scene([np.ascontiguousarray(f[:, :n]) for f in self.fields], self.sh_degree, self.seed)


def make_scene(n: int, seed: int, sh_degree: int = 0, means: str = "uniform",
               n_clusters: int = 64) -> Scene:
    """Draw a scene.  Draw order is fixed: means, log-scales, quaternions,
    opacity logits, degree-0 colours, higher-order coefficients.

    means="uniform": U[-1, 1]^3.  means="clusters": n_clusters anisotropic
    Gaussian clusters in a 20^3 box (centres U[-8, 8]^3, per-axis std
    U[0.3, 2.5] under a random rotation, clipped to [-10, 10]^3).
    """
    rng = np.random.default_rng(seed)
    if means == "uniform":
        mu = rng.uniform(-1.0, 1.0, size=(n, 3))
    elif means == "clusters":
        centres = rng.uniform(-8.0, 8.0, size=(n_clusters, 3))
        stds = rng.uniform(0.3, 2.5, size=(n_clusters, 3))
        rots = _random_rotations(rng, n_clusters)
        which = rng.integers(0, n_clusters, size=n)
        z = rng.standard_normal(size=(n, 3)) * stds[which]
        mu = centres[which] + np.einsum("nij,nj->ni", rots[which], z)
        mu = np.clip(mu, -10.0, 10.0)
    else:
        raise ValueError(means)
    log_s = rng.normal(-4.0, 0.5, size=(n, 3))
    q = rng.standard_normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = rng.normal(0.0, 1.5, size=(n, 1))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    # Degree-0 coefficient whose colour is rgb: the constant band has value
    # 1 / (2 sqrt(pi)), so the coefficient is (rgb - 1/2) * 2 sqrt(pi).
    dc = (rgb - 0.5) * (2.0 * math.sqrt(math.pi))
    n_rest = 3 * ((sh_degree + 1) ** 2 - 1)
    rest = rng.normal(0.0, 0.1, size=(n, n_rest)) if n_rest else np.zeros((n, 0))
    fields = [np.ascontiguousarray(a.T.astype(np.float32)) for a in (mu, log_s, q, opac, dc, rest)]
    return Scene(fields, sh_degree, seed)


def _random_rotations(rng, k):
    q = rng.standard_normal(size=(k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).
    World point X maps to camera point R X + t."""
    R: np.ndarray          # (3, 3) float64
    t: np.ndarray          # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.01
    far: float = 1e10


def make_camera(width: int, height: int, distance: float = 3.0, fov_x_deg: float = 60.0) -> Camera:
    """Camera on the -z axis at the given distance looking at the origin,
    horizontal field of view fov_x_deg, principal point at the image centre."""
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(np.eye(3), np.array([0.0, 0.0, distance]), f, f, width / 2.0, height / 2.0,
                  int(width), int(height))


def make_orbit_cameras(k: int, width: int, height: int, distance: float = 3.0, fov_x_deg: float = 60.0,
                       elevation_deg: float = 15.0) -> list:
    """k cameras evenly spaced in azimuth around the origin, each tilted by
    elevation_deg and looking at the origin from the given distance (R is a
    rotation about x by the elevation times a rotation about y by 2 pi j / k)."""
    base = make_camera(width, height, distance, fov_x_deg)
    e = math.radians(elevation_deg)
    rx = np.array([[1.0, 0.0, 0.0], [0.0, math.cos(e), -math.sin(e)], [0.0, math.sin(e), math.cos(e)]])
    cams = []
    for j in range(k):
        a = 2.0 * math.pi * j / k
        ry = np.array([[math.cos(a), 0.0, math.sin(a)], [0.0, 1.0, 0.0], [-math.sin(a), 0.0, math.cos(a)]])
        cams.append(Camera(rx @ ry, base.t.copy(), base.fx, base.fy, base.cx, base.cy, base.width, base.height))
    return cams


@dataclass
class Sites:
    """Fault sites (field, primitive, component, bit), Sec. 3 "Single-bit upset model"."""
    field: np.ndarray   # uint8
    comp: np.ndarray    # uint16
    prim: np.ndarray    # uint32
    bit: np.ndarray     # uint8

    def __len__(self):
        return int(self.field.shape[0])

    def take(self, idx) -> "Sites":
        return Sites(self.field[idx], self.comp[idx], self.prim[idx], self.bit[idx])


def _mk_sites(field, comp, prim, bit) -> Sites:
    return Sites(np.asarray(field, np.uint8), np.asarray(comp, np.uint16),
                 np.asarray(prim, np.uint32), np.asarray(bit, np.uint8))


def make_sites_uniform(n_prims: int, sh_degree: int, count: int, seed: int, width_bits: int = 32,
                       fields=(MEANS, LOG_SCALES, QUATS, OPACITY, SH_DC)) -> Sites:
    """Sites uniform over (field in `fields`) x primitive x component x bit."""
    rng = np.random.default_rng(seed)
    comps = field_components(sh_degree)
    f = rng.choice(np.asarray(fields), size=count)
    c = np.array([rng.integers(0, comps[x]) for x in f], dtype=np.int64) if count else np.zeros(0, np.int64)
    p = rng.integers(0, n_prims, size=count)
    b = rng.integers(0, width_bits, size=count)
    return _mk_sites(f, c, p, b)


def make_sites_stratified(n_prims: int, sh_degree: int, per_field: int, seed: int, width_bits: int,
                          fields=(MEANS, LOG_SCALES, QUATS, OPACITY, SH_DC, SH_REST)) -> Sites:
    """per_field sites for each field; site j of a field has bit j mod width_bits
    (every bit position equally represented), primitive and component uniform."""
    rng = np.random.default_rng(seed)
    comps = field_components(sh_degree)
    out_f, out_c, out_p, out_b = [], [], [], []
    for f in fields:
        out_f.append(np.full(per_field, f))
        out_c.append(rng.integers(0, comps[f], size=per_field))
        out_p.append(rng.integers(0, n_prims, size=per_field))
        out_b.append(np.arange(per_field) % width_bits)
    return _mk_sites(np.concatenate(out_f), np.concatenate(out_c), np.concatenate(out_p), np.concatenate(out_b))


def make_sites_dose(n_prims: int, sh_degree: int, k: int, seed: int, width_bits: int) -> Sites:
    """k distinct sites uniform over every stored bit of the model
    (Sec. 5.4: upsets drawn uniformly over the entire stored bit budget)."""
    rng = np.random.default_rng(seed)
    comps = np.asarray(field_components(sh_degree), np.int64)
    words_per_field = comps * n_prims
    total_bits = int(words_per_field.sum()) * width_bits
    idx = rng.choice(total_bits, size=k, replace=False)
    word, bit = idx // width_bits, idx % width_bits
    starts = np.concatenate([[0], np.cumsum(words_per_field)])
    f = np.searchsorted(starts, word, side="right") - 1
    w = word - starts[f]
    c, p = w // n_prims, w % n_prims
    return _mk_sites(f, c, p, bit)


def make_box_jitter(scene: Scene, seed: int, sigma: float = 0.2, fields=(0, 1, 2, 3, 4)):
    """Per-primitive guard box standing in for a training range: for every
    guarded component, lo <= value - |a| and hi >= value + |b| with a, b ~
    N(0, sigma) independent, each bound rounded outward to fp32 so that
    lo <= value <= hi holds exactly.  Returns (lo, hi): lists of 6 arrays
    (None for unguarded fields)."""
    rng = np.random.default_rng(seed)
    lo, hi = [None] * 6, [None] * 6
    for f in fields:
        v = scene.fields[f].astype(np.float64)
        a = np.abs(rng.normal(0.0, sigma, size=v.shape))
        b = np.abs(rng.normal(0.0, sigma, size=v.shape))
        l64, h64 = v - a, v + b
        l32, h32 = l64.astype(np.float32), h64.astype(np.float32)
        l32 = np.where(l32.astype(np.float64) > l64, np.nextafter(l32, np.float32(-np.inf)), l32)
        h32 = np.where(h32.astype(np.float64) < h64, np.nextafter(h32, np.float32(np.inf)), h32)
        lo[f], hi[f] = np.ascontiguousarray(l32), np.ascontiguousarray(h32)
    return lo, hi


def make_arrivals(rate_per_s: float, duration_s: float, seed: int) -> np.ndarray:
    """Poisson arrival times (seconds) at the given mean rate."""
    rng = np.random.default_rng(seed)
    n = rng.poisson(rate_per_s * duration_s)
    return np.sort(rng.uniform(0.0, duration_s, size=n))
