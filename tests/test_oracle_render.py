"""Pins for oracle.render / oracle.sh / oracle.metrics: closed forms of one and
several on-axis Gaussians, the transmittance stop, telescoping with white
primitives, the product form with black ones, permutation invariance, SH
orthonormality, and agreement with the independent scalar renderer."""
import json
import math
import os

import numpy as np
import pytest

from oracle import formats, metrics, render, scalar, sh
from paper_2606_21791_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
Y00 = 0.5 / math.sqrt(math.pi)


def _scene_from(prims, sh_degree=0):
    n = len(prims)
    K = (sh_degree + 1) ** 2 - 1
    f = [np.zeros((3, n)), np.zeros((3, n)), np.zeros((4, n)), np.zeros((1, n)), np.zeros((3, n)),
         np.zeros((3 * K, n))]
    for i, p in enumerate(prims):
        f[0][:, i] = p["mean"]
        f[1][:, i] = p["log_scale"]
        f[2][:, i] = p["quat"]
        f[3][0, i] = p["logit"]
        f[4][:, i] = p["dc"]
        if K:
            f[5][:, i] = np.asarray(p["rest"]).reshape(-1)
    return f


def _cam(w, h, dist=3.0, cx=None, cy=None):
    c = synth.make_camera(w, h, distance=dist)
    if cx is not None:
        c.cx, c.cy = cx, cy
    return c


def _prim(mean, s, logit, rgb, quat=(1, 0, 0, 0)):
    return dict(mean=list(mean), log_scale=[math.log(s)] * 3, quat=list(quat), logit=logit,
                dc=[(c - 0.5) / Y00 for c in rgb], rest=[])


def _render(prims, cam, deg=0):
    vals = _scene_from(prims, deg)
    pr = render.project(vals, deg, cam)
    return pr, render.render(pr, cam)


def test_single_isotropic_gaussian_closed_form():
    rng = np.random.default_rng(0)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    cam = _cam(64, 48)
    s, logit, rgb = 0.2, 0.7, (0.2, 0.6, 0.9)
    _, out = _render([_prim((0, 0, 0), s, logit, rgb, quat=q)], cam)
    var = (cam.fx * s / 3.0) ** 2 + 0.3
    o = 1 / (1 + math.exp(-logit))
    ys, xs = np.mgrid[0:48, 0:64] + 0.5
    r2 = (xs - cam.cx) ** 2 + (ys - cam.cy) ** 2
    qv = r2 / var
    al = np.minimum(0.99, o * np.exp(-qv / 2))
    inside = (qv <= 9) & (al >= 1 / 255)
    ref = np.where(inside[..., None], (1 - al)[..., None] + np.asarray(rgb) * al[..., None], 1.0)
    ok = ~out["amb"]
    assert ok.mean() > 0.99
    assert np.max(np.abs(out["image"] - ref)[ok]) < 1e-12


def test_stacked_gaussians_closed_form():
    cam = _cam(40, 40)
    prims = [_prim((0, 0, 0.5), 0.15, 0.3, (1, 0, 0)), _prim((0, 0, -0.4), 0.1, -0.2, (0, 1, 0)),
             _prim((0, 0, 0.1), 0.12, 1.1, (0, 0, 1))]
    _, out = _render(prims, cam)
    ys, xs = np.mgrid[0:40, 0:40] + 0.5
    r2 = (xs - cam.cx) ** 2 + (ys - cam.cy) ** 2
    order = sorted(range(3), key=lambda k: prims[k]["mean"][2])
    T = np.ones((40, 40))
    C = np.zeros((40, 40, 3))
    for k in order:
        p = prims[k]
        z = 3.0 + p["mean"][2]
        var = (cam.fx * math.exp(p["log_scale"][0]) / z) ** 2 + 0.3
        qv = r2 / var
        al = np.minimum(0.99, np.exp(-qv / 2) / (1 + math.exp(-p["logit"])))
        m = (qv <= 9) & (al >= 1 / 255)
        rgb = np.array([0.5 + Y00 * d for d in p["dc"]])
        C += np.where(m[..., None], rgb * (al * T)[..., None], 0)
        T = np.where(m, T * (1 - al), T)
    ref = C + T[..., None]
    ok = ~out["amb"]
    assert np.max(np.abs(out["image"] - ref)[ok]) < 1e-12


def test_transmittance_stop_excludes_terminating_contributor():
    cam = _cam(33, 33, cx=16.5, cy=16.5)             # pixel (16, 16) centred on the axis
    logit = math.log(0.95 / 0.05)
    cols = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0.5, 0.5, 0.5)]
    prims = [_prim((0, 0, -0.3 + 0.2 * k), 0.1, logit, cols[k]) for k in range(4)]
    _, out = _render(prims, cam)
    ref = sum(np.asarray(cols[k]) * 0.95 * 0.05 ** k for k in range(3)) + 0.05 ** 3
    assert np.max(np.abs(out["image"][16, 16] - ref)) < 1e-12
    assert abs(out["T"][16, 16] - 1.25e-4) < 1e-15     # the 4th would give 6.25e-6 < 1e-4


def _random_prims(rng, n, deg, rgb=None):
    prims = []
    K = (deg + 1) ** 2 - 1
    for _ in range(n):
        q = rng.standard_normal(4)
        p = dict(mean=list(rng.uniform(-1, 1, 3)), log_scale=list(rng.normal(-2.0, 0.6, 3)),
                 quat=list(q / np.linalg.norm(q)), logit=float(rng.normal(0, 1.5)),
                 dc=list((rng.uniform(0, 1, 3) - 0.5) / Y00), rest=rng.normal(0, 0.1, (K, 3)).tolist())
        if rgb is not None:
            p["dc"] = [(rgb - 0.5) / Y00] * 3
            p["rest"] = np.zeros((K, 3)).tolist()
        prims.append(p)
    return prims


def test_white_primitives_telescope_to_one():
    rng = np.random.default_rng(1)
    cam = _cam(48, 40)
    _, out = _render(_random_prims(rng, 60, 0, rgb=1.0), cam)
    assert np.max(np.abs(out["pre"] - 1.0)) < 1e-12


def test_black_primitives_give_transmittance_product():
    rng = np.random.default_rng(2)
    cam = _cam(48, 40)
    _, out = _render(_random_prims(rng, 60, 0, rgb=0.0), cam)
    assert np.max(np.abs(out["pre"] - out["T"][..., None])) < 1e-12
    assert np.all((out["T"] >= 0) & (out["T"] <= 1))


def test_permutation_invariance():
    rng = np.random.default_rng(3)
    cam = _cam(48, 40)
    prims = _random_prims(rng, 80, 1)
    _, a = _render(prims, cam, 1)
    perm = rng.permutation(len(prims))
    _, b = _render([prims[k] for k in perm], cam, 1)
    assert np.array_equal(a["image"], b["image"])


def _rotated_camera(rng, w, h):
    cam = synth.make_camera(w, h, distance=3.5)
    a = rng.normal(0, 0.15, 3)
    from scipy.spatial.transform import Rotation
    R = Rotation.from_rotvec(a).as_matrix()
    cam.R = R
    cam.t = np.array([0.1, -0.05, 3.5])
    return cam


@pytest.mark.parametrize("deg", [0, 3])
def test_scalar_oracle_agrees(deg):
    rng = np.random.default_rng(10 + deg)
    cam = _rotated_camera(rng, 16, 14)
    prims = _random_prims(rng, 10, deg)
    pr, out = _render(prims, cam, deg)
    ref = np.asarray(scalar.render_scalar(prims, deg, cam))
    ok = ~out["amb"]
    assert ok.mean() > 0.9
    assert np.max(np.abs(out["image"] - ref)[ok]) < 1e-9


def test_pixel_major_agrees_with_primitive_major():
    sc = synth.make_scene(600, seed=12, sh_degree=1)
    cam = synth.make_camera(48, 40)
    vals = render.decode_scene([formats.store(f, "f32") for f in sc.fields], "f32")
    pr = render.project(vals, 1, cam)
    out = render.render(pr, cam)
    rng = np.random.default_rng(0)
    xs, ys = rng.integers(0, 48, 120), rng.integers(0, 40, 120)
    px = render.render_pixels(pr, cam, xs, ys)
    ok = ~out["amb"][ys, xs]
    assert np.max(np.abs(px - out["image"][ys, xs])[ok]) < 1e-12


def test_sh_basis_orthonormal_and_degree1_closed_form():
    # Gauss-Legendre in cos(polar) x uniform azimuth integrates degree <= 6 products exactly
    xg, wg = np.polynomial.legendre.leggauss(12)
    phi = np.linspace(0, 2 * np.pi, 24, endpoint=False)
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(phi.size, 2 * np.pi / phi.size)[None, :]).reshape(-1)
    Y = sh.basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(16))) < 1e-12
    k1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 1:4], np.stack([-k1 * d[:, 1], k1 * d[:, 2], -k1 * d[:, 0]], 1), atol=1e-14)
    # the scalar renderer's closed-form polynomials are the same basis
    P = np.array([scalar._sh_poly(*dd, 3) for dd in d[:50]])
    assert np.max(np.abs(P - Y[:50])) < 1e-13


def test_prop1_sign_flip_worked_value():
    g = GOLD["prop1_sign_flip"]
    w = formats.store(np.array([g["theta"]], np.float32), "f32")
    th = formats.decode(formats.flip(w, 31), "f32")[0]
    assert th == g["theta_flipped"]
    assert abs(math.exp(th) / math.exp(g["theta"]) - g["scale_factor"]) < 1e-9
    assert 3.5e2 < g["scale_factor"] < 4.5e2


def test_metrics_definitions():
    clean = np.full((4, 5, 3), 0.5)
    img = clean.copy()
    m = metrics.frame_metrics(img, clean)
    assert m["psnr"] == float("inf") and m["footprint"] == 0 and not m["catastrophic"]
    img[0, 0] = [0.5 + 2 / 255, 0.5, 0.5]                # changed by more than one level
    img[1, 1] = [0.5, 0.5 + 1 / 255, 0.5]                # exactly one level: not counted
    m = metrics.frame_metrics(img, clean)
    assert m["changed_px"] == 1 and m["footprint"] == 1 / 20
    mse = ((2 / 255) ** 2 + (1 / 255) ** 2) / 60
    assert abs(m["psnr"] - 10 * math.log10(1 / mse)) < 1e-12
    assert m["catastrophic"]                              # 5% > 1% (Def. 2)
    assert metrics.frame_metrics(clean, clean, nonfinite=True)["catastrophic"]
    lo, hi = metrics.wilson_interval(0, 100)
    assert abs(lo) < 1e-15 and 0.03 < hi < 0.04
