"""Forward Gaussian-splatting render in float64 (oracle; test infrastructure only).

The paper renders each injected model with a 3DGS rasterizer (Sec. 2,
"Gaussian splatting": project every Gaussian to screen space, composite front
to back; Sec. 3 "Metrics": composite over white).  It never writes the
equations, so this module fixes the reading (listed with the others in the
design notes):

  activation   s = exp(log-scale), q = quaternion / |quaternion| (w, x, y, z),
               o = sigmoid(opacity logit), colour = max(0, 0.5 + SH(d))
               with d the unit vector from the camera centre to the mean.
  camera       p = R mu + t; primitives with p_z <= near or p_z > far are culled;
               u = fx p_x / p_z + cx, v = fy p_y / p_z + cy; pixel (i, j) has its
               centre at (i + 0.5, j + 0.5).
  EWA          Sigma = R_q diag(s^2) R_q^T; J = [[fx/z, 0, -fx tx/z^2], [0, fy/z,
               -fy ty/z^2]] with tx = clamp(p_x/p_z, +-1.3 W/(2 fx)) p_z (ty likewise);
               Sigma' = J R Sigma R^T J^T + 0.3 I.
  pixel rule   primitive i reaches pixel x iff q_i(x) = d^T Sigma'^-1 d <= 9 and
               alpha_i = min(0.99, o_i exp(-q_i / 2)) >= 1/255.
  order        contributors in increasing (depth, id), depth = p_z rounded to
               fp32 (the precision of the rasterizer's sort key), ties by id.
  compositing  T = 1, C = 0; per contributor: T' = T (1 - alpha); if T' < 1e-4
               stop without blending it; else C += colour alpha T, T = T'.
               pixel = C + T * background; image = min(pixel, 1).
  non-finite   a primitive with any non-finite stored component is culled and
               flags the render non-finite; a primitive whose scale, projected
               covariance, its largest eigenvalue, screen position or colour
               exceeds the fp32 range is culled silently; a pixel whose colour
               sum exceeds the fp32 range is non-finite (and shows as 1).

Alongside the image the oracle marks *ambiguous* pixels: pixels where one of
the discrete decisions above (the q cut, the alpha floor, the transmittance
stop, an fp32-range test) is taken within a band around its threshold that an
fp32 evaluation of the same definition cannot resolve.  Parity tests compare
every other pixel.  The bands are derived from fp32 rounding (Bands).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.spatial.transform import Rotation

from . import formats, sh

FLT_MAX = float(np.finfo(np.float32).max)


@dataclass
class Raster:
    alpha_max: float = 0.99
    alpha_min: float = 1.0 / 255.0
    t_min: float = 1e-4
    cut_q: float = 9.0
    dilation: float = 0.3
    bg: tuple = (1.0, 1.0, 1.0)


@dataclass
class Bands:
    """Half-widths of the bands in which an fp32 evaluation may take a
    threshold decision differently from float64.

    q: the fp32 quadratic form differs from the exact one by at most
       q_abs + q_rel * q + q_dir * (|d| + 1) * sqrt(q / 9) / sqrt(lambda2): a
       few ulps of q, plus the rounding of the pixel's eigenframe coordinates
       (products of the offset d from the centre with the fp32 principal
       direction, about 2^-23 per unit length of d, which moves q by
       2 sqrt(q) / sqrt(lambda2) per unit of coordinate error); at the cut the
       last term is 1.5e-6 |d| / sqrt(lambda2), twice the rounding bound.
    alpha: relative error of o * exp(-q/2) in fp32 (exp, product, rounding of o)
       plus half the q error.
    transmittance: each factor (1 - alpha) carries relative error
       2^-23 + alpha / (1 - alpha) * alpha_err (amax_rel instead for a
       contributor clamped at alpha_max: 1 - 0.99 and 1 - fp32(0.99) differ by
       9.5e-7 relative); the running sum is tracked per pixel.
    fp32 range: relative band around FLT_MAX for overflow tests.
    """
    q_abs: float = 2e-6
    q_rel: float = 1e-6
    q_dir: float = 1.5e-6
    alpha_rel: float = 4e-7
    t_base: float = 1e-6
    t_step: float = 2.4e-7
    amax_rel: float = 1.2e-6
    range_rel: float = 1e-5


def decode_scene(words, fmt):
    """float64 values (list of 6 (C_f, N) arrays) of stored words."""
    return [formats.decode(w, fmt) if w.size else np.zeros(w.shape) for w in words]


def camera_centre(cam) -> np.ndarray:
    return -cam.R.T @ cam.t


def project(vals, sh_degree: int, cam, raster: Raster = Raster()) -> dict:
    """Per-primitive screen-space quantities (float64) and cull decisions."""
    N = vals[0].shape[1]
    fin = np.ones(N, bool)
    for v in vals:
        if v.size:
            fin &= np.all(np.isfinite(v), axis=0)
    z0 = lambda a: np.where(np.isfinite(a), a, 0.0)
    mu = z0(vals[0]).T
    ls = z0(vals[1]).T
    qv = z0(vals[2]).T
    logit = z0(vals[3][0])
    dc = z0(vals[4]).T
    rest = z0(vals[5]).T if vals[5].size else np.zeros((N, 0))

    valid = fin.copy()
    amb = np.zeros(N, bool)
    rng = raster

    # camera
    p = mu @ cam.R.T + cam.t
    z = p[:, 2]
    valid &= (z > cam.near) & (z <= cam.far)
    amb |= (np.abs(z - cam.near) <= 1e-9 * cam.near) | (np.abs(z - cam.far) <= 1e-9 * cam.far)
    zs = np.where(z > 0, z, 1.0)

    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        # activations
        s = np.exp(ls)
        over = np.any(~(s <= FLT_MAX), axis=1)

        def amb_range(x):
            return np.any(np.abs(np.abs(x) / FLT_MAX - 1.0) <= Bands.range_rel, axis=tuple(range(1, x.ndim)))

        amb |= np.any(np.abs(ls - np.log(FLT_MAX)) <= 1e-9 * np.log(FLT_MAX), axis=1)

        qmax = np.max(np.abs(qv), axis=1)
        zero_q = ~(qmax > 0)
        valid &= ~zero_q
        qs = qv / np.where(zero_q, 1.0, qmax)[:, None]
        qs[zero_q] = np.array([1.0, 0.0, 0.0, 0.0])
        qn = qs / np.linalg.norm(qs, axis=1, keepdims=True)
        Rq = Rotation.from_quat(qn, scalar_first=True).as_matrix()        # (N, 3, 3)
        o = 1.0 / (1.0 + np.exp(-logit))

        # EWA projection
        limx = 1.3 * (0.5 * cam.width) / cam.fx
        limy = 1.3 * (0.5 * cam.height) / cam.fy
        tx = np.clip(p[:, 0] / zs, -limx, limx) * zs
        ty = np.clip(p[:, 1] / zs, -limy, limy) * zs
        J = np.zeros((N, 2, 3))
        J[:, 0, 0] = cam.fx / zs
        J[:, 0, 2] = -cam.fx * tx / zs ** 2
        J[:, 1, 1] = cam.fy / zs
        J[:, 1, 2] = -cam.fy * ty / zs ** 2
        T = J @ cam.R @ Rq                                                 # (N, 2, 3)
        V = T * s[:, None, :]                                              # columns s_k * (J W R_q e_k)
        over |= np.any(~(np.abs(V) <= FLT_MAX), axis=(1, 2))
        amb |= amb_range(V)
        S2 = V @ np.transpose(V, (0, 2, 1))                                # J W Sigma W^T J^T
        a = S2[:, 0, 0] + rng.dilation
        b = S2[:, 0, 1]
        c = S2[:, 1, 1] + rng.dilation
        over |= ~(a <= FLT_MAX) | ~(c <= FLT_MAX) | ~(np.abs(b) <= FLT_MAX)
        amb |= amb_range(np.stack([a, b, c], 1))
        lam1 = 0.5 * (a + c) + np.hypot(0.5 * (a - c), b)
        over |= ~(lam1 <= FLT_MAX)
        amb |= amb_range(lam1[:, None])
        det = a * c - b * b
        lam2 = det / lam1

        u = cam.fx * p[:, 0] / zs + cam.cx
        v = cam.fy * p[:, 1] / zs + cam.cy
        over |= ~(np.abs(u) <= FLT_MAX) | ~(np.abs(v) <= FLT_MAX)
        amb |= amb_range(np.stack([u, v], 1))

        # view-dependent colour
        d = mu - camera_centre(cam)
        dn = np.linalg.norm(d, axis=1, keepdims=True)
        d = d / np.where(dn > 0, dn, 1.0)
        Y = sh.basis(d, sh_degree)                                         # (N, K)
        coef = np.concatenate([dc[:, None, :], rest.reshape(N, -1, 3)], axis=1)   # (N, K, 3)
        col = 0.5 + np.einsum("nk,nkc->nc", Y, coef)
        over |= np.any(~(np.abs(col) <= FLT_MAX), axis=1)
        amb |= amb_range(col)
        rgb = np.maximum(col, 0.0)

    valid &= ~over
    depth32 = z.astype(np.float32)
    return dict(valid=valid, nonfinite_param=~fin, amb=amb & (fin), z=z, depth32=depth32,
                u=u, v=v, a=a, b=b, c=c, det=det, lam1=lam1, lam2=lam2, o=o, rgb=rgb, n=N)


def _order(proj):
    idx = np.nonzero(proj["valid"])[0]
    keys = proj["depth32"][idx].astype(np.float64)
    return idx[np.lexsort((idx, keys))]


def render(proj, cam, raster: Raster = Raster(), bands: Bands = Bands(), window=None) -> dict:
    """Full frame, primitive-major: contributors are visited in (depth, id)
    order and each pixel applies the per-contributor rule above, which is the
    same sequence of operations per pixel as a pixel-major loop.

    window=(x0, y0, x1, y1) evaluates only the pixels x0 <= i < x1,
    y0 <= j < y1 (clipped to the frame) and returns arrays of the window's
    shape.  The rule of a pixel involves no other pixel, so each of them gets
    exactly the value it has in the full frame; primitives whose support
    misses the window are not visited."""
    H, W = cam.height, cam.width
    if window is None:
        x0, y0, x1, y1 = 0, 0, W, H
    else:
        x0, y0 = max(0, int(window[0])), max(0, int(window[1]))
        x1, y1 = min(W, int(window[2])), min(H, int(window[3]))
        x1, y1 = max(x1, x0), max(y1, y0)
    h, w = y1 - y0, x1 - x0
    Tr = np.ones((h, w))
    C = np.zeros((h, w, 3))
    done = np.zeros((h, w), bool)
    amb = np.zeros((h, w), bool)
    terr = np.zeros((h, w))
    ovf = np.zeros((h, w, 3), bool)
    cut = raster.cut_q
    # a primitive culled by a range test taken inside its band may be drawn by
    # an fp32 implementation, anywhere on the frame
    if np.any(proj["amb"] & ~proj["valid"] & ~proj["nonfinite_param"]):
        amb[:] = True
    order = _order(proj)
    # pixels whose centre can satisfy q <= cut (plus a margin for the band),
    # as the pixel-index range [i0, i1] x [j0, j1] of each primitive, clipped
    # to the window
    u_all, v_all = proj["u"][order], proj["v"][order]
    rx = np.sqrt(cut * proj["a"][order]) * 1.001 + 1e-3
    ry = np.sqrt(cut * proj["c"][order]) * 1.001 + 1e-3
    I0 = np.clip(np.ceil(u_all - rx - 0.5), x0, x1).astype(np.int64)
    I1 = np.clip(np.floor(u_all + rx - 0.5), x0 - 1, x1 - 1).astype(np.int64)
    J0 = np.clip(np.ceil(v_all - ry - 0.5), y0, y1).astype(np.int64)
    J1 = np.clip(np.floor(v_all + ry - 0.5), y0 - 1, y1 - 1).astype(np.int64)
    meets = (I1 >= I0) & (J1 >= J0)
    for k in np.nonzero(meets)[0]:
        i = order[k]
        a, b, c, det = proj["a"][i], proj["b"][i], proj["c"][i], proj["det"][i]
        u, v = proj["u"][i], proj["v"][i]
        i0, i1, j0, j1 = int(I0[k]), int(I1[k]), int(J0[k]), int(J1[k])
        win = (slice(j0 - y0, j1 - y0 + 1), slice(i0 - x0, i1 - x0 + 1))
        if proj["amb"][i]:
            amb[win] = True
        dx = (np.arange(i0, i1 + 1) + 0.5)[None, :] - u
        dy = (np.arange(j0, j1 + 1) + 0.5)[:, None] - v
        q = (c * dx * dx - 2.0 * b * dx * dy + a * dy * dy) / det
        live = ~done[win]
        araw = proj["o"][i] * np.exp(-0.5 * q)
        alpha = np.minimum(raster.alpha_max, araw)
        qband = bands.q_abs + bands.q_rel * np.abs(q) + bands.q_dir * (np.sqrt(dx * dx + dy * dy) + 1.0) * \
            np.sqrt(np.abs(q) / cut) / np.sqrt(proj["lam2"][i])
        aband = bands.alpha_rel + 0.5 * qband
        inq = q <= cut
        ina = alpha >= raster.alpha_min
        contrib = live & inq & ina
        amb_q = live & (np.abs(q - cut) <= qband) & (araw >= raster.alpha_min * (1.0 - aband))
        amb_a = live & (q <= cut + qband) & (np.abs(alpha / raster.alpha_min - 1.0) <= aband)
        Tw = Tr[win]
        Tn = Tw * (1.0 - alpha)
        # relative error of the factor (1 - alpha): the alpha error amplified by
        # alpha / (1 - alpha), or, for a contributor clamped at alpha_max, the
        # difference between alpha_max and its fp32 value
        clamped = araw >= raster.alpha_max * (1.0 + aband)
        step_err = bands.t_step + np.where(clamped, bands.amax_rel, (alpha / (1.0 - alpha)) * aband)
        terr_n = terr[win] + step_err
        stop = contrib & (Tn < raster.t_min)
        amb_t = contrib & (np.abs(Tn / raster.t_min - 1.0) <= bands.t_base + 2.0 * terr_n)
        blend = contrib & ~stop
        Cw = C[win]
        Cn = Cw + proj["rgb"][i][None, None, :] * (alpha * Tw)[:, :, None]
        newovf = blend[:, :, None] & ~(Cn <= FLT_MAX)
        amb_o = blend & np.any(np.abs(Cn / FLT_MAX - 1.0) <= bands.range_rel, axis=2)
        Cw[blend] = Cn[blend]
        C[win] = Cw
        ovf[win] |= newovf
        Tr[win] = np.where(blend, Tn, Tw)
        terr[win] = np.where(blend, terr_n, terr[win])
        done[win] |= stop
        amb[win] |= amb_q | amb_a | amb_t | amb_o
    pre = C + Tr[:, :, None] * np.asarray(raster.bg)[None, None, :]
    pre[ovf] = np.inf
    image = np.minimum(pre, 1.0)
    nonfinite = bool(np.any(proj["nonfinite_param"]) or np.any(ovf))
    return dict(image=image, pre=pre, amb=amb, nonfinite=nonfinite, T=Tr, window=(x0, y0, x1, y1))


def render_pixels(proj, cam, xs, ys, raster: Raster = Raster()) -> np.ndarray:
    """Pixel-major evaluation of single pixels (x, y): every valid primitive
    is tested against the pixel, the contributors are sorted by (depth, id) and
    composited one by one.  Returns (M, 3) clamped colours."""
    valid = np.nonzero(proj["valid"])[0]
    out = np.zeros((len(xs), 3))
    bg = np.asarray(raster.bg)
    for k, (x, y) in enumerate(zip(xs, ys)):
        dx = x + 0.5 - proj["u"][valid]
        dy = y + 0.5 - proj["v"][valid]
        a, b, c, det = (proj[n][valid] for n in ("a", "b", "c", "det"))
        with np.errstate(over="ignore", invalid="ignore"):
            q = (c * dx * dx - 2.0 * b * dx * dy + a * dy * dy) / det
            alpha = np.minimum(raster.alpha_max, proj["o"][valid] * np.exp(-0.5 * q))
        sel = (q <= raster.cut_q) & (alpha >= raster.alpha_min)
        ids = valid[sel]
        al = alpha[sel]
        order = np.lexsort((ids, proj["depth32"][ids].astype(np.float64)))
        T, C = 1.0, np.zeros(3)
        ovf = np.zeros(3, bool)
        for j in order:
            Tn = T * (1.0 - al[j])
            if Tn < raster.t_min:
                break
            C = C + proj["rgb"][ids[j]] * (al[j] * T)
            ovf |= ~(C <= FLT_MAX)
            T = Tn
        pix = C + T * bg
        out[k] = np.minimum(np.where(ovf, np.inf, pix), 1.0)
    return out
