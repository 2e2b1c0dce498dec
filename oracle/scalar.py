"""Pure-Python per-pixel renderer for tiny scenes (oracle; test infrastructure only).

A second, independent statement of the same definition as `render`, written
with scalar loops and the `math` module only: the rotation matrix is written
from the quaternion formula, the SH basis from the closed-form polynomials of
degree <= 3 with normalisations sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), and every
pixel loops over every primitive.  It exists to pin `render`/`project` (which
use scipy's rotation and complex harmonics); it is far too slow for anything
but a handful of primitives and pixels.
"""
from __future__ import annotations

import math

FLT_MAX = 3.4028234663852886e38


def _sh_poly(x, y, z, degree):
    """Real SH basis values (3DGS signs and order) at unit direction (x, y, z)."""
    pi = math.pi
    out = [0.5 / math.sqrt(pi)]
    if degree >= 1:
        k1 = math.sqrt(3.0 / (4.0 * pi))
        out += [-k1 * y, k1 * z, -k1 * x]
    if degree >= 2:
        k22 = 0.5 * math.sqrt(15.0 / pi)       # |m| = 1, 2 prefactor of xy, yz, xz
        k20 = 0.25 * math.sqrt(5.0 / pi)
        k2x = 0.25 * math.sqrt(15.0 / pi)
        out += [k22 * x * y, -k22 * y * z, k20 * (3.0 * z * z - 1.0), -k22 * x * z, k2x * (x * x - y * y)]
    if degree >= 3:
        k33 = 0.25 * math.sqrt(35.0 / (2.0 * pi))
        k32 = 0.5 * math.sqrt(105.0 / pi)
        k31 = 0.25 * math.sqrt(21.0 / (2.0 * pi))
        k30 = 0.25 * math.sqrt(7.0 / pi)
        k32b = 0.25 * math.sqrt(105.0 / pi)
        out += [-k33 * y * (3.0 * x * x - y * y), k32 * x * y * z, -k31 * y * (5.0 * z * z - 1.0),
                k30 * z * (5.0 * z * z - 3.0), -k31 * x * (5.0 * z * z - 1.0), k32b * z * (x * x - y * y),
                -k33 * x * (x * x - 3.0 * y * y)]
    return out


def _rot(qw, qx, qy, qz):
    n = math.sqrt(qw * qw + qx * qx + qy * qy + qz * qz)
    w, x, y, z = qw / n, qx / n, qy / n, qz / n
    return [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
            [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
            [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]]


def _mm(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))] for i in range(len(A))]


def project_one(prim, sh_degree, cam):
    """prim: dict with mean(3), log_scale(3), quat(4), logit, dc(3), rest(list of 3-lists).
    Returns None when culled, else (depth, u, v, a, b, c, o, rgb)."""
    R = [list(r) for r in cam.R]
    mu = prim["mean"]
    p = [sum(R[i][k] * mu[k] for k in range(3)) + cam.t[i] for i in range(3)]
    if not (cam.near < p[2] <= cam.far):
        return None
    s = [math.exp(v) for v in prim["log_scale"]]
    Rq = _rot(*prim["quat"])
    limx = 1.3 * (0.5 * cam.width) / cam.fx
    limy = 1.3 * (0.5 * cam.height) / cam.fy
    tx = min(limx, max(-limx, p[0] / p[2])) * p[2]
    ty = min(limy, max(-limy, p[1] / p[2])) * p[2]
    J = [[cam.fx / p[2], 0.0, -cam.fx * tx / (p[2] * p[2])],
         [0.0, cam.fy / p[2], -cam.fy * ty / (p[2] * p[2])]]
    Sig = [[sum(Rq[i][k] * s[k] * s[k] * Rq[j][k] for k in range(3)) for j in range(3)] for i in range(3)]
    M = _mm(J, R)
    S2 = _mm(_mm(M, Sig), [list(col) for col in zip(*M)])
    a, b, c = S2[0][0] + 0.3, S2[0][1], S2[1][1] + 0.3
    u = cam.fx * p[0] / p[2] + cam.cx
    v = cam.fy * p[1] / p[2] + cam.cy
    cc = [-sum(R[k][i] * cam.t[k] for k in range(3)) for i in range(3)]
    d = [mu[i] - cc[i] for i in range(3)]
    dn = math.sqrt(sum(x * x for x in d))
    Y = _sh_poly(d[0] / dn, d[1] / dn, d[2] / dn, sh_degree)
    coefs = [prim["dc"]] + list(prim["rest"])
    rgb = [max(0.0, 0.5 + sum(Y[k] * coefs[k][ch] for k in range(len(Y)))) for ch in range(3)]
    o = 1.0 / (1.0 + math.exp(-prim["logit"]))
    return (float(p[2]), u, v, a, b, c, o, rgb)


def render_scalar(prims, sh_degree, cam, bg=(1.0, 1.0, 1.0)):
    """H x W x 3 nested lists; prims: list of dicts (see project_one)."""
    import numpy as np  # only for the fp32 rounding of the depth key
    proj = []
    for i, pr in enumerate(prims):
        r = project_one(pr, sh_degree, cam)
        if r is not None:
            proj.append((float(np.float32(r[0])), i, r))
    proj.sort(key=lambda t: (t[0], t[1]))
    img = []
    for y in range(cam.height):
        row = []
        for x in range(cam.width):
            T, C = 1.0, [0.0, 0.0, 0.0]
            for _, _, (z, u, v, a, b, c, o, rgb) in proj:
                dx, dy = x + 0.5 - u, y + 0.5 - v
                det = a * c - b * b
                q = (c * dx * dx - 2 * b * dx * dy + a * dy * dy) / det
                if q > 9.0:
                    continue
                al = min(0.99, o * math.exp(-0.5 * q))
                if al < 1.0 / 255.0:
                    continue
                Tn = T * (1.0 - al)
                if Tn < 1e-4:
                    break
                for ch in range(3):
                    C[ch] += rgb[ch] * al * T
                T = Tn
            row.append([min(1.0, C[ch] + T * bg[ch]) for ch in range(3)])
        img.append(row)
    return img
