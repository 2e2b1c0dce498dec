"""Real spherical-harmonic colour basis (oracle; test infrastructure only).

Sec. 3, "Parameter layout": colour is a direct-current coefficient plus
higher-order coefficients of degree <= L.  The paper does not write the
basis; the reading is the real basis used by 3D Gaussian splatting, which in
terms of the complex harmonics Y_l^m (with the Condon-Shortley phase, as
scipy.special.sph_harm_y defines them) is

    m = 0 :  Y_l^0
    m > 0 :  sqrt(2) Re Y_l^m
    m < 0 :  sqrt(2) Im Y_l^|m|

with the polar axis along +z, ordered by degree and then m = -l .. l
(index l^2 + l + m).  The colour of direction d is 0.5 + sum_k c_k Y_k(d),
clamped below at 0.
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def basis(dirs: np.ndarray, degree: int) -> np.ndarray:
    """(M, (degree+1)^2) real SH values at unit directions dirs (M, 3)."""
    d = np.asarray(dirs, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    polar = np.arccos(np.clip(z, -1.0, 1.0))
    azim = np.arctan2(y, x)
    cols = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), polar, azim)
            if m == 0:
                cols.append(Y.real)
            elif m > 0:
                cols.append(np.sqrt(2.0) * Y.real)
            else:
                cols.append(np.sqrt(2.0) * Y.imag)
    return np.stack(cols, axis=1)
