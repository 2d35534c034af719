"""HEALPix RING geometry for the oracle (Sec. 2.1; Gorski et al. 2005).

Rings i = 1 .. 4 N_side - 1 run north to south.  For the north polar cap
(i < N_side) a ring holds 4i pixels at z = 1 - i^2 / (3 N_side^2), the first
at phi = pi / (4 i); belt rings (N_side <= i <= 3 N_side) hold 4 N_side pixels
at z = 4/3 - 2 i / (3 N_side), the first at (pi / (2 N_side)) (1 - s / 2)
with s = (i - N_side + 1) mod 2; south-cap rings mirror the north cap.

sin(theta) is evaluated as sqrt((1 - z)(1 + z)) with 1 - z formed exactly
from integers, so it keeps full relative precision at the poles.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
import math

import numpy as np


@dataclass
class RingGeometry:
    nside: int
    z: np.ndarray        # cos(theta) per ring
    sint: np.ndarray     # sin(theta) per ring
    nphi: np.ndarray     # pixels per ring
    phi0: np.ndarray     # phi of the first pixel
    start: np.ndarray    # RING index of the first pixel

    @property
    def nrings(self) -> int:
        return len(self.z)

    @property
    def npix(self) -> int:
        return int(self.nphi.sum())

    def ring_phi(self, k: int) -> np.ndarray:
        n = int(self.nphi[k])
        return self.phi0[k] + 2.0 * math.pi * np.arange(n) / n


def healpix_rings(nside: int) -> RingGeometry:
    nr = 4 * nside - 1
    z = np.empty(nr)
    st = np.empty(nr)
    nphi = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    for i in range(1, nr + 1):
        if i < nside or i > 3 * nside:
            ii = i if i < nside else 4 * nside - i
            one_minus = Fraction(ii * ii, 3 * nside * nside)          # 1 - |z|
            zabs = 1 - one_minus
            nphi[i - 1] = 4 * ii
            phi0[i - 1] = math.pi / (4.0 * ii)
        else:
            zabs = abs(Fraction(4 * nside - 2 * i, 3 * nside))
            one_minus = 1 - zabs
            nphi[i - 1] = 4 * nside
            s = (i - nside + 1) % 2
            phi0[i - 1] = (math.pi / (2.0 * nside)) * (1.0 - s / 2.0)
        sign = -1.0 if i > 2 * nside else 1.0
        z[i - 1] = sign * float(zabs)
        st[i - 1] = math.sqrt(float(one_minus * (1 + zabs)))
    start = np.concatenate([[0], np.cumsum(nphi)[:-1]]).astype(np.int64)
    return RingGeometry(nside, z, st, nphi, phi0, start)


def pixel_angles(geom: RingGeometry):
    """(theta, phi) of every pixel centre in RING order."""
    th = np.arctan2(geom.sint, geom.z)
    theta = np.repeat(th, geom.nphi)
    phi = np.concatenate([geom.ring_phi(k) for k in range(geom.nrings)])
    return theta, phi
