"""HEALPix RING geometry for the oracle (Sec. 2.1; Gorski et al. 2005).

Rings i = 1 .. 4 N_side - 1 run north to south.  For the north polar cap
(i < N_side) a ring holds 4i pixels at z = 1 - i^2 / (3 N_side^2), the first
at phi = pi / (4 i); belt rings (N_side <= i <= 3 N_side) hold 4 N_side pixels
at z = 4/3 - 2 i / (3 N_side), the first at pi / (4 N_side) when i - N_side
is even and at phi = 0 when it is odd (the numbering of the HEALPix reference
code, base pixel 4 centred on phi = 0); south-cap rings mirror the north cap.

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
            phi0[i - 1] = math.pi / (4.0 * nside) if (i - nside) % 2 == 0 else 0.0
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


def gauss_legendre_rings(nrings: int, nphi: int):
    """Gauss-Legendre rings (Sec. 3.4): the nodes z_k of P_nrings, north to
    south, each with nphi equispaced pixels from phi = 0.  Returns the ring
    geometry and the quadrature weight of one pixel of each ring,
    W_k = w_k 2 pi / nphi with w_k = 2 / ((1 - z_k^2) P'_n(z_k)^2).

    Nodes by Newton's method on P_n (three-term recurrence) from the
    Tricomi-type guesses cos(pi (k + 3/4) / (n + 1/2)), in long double; the
    south half mirrors the north."""
    n = int(nrings)
    z = np.empty(n, dtype=np.longdouble)
    w = np.empty(n, dtype=np.longdouble)
    half = (n + 1) // 2
    k = np.arange(half)
    x = np.cos(np.pi * (k + 0.75) / (n + 0.5)).astype(np.longdouble)
    for _ in range(100):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for j in range(2, n + 1):
            p0, p1 = p1, ((2 * j - 1) * x * p1 - (j - 1) * p0) / j
        dp = n * (x * p1 - p0) / (x * x - 1) if n > 1 else np.ones_like(x)
        if n == 1:
            p1 = x
        dx = p1 / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-19:
            break
    z[:half] = x
    w[:half] = 2 / ((1 - x * x) * dp * dp)
    z[n - half:] = -x[::-1]
    w[n - half:] = w[:half][::-1]
    if n % 2 == 1:
        z[n // 2] = 0
    zf = z.astype(np.float64)
    st = np.sqrt(((1 - z) * (1 + z)).astype(np.float64))
    nph = np.full(n, int(nphi), dtype=np.int64)
    start = (np.arange(n) * int(nphi)).astype(np.int64)
    geom = RingGeometry(0, zf, st, nph, np.zeros(n), start)
    W = (w * 2 * np.pi / int(nphi)).astype(np.float64)
    return geom, W


def nest_to_ring(nside: int, nest) -> np.ndarray:
    """HEALPix NESTED -> RING pixel index (Gorski et al. 2005).

    A nested index holds the base face f (12 faces of nside^2 pixels) and the
    pixel's (x, y) position inside the face, bit-interleaved.  The ring number
    counts down from the face's northernmost corner: i = r_f nside - x - y - 1
    with r_f = 2, 3, 4 for the northern, equatorial and southern faces; the
    position along the ring follows from the face's longitude offset
    (1, 3, 5, 7 or 0, 2, 4, 6 in units of pi / 4, times the ring length
    quarter) and x - y."""
    nest = np.asarray(nest, dtype=np.int64)
    npf = nside * nside
    f = nest // npf
    p = nest % npf
    x = np.zeros_like(p)
    y = np.zeros_like(p)
    for b in range(max(1, int(nside).bit_length())):
        x |= ((p >> (2 * b)) & 1) << b
        y |= ((p >> (2 * b + 1)) & 1) << b
    row = f // 4
    i = (row + 2) * nside - x - y - 1                     # ring number, 1 .. 4 nside - 1
    lon = np.where(row == 1, 2 * (f % 4), 2 * (f % 4) + 1)
    north, south = i < nside, i > 3 * nside
    nr = np.where(north, i, np.where(south, 4 * nside - i, nside))
    shift = np.where(north | south, 0, (i - nside) & 1)
    jp = (lon * nr + x - y + 1 + shift) // 2
    jp = np.where(jp > 4 * nr, jp - 4 * nr, jp)
    jp = np.where(jp < 1, jp + 4 * nr, jp)
    # pixels before ring i
    before = np.where(north, 2 * i * (i - 1),
                      np.where(south, 12 * npf - 2 * (4 * nside - i + 1) * (4 * nside - i),
                               2 * nside * (nside - 1) + (i - nside) * 4 * nside))
    return before + jp - 1
