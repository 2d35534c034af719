"""Normalized associated Legendre functions for the oracle.

lambda_lm(theta) = P~_lm(cos theta) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_lm(cos theta)
(Sec. 3.2, the normalization stated beside eq. Ni-dense), with the
Condon-Shortley phase (-1)^m included in P_lm, so that the complex
spherical harmonic is Y_lm = lambda_lm(theta) e^{i m phi}.

Computed by the textbook three-term recurrence in l at fixed m:

    lambda_mm     = (-1)^m sqrt((2m+1)/(4 pi) * prod_{k=1..m} (2k-1)/(2k)) sin^m theta
    lambda_m+1,m  = sqrt(2m+3) cos theta lambda_mm
    lambda_lm     = a_lm (cos theta lambda_l-1,m - lambda_l-2,m / a_l-1,m),
    a_lm          = sqrt((4 l^2 - 1) / (l^2 - m^2)).

sin^m theta underflows float64 for large m near the poles (m = 4096 at
sin theta ~ 4e-4 gives ~1e-13900), so values are carried as
mantissa * 2^exponent with an integer exponent per ring (extended-exponent
arithmetic in the manner of Fukushima 2012).  The mantissa is renormalized
whenever its binary exponent leaves [-300, 300].  The emitted value is
ldexp(mantissa, exponent): it is exactly 0 where the true value underflows
float64.  No value is skipped or thresholded here.

The product in the seed is evaluated exactly as binom(2m, m) / 4^m with
integer arithmetic and rounded once.
"""
from __future__ import annotations

from fractions import Fraction
import math

import numpy as np


_BINOM = [1]          # binom(2m, m) for m = 0, 1, ..., exact integers


def _binom_2m_m(m: int) -> int:
    """binom(2m, m), extended exactly: binom(2m+2, m+1) = binom(2m, m) 2 (2m+1) / (m+1)."""
    while len(_BINOM) <= m:
        k = len(_BINOM) - 1
        _BINOM.append(_BINOM[k] * 2 * (2 * k + 1) // (k + 1))
    return _BINOM[m]


def seed_constant(m: int) -> float:
    """(-1)^m sqrt((2m+1)/(4 pi) * binom(2m,m)/4^m), the factor of sin^m theta."""
    t = float(Fraction(_binom_2m_m(m) * (2 * m + 1), 4 ** m))
    c = math.sqrt(t / (4.0 * math.pi))
    return -c if (m & 1) else c


def _pow_ext(s: np.ndarray, m: int):
    """s^m as (mantissa, int exponent) by binary powering with renormalization."""
    fs, es = np.frexp(s)
    es = es.astype(np.int64)
    mant = np.ones_like(fs)
    expo = np.zeros_like(es)
    base, bexp = fs.copy(), es.copy()
    e = m
    while e:
        if e & 1:
            mant = mant * base
            expo = expo + bexp
            mant, k = np.frexp(mant)
            expo = expo + k
        e >>= 1
        if e:
            base = base * base
            bexp = 2 * bexp
            base, k = np.frexp(base)
            bexp = bexp + k
    return mant, expo


def _renorm(cur, prev, expo):
    _, k = np.frexp(cur)
    k = k.astype(np.int64)
    big = np.abs(k) > 300
    if big.any():
        sh = np.where(big, k, 0)
        cur = np.ldexp(cur, -sh)
        prev = np.ldexp(prev, -sh)
        expo = expo + sh
    return cur, prev, expo


def recurrence_coeff(l: int, m: int) -> float:
    """a_lm = sqrt((4 l^2 - 1) / (l^2 - m^2)), l > m."""
    return math.sqrt((4.0 * l * l - 1.0) / ((l - m) * (l + m)))


def lambda_table(m: int, lmax: int, z: np.ndarray, s: np.ndarray) -> np.ndarray:
    """lambda_lm at every ring for l = m..lmax; shape (lmax-m+1, nrings)."""
    z = np.asarray(z, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros((lmax - m + 1, z.size))
    if lmax < m:
        return out
    mant, expo = _pow_ext(s, m)
    cur = mant * seed_constant(m)
    prev = np.zeros_like(cur)
    cur, prev, expo = _renorm(cur, prev, expo)
    out[0] = np.ldexp(cur, expo)
    a_prev = 0.0
    for l in range(m + 1, lmax + 1):
        a = recurrence_coeff(l, m)
        if l == m + 1:
            nxt = a * z * cur                      # a_{m+1,m} = sqrt(2m+3)
        else:
            nxt = a * (z * cur - prev / a_prev)
        prev, cur = cur, nxt
        a_prev = a
        cur, prev, expo = _renorm(cur, prev, expo)
        out[l - m] = np.ldexp(cur, expo)
    return out


def lambda_all_m(lmax: int, z: float, s: float) -> np.ndarray:
    """lambda_lm(theta) for one theta and all 0 <= m <= l <= lmax.

    The same recurrence, stepped in l for all m at once (vectorized over m).
    Returns a (lmax+1, lmax+1) array indexed [l, m]; entries with m > l are 0.
    """
    out = np.zeros((lmax + 1, lmax + 1))
    ms = np.arange(lmax + 1)
    mant = np.empty(lmax + 1)
    expo = np.empty(lmax + 1, dtype=np.int64)
    for m in range(lmax + 1):
        mm, ee = _pow_ext(np.array([s]), m)
        mant[m] = mm[0] * seed_constant(m)
        expo[m] = ee[0]
    cur = mant.copy()
    prev = np.zeros(lmax + 1)
    cur, prev, expo = _renorm(cur, prev, expo)
    # a_prev[m] = a_{l-1,m} for the active entries
    a_prev = np.zeros(lmax + 1)
    active = np.zeros(lmax + 1, dtype=bool)     # m with m < l (already seeded)
    for l in range(lmax + 1):
        if l > 0:
            idx = np.nonzero(active)[0]
            first = idx[idx == l - 1]
            rest = idx[idx < l - 1]
            if rest.size:
                lm = rest.astype(np.float64)
                a = np.sqrt((4.0 * l * l - 1.0) / ((l - lm) * (l + lm)))
                nxt = a * (z * cur[rest] - prev[rest] / a_prev[rest])
                prev[rest] = cur[rest]
                cur[rest] = nxt
                a_prev[rest] = a
            if first.size:
                a = math.sqrt(2.0 * (l - 1) + 3.0)
                nxt = a * z * cur[first]
                prev[first] = cur[first]
                cur[first] = nxt
                a_prev[first] = a
        active[l] = True
        sel = ms[: l + 1]
        c, p, e = _renorm(cur[sel], prev[sel], expo[sel])
        cur[sel], prev[sel], expo[sel] = c, p, e
        out[l, : l + 1] = np.ldexp(cur[sel], expo[sel])
    return out
