"""Pins of the oracle's normalized Legendre recurrence (oracle/legendre.py).

* closed forms of Y_lm for l <= 2 (textbook; Condon-Shortley phase);
* scipy.special.sph_harm_y (library routine) for l <= 64;
* Gauss-Legendre exactness at lmax = 4096: for n = lmax+1 GL nodes,
  2 pi sum_k w_k lambda_lm(z_k) lambda_l'm(z_k) = delta_ll' exactly (the
  integrand is a polynomial of degree <= 2 lmax in z), which tests the
  extended-exponent seeds and every recurrence step up to l = 4096;
* the two loop orders of the same recurrence agree (per m over rings vs.
  per ring over m).
"""
import math

import numpy as np
import pytest
from scipy.special import roots_legendre, sph_harm_y

from oracle import geometry, legendre


def _gl_nodes(n):
    """GL nodes/weights refined in long double (numpy/scipy weights lose
    ~1e-7 relative accuracy next to the poles at n ~ 4000)."""
    x, _ = roots_legendre(n)
    x = x.astype(np.longdouble)
    for _ in range(2):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = n * (x * p1 - p0) / ((x - 1) * (x + 1))
        x = x - p1 / dp
    p0 = np.ones_like(x)
    p1 = x.copy()
    for k in range(2, n):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    w = 2 * (1 - x) * (1 + x) / (n * p1) ** 2
    s = np.sqrt((1 - x) * (1 + x))
    return x.astype(np.float64), s.astype(np.float64), w.astype(np.float64)


def test_closed_forms():
    th = np.linspace(0.01, math.pi - 0.01, 37)
    z, s = np.cos(th), np.sin(th)
    pi = math.pi
    expect = {
        (0, 0): np.full_like(th, 1 / math.sqrt(4 * pi)),
        (1, 0): math.sqrt(3 / (4 * pi)) * z,
        (1, 1): -math.sqrt(3 / (8 * pi)) * s,
        (2, 0): math.sqrt(5 / (16 * pi)) * (3 * z * z - 1),
        (2, 1): -math.sqrt(15 / (8 * pi)) * s * z,
        (2, 2): 0.25 * math.sqrt(15 / (2 * pi)) * s * s,
    }
    for (l, m), ref in expect.items():
        lam = legendre.lambda_table(m, 2, z, s)[l - m]
        np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-15)


def test_scipy_low_l():
    g = geometry.healpix_rings(16)
    th = np.arctan2(g.sint, g.z)
    lmax = 64
    worst = 0.0
    for m in [0, 1, 2, 5, 17, 33, 63, 64]:
        lam = legendre.lambda_table(m, lmax, g.z, g.sint)
        for l in range(m, lmax + 1):
            ref = sph_harm_y(l, m, th, np.zeros_like(th)).real
            worst = max(worst, float(np.max(np.abs(lam[l - m] - ref))))
    assert worst < 5e-14


def test_gauss_legendre_orthonormality_lmax4096():
    lmax = 4096
    z, s, w = _gl_nodes(lmax + 1)
    for m in [0, 1, 100, 1000, 2047, 4000, 4096]:
        lam = legendre.lambda_table(m, lmax, z, s)
        G = 2 * math.pi * (lam * w) @ lam.T
        err = np.abs(G - np.eye(G.shape[0])).max()
        assert err < 2e-12, (m, err)


def test_loop_orders_agree():
    g = geometry.healpix_rings(32)
    lmax = 96
    for k in [0, 5, 60, 63, 100]:
        tab = legendre.lambda_all_m(lmax, float(g.z[k]), float(g.sint[k]))
        for m in range(lmax + 1):
            col = legendre.lambda_table(m, lmax, g.z[k:k + 1], g.sint[k:k + 1])[:, 0]
            np.testing.assert_allclose(tab[m:, m], col, rtol=0, atol=1e-15)


def test_extended_range_underflow_is_exact_zero_or_tiny():
    # m = 4096 at the polar ring of N_side 2048: sin^m theta ~ 1e-13900
    g = geometry.healpix_rings(2048)
    lam = legendre.lambda_table(4096, 4096, g.z[:3], g.sint[:3])
    assert np.all(lam == 0.0)
    # a ring where the seed is representable gives a finite, nonzero value
    mid = g.nrings // 2
    lam2 = legendre.lambda_table(4096, 4096, g.z[mid:mid + 1], g.sint[mid:mid + 1])
    assert np.isfinite(lam2).all() and lam2[0, 0] != 0.0


def test_parity_mirror_symmetry():
    # lambda_lm(-z) = (-1)^(l+m) lambda_lm(z)
    g = geometry.healpix_rings(64)
    n = g.nrings
    for m in [0, 3, 50]:
        lam = legendre.lambda_table(m, 180, g.z, g.sint)
        sign = np.array([(-1) ** (l + m) for l in range(m, 181)])[:, None]
        np.testing.assert_allclose(lam[:, ::-1], sign * lam, rtol=0, atol=1e-13)
        assert n % 2 == 1
