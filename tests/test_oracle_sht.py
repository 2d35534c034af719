"""Pins of the oracle SHT (oracle/sht.py) and geometry (oracle/geometry.py).

* brute-force dense Y built from scipy.special.sph_harm_y vs. the oracle's
  Legendre-then-ring-FFT route, including under-pixelized band limits
  (lmax > 2 N_side, where m folds modulo the ring length);
* adjointness <Y x, y> = <x, Y^T y>;
* Unsold's theorem: sum over all (l, m) of Y_lm(p)^2 = (lmax+1)^2 / (4 pi)
  at every pixel;
* addition theorem (eq. addition-theorem): synthesizing
  x_lm = g_l Y_lm(n0) gives sum_l (2l+1)/(4 pi) g_l P_l(cos gamma);
* geometry against an independent implementation and HEALPix invariants.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

import workloads
from oracle import geometry, sht


@pytest.mark.parametrize("nside,lmax", [(2, 5), (4, 12), (4, 20), (8, 16), (8, 40)])
def test_dense_vs_fast(nside, lmax):
    Y = sht.dense_Y(nside, lmax)
    rng = np.random.default_rng(nside * 100 + lmax)
    x = rng.standard_normal(sht.nalm(lmax))
    y = rng.standard_normal(12 * nside * nside)
    f = sht.synth(x, lmax, nside)
    a = sht.adjoint(y, lmax, nside)
    scale_f = np.abs(Y).sum(axis=1).max() * np.abs(x).max()
    assert np.max(np.abs(Y @ x - f)) < 1e-14 * scale_f
    scale_a = np.abs(Y).sum(axis=0).max() * np.abs(y).max()
    assert np.max(np.abs(Y.T @ y - a)) < 1e-14 * scale_a


@pytest.mark.parametrize("nside,lmax", [(8, 20), (16, 32), (32, 100)])
def test_adjointness(nside, lmax):
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, sht.nalm(lmax)))
    y = rng.standard_normal((2, 12 * nside * nside))
    f = sht.synth(x, lmax, nside)
    lhs = np.sum(f * y, axis=-1)
    rhs = np.sum(x * sht.adjoint(y, lmax, nside), axis=-1)
    # the inner products cancel: bound the difference by the size of their terms
    scale = np.linalg.norm(f, axis=-1) * np.linalg.norm(y, axis=-1)
    assert np.all(np.abs(lhs - rhs) <= 1e-14 * scale), (lhs, rhs, scale)


def test_unsold():
    nside, lmax = 4, 14
    Y = sht.dense_Y(nside, lmax)
    # the same sum from the fast route: row norms of Y = diag(Y Y^T)
    rng = np.random.default_rng(3)
    probe = rng.standard_normal(12 * nside * nside)
    np.testing.assert_allclose((Y * Y).sum(axis=1), (lmax + 1) ** 2 / (4 * math.pi), rtol=1e-13)
    # fast route: Y Y^T e_p at pixel p equals the same constant
    for p in [0, 17, 100, 191]:
        e = np.zeros(12 * nside * nside)
        e[p] = 1.0
        v = sht.synth(sht.adjoint(e, lmax, nside), lmax, nside)[p]
        assert abs(v - (lmax + 1) ** 2 / (4 * math.pi)) < 1e-12
    assert probe.size == Y.shape[0]


def test_addition_theorem():
    nside, lmax = 16, 40
    g = geometry.healpix_rings(nside)
    theta, phi = geometry.pixel_angles(g)
    th0, ph0 = 1.1, 0.7
    gl = np.exp(-0.002 * np.arange(lmax + 1) ** 2)
    L, M, S = sht.packed_index(lmax)
    x = np.empty(L.size)
    for j in range(L.size):
        y0 = sph_harm_y(int(L[j]), int(M[j]), th0, ph0)
        if M[j] == 0:
            x[j] = y0.real
        elif S[j] == 0:
            x[j] = math.sqrt(2) * y0.real
        else:
            x[j] = math.sqrt(2) * y0.imag
        x[j] *= gl[L[j]]
    f = sht.synth(x, lmax, nside)
    cosg = np.cos(theta) * math.cos(th0) + np.sin(theta) * math.sin(th0) * np.cos(phi - ph0)
    ref = sum((2 * l + 1) / (4 * math.pi) * gl[l] * eval_legendre(l, cosg) for l in range(lmax + 1))
    np.testing.assert_allclose(f, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("nside", [1, 2, 16, 256, 2048])
def test_geometry_invariants(nside):
    g = geometry.healpix_rings(nside)
    assert g.npix == 12 * nside * nside
    assert g.nrings == 4 * nside - 1
    np.testing.assert_allclose(g.z ** 2 + g.sint ** 2, 1.0, rtol=0, atol=4.5e-16)
    z, npr, phi0 = workloads.ring_layout(nside)
    np.testing.assert_array_equal(npr, g.nphi)
    np.testing.assert_allclose(z, g.z, rtol=0, atol=1e-15)
    np.testing.assert_allclose(phi0, g.phi0, rtol=0, atol=1e-15)
    # equal-area: the z-extent of the caps matches pixel counts (ring z is
    # symmetric about the equator)
    np.testing.assert_allclose(g.z, -g.z[::-1], rtol=0, atol=1e-15)


def test_sampled_rings_match_full():
    nside, lmax = 16, 40
    x = np.random.default_rng(11).standard_normal(sht.nalm(lmax))
    full = sht.synth(x, lmax, nside)
    g = geometry.healpix_rings(nside)
    got = sht.synth_rings(x, lmax, nside, [0, 7, 31, 62])
    for k, v in got.items():
        np.testing.assert_allclose(v, full[g.start[k]: g.start[k] + g.nphi[k]], rtol=0, atol=1e-12)


def test_sampled_orders_match_full():
    """The per-order direct-sum adjoint equals the full FFT-based adjoint,
    including orders above the rings' Nyquist frequency (m >= N_k / 2)."""
    nside, lmax = 8, 40
    y = np.random.default_rng(12).standard_normal((2, 12 * nside * nside))
    full = sht.adjoint(y, lmax, nside)
    got = sht.adjoint_orders(y, lmax, nside, [0, 1, 17, 33, 40])
    for m, (c, s) in got.items():
        if m == 0:
            np.testing.assert_allclose(c, full[:, : lmax + 1], rtol=0, atol=1e-12)
            continue
        b = sht.block_base(m, lmax)
        n = lmax - m + 1
        np.testing.assert_allclose(c, full[:, b: b + n], rtol=0, atol=1e-12)
        np.testing.assert_allclose(s, full[:, b + n: b + 2 * n], rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 7, 64, 100])
def test_gauss_legendre_rings(n):
    """Nodes match numpy's Gauss-Legendre rule; weights integrate z^k exactly
    for k < 2n (sum over rings of W_k nphi / (2 pi) = Gauss-Legendre weights)."""
    g, W = geometry.gauss_legendre_rings(n, 8)
    x, w = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(np.sort(g.z), np.sort(x), rtol=0, atol=1e-14)
    wl = W * 8 / (2 * np.pi)
    for k in range(0, 2 * n, max(1, n // 8)):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(wl * g.z ** k) - exact) < 1e-13, k
    np.testing.assert_allclose(g.z, -g.z[::-1], rtol=0, atol=0)


def test_gauss_legendre_quadrature_is_exact():
    """Y^T W Y = I on a Gauss-Legendre grid with lmax + 1 rings and
    nphi > 2 lmax (the exact quadrature the coarse levels rely on, Sec. 3.4)."""
    lmax = 24
    g, W = geometry.gauss_legendre_rings(lmax + 1, 52)
    x = np.random.default_rng(21).standard_normal(sht.nalm(lmax))
    m = sht.synth_geom(x, lmax, g)
    y = sht.adjoint_geom(m * np.repeat(W, g.nphi), lmax, g)
    np.testing.assert_allclose(y, x, rtol=0, atol=1e-13)


def test_downgraded_inverse_noise_identity():
    """Sec. 3.4: for modes l, l' <= lh, Y_obs^T N^-1 Y_obs equals
    Y_GL^T W Ntilde Y_GL with Ntilde the synthesis of xi = Y_obs^T N^-1
    truncated at 2 lh on 2 lh + 1 Gauss-Legendre rings of > 4 lh pixels."""
    nside, lh = 8, 9
    cfg = workloads.WorkloadConfig("t", nside, 2 * lh, -1.0, 10.0, 20.0, 3, 8.0, 1)
    ninv, _, _ = workloads.inverse_noise_map(cfg)
    x = np.random.default_rng(22).standard_normal(sht.nalm(lh))
    ref = sht.adjoint(ninv * sht.synth(x, lh, nside), lh, nside)
    xi = sht.adjoint(ninv, 2 * lh, nside)
    g, W = geometry.gauss_legendre_rings(2 * lh + 1, 64)
    nt = sht.synth_geom(xi, 2 * lh, g) * np.repeat(W, g.nphi)
    got = sht.adjoint_geom(nt * sht.synth_geom(x, lh, g), lh, g)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
