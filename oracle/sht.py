"""Spherical harmonic synthesis Y and adjoint synthesis Y^T for the oracle.

Synthesis is eq. sh-synthesis (Sec. 2.1) written in a real orthonormal basis:

    f(theta, phi) = sum_l x_l0 lambda_l0(theta)
                  + sum_{m>=1} sum_{l>=m} sqrt(2) lambda_lm(theta) (x^c_lm cos m phi + x^s_lm sin m phi)

evaluated at the HEALPix RING pixel centres.  Adjoint synthesis Y^T is the
literal matrix transpose of Y (Sec. 2.1: no quadrature weights), which the
paper uses instead of analysis.  x is real packed, m-major (m = 0 block of
x_l0, then for every m >= 1 a cosine block l = m..lmax and a sine block).

Fast route (two steps, in the order the definition factorizes):
  1. Legendre step per m:  F^c_m(theta_k) = sum_l lambda_lm(theta_k) x^c_lm (and sine).
  2. Ring step per ring k: f_j = sum_m w_m (F^c_m cos m phi_kj + F^s_m sin m phi_kj),
     w_0 = 1, w_m = sqrt(2), phi_kj = phi0_k + 2 pi j / N_k, done with one
     length-N_k inverse FFT after folding m modulo N_k (H_m = w_m (F^c - i F^s)
     e^{i m phi0}).  The adjoint takes Y_q = FFT(y)_q and forms
     G^c_m = w_m Re(e^{i m phi0} conj(Y_{m mod N})), G^s_m = w_m Im(...).
A brute-force route builds the dense matrix Y element by element from
``scipy.special.sph_harm_y`` (a library routine, independent of the
recurrence in ``legendre``), for tiny grids.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import RingGeometry, healpix_rings, pixel_angles
from .legendre import lambda_table

SQRT2 = math.sqrt(2.0)


def nalm(lmax: int) -> int:
    return (lmax + 1) ** 2


def block_base(m: int, lmax: int) -> int:
    """Offset of the cosine block of m >= 1 in the real packed vector."""
    return (lmax + 1) + (m - 1) * (2 * lmax - m + 2)


def split_m(x: np.ndarray, m: int, lmax: int):
    """(cos block, sin block) of order m; the sine block of m = 0 is zeros."""
    if m == 0:
        c = x[..., : lmax + 1]
        return c, np.zeros_like(c)
    b = block_base(m, lmax)
    n = lmax - m + 1
    return x[..., b: b + n], x[..., b + n: b + 2 * n]


def packed_index(lmax: int):
    """(l, m, is_sine) for every entry of the packed vector."""
    L, M, S = [], [], []
    L += list(range(lmax + 1)); M += [0] * (lmax + 1); S += [0] * (lmax + 1)
    for m in range(1, lmax + 1):
        ls = list(range(m, lmax + 1))
        L += ls; M += [m] * len(ls); S += [0] * len(ls)
        L += ls; M += [m] * len(ls); S += [1] * len(ls)
    return np.array(L), np.array(M), np.array(S)


# --------------------------------------------------------------------------
# Legendre step
# --------------------------------------------------------------------------
def legendre_pair_m(x: np.ndarray, G, m: int, lmax: int, geom: RingGeometry):
    """Legendre step of one order m in both directions.

    Returns (F^c_m, F^s_m) = (sum_l lambda_lm x^c_lm, sum_l lambda_lm x^s_lm) per ring
    for the packed input x (..., nalm), and, if G = (G^c_m, G^s_m) per ring is
    given, the adjoint blocks (sum_k lambda_lm(theta_k) G^c_m(k), ...) per l.
    """
    lam = lambda_table(m, lmax, geom.z, geom.sint)          # (nl, nrings)
    F = None
    if x is not None:
        xc, xs = split_m(x, m, lmax)
        F = (xc @ lam, xs @ lam)
    A = None
    if G is not None:
        A = (G[0] @ lam.T, G[1] @ lam.T)
    return F, A


def _synth_orders(lmax: int, geom: RingGeometry, items):
    """Legendre synthesis of the orders in items [(m, x^c_m, x^s_m)]."""
    out = []
    for m, xc, xs in items:
        lam = lambda_table(m, lmax, geom.z, geom.sint)
        out.append((m, xc @ lam, xs @ lam))
    return out


def _adjoint_orders(lmax: int, geom: RingGeometry, items):
    """Legendre adjoint of the orders in items [(m, G^c_m, G^s_m)]."""
    out = []
    for m, gc, gs in items:
        lam = lambda_table(m, lmax, geom.z, geom.sint)
        out.append((m, gc @ lam.T, gs @ lam.T))
    return out


def _order_groups(lmax: int, geom: RingGeometry):
    """Orders in interleaved groups, one per worker task; a single group for
    small transforms (worker start-up would cost more than it saves)."""
    from . import pool
    if (lmax + 1) ** 2 * geom.nrings < 2e7:
        return [list(range(lmax + 1))]
    return pool.interleave(lmax + 1, 4 * pool.worker_count())


def legendre_synth(x: np.ndarray, lmax: int, geom: RingGeometry):
    """F^c, F^s of shape (..., nrings, lmax+1) from packed x of shape (..., nalm).

    Orders are independent; large transforms spread them over the oracle's
    worker processes (``pool``), with the same per-order arithmetic."""
    from . import pool
    x = np.asarray(x, dtype=np.float64)
    lead = x.shape[:-1]
    Fc = np.zeros(lead + (geom.nrings, lmax + 1))
    Fs = np.zeros_like(Fc)
    groups = [(lmax, geom, [(m,) + tuple(np.ascontiguousarray(v) for v in split_m(x, m, lmax))
                            for m in ms]) for ms in _order_groups(lmax, geom)]
    for res in pool.run(_synth_orders, groups):
        for m, fc, fs in res:
            Fc[..., :, m] = fc
            Fs[..., :, m] = fs
    return Fc, Fs


def legendre_adjoint(Gc: np.ndarray, Gs: np.ndarray, lmax: int, geom: RingGeometry):
    """Transpose of ``legendre_synth``: packed x from G^c, G^s (..., nrings, lmax+1)."""
    from . import pool
    lead = Gc.shape[:-2]
    x = np.zeros(lead + (nalm(lmax),))
    groups = [(lmax, geom, [(m, np.ascontiguousarray(Gc[..., :, m]), np.ascontiguousarray(Gs[..., :, m]))
                            for m in ms]) for ms in _order_groups(lmax, geom)]
    for res in pool.run(_adjoint_orders, groups):
        for m, ac, as_ in res:
            if m == 0:
                x[..., : lmax + 1] = ac
            else:
                b = block_base(m, lmax)
                n = lmax - m + 1
                x[..., b: b + n] = ac
                x[..., b + n: b + 2 * n] = as_
    return x


# --------------------------------------------------------------------------
# ring step
# --------------------------------------------------------------------------
def _weights(lmax: int) -> np.ndarray:
    w = np.full(lmax + 1, SQRT2)
    w[0] = 1.0
    return w


def ring_synth(Fc: np.ndarray, Fs: np.ndarray, geom: RingGeometry) -> np.ndarray:
    """Map (..., npix) from F^c, F^s (..., nrings, lmax+1)."""
    lmax = Fc.shape[-1] - 1
    lead = Fc.shape[:-2]
    w = _weights(lmax)
    ms = np.arange(lmax + 1)
    out = np.zeros(lead + (geom.npix,))
    for k in range(geom.nrings):
        n = int(geom.nphi[k])
        H = w * (Fc[..., k, :] - 1j * Fs[..., k, :]) * np.exp(1j * ms * geom.phi0[k])
        Hf = np.zeros(lead + (n,), dtype=np.complex128)
        for q0 in range(0, lmax + 1, n):
            seg = H[..., q0: q0 + n]
            Hf[..., : seg.shape[-1]] += seg
        f = (np.fft.ifft(Hf, axis=-1) * n).real
        out[..., geom.start[k]: geom.start[k] + n] = f
    return out


def ring_adjoint(y: np.ndarray, lmax: int, geom: RingGeometry):
    """Transpose of ``ring_synth``: G^c, G^s (..., nrings, lmax+1) from a map."""
    lead = y.shape[:-1]
    w = _weights(lmax)
    ms = np.arange(lmax + 1)
    Gc = np.zeros(lead + (geom.nrings, lmax + 1))
    Gs = np.zeros_like(Gc)
    for k in range(geom.nrings):
        n = int(geom.nphi[k])
        Y = np.fft.fft(y[..., geom.start[k]: geom.start[k] + n], axis=-1)
        t = np.exp(1j * ms * geom.phi0[k]) * np.conj(Y[..., ms % n])
        Gc[..., k, :] = w * t.real
        Gs[..., k, :] = w * t.imag
    return Gc, Gs


# --------------------------------------------------------------------------
# full transforms
# --------------------------------------------------------------------------
def synth(x: np.ndarray, lmax: int, nside: int) -> np.ndarray:
    return synth_geom(x, lmax, healpix_rings(nside))


def adjoint(y: np.ndarray, lmax: int, nside: int) -> np.ndarray:
    return adjoint_geom(y, lmax, healpix_rings(nside))


def synth_geom(x: np.ndarray, lmax: int, geom: RingGeometry) -> np.ndarray:
    """Synthesis at the pixels of any iso-latitude ring geometry."""
    Fc, Fs = legendre_synth(x, lmax, geom)
    return ring_synth(Fc, Fs, geom)


def adjoint_geom(y: np.ndarray, lmax: int, geom: RingGeometry) -> np.ndarray:
    """Adjoint synthesis (plain transpose) for any iso-latitude ring geometry."""
    Gc, Gs = ring_adjoint(y, lmax, geom)
    return legendre_adjoint(Gc, Gs, lmax, geom)


def dense_Y(nside: int, lmax: int) -> np.ndarray:
    """Brute-force dense Y (npix x nalm) from scipy.special.sph_harm_y.

    Column (l, 0): Y_l0; column (l, m, cos): sqrt(2) Re Y_lm; (l, m, sin):
    sqrt(2) Im Y_lm, with Y_lm = lambda_lm(theta) e^{i m phi}.
    """
    from scipy.special import sph_harm_y

    geom = healpix_rings(nside)
    theta, phi = pixel_angles(geom)
    L, M, S = packed_index(lmax)
    Yd = np.empty((theta.size, L.size))
    for j in range(L.size):
        ylm = sph_harm_y(int(L[j]), int(M[j]), theta, phi)
        if M[j] == 0:
            Yd[:, j] = ylm.real
        elif S[j] == 0:
            Yd[:, j] = SQRT2 * ylm.real
        else:
            Yd[:, j] = SQRT2 * ylm.imag
    return Yd


# --------------------------------------------------------------------------
# sampled evaluation (one ring, all m) for large grids
# --------------------------------------------------------------------------
def synth_rings(x: np.ndarray, lmax: int, nside: int, rings) -> dict:
    """Synthesized pixel values on selected rings only: {ring k: values}.

    Uses the same definition, with the Legendre step stepped over all m at
    once for each selected ring (``legendre.lambda_all_m``)."""
    from .legendre import lambda_all_m

    geom = healpix_rings(nside)
    x = np.asarray(x, dtype=np.float64)
    w = _weights(lmax)
    out = {}
    for k in rings:
        lam = lambda_all_m(lmax, float(geom.z[k]), float(geom.sint[k]))   # [l, m]
        Fc = np.zeros(x.shape[:-1] + (lmax + 1,))
        Fs = np.zeros_like(Fc)
        for m in range(lmax + 1):
            xc, xs = split_m(x, m, lmax)
            Fc[..., m] = xc @ lam[m:, m]
            Fs[..., m] = xs @ lam[m:, m]
        phi = geom.ring_phi(k)
        ms = np.arange(lmax + 1)
        cosm = np.cos(np.outer(ms, phi))
        sinm = np.sin(np.outer(ms, phi))
        out[k] = (w * Fc) @ cosm + (w * Fs) @ sinm
    return out


def adjoint_orders(y: np.ndarray, lmax: int, nside: int, orders) -> dict:
    """Adjoint synthesis restricted to selected orders: {m: (cos block, sin block)}.

    Each ring's weighted trigonometric sums at frequency m are evaluated
    directly from the definition (no FFT, no folding), then contracted with
    the lambda_lm table of that order over all rings, for grids too large for
    the full transform."""
    geom = healpix_rings(nside)
    y = np.asarray(y, dtype=np.float64)
    out = {}
    for m in orders:
        w = 1.0 if m == 0 else SQRT2
        gc = np.zeros(y.shape[:-1] + (geom.nrings,))
        gs = np.zeros_like(gc)
        for k in range(geom.nrings):
            phi = geom.ring_phi(k)
            seg = y[..., geom.start[k]: geom.start[k] + int(geom.nphi[k])]
            gc[..., k] = w * (seg @ np.cos(m * phi))
            gs[..., k] = w * (seg @ np.sin(m * phi))
        lam = lambda_table(m, lmax, geom.z, geom.sint)        # (lmax - m + 1, nrings)
        out[m] = (gc @ lam.T, gs @ lam.T)
    return out
