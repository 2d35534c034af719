"""The CR system operator for the oracle.

A = S^-1 + B Y^T N^-1 Y B                          (eq. system-explicit, Sec. 2.3)
A_h = F_h A F_h^T = D_h + B_h Y^T N^-1 Y B_h      (eq. A_h, Sec. 3.2)

with S = diag(C_l), B = diag(b_l p_l), D_h = diag(f_l^2 / C_l),
B_h = diag(f_l b_l p_l), N^-1 a pixel diagonal that is 0 inside the mask
(Sec. 2.3).  Unknowns are restricted to the active modes {(l, m): C_l > 0,
l <= lmax_h}: inputs there are ignored and outputs there are 0 (the
projection reading of C_0 = C_1 = 0).

Dense Y^T N^-1 Y is built two independent ways: (1) brute force from the
dense Y of ``sht.dense_Y``; (2) the ring-DFT formula of eq. Ni-dense, which
needs, per ring k, xi-weighted Fourier sums Xi_k(D) = sum_j xi_kj e^{i D phi_kj}
at the frequencies D = m1 - m2 and m1 + m2 (the real basis mixes both).
"""
from __future__ import annotations

import numpy as np

from . import sht
from .geometry import healpix_rings
from .legendre import lambda_table


def mode_ell(lmax: int) -> np.ndarray:
    L, _, _ = sht.packed_index(lmax)
    return L


def level_diagonals(cl, bl, lmax_h: int, fl=None):
    """(d, bh) per l for a level: d = f^2 / C (0 where C = 0), bh = f b (0 where C = 0)."""
    cl = np.asarray(cl, dtype=np.float64)[: lmax_h + 1]
    bl = np.asarray(bl, dtype=np.float64)[: lmax_h + 1]
    f = np.ones(lmax_h + 1) if fl is None else np.asarray(fl, dtype=np.float64)[: lmax_h + 1]
    act = cl > 0
    d = np.where(act, f * f / np.where(act, cl, 1.0), 0.0)
    bh = np.where(act, f * bl, 0.0)
    return d, bh


def apply_A(x, cl, bl, ninv, nside: int, lmax_h: int | None = None, fl=None):
    """y = D_h x + B_h Y^T N^-1 Y B_h x (top level: f = 1, D = S^-1, B_h = B)."""
    x = np.asarray(x, dtype=np.float64)
    lmax_h = (len(cl) - 1) if lmax_h is None else lmax_h
    d, bh = level_diagonals(cl, bl, lmax_h, fl)
    L = mode_ell(lmax_h)
    u = bh[L] * x
    f = sht.synth(u, lmax_h, nside)
    v = sht.adjoint(ninv * f, lmax_h, nside)
    return d[L] * x + bh[L] * v


def dense_YtNY_bruteforce(nside: int, lmax: int, ninv) -> np.ndarray:
    Y = sht.dense_Y(nside, lmax)
    return Y.T @ (np.asarray(ninv)[:, None] * Y)


def ring_fourier_sums(nside: int, xi, dmax: int) -> np.ndarray:
    """Xi[k, D] = sum_j xi_kj e^{i D phi_kj}, D = 0..dmax, from one FFT per ring."""
    geom = healpix_rings(nside)
    xi = np.asarray(xi, dtype=np.float64)
    D = np.arange(dmax + 1)
    Xi = np.zeros((geom.nrings, dmax + 1), dtype=np.complex128)
    for k in range(geom.nrings):
        n = int(geom.nphi[k])
        Fk = np.fft.fft(xi[geom.start[k]: geom.start[k] + n])
        Xi[k] = np.exp(1j * D * geom.phi0[k]) * np.conj(Fk[D % n])
    return Xi


def dense_YtNY_ringdft(nside: int, lmax: int, ninv) -> np.ndarray:
    """Eq. Ni-dense in the real basis.

    For basis functions u_1 = w_{m1} lambda_{l1 m1} t_1(m1 phi) and
    u_2 = w_{m2} lambda_{l2 m2} t_2(m2 phi), t in {cos, sin}:
      cos a cos b = (cos(a-b) + cos(a+b)) / 2
      sin a sin b = (cos(a-b) - cos(a+b)) / 2
      cos a sin b = (sin(a+b) - sin(a-b)) / 2
      sin a cos b = (sin(a+b) + sin(a-b)) / 2
    and sum_j xi_kj cos(D phi_kj) = Re Xi_k(D), sin -> Im (Xi(-D) = conj Xi(D)).
    """
    geom = healpix_rings(nside)
    Xi = ring_fourier_sums(nside, ninv, 2 * lmax)
    L, M, S = sht.packed_index(lmax)
    n = L.size
    # lambda for every packed entry at every ring
    lam = np.zeros((n, geom.nrings))
    tabs = [lambda_table(m, lmax, geom.z, geom.sint) for m in range(lmax + 1)]
    for j in range(n):
        lam[j] = tabs[M[j]][L[j] - M[j]]
    w = np.where(M == 0, 1.0, np.sqrt(2.0))
    out = np.empty((n, n))
    for i in range(n):
        m1, s1 = M[i], S[i]
        dm = m1 - M                 # may be negative
        sm = m1 + M
        Xd = Xi[:, np.abs(dm)]
        Xd = np.where(dm[None, :] < 0, np.conj(Xd), Xd)   # Xi(-D) = conj Xi(D)
        Xs = Xi[:, sm]
        cc = 0.5 * (Xd.real + Xs.real)
        ss = 0.5 * (Xd.real - Xs.real)
        cs = 0.5 * (Xs.imag - Xd.imag)      # cos(m1) sin(m2)
        sc = 0.5 * (Xs.imag + Xd.imag)      # sin(m1) cos(m2)
        if s1 == 0:
            trig = np.where(S[None, :] == 0, cc, cs)
        else:
            trig = np.where(S[None, :] == 0, sc, ss)
        out[i] = w[i] * w * np.einsum("k,jk,kj->j", lam[i], lam, trig)
    return out


def dense_A(cl, bl, ninv, nside: int, lmax_h: int | None = None, fl=None, route: str = "ringdft"):
    """Dense A_h over ALL packed modes (excluded modes give zero rows/columns)."""
    lmax_h = (len(cl) - 1) if lmax_h is None else lmax_h
    d, bh = level_diagonals(cl, bl, lmax_h, fl)
    L = mode_ell(lmax_h)
    if route == "bruteforce":
        K = dense_YtNY_bruteforce(nside, lmax_h, ninv)
    else:
        K = dense_YtNY_ringdft(nside, lmax_h, ninv)
    return np.diag(d[L]) + bh[L][:, None] * K * bh[L][None, :]


def diag_YtNY(nside: int, lmax: int, ninv) -> np.ndarray:
    """Diagonal of Y^T N^-1 Y from eq. Ni-dense (D = 0 and D = 2m terms)."""
    geom = healpix_rings(nside)
    Xi = ring_fourier_sums(nside, ninv, 2 * lmax)
    out = np.zeros(sht.nalm(lmax))
    for m in range(lmax + 1):
        lam2 = lambda_table(m, lmax, geom.z, geom.sint) ** 2     # (nl, nrings)
        X0 = Xi[:, 0].real
        X2 = Xi[:, 2 * m].real
        if m == 0:
            out[: lmax + 1] = lam2 @ X0
        else:
            b = sht.block_base(m, lmax)
            n = lmax - m + 1
            out[b: b + n] = lam2 @ (X0 + X2)         # 2 cos^2 = 1 + cos 2a
            out[b + n: b + 2 * n] = lam2 @ (X0 - X2)  # 2 sin^2 = 1 - cos 2a
    return out
