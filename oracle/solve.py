"""Exact solutions, right-hand sides and error certificates for the oracle.

The multi-level method is an iterative solver for the symmetric positive
definite CR system (Sec. 2.4), so what it must reach is the plain definition
x* = A^-1 b.  The oracle computes that directly:

* ``solve_dense``   Cholesky of the dense A on the active modes (tiny grids).
* ``solve_cg``      Jacobi-preconditioned conjugate gradients (Sec. 2.4 names
                    CG as the standard approach) for mid-size grids.
* ``cr_rhs``        b = B Y^T N^-1 d + S^{-1/2} w1 + B Y^T N^{-1/2} w2 with
                    d = Y B s + n (eq. Y-data-model, eq. cr-system and the
                    fluctuation terms that make x a posterior sample).
* ``manufactured``  b = A x_true with x_true drawn from the prior (Sec. 4.1).
* ``certificate``   an a-posteriori bound on the max pixel error of any x:
                    since A = S^-1 + (PSD), S^{1/2} A S^{1/2} >= I, so for every
                    pixel p, |Y(x - x*)|_p <= sigma_prior ||S^{1/2}(b - A x)||_2
                    with sigma_prior^2 = sum_l (2l+1) C_l / (4 pi) (addition
                    theorem, eq. addition-theorem, at zero separation).
* ``s_inv_ratio``   the stopping quantity of CR-Solve (Fig. code:mg):
                    sqrt(r^T S^-1 r / b^T S^-1 b).
"""
from __future__ import annotations

import math

import numpy as np

from . import sht
from .operator import apply_A, mode_ell


def active_modes(cl) -> np.ndarray:
    cl = np.asarray(cl)
    return cl[mode_ell(len(cl) - 1)] > 0


def cr_rhs(cl, bl, ninv, sigma, nside: int, w1, w2, gs, gn):
    """b of the CR system for one realization from white draws."""
    cl = np.asarray(cl, dtype=np.float64)
    lmax = len(cl) - 1
    L = mode_ell(lmax)
    act = cl[L] > 0
    sq = np.sqrt(np.where(act, cl[L], 0.0))
    bh = np.where(act, np.asarray(bl)[L], 0.0)
    s = sq * gs                                    # s ~ N(0, S)
    d = sht.synth(bh * s, lmax, nside) + np.asarray(sigma) * gn
    ninv = np.asarray(ninv)
    pix = ninv * d + np.sqrt(ninv) * w2
    b = bh * sht.adjoint(pix, lmax, nside)
    b = b + np.where(act, w1 / np.where(act, sq, 1.0), 0.0)
    return np.where(act, b, 0.0)


def manufactured(x_true, cl, bl, ninv, nside: int):
    return apply_A(x_true, cl, bl, ninv, nside)


def solve_dense(Adense: np.ndarray, b, cl) -> np.ndarray:
    """x* = A^-1 b on the active modes by Cholesky (scipy.linalg.cho_factor)."""
    from scipy.linalg import cho_factor, cho_solve

    act = active_modes(cl)
    idx = np.nonzero(act)[0]
    sub = Adense[np.ix_(idx, idx)]
    c = cho_factor(sub, lower=True)
    x = np.zeros(len(act))
    x[idx] = cho_solve(c, np.asarray(b)[idx])
    return x


def solve_cg(apply, b, mdiag, rtol: float = 1e-12, maxiter: int = 100000, x0=None, callback=None):
    """Preconditioned CG; stops when ||r|| <= rtol ||b|| (Euclidean)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    z = mdiag * r
    p = z.copy()
    rz = float(r @ z)
    bn = float(np.linalg.norm(b))
    it = 0
    for it in range(1, maxiter + 1):
        Ap = apply(p)
        alpha = rz / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rn = float(np.linalg.norm(r))
        if callback is not None:
            callback(it, rn / bn)
        if rn <= rtol * bn:
            break
        z = mdiag * r
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it


def sigma_prior(cl) -> float:
    cl = np.asarray(cl, dtype=np.float64)
    ell = np.arange(len(cl))
    return math.sqrt(float(np.sum((2 * ell + 1) * cl) / (4.0 * math.pi)))


def s_half_norm(r, cl) -> float:
    cl = np.asarray(cl, dtype=np.float64)
    L = mode_ell(len(cl) - 1)
    return float(np.linalg.norm(np.sqrt(cl[L]) * np.asarray(r)))


def certificate(x, b, cl, bl, ninv, nside: int):
    """(bound on max pixel error in uK, ||S^{1/2} r||) for a candidate x."""
    act = active_modes(cl)
    r = np.where(act, np.asarray(b) - apply_A(x, cl, bl, ninv, nside), 0.0)
    sn = s_half_norm(r, cl)
    return sigma_prior(cl) * sn, sn


def s_inv_ratio(r, b, cl) -> float:
    cl = np.asarray(cl, dtype=np.float64)
    L = mode_ell(len(cl) - 1)
    act = cl[L] > 0
    sinv = np.where(act, 1.0 / np.where(act, cl[L], 1.0), 0.0)
    r = np.asarray(r); b = np.asarray(b)
    return math.sqrt(float(np.sum(sinv * r * r)) / float(np.sum(sinv * b * b)))


def max_pixel_error(x, xref, lmax: int, nside: int) -> float:
    """max_p |Y (x - x_ref)|_p over all pixels (masked ones included)."""
    return float(np.max(np.abs(sht.synth(np.asarray(x) - np.asarray(xref), lmax, nside))))
