"""Pins of the oracle operator and solves (oracle/operator.py, oracle/solve.py).

* eq. Ni-dense (ring-DFT route) against brute-force Y^T N^-1 Y built from
  scipy's Y_lm, with a masked, inhomogeneous N^-1;
* the operator is symmetric positive definite and A >= S^-1, so its
  smallest eigenvalue is at least 1 / max C_l;
* special case N^-1 = 0: A = S^-1 and x* = S b exactly;
* A_h = F_h A F_h (eq. A_h) for a level filter;
* Cholesky solve against numpy.linalg.solve, CG against Cholesky, the
  manufactured solution is recovered, and the max-pixel-error certificate
  bounds the true error of perturbed solutions;
* the CR right-hand side reduces to S^{-1/2} w1 when N^-1 = 0 and to
  (A - S^-1) s when w1 = w2 = n = 0.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import operator as op
from oracle import sht, solve


def _c1():
    cfg = workloads.get_config("c1")
    d = workloads.workload_inputs(cfg)
    return cfg, d


def test_ringdft_vs_bruteforce_masked():
    nside, lmax = 8, 18
    cfg = workloads.WorkloadConfig("t", nside, lmax, -1.0, 10.0, 20.0, 3, 8.0, 1)
    ninv, _, mask = workloads.inverse_noise_map(cfg)
    assert mask.any() and (~mask).any()
    K1 = op.dense_YtNY_bruteforce(nside, lmax, ninv)
    K2 = op.dense_YtNY_ringdft(nside, lmax, ninv)
    assert np.abs(K1 - K2).max() < 1e-14 * np.abs(K1).max()
    np.testing.assert_allclose(op.diag_YtNY(nside, lmax, ninv), np.diag(K1), rtol=1e-13, atol=0)


@pytest.mark.parametrize("project", [False, True])
def test_apply_matches_dense_and_is_spd(project):
    """project: C_0 = C_1 = 0 removes the monopole and dipole from the unknowns
    (their rows and columns of A vanish)."""
    cfg, d = _c1()
    d = dict(d)
    d["cl"] = d["cl"].copy()
    d["cl"][:2] = 0.0 if project else d["cl"][2]
    A = op.dense_A(d["cl"], d["bl"], d["ninv"], cfg.nside)
    x = np.random.default_rng(0).standard_normal(cfg.nalm)
    act = solve.active_modes(d["cl"])
    assert act.sum() == (cfg.nalm - 4 if project else cfg.nalm)
    y = op.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside)
    np.testing.assert_allclose(y, A @ np.where(act, x, 0.0), rtol=0, atol=1e-11 * np.abs(y).max())
    assert np.all(y[~act] == 0.0)
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
    idx = np.nonzero(act)[0]
    ev = np.linalg.eigvalsh(A[np.ix_(idx, idx)])
    assert ev.min() >= (1.0 / d["cl"].max()) * (1 - 1e-10)


def test_zero_noise_gives_prior():
    cfg, d = _c1()
    ninv0 = np.zeros(cfg.npix)
    b = np.random.default_rng(1).standard_normal(cfg.nalm)
    A = op.dense_A(d["cl"], d["bl"], ninv0, cfg.nside)
    L = op.mode_ell(cfg.lmax)
    act = d["cl"][L] > 0
    np.testing.assert_allclose(np.diag(A)[act], 1.0 / d["cl"][L][act], rtol=1e-15)
    x = solve.solve_dense(A, b, d["cl"])
    np.testing.assert_allclose(x, np.where(act, d["cl"][L] * b, 0.0), rtol=1e-14)


def test_level_operator_is_filtered_top_operator():
    cfg, d = _c1()
    lmax_h = 24
    f = np.exp(-((np.arange(cfg.lmax + 1) / 15.0) ** 4))
    A = op.dense_A(d["cl"], d["bl"], d["ninv"], cfg.nside)
    Ah = op.dense_A(d["cl"], d["bl"], d["ninv"], cfg.nside, lmax_h=lmax_h, fl=f)
    L, M, S = sht.packed_index(cfg.lmax)
    Lh, Mh, Sh = sht.packed_index(lmax_h)
    # position of every level mode in the top packed vector
    pos = {(l, m, s): i for i, (l, m, s) in enumerate(zip(L, M, S))}
    sel = np.array([pos[(l, m, s)] for l, m, s in zip(Lh, Mh, Sh)])
    F = f[Lh]
    ref = F[:, None] * A[np.ix_(sel, sel)] * F[None, :]
    np.testing.assert_allclose(Ah, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    x = np.random.default_rng(5).standard_normal(Lh.size)
    np.testing.assert_allclose(op.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside, lmax_h=lmax_h, fl=f),
                               Ah @ x, rtol=0, atol=1e-11 * np.abs(Ah @ x).max())


def test_solves_and_certificate():
    cfg, d = _c1()
    cl, bl, ninv = d["cl"], d["bl"], d["ninv"]
    A = op.dense_A(cl, bl, ninv, cfg.nside)
    act = solve.active_modes(cl)
    w1, w2, gs, gn = workloads.draw_rhs_white(cfg, 0)
    b = solve.cr_rhs(cl, bl, ninv, d["sigma"], cfg.nside, w1, w2, gs, gn)
    x = solve.solve_dense(A, b, cl)
    idx = np.nonzero(act)[0]
    xr = np.linalg.solve(A[np.ix_(idx, idx)], b[idx])
    np.testing.assert_allclose(x[idx], xr, rtol=1e-10, atol=1e-10 * np.abs(xr).max())
    # CG to 1e-13 agrees with Cholesky
    Ld = op.mode_ell(cfg.lmax)
    mdiag = np.where(act, 1.0 / np.where(act, np.diag(A), 1.0), 0.0)
    xc, it = solve.solve_cg(lambda v: np.where(act, A @ v, 0.0), b, mdiag, rtol=1e-13)
    assert np.linalg.norm(xc - x) <= 1e-10 * np.linalg.norm(x), it
    # manufactured solution
    xt = np.sqrt(cl[Ld]) * workloads.draw_prior_white(cfg, 0)
    bt = solve.manufactured(xt, cl, bl, ninv, cfg.nside)
    np.testing.assert_allclose(solve.solve_dense(A, bt, cl), xt, rtol=0, atol=1e-9 * np.abs(xt).max())
    # certificate bounds the true max pixel error of perturbed solutions
    rng = np.random.default_rng(9)
    for scale in [1e-3, 1e-6]:
        xp = x + np.where(act, scale * np.sqrt(cl[Ld]) * rng.standard_normal(cfg.nalm), 0.0)
        bound, _ = solve.certificate(xp, b, cl, bl, ninv, cfg.nside)
        true = solve.max_pixel_error(xp, x, cfg.lmax, cfg.nside)
        assert true <= bound * (1 + 1e-12)
        assert true > 0.0


def test_rhs_special_cases():
    cfg, d = _c1()
    cl, bl = d["cl"], d["bl"]
    w1, w2, gs, gn = workloads.draw_rhs_white(cfg, 0)
    L = op.mode_ell(cfg.lmax)
    act = cl[L] > 0
    b0 = solve.cr_rhs(cl, bl, np.zeros(cfg.npix), d["sigma"], cfg.nside, w1, w2, gs, gn)
    np.testing.assert_allclose(b0, np.where(act, w1 / np.sqrt(np.where(act, cl[L], 1.0)), 0.0), rtol=1e-14)
    z = np.zeros
    b1 = solve.cr_rhs(cl, bl, d["ninv"], d["sigma"], cfg.nside, z(cfg.nalm), z(cfg.npix), gs, z(cfg.npix))
    s = np.sqrt(cl[L]) * gs
    A = op.dense_A(cl, bl, d["ninv"], cfg.nside)
    ref = A @ s - np.where(act, s / np.where(act, cl[L], 1.0), 0.0)
    np.testing.assert_allclose(b1, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_s_inv_ratio_and_sigma_prior():
    cfg, d = _c1()
    assert abs(solve.sigma_prior(d["cl"]) - 100.0) < 1e-10       # C_0 = C_1 = 0 here
    b = np.random.default_rng(2).standard_normal(cfg.nalm)
    assert solve.s_inv_ratio(b, b, d["cl"]) == pytest.approx(1.0)


def test_s_inv_ratio_hand_computed():
    """sqrt(r^T S^-1 r / b^T S^-1 b) (Fig. code:mg's stopping quantity) on a
    hand-computed case: lmax 3, C = (0, 0, 4, 9), so l < 2 is excluded and the
    two active l carry different weights 1/4 and 1/9.  r has 2 at (l=2, m=0)
    and 3 at (l=3, m=0); b has 1 at both; both have large values on excluded
    modes, which must not count.  r^T S^-1 r = 4/4 + 9/9 = 2 and
    b^T S^-1 b = 1/4 + 1/9 = 13/36, so the ratio is sqrt(72/13).  Weighting
    by C instead of 1/C would give sqrt(97/13)."""
    cl = np.array([0.0, 0.0, 4.0, 9.0])
    n = sht.nalm(3)
    r = np.zeros(n); b = np.zeros(n)
    r[2], r[3] = 2.0, 3.0
    b[2], b[3] = 1.0, 1.0
    r[0], r[1], b[0], b[1] = 100.0, -50.0, 30.0, 7.0          # l = 0, 1: excluded
    base = sht.block_base(1, 3)                               # m = 1 cosine block, l = 1 first
    r[base], b[base] = 40.0, 11.0                             # (l=1, m=1): excluded
    assert solve.s_inv_ratio(r, b, cl) == pytest.approx(math.sqrt(72.0 / 13.0), rel=1e-15)
    # a sine entry at (l=3, m=2) enters with weight 1/9
    s32 = sht.block_base(2, 3) + 2 + 1
    r2 = r.copy(); r2[s32] = 3.0
    assert solve.s_inv_ratio(r2, b, cl) == pytest.approx(math.sqrt(3.0 * 36.0 / 13.0), rel=1e-15)


def test_certificate_is_attained_at_zero_noise():
    """The certificate max_p |Y(x - x*)|_p <= sigma_prior ||S^{1/2} (b - A x)||
    is tight: with N^-1 = 0 (A = S^-1) and a residual r proportional to the
    row of Y at one pixel p, the error e = S r has e_p = sigma_prior^2 (Unsold,
    sum_m Y_lm(p)^2 = (2l+1)/4 pi) while ||S^{1/2} r|| = sigma_prior, so the bound
    equals the true max pixel error.  A sigma_prior or an S^{1/2} weighting
    that is too large, or a residual taken against the wrong operator, breaks
    the equality."""
    cfg, d = _c1()
    cl, bl = d["cl"], d["bl"]
    L = op.mode_ell(cfg.lmax)
    act = cl[L] > 0
    rng = np.random.default_rng(5)
    xstar = np.where(act, np.sqrt(np.where(act, cl[L], 0.0)) * rng.standard_normal(cfg.nalm), 0.0)
    ninv0 = np.zeros(cfg.npix)
    b = op.apply_A(xstar, cl, bl, ninv0, cfg.nside)
    for p in (0, 1234, cfg.npix - 1):
        delta = np.zeros(cfg.npix); delta[p] = 1.0
        r = np.where(act, sht.adjoint(delta, cfg.lmax, cfg.nside), 0.0)     # row p of Y
        x = xstar - np.where(act, cl[L], 0.0) * r                           # b - A x = r
        bound, sn = solve.certificate(x, b, cl, bl, ninv0, cfg.nside)
        assert sn == pytest.approx(solve.sigma_prior(cl), rel=1e-12)
        true = solve.max_pixel_error(x, xstar, cfg.lmax, cfg.nside)
        assert true == pytest.approx(bound, rel=1e-12), (p, true, bound)
        e_p = sht.synth(xstar - x, cfg.lmax, cfg.nside)[p]
        assert e_p == pytest.approx(solve.sigma_prior(cl) ** 2, rel=1e-12)
