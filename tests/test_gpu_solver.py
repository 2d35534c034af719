"""GPU solver parity: wcycle_solve against the oracle.

* C1 (N_side 16, lmax 32): the ladder is a single dense level; the GPU solve
  must match the oracle's dense Cholesky solve of A to 1e-10 relative.
* top-level diagonal smoother: 1/diag(A) from eq. Ni-dense on the GPU vs the
  oracle's diagonal, 1e-12 relative.
* C2 (N_side 256, lmax 512): multi-level W-cycles to relative residual 1e-8
  on a manufactured right-hand side b = A x_true (Sec. 4.1); the true max
  pixel error (oracle synthesis) must be below 1e-3 uK and below the
  a-posteriori certificate sigma_prior ||S^1/2 r|| (oracle residual).
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import operator as oop
from oracle import solve as osolve
from tests.gpu_util import dev, host, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


def _problem(mlcr, name, max_nrhs=1):
    cfg = workloads.get_config(name)
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    ninv = dev(d["ninv"])
    op = mlcr.Operator(g, d["cl"], d["bl"], ninv, max_nrhs=max_nrhs)
    return cfg, d, g, ninv, op


def test_c1_dense_solve_matches_cholesky(mlcr):
    print("case c1 dense solve", flush=True)
    cfg, d, g, ninv, op = _problem(mlcr, "c1")
    S = mlcr.Solver(op, max_nrhs=1)
    assert S.info()["nlevels"] == 0
    w1, w2, gs, gn = workloads.draw_rhs_white(cfg, 0)
    b = osolve.cr_rhs(d["cl"], d["bl"], d["ninv"], d["sigma"], cfg.nside, w1, w2, gs, gn)
    x, info = S.solve(dev(b[None]), rtol=1e-12, max_cycles=4)
    A = oop.dense_A(d["cl"], d["bl"], d["ninv"], cfg.nside)
    xr = osolve.solve_dense(A, b, d["cl"])
    assert rel2(host(x)[0], xr) <= 1e-10, rel2(host(x)[0], xr)
    assert info[0]["converged"] == 1


def test_top_diagonal_parity(mlcr):
    print("case top diagonal nside 64 lmax 128", flush=True)
    cfg = workloads.WorkloadConfig("t64", 64, 128, 60.0, 15.0, 20.0, 20, 2.0, 1)
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=1)
    S = mlcr.Solver(op, max_nrhs=1)
    assert S.info()["nlevels"] >= 1
    got = host(S.top_dinv())
    dl, bh = oop.level_diagonals(d["cl"], d["bl"], cfg.lmax)
    L = oop.mode_ell(cfg.lmax)
    diag = dl[L] + bh[L] ** 2 * oop.diag_YtNY(cfg.nside, cfg.lmax, d["ninv"])
    ref = np.where(dl[L] > 0, 1.0 / np.where(dl[L] > 0, diag, 1.0), 0.0)
    assert rel2(got, ref) <= 1e-12, rel2(got, ref)


@pytest.mark.parametrize("prec_name", ["fp64", "fp32", "bf16x3"])
def test_c2_wcycle_manufactured(mlcr, prec_name):
    """fp32 / bf16x3: the cycle's transforms with that contraction (matrix
    cores), residual and update in float64 -- iterative refinement to the
    same bar."""
    print(f"case c2 w-cycle manufactured {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}[prec_name]
    cfg, d, g, ninv, op = _problem(mlcr, "c2")
    S = mlcr.Solver(op, max_nrhs=1)
    xt = workloads.prior_sample(cfg, 0)
    b = oop.apply_A(xt, d["cl"], d["bl"], d["ninv"], cfg.nside)
    x, info = S.solve(dev(b[None]), rtol=1e-8, max_cycles=40, prec=prec)
    xg = host(x)[0]
    print("c2 info", info[0], flush=True)
    assert info[0]["converged"] == 1 and info[0]["rho"] <= 1e-8
    mpe = osolve.max_pixel_error(xg, xt, cfg.lmax, cfg.nside)
    bound, _ = osolve.certificate(xg, b, d["cl"], d["bl"], d["ninv"], cfg.nside)
    print(f"c2 max pixel error {mpe:.3e} uK, certificate {bound:.3e} uK", flush=True)
    assert mpe <= bound * (1 + 1e-9)        # the a-posteriori bound holds
    assert mpe <= 1e-3


def test_solver_errors(mlcr):
    from paper_1308_5299_amd import MLCRError
    cfg, d, g, ninv, op = _problem(mlcr, "c1")
    S = mlcr.Solver(op, max_nrhs=1)
    b = dev(np.ones((2, cfg.nalm)))
    with pytest.raises(MLCRError):
        S.solve(b)                      # more RHS than max_nrhs
    x, info = S.solve(dev(np.ones((1, cfg.nalm))), rtol=0.0, max_cycles=1,
                      raise_on_noconv=False)
    assert info[0]["cycles"] == 1
    with pytest.raises(MLCRError) as e:
        S.solve(dev(np.ones((1, cfg.nalm))), rtol=0.0, max_cycles=1)
    assert e.value.code == -5
    # the multi-level solver needs every mode in the unknowns (no C_l = 0)
    cfg = workloads.WorkloadConfig("t64", 64, 128, 60.0, 15.0, 20.0, 20, 2.0, 1)
    d = workloads.workload_inputs(cfg)
    cl = d["cl"].copy()
    cl[:2] = 0.0
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, cl, d["bl"], dev(d["ninv"]), max_nrhs=1)
    with pytest.raises(MLCRError) as e:
        mlcr.Solver(op, max_nrhs=1)
    assert e.value.code == -1 and "C_l > 0" in str(e.value)
