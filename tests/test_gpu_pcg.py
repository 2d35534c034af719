"""Conjugate gradients with the CR-Cycle as preconditioner, and the CR
right-hand side on the GPU (Sec. 2.3, eq. cr-system; caption of Fig.
code:mg).

* mlcr_cr_rhs against the oracle's CR right-hand side from the same white
  draws, with and without the fluctuation terms (the latter is the
  Wiener-filter system): float64, 1e-12.
* pcg_solve on a manufactured right-hand side at N_side 256 / lmax 512 in
  all three precisions: max pixel error <= 1e-3 uK and below the oracle's
  a-posteriori certificate; not more iterations than W-cycle iterations.
* the Wiener-filtered map at N_side 16 / lmax 32 by pcg_solve against the
  oracle's dense Cholesky solve, 1e-10.
"""
import numpy as np
import pytest

import workloads
from oracle import operator as oop
from oracle import sht as osht
from oracle import solve as osolve
from tests.gpu_util import dev, host, parity

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
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=max_nrhs)
    return cfg, d, op


def _data_map(cfg, d, gs, gn):
    """d = Y B s + n with s = S^1/2 gs, n = sigma gn (the oracle's data model)."""
    L = workloads.packed_ell(cfg.lmax)
    act = d["cl"][L] > 0
    s = np.sqrt(np.where(act, d["cl"][L], 0.0)) * gs
    return osht.synth((np.where(act, d["bl"][L], 0.0) * s)[None], cfg.lmax, cfg.nside)[0] + d["sigma"] * gn


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_cr_rhs_matches_oracle(mlcr, name):
    print(f"case cr rhs {name}", flush=True)
    cfg, d, op = _problem(mlcr, name, max_nrhs=2)
    rows = [workloads.draw_rhs_white(cfg, r) for r in range(2)]
    dm = np.stack([_data_map(cfg, d, gs, gn) for _, _, gs, gn in rows])
    w1 = np.stack([r[0] for r in rows])
    w2 = np.stack([r[1] for r in rows])
    b = host(mlcr.cr_rhs(op, dev(dm), dev(w1), dev(w2)))
    ref = np.stack([osolve.cr_rhs(d["cl"], d["bl"], d["ninv"], d["sigma"], cfg.nside, *r) for r in rows])
    assert parity(b, ref) <= 1e-12, parity(b, ref)
    # Wiener filter: no fluctuation terms
    bw = host(mlcr.cr_rhs(op, dev(dm)))
    zero_a, zero_p = np.zeros(cfg.nalm), np.zeros(cfg.npix)
    refw = np.stack([osolve.cr_rhs(d["cl"], d["bl"], d["ninv"], d["sigma"], cfg.nside, zero_a, zero_p,
                                   gs, gn) for _, _, gs, gn in rows])
    assert parity(bw, refw) <= 1e-12, parity(bw, refw)


@pytest.mark.parametrize("prec_name", ["fp64", "fp32", "bf16x3"])
def test_pcg_c2_manufactured(mlcr, prec_name):
    print(f"case pcg c2 {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}[prec_name]
    cfg, d, op = _problem(mlcr, "c2")
    S = mlcr.Solver(op, max_nrhs=1)
    xt = workloads.prior_sample(cfg, 0)
    b = oop.apply_A(xt, d["cl"], d["bl"], d["ninv"], cfg.nside)
    x, info = S.solve_pcg(dev(b[None]), rtol=1e-8, max_iter=40, prec=prec)
    _, info_w = S.solve(dev(b[None]), rtol=1e-8, max_cycles=40, prec=prec)
    xg = host(x)[0]
    mpe = osolve.max_pixel_error(xg, xt, cfg.lmax, cfg.nside)
    bound, _ = osolve.certificate(xg, b, d["cl"], d["bl"], d["ninv"], cfg.nside)
    print(f"pcg {prec_name}: {info[0]['cycles']} iterations (W-cycle {info_w[0]['cycles']}), "
          f"rho {info[0]['rho']:.2e}, max pixel error {mpe:.3e} uK, certificate {bound:.3e} uK", flush=True)
    assert info[0]["converged"] == 1
    assert mpe <= bound * (1 + 1e-9) and mpe <= 1e-3
    assert info[0]["cycles"] <= info_w[0]["cycles"]


def test_wiener_filter_c1(mlcr):
    print("case wiener filter c1", flush=True)
    cfg, d, op = _problem(mlcr, "c1")
    S = mlcr.Solver(op, max_nrhs=1)
    _, _, gs, gn = workloads.draw_rhs_white(cfg, 3)
    dm = _data_map(cfg, d, gs, gn)
    b = mlcr.cr_rhs(op, dev(dm[None]))
    x, info = S.solve_pcg(b, rtol=1e-12, max_iter=10)
    A = oop.dense_A(d["cl"], d["bl"], d["ninv"], cfg.nside)
    bref = osolve.cr_rhs(d["cl"], d["bl"], d["ninv"], d["sigma"], cfg.nside, np.zeros(cfg.nalm),
                         np.zeros(cfg.npix), gs, gn)
    xr = osolve.solve_dense(A, bref, d["cl"])
    assert parity(host(x)[0], xr) <= 1e-10, parity(host(x)[0], xr)
    assert info[0]["converged"] == 1
