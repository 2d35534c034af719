"""Full-size checks in the launch configuration the benchmark times
(N_side 2048, lmax 4096, 8 RHS per launch), and the multi-level solve at
N_side 1024 / lmax 2048 in both precisions.

At these sizes the oracle cannot run whole transforms, so it is asked for
samples it computes one by one:
* synthesis: every pixel of a few whole rings (all m, all l, by the definition);
* adjoint: a few whole orders m (direct trigonometric ring sums, all rings).
The operator is then checked through properties that hold at any size:
symmetry <u, A v> = <A u, v>; the fused ring kernel equals the composition
of the sampled-checked transforms; the float32 path stays within its
rounding bound of the float64 path.  The solves use a manufactured solution
b = A x_true (Sec. 4.1) and measure the max pixel error with the float64
synthesis.
"""
import math
import time

import numpy as np
import pytest
import torch

import workloads
from oracle import sht as osht
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

R = 8
TOL = 1e-12
TOL32 = 2e-5          # float32 contraction: ~2^-24 sqrt(lmax) relative
TOLB3 = 1e-4          # split-bfloat16 contraction: 3 * 2^-18 per product, 9x margin


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def c5(mlcr):
    cfg = workloads.get_config("c5")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    x = np.stack([workloads.prior_sample(cfg, r) for r in range(R)])
    return cfg, d, g, x


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_c5_synthesis_sampled_rings(mlcr, c5):
    cfg, d, g, x = c5
    print("case c5 synthesis, 8 RHS, sampled rings", flush=True)
    rings = [3, 2047, 4095]             # polar cap, cap/belt edge, equator
    geo = osht.healpix_rings(cfg.nside)
    ref = osht.synth_rings(x, cfg.lmax, cfg.nside, rings)
    # the relative 2-norm bar applies to the sampled output as a whole; a
    # single ring near a pole holds only a few pixels, so it gets 4x slack
    for prec, tol in [(mlcr.FP64, TOL), (mlcr.FP32, TOL32), (mlcr.BF16X3, TOLB3)]:
        f = mlcr.sht_synth(g, dev(x), prec=prec)
        got = {k: host(f[:, geo.start[k]: geo.start[k] + geo.nphi[k]]) for k in rings}
        del f
        allg = np.concatenate([got[k] for k in rings], axis=1)
        allr = np.concatenate([ref[k] for k in rings], axis=1)
        print(f"prec {prec}: sampled rings rel {_rel(allg, allr):.2e}, per ring "
              + ", ".join(f"{_rel(got[k], ref[k]):.2e}" for k in rings), flush=True)
        assert _rel(allg, allr) <= tol, (prec, _rel(allg, allr))
        for k in rings:
            assert _rel(got[k], ref[k]) <= 4 * tol, (prec, k, _rel(got[k], ref[k]))


def test_c5_adjoint_sampled_orders(mlcr, c5):
    cfg, d, g, x = c5
    print("case c5 adjoint, 8 RHS, sampled orders", flush=True)
    y = np.random.default_rng(77).standard_normal((R, cfg.npix))
    orders = [0, 1, 2048, 4096]
    ref = osht.adjoint_orders(y, cfg.lmax, cfg.nside, orders)
    for prec, tol in [(mlcr.FP64, TOL), (mlcr.FP32, TOL32), (mlcr.BF16X3, TOLB3)]:
        a = mlcr.sht_adjoint(g, dev(y), prec=prec)
        got, want = [], []
        for m in orders:
            c, s = ref[m]
            if m == 0:
                got.append(host(a[:, : cfg.lmax + 1]))
                want.append(c)
                continue
            b = osht.block_base(m, cfg.lmax)
            n = cfg.lmax - m + 1
            got += [host(a[:, b: b + n]), host(a[:, b + n: b + 2 * n])]
            want += [c, s]
        del a
        per = [_rel(u, v) for u, v in zip(got, want)]
        tot = _rel(np.concatenate(got, axis=1), np.concatenate(want, axis=1))
        print(f"prec {prec}: sampled orders rel {tot:.2e}, per block "
              + ", ".join(f"{p:.2e}" for p in per), flush=True)
        # bar over the sampled output as a whole; the m = lmax blocks hold a
        # single coefficient each, so blocks get 4x slack
        assert tot <= tol, (prec, tot)
        assert max(per) <= 4 * tol, (prec, per)


def test_c5_apply_properties(mlcr, c5):
    cfg, d, g, x = c5
    print("case c5 apply_A properties, 8 RHS", flush=True)
    ninv = dev(d["ninv"])
    op = mlcr.Operator(g, d["cl"], d["bl"], ninv, max_nrhs=R)
    u = dev(x)
    v = dev(np.stack([workloads.prior_sample(cfg, R + r) for r in range(R)]))
    Au = mlcr.apply_A(op, u)
    Av = mlcr.apply_A(op, v)
    # symmetry, per RHS
    lhs = (u * Av).sum(dim=1)
    rhs = (Au * v).sum(dim=1)
    assert float(((lhs - rhs).abs() / lhs.abs()).max()) <= 1e-12
    # the fused ring step equals synthesis -> N^-1 -> adjoint, plus the prior
    L = workloads.packed_ell(cfg.lmax)
    bl = dev(d["bl"][L])
    sinv = dev(np.where(d["cl"][L] > 0, 1.0 / np.where(d["cl"][L] > 0, d["cl"][L], 1.0), 0.0))
    mp = mlcr.sht_synth(g, bl * u)
    comp = sinv * u + bl * mlcr.sht_adjoint(g, mp * ninv)
    del mp
    assert float((comp - Au).norm() / Au.norm()) <= 1e-12
    # float32 contraction within its rounding bound of the float64 path
    Au32 = mlcr.apply_A(op, u, prec=mlcr.FP32)
    assert float((Au32 - Au).norm() / Au.norm()) <= TOL32
    Aub3 = mlcr.apply_A(op, u, prec=mlcr.BF16X3)
    print(f"apply rel vs float64: fp32 {float((Au32 - Au).norm() / Au.norm()):.2e}, "
          f"bf16x3 {float((Aub3 - Au).norm() / Au.norm()):.2e}", flush=True)
    assert float((Aub3 - Au).norm() / Au.norm()) <= TOLB3


@pytest.mark.parametrize("prec_name", ["fp64", "fp32", "bf16x3"])
def test_c3_solve_to_1e3_uK(mlcr, prec_name):
    """W-cycles reach 1e-3 uK max pixel error on a manufactured solution at
    N_side 1024 / lmax 2048; fp32 runs the cycle's transforms in float32 with
    the float64 residual and update (iterative refinement)."""
    cfg = workloads.get_config("c3")
    d = workloads.workload_inputs(cfg)
    print(f"case c3 solve {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}[prec_name]
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=1)
    S = mlcr.Solver(op, max_nrhs=1)
    xt = dev(workloads.prior_sample(cfg, 0)[None])
    b = mlcr.apply_A(op, xt)
    torch.cuda.synchronize()
    t0 = time.time()
    x, info = S.solve(b, rtol=1e-7, max_cycles=20, prec=prec)
    torch.cuda.synchronize()
    dt = time.time() - t0
    err = float(mlcr.sht_synth(g, x - xt).abs().max())
    print(f"c3 {prec_name}: {info[0]['cycles']} cycles, {dt:.2f} s, max pixel error {err:.3e} uK",
          flush=True)
    assert info[0]["converged"] == 1
    assert err <= 1e-3


@pytest.mark.parametrize("nrhs", [1, 2])
def test_adjoint_ignores_stale_workspace(mlcr, nrhs):
    """Regression: the vector adjoint's split-K chunks each store their
    partial sums; no chunk may be left empty (its slice would be stale when a
    larger transform used the workspace before).  N_side 300 / lmax 2048 has 5
    ring-pair blocks, the shape that once produced an empty chunk."""
    print(f"case stale workspace nrhs={nrhs}", flush=True)
    nside, lmax = 300, 2048
    g = mlcr.Geometry(nside, lmax)
    y = dev(np.random.default_rng(88).standard_normal((nrhs, 12 * nside * nside)))
    a1 = mlcr.sht_adjoint(g, y).clone()
    big = dev(np.random.default_rng(89).standard_normal((16, 12 * nside * nside)))
    mlcr.sht_adjoint(g, big)                 # fills the workspaces with other data
    del big
    a2 = mlcr.sht_adjoint(g, y)
    assert torch.equal(a1, a2)
    # and against the oracle on a few whole orders
    ref = osht.adjoint_orders(host(y), lmax, nside, [0, 700, 2048])
    got = [host(a2[:, : lmax + 1])]
    want = [ref[0][0]]
    for m in (700, 2048):
        b = osht.block_base(m, lmax)
        n = lmax - m + 1
        got += [host(a2[:, b: b + n]), host(a2[:, b + n: b + 2 * n])]
        want += [ref[m][0], ref[m][1]]
    assert _rel(np.concatenate(got, axis=1), np.concatenate(want, axis=1)) <= TOL
