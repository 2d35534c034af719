"""Batched right-hand sides (independent realizations, Sec. 2.3) through one
launch, against the oracle.

* Wide batches at N_side 256 / lmax 512: 61 RHS (a ragged last chunk of 5)
  and 64 RHS, synthesis and adjoint in all three precisions vs the oracle's
  whole transforms.
* A grid whose ring-pair blocks do not fill the adjoint's last workgroup
  (N_side 300: 600 ring pairs, 10 blocks of 64, so the second 8-wave chunk has
  6 idle waves), with 9 and 16 RHS, in all three precisions.
* The batching workload at N_side 1024 / lmax 2048 with 32 RHS in one launch:
  synthesis on sampled rings and adjoint on sampled orders vs the oracle, and
  a batched W-cycle solve of manufactured right-hand sides to 1e-3 uK in
  bf16x3 with float64 refinement.
* The mixed batch of 8 independent problems (3 x N_side 256 / lmax 512,
  3 x 512 / 1024, 2 x 1024 / 2048): the grouped solve equals the single
  solves bit for bit and every problem converges.
Every parity bar applies to the relative 2-norm and to the per-element
max |y - y_ref| / max |y_ref|.
"""
import time

import numpy as np
import pytest
import torch

import workloads
from oracle import sht as osht
from tests.gpu_util import check, dev, host, parity

pytestmark = pytest.mark.gpu

TOLS = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


def _precs(mlcr):
    return {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}


@pytest.mark.parametrize("nside,lmax,nrhs", [(256, 512, 61), (256, 512, 64), (300, 600, 9),
                                             (300, 600, 16)])
def test_wide_and_ragged_batches(mlcr, nside, lmax, nrhs):
    print(f"case batch nside={nside} lmax={lmax} nrhs={nrhs}", flush=True)
    g = mlcr.Geometry(nside, lmax)
    rng = np.random.default_rng(1300 + nrhs + nside)
    x = rng.standard_normal((nrhs, osht.nalm(lmax)))
    y = rng.standard_normal((nrhs, 12 * nside * nside))
    t0 = time.time()
    fr = osht.synth(x, lmax, nside)
    ar = osht.adjoint(y, lmax, nside)
    print(f"oracle in {time.time() - t0:.1f}s", flush=True)
    for name, prec in _precs(mlcr).items():
        f = host(mlcr.sht_synth(g, dev(x), prec=prec))
        a = host(mlcr.sht_adjoint(g, dev(y), prec=prec))
        fp64 = name == "fp64"
        okf, ef = check(f, fr, TOLS[name], lmax, fp64)
        oka, ea = check(a, ar, TOLS[name], lmax, fp64)
        # each RHS on its own too: a wrong column block cannot hide in the batch
        wf = max(parity(f[r], fr[r]) for r in range(nrhs))
        wa = max(parity(a[r], ar[r]) for r in range(nrhs))
        print(f"{name}: synth {ef} (worst RHS {wf:.2e}), adjoint {ea} (worst RHS {wa:.2e})",
              flush=True)
        assert okf and oka, (name, ef, ea)
        for r in range(nrhs):
            assert check(f[r], fr[r], TOLS[name], lmax, fp64, slack=2.0)[0], (name, r)
            assert check(a[r], ar[r], TOLS[name], lmax, fp64, slack=2.0)[0], (name, r)
    # the 4-wave adjoint shape: from 16 RHS on, the split-bfloat16 adjoint
    # feeds each lambda tile to two column blocks
    g.set_tuning(mlcr.BF16X3, 4, 4, 1024)
    a4 = host(mlcr.sht_adjoint(g, dev(y), prec=mlcr.BF16X3))
    ok4, e4 = check(a4, ar, TOLS["bf16x3"])
    print(f"bf16x3 adjoint, 4-wave shape: {e4}", flush=True)
    assert ok4, e4
    for r in range(nrhs):
        assert check(a4[r], ar[r], TOLS["bf16x3"], slack=2.0)[0], r


@pytest.fixture(scope="module")
def c4(mlcr):
    cfg = workloads.get_config("c4")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    x = np.stack([workloads.prior_sample(cfg, r) for r in range(cfg.nrhs)])
    return cfg, d, g, x


def test_c4_32_rhs_sampled_parity(mlcr, c4):
    cfg, d, g, x = c4
    R = cfg.nrhs
    print(f"case c4 {R} RHS sampled parity", flush=True)
    geo = osht.healpix_rings(cfg.nside)
    rings = [0, 150, 511, 700, 1023, 2047, 3500, 4094]
    orders = [0, 1, 8, 15, 333, 1024, 1999, 2048]
    y = np.random.default_rng(91).standard_normal((R, cfg.npix))
    t0 = time.time()
    fr = osht.synth_rings(x, cfg.lmax, cfg.nside, rings)
    ar = osht.adjoint_orders(y, cfg.lmax, cfg.nside, orders)
    print(f"oracle samples in {time.time() - t0:.1f}s", flush=True)
    allr = np.concatenate([fr[k] for k in rings], axis=1)
    for name, prec in _precs(mlcr).items():
        f = mlcr.sht_synth(g, dev(x), prec=prec)
        allg = np.concatenate([host(f[:, geo.start[k]: geo.start[k] + geo.nphi[k]]) for k in rings],
                              axis=1)
        del f
        a = mlcr.sht_adjoint(g, dev(y), prec=prec)
        got, want = [host(a[:, : cfg.lmax + 1])], [ar[0][0]]
        for m in orders[1:]:
            b = osht.block_base(m, cfg.lmax)
            n = cfg.lmax - m + 1
            got += [host(a[:, b: b + n]), host(a[:, b + n: b + 2 * n])]
            want += [ar[m][0], ar[m][1]]
        del a
        oks, es = check(allg, allr, TOLS[name], cfg.lmax, name == "fp64")
        oka, ea = check(np.concatenate(got, axis=1), np.concatenate(want, axis=1), TOLS[name],
                        cfg.lmax, name == "fp64")
        print(f"{name}: sampled rings {es}, sampled orders {ea}", flush=True)
        assert oks and oka, (name, es, ea)


@pytest.mark.timeout(600)
def test_c4_batched_solve(mlcr, c4):
    """32 manufactured right-hand sides solved together in bf16x3 with float64
    refinement to 1e-3 uK (float64 synthesis over all pixels, and the oracle
    on sampled rings), and the batched solve equals the solve of a 5-RHS
    slice up to the cycle's rounding (the RHS are independent)."""
    cfg, d, g, xt = c4
    R = cfg.nrhs
    print(f"case c4 batched solve, {R} RHS, bf16x3", flush=True)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=R)
    S = mlcr.Solver(op, max_nrhs=R)
    xtd = dev(xt)
    b = mlcr.apply_A(op, xtd)
    torch.cuda.synchronize()
    t0 = time.time()
    x, info = S.solve(b, rtol=0.0, max_cycles=9, prec=mlcr.BF16X3, raise_on_noconv=False)
    torch.cuda.synchronize()
    dt = time.time() - t0
    e = float(mlcr.sht_synth(g, x - xtd).abs().max())
    print(f"c4 bf16x3 {R} RHS: 9 cycles {dt:.2f} s, max pixel error {e:.3e} uK", flush=True)
    assert e <= 1e-3
    rings = [0, 700, 2047, 4094]
    err = host(x) - xt
    ref = osht.synth_rings(err, cfg.lmax, cfg.nside, rings)
    eo = max(float(np.abs(ref[k]).max()) for k in rings)
    print(f"oracle-sampled rings: {eo:.3e} uK", flush=True)
    assert eo <= 1e-3
    x5, _ = S.solve(b[3:8].contiguous(), rtol=0.0, max_cycles=9, prec=mlcr.BF16X3,
                    raise_on_noconv=False)
    assert parity(host(x5), host(x[3:8])) <= 1e-9


@pytest.mark.timeout(600)
def test_mixed_batch_grouped_solve(mlcr):
    """The batching workload's mixed batch: 8 independent problems with their
    own grids and band limits, solved by one grouped call; results equal the
    single solves bit for bit, every problem converges."""
    print(f"case mixed batch {workloads.MIXED_BATCH}", flush=True)
    grids, probs = {}, []
    for k, name in enumerate(workloads.MIXED_BATCH):
        cfg = workloads.get_config(name)
        if name not in grids:
            d = workloads.workload_inputs(cfg)
            g = mlcr.Geometry(cfg.nside, cfg.lmax)
            grids[name] = (g, mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=1))
        g, op = grids[name]
        S = mlcr.Solver(op, max_nrhs=1)
        xt = dev(workloads.prior_sample(cfg, k)[None])
        probs.append((name, S, mlcr.apply_A(op, xt)))
    for prec_name in ["fp64", "bf16x3"]:
        prec = _precs(mlcr)[prec_name]
        single = [S.solve(b, rtol=1e-8, max_cycles=40, prec=prec) for _, S, b in probs]
        torch.cuda.synchronize()
        xs, infos = mlcr.solve_grouped([S for _, S, _ in probs], [b for _, _, b in probs], rtol=1e-8,
                                       max_cycles=40, prec=prec)
        torch.cuda.synchronize()
        print(prec_name, [i[0]["cycles"] for i in infos], flush=True)
        for (name, _, _), (x1, i1), x2, i2 in zip(probs, single, xs, infos):
            assert torch.equal(x1, x2), name
            assert i1 == i2
            assert i2[0]["converged"] == 1, name
