"""Grouped entry points for a mixed batch (independent problems with their
own grids and band limits, run concurrently on library streams).

The grouped calls must return exactly what the single calls return: the
problems share no arithmetic, so the results are compared bit for bit, for
a batch that includes two problems on one grid (serialized on one stream)
and RHS counts that are not multiples of 8.
"""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def batch(mlcr):
    out = []
    grids = {}
    for name, nrhs in [("c1", 1), ("c2", 3), ("c2", 1), ("m512", 2)]:
        cfg = workloads.get_config(name)
        d = workloads.workload_inputs(cfg)
        if name not in grids:
            grids[name] = (mlcr.Geometry(cfg.nside, cfg.lmax), dev(d["ninv"]))
        g, ninv = grids[name]
        op = mlcr.Operator(g, d["cl"], d["bl"], ninv, max_nrhs=nrhs)
        x = dev(np.stack([workloads.prior_sample(cfg, 10 + r) for r in range(nrhs)]))
        out.append((cfg, op, x))
    return out, grids


@pytest.mark.parametrize("prec_name", ["fp64", "bf16x3"])
def test_apply_grouped_equals_single(mlcr, batch, prec_name):
    print(f"case grouped apply {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "bf16x3": mlcr.BF16X3}[prec_name]
    probs, _ = batch
    single = [mlcr.apply_A(op, x, prec=prec) for _, op, x in probs]
    torch.cuda.synchronize()
    grouped = mlcr.apply_A_grouped([op for _, op, _ in probs], [x for _, _, x in probs], prec=prec)
    torch.cuda.synchronize()
    for (cfg, _, _), a, b in zip(probs, single, grouped):
        assert torch.equal(a, b), cfg.name


def test_solve_grouped_equals_single(mlcr, batch):
    print("case grouped solve", flush=True)
    probs, _ = batch
    solvers, bs = [], []
    for cfg, op, x in probs:
        solvers.append(mlcr.Solver(op, max_nrhs=x.shape[0]))
        bs.append(mlcr.apply_A(op, x))
    single = [S.solve(b, rtol=1e-8, max_cycles=40) for S, b in zip(solvers, bs)]
    torch.cuda.synchronize()
    xs, infos = mlcr.solve_grouped(solvers, bs, rtol=1e-8, max_cycles=40)
    torch.cuda.synchronize()
    for (cfg, _, _), (xs1, inf1), x2, inf2 in zip(probs, single, xs, infos):
        print(cfg.name, [i["cycles"] for i in inf2], [f"{i['rho']:.2e}" for i in inf2], flush=True)
        assert torch.equal(xs1, x2), cfg.name
        assert inf1 == inf2
        assert all(i["converged"] == 1 for i in inf2)


def test_grouped_errors(mlcr, batch):
    from paper_1308_5299_amd import MLCRError
    probs, _ = batch
    cfg, op, x = probs[1]
    S = mlcr.Solver(op, max_nrhs=x.shape[0])
    b = mlcr.apply_A(op, x)
    with pytest.raises(MLCRError):
        mlcr.solve_grouped([S, S], [b, b])                 # one solver twice
    with pytest.raises(ValueError):
        mlcr.apply_A_grouped([op], [x, x])                 # lengths differ
    with pytest.raises(ValueError):
        mlcr.apply_A_grouped([op], [torch.cat([x, x, x])])  # nrhs above max_nrhs
