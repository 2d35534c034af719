"""W-cycle solves with the cycle replayed from a captured HIP graph.

Graph mode runs cycle 1 directly, captures cycle 2 and replays it for the
later cycles, with the host reading the residual norms back (a stream
synchronization) between replays.  Every replay must do exactly what the
direct launches do, so the graph-mode solutions are compared bit for bit
with direct-launch solutions: float64 and bf16x3 cycles, two calls in a row
with different RHS counts, a dense-only solver, and a grouped solve.
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


def _problem(mlcr, name, nrhs):
    cfg = workloads.get_config(name)
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    ninv = dev(d["ninv"])
    op = mlcr.Operator(g, d["cl"], d["bl"], ninv, max_nrhs=nrhs)
    x = dev(np.stack([workloads.prior_sample(cfg, 20 + r) for r in range(nrhs)]))
    return cfg, (g, ninv), op, mlcr.apply_A(op, x)


@pytest.mark.parametrize("prec_name", ["fp64", "bf16x3"])
def test_graph_solve_equals_direct(mlcr, prec_name):
    print(f"case graph solve c2 {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "bf16x3": mlcr.BF16X3}[prec_name]
    cfg, keep, op, b = _problem(mlcr, "c2", 2)
    S = mlcr.Solver(op, max_nrhs=2)
    for rhs in (b, b[:1].contiguous()):
        S.set_graph(False)
        x1, i1 = S.solve(rhs, rtol=1e-9, max_cycles=30, prec=prec)
        S.set_graph(True)
        x2, i2 = S.solve(rhs, rtol=1e-9, max_cycles=30, prec=prec)
        torch.cuda.synchronize()
        st = S.graph_stats()
        print(rhs.shape[0], "RHS, cycles", [i["cycles"] for i in i2], st, flush=True)
        assert all(i["cycles"] >= 3 for i in i2)
        assert st["fallbacks"] == 0 and st["replays"] >= 1
        assert torch.equal(x1, x2)
        assert i1 == i2


def test_graph_dense_only_and_grouped(mlcr):
    print("case graph dense c1 and grouped", flush=True)
    cfg1, keep1, op1, b1 = _problem(mlcr, "c1", 1)
    S1 = mlcr.Solver(op1, max_nrhs=1)
    x1, _ = S1.solve(b1, rtol=1e-12, max_cycles=4)
    S1.set_graph(True)
    x2, _ = S1.solve(b1, rtol=1e-12, max_cycles=4)
    assert torch.equal(x1, x2)
    cfg2, keep2, op2, b2 = _problem(mlcr, "c2", 1)
    cfg3, keep3, op3, b3 = _problem(mlcr, "m512", 1)
    solvers = [mlcr.Solver(op2, max_nrhs=1), mlcr.Solver(op2, max_nrhs=1), mlcr.Solver(op3, max_nrhs=1)]
    bs = [b2, 2.0 * b2, b3]
    xs_d, inf_d = mlcr.solve_grouped(solvers, bs, rtol=1e-8, max_cycles=30)
    for S in solvers:
        S.set_graph(True)
    xs_g, inf_g = mlcr.solve_grouped(solvers, bs, rtol=1e-8, max_cycles=30)
    torch.cuda.synchronize()
    for a, c in zip(xs_d, xs_g):
        assert torch.equal(a, c)
    assert inf_d == inf_g
    for S in solvers:
        st = S.graph_stats()
        assert st["fallbacks"] == 0 and st["replays"] >= 1, st
