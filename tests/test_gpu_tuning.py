"""Launch shapes (mlcr_geom_set_tuning) and the autotuner on the GPU.

Every launch shape must give the default shape's result up to rounding
order: the adjoint's waves per workgroup change the split-K chunking (and so
the order of the float32 / float64 partial sums), the synthesis chains per
lane and the ring threads change only which thread computes what.  The
default shapes are pinned to the oracle by the parity tests; here each other
shape is compared with them, and with tolerances set by that rounding.
"""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu

DEFAULT = {"adjoint_waves": 8, "synth_chains": 4, "ring_threads": 1024}
OTHERS = [{"adjoint_waves": 4}, {"synth_chains": 2}, {"ring_threads": 512},
          {"adjoint_waves": 4, "synth_chains": 2, "ring_threads": 512}]
TOL = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 2e-5}


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


def _rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def test_set_get_and_errors(mlcr):
    print("case tuning set/get", flush=True)
    g = mlcr.Geometry(16, 32)
    for p in (mlcr.FP64, mlcr.FP32, mlcr.BF16X3):
        assert g.get_tuning(p) == DEFAULT
    g.set_tuning(mlcr.BF16X3, 4, 2, 512)
    assert g.get_tuning(mlcr.BF16X3) == {"adjoint_waves": 4, "synth_chains": 2, "ring_threads": 512}
    assert g.get_tuning(mlcr.FP32) == DEFAULT
    for bad in [(6, 4, 1024), (8, 3, 1024), (8, 4, 256), (0, 4, 1024)]:
        with pytest.raises(mlcr.MLCRError):
            g.set_tuning(mlcr.FP32, *bad)
    with pytest.raises(mlcr.MLCRError):
        g.set_tuning(7, 8, 4, 1024)
    assert g.get_tuning(mlcr.FP32) == DEFAULT


@pytest.mark.parametrize("prec_name", ["fp64", "fp32", "bf16x3"])
def test_apply_agrees_under_every_shape(mlcr, prec_name):
    # N_side 256: 8 ring-pair blocks, so 4 waves per adjoint workgroup
    # changes the chunking
    print(f"case tuning apply {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}[prec_name]
    cfg = workloads.get_config("c2")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=8)
    x = dev(np.stack([workloads.prior_sample(cfg, 30 + r) for r in range(8)]))
    y0 = mlcr.apply_A(op, x, prec=prec)
    for change in OTHERS:
        t = dict(DEFAULT, **change)
        g.set_tuning(prec, **t)
        y = mlcr.apply_A(op, x, prec=prec)
        torch.cuda.synchronize()
        assert _rel(y, y0) <= TOL[prec_name], (change, _rel(y, y0))
    g.set_tuning(prec, **DEFAULT)
    assert torch.equal(mlcr.apply_A(op, x, prec=prec), y0)


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_ring_threads_on_the_largest_ffts(mlcr, prec_name):
    # FFT sizes above 4096 occur at N_side 2048; a small lmax keeps the
    # Legendre part cheap
    print(f"case tuning ring threads {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "fp32": mlcr.FP32}[prec_name]
    nside, lmax = 2048, 256
    g = mlcr.Geometry(nside, lmax)
    gen = torch.Generator(device="cuda").manual_seed(5)
    ninv = torch.rand(12 * nside * nside, dtype=torch.float64, device="cuda", generator=gen)
    op = mlcr.Operator(g, np.ones(lmax + 1), np.ones(lmax + 1), ninv, max_nrhs=8)
    x = torch.randn(8, (lmax + 1) ** 2, dtype=torch.float64, device="cuda", generator=gen)
    y0 = mlcr.apply_A(op, x, prec=prec)
    g.set_tuning(prec, **dict(DEFAULT, ring_threads=512))
    y = mlcr.apply_A(op, x, prec=prec)
    torch.cuda.synchronize()
    assert _rel(y, y0) <= TOL[prec_name]


def test_autotune_chooses_and_caches(mlcr, tmp_path):
    print("case autotune", flush=True)
    from paper_1308_5299_amd import autotune
    cfg = workloads.get_config("c2")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=8)
    path = str(tmp_path / "tune.json")
    r = autotune.tune(op, 8, mlcr.BF16X3, reps=2, cache_path=path)
    assert not r["cached"] and autotune.valid(r["tuning"])
    assert g.get_tuning(mlcr.BF16X3) == r["tuning"]
    assert set(r["timings_ms"]) == set(autotune.CANDIDATES)
    g.set_tuning(mlcr.BF16X3, **DEFAULT)
    r2 = autotune.tune(op, 8, mlcr.BF16X3, cache_path=path)
    assert r2["cached"] and r2["tuning"] == r["tuning"]
    assert g.get_tuning(mlcr.BF16X3) == r["tuning"]
