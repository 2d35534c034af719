"""GPU parity of the float64 transforms and operator against the oracle.

Bar (FP64 path): ||y - y_oracle||_2 / ||y_oracle||_2 <= 1e-12 and
max |y - y_oracle| / max |y_oracle| <= 1e-12, computed on the same seeded
inputs.  Cases span several Legendre tiles and FFT length
classes with ragged tails: power-of-two and Bluestein rings, lmax above the
grid's Nyquist (m folded modulo ring length), tiny grids and lmax = 0.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import operator as oop
from oracle import sht as osht
from tests.gpu_util import dev, host, maxrel, parity, rel2

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = [(1, 0), (1, 3), (2, 5), (4, 12), (4, 30), (8, 16), (8, 40), (16, 32), (32, 100),
         (64, 128), (128, 200), (256, 512)]


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


@pytest.mark.parametrize("nside,lmax", CASES)
def test_synth_adjoint_parity(mlcr, nside, lmax):
    print(f"case nside={nside} lmax={lmax}", flush=True)
    g = mlcr.Geometry(nside, lmax)
    rng = np.random.default_rng(1000 * nside + lmax)
    x = rng.standard_normal((2, osht.nalm(lmax)))
    y = rng.standard_normal((2, 12 * nside * nside))
    f = host(mlcr.sht_synth(g, dev(x)))
    a = host(mlcr.sht_adjoint(g, dev(y)))
    fr = osht.synth(x, lmax, nside)
    ar = osht.adjoint(y, lmax, nside)
    assert parity(f, fr) <= TOL, parity(f, fr)
    assert parity(a, ar) <= TOL, parity(a, ar)


def test_batch_equals_singles(mlcr):
    nside, lmax = 32, 80
    g = mlcr.Geometry(nside, lmax)
    x = np.random.default_rng(3).standard_normal((5, osht.nalm(lmax)))
    fb = host(mlcr.sht_synth(g, dev(x)))
    # 5 RHS run on the float64 matrix cores, a single RHS on the vector
    # kernels: same sums, different rounding order (a few units in the last
    # place of the largest value per element, ~1e-14 in the 2-norm)
    for r in range(5):
        fs = host(mlcr.sht_synth(g, dev(x[r:r + 1])))
        assert rel2(fb[r:r + 1], fs) <= 1e-14 and maxrel(fb[r:r + 1], fs) <= 1e-13
    yb = host(mlcr.sht_adjoint(g, dev(fb)))
    for r in range(5):
        ys = host(mlcr.sht_adjoint(g, dev(fb[r:r + 1])))
        assert rel2(yb[r:r + 1], ys) <= 1e-14 and maxrel(yb[r:r + 1], ys) <= 1e-13


def test_smaller_lmax_than_geometry(mlcr):
    nside, lmax_g, lmax = 16, 40, 23
    g = mlcr.Geometry(nside, lmax_g)
    x = np.random.default_rng(4).standard_normal((1, osht.nalm(lmax)))
    f = host(mlcr.sht_synth(g, dev(x), lmax=lmax))
    assert parity(f, osht.synth(x, lmax, nside)) <= TOL
    a = host(mlcr.sht_adjoint(g, dev(f), lmax=lmax))
    assert parity(a, osht.adjoint(f, lmax, nside)) <= TOL


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_apply_A_parity(mlcr, name):
    cfg = workloads.get_config(name)
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=2)
    x = np.stack([workloads.prior_sample(cfg, r) for r in range(2)])
    y = host(mlcr.apply_A(op, dev(x)))
    yr = oop.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside)
    assert parity(y, yr) <= TOL, parity(y, yr)
    L = oop.mode_ell(cfg.lmax)
    assert np.all(y[:, d["cl"][L] == 0] == 0.0)


@pytest.mark.parametrize("nside,lmax,nrhs", [(1, 3, 4), (4, 12, 4), (16, 32, 9), (32, 100, 8),
                                             (64, 128, 16), (256, 512, 8)])
def test_fp64_mfma_parity(mlcr, nside, lmax, nrhs):
    """Batches of >= 4 RHS take the float64 matrix-core kernels (16 columns =
    8 RHS x cos/sin per wave, ragged last chunk); same 1e-12 bar."""
    print(f"case fp64 mfma nside={nside} lmax={lmax} nrhs={nrhs}", flush=True)
    g = mlcr.Geometry(nside, lmax)
    rng = np.random.default_rng(700 + lmax + nrhs)
    x = rng.standard_normal((nrhs, osht.nalm(lmax)))
    y = rng.standard_normal((nrhs, 12 * nside * nside))
    f = host(mlcr.sht_synth(g, dev(x)))
    a = host(mlcr.sht_adjoint(g, dev(y)))
    assert parity(f, osht.synth(x, lmax, nside)) <= TOL, parity(f, osht.synth(x, lmax, nside))
    assert parity(a, osht.adjoint(y, lmax, nside)) <= TOL, parity(a, osht.adjoint(y, lmax, nside))


def test_fp64_mfma_apply_parity(mlcr):
    cfg = workloads.get_config("c2")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=8)
    x = np.stack([workloads.prior_sample(cfg, r) for r in range(8)])
    y = host(mlcr.apply_A(op, dev(x)))
    yr = oop.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside)
    assert parity(y, yr) <= TOL, parity(y, yr)


def test_level_operator_parity(mlcr):
    cfg = workloads.get_config("c1")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=1)
    lmax_h = 24
    f = np.exp(-((np.arange(lmax_h + 1) / 15.0) ** 4))
    op.set_level(1, lmax_h, f)
    x = np.random.default_rng(6).standard_normal((1, osht.nalm(lmax_h)))
    y = host(mlcr.apply_A(op, dev(x), level=1))
    yr = oop.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside, lmax_h=lmax_h, fl=f)
    assert parity(y, yr) <= TOL


def test_errors(mlcr):
    from paper_1308_5299_amd import MLCRError
    g = mlcr.Geometry(4, 8)
    with pytest.raises(MLCRError):
        mlcr.sht_synth(g, dev(np.zeros(100)), lmax=9)      # above the geometry's lmax
    with pytest.raises(MLCRError):
        mlcr.sht_synth(g, dev(np.zeros(81)), prec=7)
    with pytest.raises(ValueError):
        mlcr.sht_synth(g, dev(np.zeros(80)))                # not a whole vector


def test_empty_batch_rejected(mlcr):
    """nrhs = 0 is outside every entry point's range (nrhs >= 1): MLCR_EINVAL
    through the C ABI, nothing launched."""
    import ctypes
    from paper_1308_5299_amd import _lib
    lib = _lib.load()
    g = mlcr.Geometry(4, 8)
    buf = dev(np.zeros(12 * 16 + 81))
    p = ctypes.c_void_p(buf.data_ptr())
    for prec in (mlcr.FP64, mlcr.FP32, mlcr.BF16X3):
        assert lib.sht_synth(g.handle, 8, 0, p, p, prec, None) == -1
        assert lib.sht_adjoint(g.handle, 8, 0, p, p, prec, None) == -1
    op = mlcr.Operator(g, np.ones(9), np.ones(9), dev(np.ones(12 * 16)), max_nrhs=2)
    assert lib.apply_A(op.handle, 0, 0, p, p, mlcr.FP64, None) == -1
    assert lib.apply_A(op.handle, 0, 3, p, p, mlcr.FP64, None) == -1        # above max_nrhs


@pytest.mark.parametrize("prec_name", ["fp64", "fp32", "bf16x3"])
def test_apply_without_data_is_the_prior(mlcr, prec_name):
    """N^-1 = 0 everywhere (a fully masked sky, Sec. 2.3): A = S^-1, so the
    apply returns x / C_l whatever the transform arithmetic (v is exactly 0)."""
    prec = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}[prec_name]
    nside, lmax = 32, 64
    rng = np.random.default_rng(77)
    cl = rng.uniform(0.5, 2.0, lmax + 1)
    bl = rng.uniform(0.2, 1.0, lmax + 1)
    g = mlcr.Geometry(nside, lmax)
    op = mlcr.Operator(g, cl, bl, dev(np.zeros(12 * nside * nside)), max_nrhs=9)
    x = rng.standard_normal((9, osht.nalm(lmax)))
    y = host(mlcr.apply_A(op, dev(x), prec=prec))
    L, _, _ = osht.packed_index(lmax)
    want = x / cl[L]
    assert np.max(np.abs(y - want) / np.abs(want)) <= 4e-16


# Float32 contraction on the matrix cores: lambda and the coefficients are
# rounded to float32 (2^-24) and summed in float32 over <= lmax + 1 terms,
# so the relative 2-norm error is ~ 2^-24 sqrt(lmax); 2e-5 covers lmax 512.
TOL32 = 2e-5


@pytest.mark.parametrize("nside,lmax,nrhs", [(4, 12, 1), (16, 32, 3), (32, 100, 8), (64, 128, 9),
                                             (256, 512, 2)])
def test_fp32_synth_adjoint_parity(mlcr, nside, lmax, nrhs):
    print(f"case fp32 nside={nside} lmax={lmax} nrhs={nrhs}", flush=True)
    g = mlcr.Geometry(nside, lmax)
    rng = np.random.default_rng(500 + lmax)
    x = rng.standard_normal((nrhs, osht.nalm(lmax)))
    y = rng.standard_normal((nrhs, 12 * nside * nside))
    f = host(mlcr.sht_synth(g, dev(x), prec=mlcr.FP32))
    a = host(mlcr.sht_adjoint(g, dev(y), prec=mlcr.FP32))
    assert parity(f, osht.synth(x, lmax, nside)) <= TOL32, parity(f, osht.synth(x, lmax, nside))
    assert parity(a, osht.adjoint(y, lmax, nside)) <= TOL32, parity(a, osht.adjoint(y, lmax, nside))


def test_fp32_apply_parity(mlcr):
    cfg = workloads.get_config("c2")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=1)
    x = workloads.prior_sample(cfg, 0)[None, :]
    y = host(mlcr.apply_A(op, dev(x), prec=mlcr.FP32))
    yr = oop.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside)
    assert parity(y, yr) <= TOL32, parity(y, yr)


# Split-bfloat16 contraction: each float32 operand is carried as hi + lo
# bfloat16 to 2^-18 relative and the dropped lo*lo term is below 2^-18 of the
# product, so a product is good to 3 * 2^-18 = 1.1e-5; sums of terms of
# random sign keep that relative 2-norm error.  The bar is 9x that.
TOLB3 = 1e-4


@pytest.mark.parametrize("nside,lmax,nrhs", [(1, 3, 1), (4, 12, 1), (16, 32, 3), (32, 100, 8),
                                             (64, 128, 9), (256, 512, 2), (64, 255, 17)])
def test_bf16x3_synth_adjoint_parity(mlcr, nside, lmax, nrhs):
    print(f"case bf16x3 nside={nside} lmax={lmax} nrhs={nrhs}", flush=True)
    g = mlcr.Geometry(nside, lmax)
    rng = np.random.default_rng(700 + lmax)
    x = rng.standard_normal((nrhs, osht.nalm(lmax)))
    y = rng.standard_normal((nrhs, 12 * nside * nside))
    f = host(mlcr.sht_synth(g, dev(x), prec=mlcr.BF16X3))
    a = host(mlcr.sht_adjoint(g, dev(y), prec=mlcr.BF16X3))
    ef, ea = parity(f, osht.synth(x, lmax, nside)), parity(a, osht.adjoint(y, lmax, nside))
    print(f"bf16x3 synth rel {ef:.2e} adjoint rel {ea:.2e}", flush=True)
    assert ef <= TOLB3 and ea <= TOLB3, (ef, ea)


def test_bf16x3_apply_parity(mlcr):
    cfg = workloads.get_config("c2")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=1)
    x = workloads.prior_sample(cfg, 0)[None, :]
    y = host(mlcr.apply_A(op, dev(x), prec=mlcr.BF16X3))
    yr = oop.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside)
    print(f"bf16x3 apply rel {parity(y, yr):.2e}", flush=True)
    assert parity(y, yr) <= TOLB3, parity(y, yr)


@pytest.mark.parametrize("prec_name,nrhs,tol", [("fp64", 8, TOL), ("fp32", 3, TOL32),
                                                ("bf16x3", 9, TOLB3)])
def test_matrix_core_smaller_lmax_than_geometry(mlcr, prec_name, nrhs, tol):
    """The matrix-core kernels index their recurrence tables (alpha_lm, c_lm)
    by the geometry's band limit; a transform at a smaller band limit must
    match the oracle at that band limit."""
    print(f"case matrix-core lmax < geometry lmax {prec_name}", flush=True)
    prec = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}[prec_name]
    nside, lmax_g, lmax = 32, 100, 57
    g = mlcr.Geometry(nside, lmax_g)
    rng = np.random.default_rng(900 + nrhs)
    x = rng.standard_normal((nrhs, osht.nalm(lmax)))
    y = rng.standard_normal((nrhs, 12 * nside * nside))
    f = host(mlcr.sht_synth(g, dev(x), lmax=lmax, prec=prec))
    a = host(mlcr.sht_adjoint(g, dev(y), lmax=lmax, prec=prec))
    ef, ea = parity(f, osht.synth(x, lmax, nside)), parity(a, osht.adjoint(y, lmax, nside))
    assert ef <= tol and ea <= tol, (ef, ea)
