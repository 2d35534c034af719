"""Gauss-Legendre grids on the GPU (Sec. 3.4).

* transforms on a Gauss-Legendre geometry against the oracle's transforms on
  its own Gauss-Legendre rings (power-of-two and Bluestein ring lengths);
* quadrature weights against the oracle's;
* a level operator whose Y^T N^-1 Y runs on a Gauss-Legendre grid with the
  downgraded N^-1 against the oracle's level operator on the observation
  grid: the identity is exact, so the bar is the float64 one, 1e-12.
"""
import numpy as np
import pytest

import workloads
from oracle import geometry as ogeo
from oracle import operator as oop
from oracle import sht as osht
from tests.gpu_util import dev, host, parity

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


@pytest.mark.parametrize("lmax,nrings,nphi,nrhs", [(0, 1, 4, 1), (12, 25, 52, 2), (64, 129, 256, 3),
                                                   (100, 201, 404, 5), (100, 201, 512, 9)])
def test_gl_transforms_parity(mlcr, lmax, nrings, nphi, nrhs):
    print(f"case gl lmax={lmax} nrings={nrings} nphi={nphi} nrhs={nrhs}", flush=True)
    g = mlcr.Geometry.gauss_legendre(lmax, nrings, nphi)
    og, W = ogeo.gauss_legendre_rings(nrings, nphi)
    np.testing.assert_allclose(g.weights(), W, rtol=1e-15, atol=0)
    rng = np.random.default_rng(300 + lmax + nphi)
    x = rng.standard_normal((nrhs, osht.nalm(lmax)))
    y = rng.standard_normal((nrhs, nrings * nphi))
    f = host(mlcr.sht_synth(g, dev(x)))
    a = host(mlcr.sht_adjoint(g, dev(y)))
    assert parity(f, osht.synth_geom(x, lmax, og)) <= TOL
    assert parity(a, osht.adjoint_geom(y, lmax, og)) <= TOL


@pytest.mark.parametrize("name,lmax_h", [("c1", 12), ("c2", 192)])
def test_gl_level_operator_parity(mlcr, name, lmax_h):
    """A_h with Y^T N^-1 Y on the Gauss-Legendre grid equals the oracle's A_h
    on the observation grid (Sec. 3.4, eqs. Ni-rewrite and Xi)."""
    print(f"case gl level {name} lmax_h={lmax_h}", flush=True)
    cfg = workloads.get_config(name)
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=2)
    ell = np.arange(lmax_h + 1)
    f = np.exp(-0.5 * ell * (ell + 1) * (2.5 / lmax_h) ** 2)
    op.set_level_gl(1, lmax_h, f)
    x = np.random.default_rng(31).standard_normal((2, osht.nalm(lmax_h)))
    y = host(mlcr.apply_A(op, dev(x), level=1))
    yr = oop.apply_A(x, d["cl"], d["bl"], d["ninv"], cfg.nside, lmax_h=lmax_h, fl=f)
    assert parity(y, yr) <= TOL, parity(y, yr)
    # the same level on the observation grid agrees too (returns the level to it)
    op.set_level(1, lmax_h, f)
    y2 = host(mlcr.apply_A(op, dev(x), level=1))
    assert parity(y2, yr) <= TOL


def test_gl_errors(mlcr):
    from paper_1308_5299_amd import MLCRError
    cfg = workloads.get_config("c1")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=1)
    with pytest.raises(MLCRError):
        op.set_level_gl(1, cfg.lmax // 2 + 1, np.ones(cfg.lmax))     # 2 lmax_h > lmax
    with pytest.raises(MLCRError):
        mlcr.Geometry.gauss_legendre(10, 11, 30)                       # nphi not a multiple of 4
