"""sht_synth_noalloc: the synthesis for callers that cannot allocate device
memory, through the C ABI, against the allocating sht_synth (float64 path)
on two calls in a row, the second with a smaller input, and the size limit.
"""
import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_util import dev, host, check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


def _noalloc(mlcr, g, lmax, alm):
    from paper_1308_5299_amd import _lib
    nrhs = alm.shape[0]
    out = torch.full((nrhs, g.npix), np.nan, dtype=torch.float64, device="cuda")
    rc = _lib.load().sht_synth_noalloc(g.handle, lmax, nrhs, ctypes.c_void_p(alm.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


def test_noalloc_matches_sht_synth(mlcr):
    print("case sht_synth_noalloc vs sht_synth, N_side 256 / lmax 512, then N_side 64 / lmax 100",
          flush=True)
    g = mlcr.Geometry(256, 512)
    rng = np.random.default_rng(2024)
    x1 = dev(rng.standard_normal((4, (512 + 1) ** 2)))
    rc, f1 = _noalloc(mlcr, g, 512, x1)
    assert rc == 0
    ref1 = host(mlcr.sht_synth(g, x1))
    ok, err = check(host(f1), ref1, 1e-12, 512, True)
    print("first call", err, flush=True)
    assert ok, err
    # second call, smaller: fewer RHS, a lower band limit and another grid
    g2 = mlcr.Geometry(64, 100)
    x2 = dev(rng.standard_normal((1, (100 + 1) ** 2)))
    rc, f2 = _noalloc(mlcr, g2, 100, x2)
    assert rc == 0
    ref2 = host(mlcr.sht_synth(g2, x2))
    ok, err = check(host(f2), ref2, 1e-12, 100, True)
    print("second call", err, flush=True)
    assert ok, err
    # and the first shape again on the same grid after the smaller call
    rc, f3 = _noalloc(mlcr, g, 300, x1[:, : 301 ** 2].contiguous())
    assert rc == 0
    ok, err = check(host(f3), host(mlcr.sht_synth(g, x1[:, : 301 ** 2].contiguous(), lmax=300)),
                    1e-12, 300, True)
    assert ok, err


def test_noalloc_rejects_oversize(mlcr):
    from paper_1308_5299_amd import _lib
    g = mlcr.Geometry(1024, 2048)
    x = dev(np.zeros((1, 2049 ** 2)))
    rc, _ = _noalloc(mlcr, g, 2048, x)       # F alone is 134 MB > 64 MiB
    assert rc == -1
    assert b"scratch" in _lib.load().mlcr_last_error()
