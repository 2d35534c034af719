"""Host logic of the solver, checked without a GPU.

* the CR-Cycle recursion with the partial W-cycle of Sec. 4.1 reproduces
  the operation counts the paper prints in Table cycle-cost
  (tests/golden/cycle_cost_table.txt);
* HEALPix NESTED -> RING: a bijection, and each smoother tile (a nested
  block of 64 pixels) is compact on the sphere, checked with the
  independent pixel-centre code of ``workloads``;
* the default ladder follows the paper's band-limit rules.
"""
import math
import os

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = []
    for line in open(os.path.join(HERE, "golden", "cycle_cost_table.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append([0 if v == "-" else int(v) for v in f[1:]])
    return np.array(rows)


def test_cycle_counts_match_paper_table():
    import paper_1308_5299_amd as m
    g = _golden()
    # paper ladder: 6 pixel levels; W on levels <= 1024 except the finest
    # smoother and the top SHTs, which run once down and once up
    c = m.cycle_counts([2, 2, 2, 2, 2, 1], nrec_top=1, ncycles=1)
    visits, applies, yh, smooth = c[:, 0], c[:, 1], c[:, 2], c[:, 3]
    np.testing.assert_array_equal(visits, g[:, 1])
    np.testing.assert_array_equal(yh[1:-1], g[1:-1, 2])
    np.testing.assert_array_equal(2 * applies, g[:, 3])          # Y_obs = 2 per A_h
    np.testing.assert_array_equal(smooth[1:], g[1:, 4])


def test_cycle_counts_scale_with_cycles():
    import paper_1308_5299_amd as m
    c1 = m.cycle_counts([2, 1], 1, 1)
    c3 = m.cycle_counts([2, 1], 1, 3)
    np.testing.assert_array_equal(c3, 3 * c1)


@pytest.mark.parametrize("nside", [1, 2, 8, 32, 64])
def test_nest2ring_bijection_and_tiles(nside):
    import paper_1308_5299_amd as m
    npix = 12 * nside * nside
    ring = m.nest2ring(nside, np.arange(npix))
    assert np.array_equal(np.sort(ring), np.arange(npix))
    if nside >= 8:
        z, phi = workloads.pixel_centres(nside)
        v = np.stack([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z], 1)
        pix = math.sqrt(4 * math.pi / npix)
        tiles = ring.reshape(-1, 64)
        worst = 0.0
        for t in tiles:
            c = v[t].mean(0)
            c /= np.linalg.norm(c)
            worst = max(worst, float(np.max(np.arccos(np.clip(v[t] @ c, -1, 1)))))
        assert worst < 8.0 * pix, worst / pix       # a tile spans about 8 x 8 pixels
        # the four children of a nested pixel are neighbours
        quad = ring.reshape(-1, 4)
        d = np.arccos(np.clip(np.einsum("ij,ij->i", v[quad[:, 0]], v[quad[:, 3]]), -1, 1))
        assert d.max() < 2.5 * pix


def test_ladder_plan_rules():
    import paper_1308_5299_amd as m
    p = m.ladder_plan(2048, 4096)
    assert p["nside"] == [1024, 512, 256, 128, 64, 32]
    assert p["lmax"][0] == 4096 and p["lmax"][1] == 4 * 512
    assert all(l <= 6 * n for l, n in zip(p["lmax"][2:], p["nside"][2:]))
    assert p["nrec"] == [2, 2, 2, 2, 2, 1] and p["nrec_top"] == 1 and p["lmax_bottom"] == 40
    small = m.ladder_plan(16, 32)
    assert small["nlevels"] == 0 and small["lmax_bottom"] == 32     # direct dense solve
