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


def _tile_distances(nside):
    """Nearest pixel-centre distance between every pair of 8 x 8 nested tiles,
    in pixel widths (brute force over all pixel centres)."""
    import paper_1308_5299_amd as m
    npix = 12 * nside * nside
    ring = m.nest2ring(nside, np.arange(npix)).reshape(-1, 64)
    z, phi = workloads.pixel_centres(nside)
    v = np.stack([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z], 1)
    vt = v[ring]                                            # [ntiles, 64, 3]
    flat = vt.reshape(-1, 3)
    nt = len(ring)
    dmin = np.empty((nt, nt))
    for a in range(nt):
        dots = (vt[a] @ flat.T).reshape(64, nt, 64)
        dmin[a] = np.arccos(np.clip(dots.max(axis=(0, 2)), -1, 1))
    return dmin / math.sqrt(4 * math.pi / npix)


@pytest.mark.parametrize("nside", [32, 64])
def test_tile_graph(nside):
    """Neighbour lists hold exactly the tiles nearer than 4 pixel widths;
    neighbours never share a sweep colour; the response of a probed tile,
    read at the tile and its neighbours, stays 6 pixel widths away from every
    other tile of its probe colour."""
    import paper_1308_5299_amd as m
    g = m.tile_graph(nside)
    d = _tile_distances(nside)
    nt = d.shape[0]
    nb = [set(int(u) for u in row if u >= 0) for row in g["nb"]]
    for t in range(nt):
        want = set(np.flatnonzero(d[t] < 4.0).tolist()) - {t}
        assert nb[t] == want, t
        assert list(row for row in g["nb"][t] if row >= 0) == sorted(want)
    sc, pc = g["sweep_color"], g["probe_color"]
    for t in range(nt):
        assert all(sc[u] != sc[t] for u in nb[t])
    worst = np.inf
    for c in range(g["n_probe"]):
        ts = np.flatnonzero(pc == c)
        for u in ts:
            read_at = [u] + sorted(nb[u])
            others = ts[ts != u]
            if len(others):
                worst = min(worst, d[np.ix_(read_at, others)].min())
    assert worst >= 6.0, worst
    # a regular patch has 8 neighbours; colour counts stay small
    assert np.bincount((g["nb"] >= 0).sum(1)).argmax() == 8
    assert g["n_sweep"] <= 8 and g["n_probe"] <= 20


def test_ladder_plan_rules():
    import paper_1308_5299_amd as m
    p = m.ladder_plan(2048, 4096)
    assert p["nside"] == [1024, 512, 256, 128, 64, 32]
    assert p["lmax"][0] == 4096 and p["lmax"][1] == 4 * 512
    assert p["lmax"][2:] == [6 * n for n in p["nside"][2:]]
    c2 = m.ladder_plan(256, 512)
    assert c2["nside"] == [128, 64, 32] and c2["lmax"] == [512, 384, 192]
    assert p["nrec"] == [2, 2, 2, 2, 2, 1] and p["nrec_top"] == 1 and p["lmax_bottom"] == 40
    small = m.ladder_plan(16, 32)
    assert small["nlevels"] == 0 and small["lmax_bottom"] == 32     # direct dense solve
