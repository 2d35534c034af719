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


def test_ladder_default_matches_plan():
    """mlcr_ladder_default reproduces mlcr_ladder_plan and its filters follow
    the Sec. 3.3 forms: the q_l filter of eq. fourth-power-beam with
    q = 0.1 at 2570/3000 of the band limit on the first level of N_side >= 512,
    and a Gaussian of FWHM two level pixels on levels of N_side <= 256."""
    import paper_1308_5299_amd as m
    for nside, lmax in [(16, 32), (256, 512), (2048, 4096)]:
        lad = m.Ladder.default(nside, lmax)
        plan = m.ladder_plan(nside, lmax)
        assert len(lad.nside) == plan["nlevels"]
        assert lad.nside == plan["nside"] and lad.lmax == plan["lmax"] and lad.nrec == plan["nrec"]
        assert lad.nrec_top == plan["nrec_top"] and lad.lmax_dense == plan["lmax_bottom"]
        lad.check(nside, lmax)
    lad = m.Ladder.default(2048, 4096)
    ls = round(lad.lmax[0] * 2570 / 3000)
    assert lad.filters[0][ls] == pytest.approx(0.1, rel=1e-12)
    h = lad.nside.index(256)
    pix = math.sqrt(4 * math.pi / (12 * 256 ** 2))
    sig = 2 * pix / math.sqrt(8 * math.log(2))
    ell = np.arange(lad.lmax[h] + 1)
    np.testing.assert_allclose(lad.filters[h], np.exp(-0.5 * ell * (ell + 1) * sig * sig), rtol=1e-13)


def _gauss(lmax, fwhm_px, nside):
    pix = math.sqrt(4 * math.pi / (12 * nside ** 2))
    sig = fwhm_px * pix / math.sqrt(8 * math.log(2))
    ell = np.arange(lmax + 1)
    return np.exp(-0.5 * ell * (ell + 1) * sig * sig)


@pytest.mark.parametrize("field,value,msg", [
    ("nlevels", 9, b"nlevels"),
    ("nside", [100, 64], b"multiple of 8"),
    ("lmax", [600, 300], b"lmax must be in"),
    ("lmax", [300, 384], b"lmax must be in"),
    ("nrec", [2, 0], b"nrec must be in"),
    ("nrec_top", 4, b"nrec_top"),
    ("lmax_dense", 80, b"lmax_dense"),
    ("gl_levels", 2, b"gl_levels"),
    ("smoother", 2, b"smoother must be 0 or 1"),
    ("keep_blocks", 3, b"keep_blocks"),
    ("ridge_max", -1.0, b"ridge_max"),
    ("ridge_max", float("inf"), b"ridge_max"),
    ("ridge_min", -1.0, b"ridge_min"),
    ("ridge_min", 2.0, b"ridge_min"),
    ("ridge_min", float("nan"), b"ridge_min"),
    ("smoother_ratio", [96, 64], b"power of two"),
    ("filter0", "zero", b"filter must be > 0"),
    ("filter0", "nan", b"finite"),
])
def test_ladder_check_rejects(field, value, msg):
    """A custom ladder is validated on the host before any device work."""
    import ctypes
    import paper_1308_5299_amd as m
    from paper_1308_5299_amd import _lib
    f0, f1 = _gauss(384, 2.0, 128), _gauss(300, 2.0, 64)
    lad = m.Ladder([128, 64], [384, 300], [2, 1], [f0, f1], nrec_top=1, lmax_dense=40)
    lad.check(256, 512)
    if field == "filter0":
        bad = f0.copy()
        bad[10] = 0.0 if value == "zero" else np.nan
        lad.filters[0] = bad
    elif field == "smoother_ratio":
        # 256 / 96 is no power of two: the addition-theorem smoother's tiles
        # would not nest in the observation grid's
        lad.nside = value
        lad.smoother = 1
    elif field in ("nside", "lmax", "nrec"):
        setattr(lad, field, value)
    else:
        setattr(lad, field, value)
    d = lad.desc()
    if field in ("nlevels", "gl_levels", "smoother", "keep_blocks"):
        setattr(d, field, value)
    lib = _lib.load()
    assert lib.mlcr_ladder_check(256, 512, ctypes.byref(d)) == -1
    assert msg in lib.mlcr_last_error(), lib.mlcr_last_error()


def test_ladder_without_pixel_levels():
    import ctypes
    import paper_1308_5299_amd as m
    from paper_1308_5299_amd import _lib
    lib = _lib.load()
    lad = m.Ladder([], [], [], [], nrec_top=1, lmax_dense=32)
    lad.check(16, 32)
    d = m.Ladder([], [], [], [], nrec_top=1, lmax_dense=40).desc()
    assert lib.mlcr_ladder_check(16, 32, ctypes.byref(d)) == -1       # must cover lmax exactly
    d = m.Ladder([], [], [], [], nrec_top=1, lmax_dense=100).desc()
    assert lib.mlcr_ladder_check(64, 100, ctypes.byref(d)) == -1      # too large to be dense


def test_schedule_visits_for_custom_counts():
    """The cycle schedule visits level h prod_{k < h} n_rec^k times (the
    recursion of Fig. code:mg), for counts the paper's table does not use."""
    import paper_1308_5299_amd as m
    nrec, top = [3, 1, 2], 2
    c = m.cycle_counts(nrec, nrec_top=top, ncycles=1)
    want = [1, top, top * 3, top * 3 * 1, top * 3 * 1 * 2]
    np.testing.assert_array_equal(c[:, 0], want)
    # pixel levels smooth twice per visit, two level SHTs per smoothing;
    # the bottom is solved once per visit
    np.testing.assert_array_equal(c[1:4, 3], 2 * np.array(want[1:4]))
    np.testing.assert_array_equal(c[1:4, 2], 4 * np.array(want[1:4]))
    assert c[4, 3] == want[4]


@pytest.mark.parametrize("nside", [16, 32, 64])
def test_tiles_match_the_oracle(nside):
    """The library's NESTED -> RING map and its tile graph (neighbour lists,
    sweep colours) equal the oracle's, integer for integer."""
    import paper_1308_5299_amd as m
    from oracle import smoother as osm
    from oracle.geometry import nest_to_ring
    n = 12 * nside * nside
    assert np.array_equal(m.nest2ring(nside, np.arange(n)), nest_to_ring(nside, np.arange(n)))
    g = m.tile_graph(nside)
    nbptr, nbs, color = osm.tile_graph(nside)
    nt = len(nbptr) - 1
    for t in range(nt):
        assert sorted(int(u) for u in g["nb"][t] if u >= 0) == list(nbs[nbptr[t]: nbptr[t + 1]])
    assert np.array_equal(np.asarray(g["sweep_color"]), color)
