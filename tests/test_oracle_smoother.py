"""Pins of the oracle's smoother reference (Sec. 3.5) against facts that do not
come from it:

* NESTED -> RING (Gorski et al. 2005): a bijection; at N_side 1 the two
  orders agree; the four nested children 4p .. 4p + 3 at 2 N_side lie around
  their parent pixel p (within one parent pixel width); a tile of 64 nested
  pixels is a compact 8 x 8 patch.
* D_hat = Y_h diag(g) Y_h^T and B_hat = Y_obs diag(g) Y_h^T equal the
  addition-theorem sum  sum_l (2l+1)/(4 pi) g_l P_l(cos theta)
  (eq. addition-theorem) between the pixel centres, with P_l from scipy.
* The no-fill product over a complete pattern equals the full block of
  B_hat^T N^-1 B_hat; over a sparse pattern each block sums only the common
  tiles (checked against a direct masked sum).
* Block ICC(0): with the complete pattern it is the dense Cholesky factor of
  the matrix in colour order; with no neighbours it is the Cholesky factor of
  each diagonal block; on a sparse pattern L L^T reproduces the matrix on
  every block of the pattern (the defining property of zero fill-in).
* The tile graph: symmetric, neighbours never share a colour, and every pair
  of tiles closer than 4 pixel widths (brute force over all pixel pairs) is
  listed.
"""
import numpy as np
import pytest
from scipy.linalg import cholesky
from scipy.special import eval_legendre

from oracle import smoother as sm
from oracle.geometry import nest_to_ring


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 64])
def test_nest_to_ring_bijection_and_children(nside):
    n = 12 * nside * nside
    r = nest_to_ring(nside, np.arange(n))
    assert np.array_equal(np.sort(r), np.arange(n))
    if nside == 1:
        assert np.array_equal(r, np.arange(12))
    vp = sm.unit_vectors(nside)[r]                          # nested order
    vc = sm.unit_vectors(2 * nside)[nest_to_ring(2 * nside, np.arange(4 * n))].reshape(n, 4, 3)
    pix = np.sqrt(4 * np.pi / n)
    d = np.linalg.norm(vc - vp[:, None, :], axis=2)
    assert d.max() < 1.0 * pix, d.max() / pix
    # a child's nearest parent centre is its own parent
    cos = np.einsum("pcd,qd->pcq", vc[: min(n, 48)], vp)
    assert np.all(cos.argmax(axis=2) == np.arange(min(n, 48))[:, None])


def test_tiles_are_compact_patches():
    nside = 32
    v = sm.unit_vectors(nside)[sm.tile_pixels(nside, 12 * 16, 64)]
    pix = np.sqrt(4 * np.pi / (12 * nside * nside))
    span = max(np.linalg.norm(t[:, None, :] - t[None, :, :], axis=2).max() for t in v)
    assert span < 14.0 * pix      # an 8 x 8 patch: ~ 10 widths across, stretched near the poles


def _addthm(g, va, vb):
    c = np.clip(va @ vb.T, -1.0, 1.0)
    return sum((2 * l + 1) / (4 * np.pi) * g[l] * eval_legendre(l, c) for l in range(len(g)))


def test_level_matrices_are_addition_theorem_sums():
    rng = np.random.default_rng(5)
    lh, nh, no = 24, 8, 16
    cl = rng.uniform(0.5, 2.0, lh + 1)
    cl[:2] = 0.0                                  # inactive modes are projected out
    bl = rng.uniform(0.2, 1.0, lh + 1)
    fl = np.exp(-0.01 * np.arange(lh + 1) ** 2)
    D, B = sm.level_matrices(cl, bl, fl, lh, nh, no)
    act = cl > 0
    gd = np.where(act, fl * fl / np.where(act, cl, 1), 0)
    gb = np.where(act, fl * bl, 0)
    vh, vo = sm.unit_vectors(nh), sm.unit_vectors(no)
    Dw, Bw = _addthm(gd, vh, vh), _addthm(gb, vo, vh)
    assert np.abs(D - Dw).max() <= 1e-12 * np.abs(Dw).max()
    assert np.abs(B - Bw).max() <= 1e-12 * np.abs(Bw).max()
    assert D.shape == (12 * nh * nh,) * 2 and B.shape == (12 * no * no, 12 * nh * nh)


def _small_system(nside=16, nobs=32, seed=0):
    rng = np.random.default_rng(seed)
    nt = 12 * (nside // 8) ** 2
    lev = sm.tile_pixels(nside, nt, 64)
    obs = sm.tile_pixels(nobs, nt, 64 * (nobs // nside) ** 2)
    B = rng.standard_normal((12 * nobs * nobs, 12 * nside * nside))
    ninv = rng.uniform(0.0, 2.0, 12 * nobs * nobs)
    return nt, lev, obs, B, ninv


def _complete(nt):
    nbptr = np.arange(nt + 1) * (nt - 1)
    nbs = np.concatenate([[u for u in range(nt) if u != t] for t in range(nt)])
    return nbptr, nbs


def test_no_fill_product_complete_pattern_is_full_product():
    nt, lev, obs, B, ninv = _small_system(16, 16)
    nbptr, nbs = _complete(nt)
    diag, off = sm.no_fill_product(B, ninv, obs, lev, nbptr, nbs)
    full = B.T @ (ninv[:, None] * B)
    for t in range(nt):
        assert np.allclose(diag[t], full[np.ix_(lev[t], lev[t])], rtol=0, atol=1e-10)
    for t in [0, 5, nt - 1]:
        for s in range(nbptr[t], nbptr[t + 1]):
            u = nbs[s]
            assert np.allclose(off[s], full[np.ix_(lev[t], lev[u])], rtol=0, atol=1e-10)


def test_no_fill_product_sparse_pattern_sums_common_tiles():
    nt, lev, obs, B, ninv = _small_system(16, 32)
    nbptr, nbs, _ = sm.tile_graph(16)
    diag, off = sm.no_fill_product(B, ninv, obs, lev, nbptr, nbs)
    nb = [set(nbs[nbptr[t]: nbptr[t + 1]]) | {t} for t in range(nt)]
    for t in [0, 7, 30]:
        for s in range(nbptr[t], nbptr[t + 1]):
            u = nbs[s]
            rows = np.zeros(B.shape[0], dtype=bool)
            for T in nb[t] & nb[u]:
                rows[obs[T]] = True
            Bm = np.where(rows[:, None], B, 0.0)
            want = Bm[:, lev[t]].T @ (ninv[:, None] * Bm[:, lev[u]])
            assert np.allclose(off[s], want, rtol=0, atol=1e-10)
        rows = np.zeros(B.shape[0], dtype=bool)
        for T in nb[t]:
            rows[obs[T]] = True
        Bm = np.where(rows[:, None], B, 0.0)
        assert np.allclose(diag[t], Bm[:, lev[t]].T @ (ninv[:, None] * Bm[:, lev[t]]), atol=1e-10)


def _spd_blocks(nt, nbptr, nbs, seed):
    """Blocks of a random SPD matrix on the pattern (diagonally dominant)."""
    rng = np.random.default_rng(seed)
    n = nt * 64
    M = np.zeros((n, n))
    for t in range(nt):
        for u in list(nbs[nbptr[t]: nbptr[t + 1]]) + [t]:
            if u >= t:
                blk = 0.1 * rng.standard_normal((64, 64))
                M[t * 64:(t + 1) * 64, u * 64:(u + 1) * 64] = blk
                M[u * 64:(u + 1) * 64, t * 64:(t + 1) * 64] = blk.T
    M = 0.5 * (M + M.T) + n ** 0.5 * np.eye(n)
    diag = np.stack([M[t * 64:(t + 1) * 64, t * 64:(t + 1) * 64] for t in range(nt)])
    off = np.stack([M[t * 64:(t + 1) * 64, u * 64:(u + 1) * 64]
                    for t in range(nt) for u in nbs[nbptr[t]: nbptr[t + 1]]])
    return M, diag, off


def test_block_icc_complete_pattern_is_cholesky():
    nt = 6
    nbptr, nbs = _complete(nt)
    color = np.array([3, 0, 5, 1, 4, 2])
    M, diag, off = _spd_blocks(nt, nbptr, nbs, 1)
    Ltt, L = sm.block_icc(diag, off, nbptr, nbs, color)
    order = np.argsort(color)
    perm = np.concatenate([np.arange(t * 64, (t + 1) * 64) for t in order])
    C = cholesky(M[np.ix_(perm, perm)], lower=True)
    pos = {int(t): i for i, t in enumerate(order)}
    for t in range(nt):
        i = pos[t]
        assert np.allclose(Ltt[t], C[i * 64:(i + 1) * 64, i * 64:(i + 1) * 64], atol=1e-10)
        for s in range(nbptr[t], nbptr[t + 1]):
            u = int(nbs[s]); j = pos[u]
            if color[u] < color[t]:
                want = C[i * 64:(i + 1) * 64, j * 64:(j + 1) * 64]
            else:
                want = C[j * 64:(j + 1) * 64, i * 64:(i + 1) * 64].T
            assert np.allclose(L[s], want, atol=1e-10)


def test_block_icc_without_neighbours_is_blockwise_cholesky():
    nt = 4
    nbptr = np.zeros(nt + 1, dtype=np.int64)
    nbs = np.zeros(0, dtype=np.int64)
    rng = np.random.default_rng(2)
    diag = np.stack([(lambda a: a @ a.T + 64 * np.eye(64))(rng.standard_normal((64, 64)))
                     for _ in range(nt)])
    Ltt, L = sm.block_icc(diag, np.zeros((0, 64, 64)), nbptr, nbs, np.zeros(nt, dtype=int))
    for t in range(nt):
        assert np.allclose(Ltt[t], cholesky(diag[t], lower=True), atol=1e-12)


def test_block_icc_reproduces_pattern_blocks():
    """Zero fill-in: (L L^T)_tu = A_tu (+ shift on the diagonal) on the pattern."""
    nbptr, nbs, color = sm.tile_graph(16)
    nt = len(nbptr) - 1
    M, diag, off = _spd_blocks(nt, nbptr, nbs, 3)
    shift = 0.25
    Ltt, L = sm.block_icc(diag, off, nbptr, nbs, color, shift=shift)
    # the lower factor in tile blocks: F[t][u] for colour(u) < colour(t), F[t][t] = L_tt
    F = {(t, t): Ltt[t] for t in range(nt)}
    for t in range(nt):
        for s in range(nbptr[t], nbptr[t + 1]):
            u = int(nbs[s])
            if color[u] < color[t]:
                F[(t, u)] = L[s]
    def LLt(t, u):
        acc = np.zeros((64, 64))
        for k in range(nt):
            if (t, k) in F and (u, k) in F:
                acc += F[(t, k)] @ F[(u, k)].T
        return acc
    for t in range(nt):
        assert np.allclose(LLt(t, t), diag[t] + shift * np.eye(64), atol=1e-9)
        for s in range(nbptr[t], nbptr[t + 1]):
            assert np.allclose(LLt(t, int(nbs[s])), off[s], atol=1e-9)


def test_block_icc_reports_failed_pivot():
    nbptr, nbs = _complete(2)
    diag = np.stack([np.eye(64), -np.eye(64)])
    assert sm.block_icc(diag, np.zeros((2, 64, 64)), nbptr, nbs, np.array([0, 1])) is None


@pytest.mark.parametrize("nside", [16, 32])
def test_tile_graph_brute_force(nside):
    nbptr, nbs, color = sm.tile_graph(nside)
    nt = len(nbptr) - 1
    v = sm.unit_vectors(nside)[sm.tile_pixels(nside, nt, 64)]
    pix = np.sqrt(4 * np.pi / (12 * nside * nside))
    for t in range(0, nt, max(1, nt // 24)):
        d = np.linalg.norm(v[t][:, None, None, :] - v[None, :, :, :], axis=3).min(axis=(0, 2))
        want = [u for u in range(nt) if u != t and d[u] < 4 * pix]
        assert list(nbs[nbptr[t]: nbptr[t + 1]]) == want
    for t in range(nt):
        for u in nbs[nbptr[t]: nbptr[t + 1]]:
            assert t in nbs[nbptr[u]: nbptr[u + 1]]
            assert color[t] != color[u]
    assert 4 <= color.max() + 1 <= 12
