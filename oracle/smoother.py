"""Pixel-domain level operator and its sparse approximant, for the oracle
(test infrastructure only).

Sec. 3.5 builds the pixel levels' error smoother from
    A_hat_h = Y_h A_h Y_h^T = D_hat_h + B_hat_h^T N^-1 B_hat_h     (eq. pixel-domain)
    D_hat_h = Y_h F_h S^-1 F_h Y_h^T,  B_hat_h = Y_obs B F_h Y_h^T  (eqs. Dhat, Bhat)
restricted to a block pattern of k x k tiles and their neighbour tiles, with
B_hat^T N^-1 B_hat formed by block products without fill-in, and factors the
result by a zero-fill incomplete Cholesky.  Here everything is dense and
plain, for small grids:

* ``synth_matrix``     the dense synthesis matrix of a grid from the oracle's
                       own transform (Y = synth applied to the identity);
* ``level_matrices``   D_hat_h (level x level) and B_hat_h (obs x level);
* ``tile_blocks``      the blocks of a dense level matrix on the pattern;
* ``no_fill_product``  sum over the tiles T common to both patterns of
                       B_hat[obs(T), t]^T diag(N^-1) B_hat[obs(T), u];
* ``block_icc``        block incomplete Cholesky with no fill-in, tiles taken
                       colour by colour.

Tiles are nested pixel blocks: tile t holds level pixels (nested) 64 t ..
64 t + 63; obs(T) are the observation pixels (nested) inside tile T.  Blocks
are returned row-major [t][i][j] with i, j the nested position in the tile.
"""
from __future__ import annotations

import numpy as np

from . import sht
from .geometry import healpix_rings, nest_to_ring, pixel_angles

K = 8
K2 = K * K


def synth_matrix(nside: int, lmax: int) -> np.ndarray:
    """Y of the grid: (npix, (lmax+1)^2), column j the map of packed unit vector j."""
    return sht.synth(np.eye(sht.nalm(lmax)), lmax, nside).T


def level_matrices(cl, bl, fl, lmax_h: int, nside_h: int, nside_obs: int):
    """(D_hat_h, B_hat_h) with D_hat = Y_h diag(f^2 / C) Y_h^T and
    B_hat = Y_obs diag(f b) Y_h^T, over the modes l <= lmax_h (C > 0)."""
    from .operator import mode_ell
    L = mode_ell(lmax_h)
    cl = np.asarray(cl, dtype=np.float64)[L]
    f = np.asarray(fl, dtype=np.float64)[L]
    b = np.asarray(bl, dtype=np.float64)[L]
    act = cl > 0
    gd = np.where(act, f * f / np.where(act, cl, 1.0), 0.0)
    gb = np.where(act, f * b, 0.0)
    Yh = synth_matrix(nside_h, lmax_h)
    Yo = synth_matrix(nside_obs, lmax_h)
    return (Yh * gd) @ Yh.T, (Yo * gb) @ Yh.T


def unit_vectors(nside: int) -> np.ndarray:
    """Pixel-centre unit vectors of a HEALPix grid, RING order."""
    th, ph = pixel_angles(healpix_rings(nside))
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def tile_graph(nside: int, adj_px: float = 4.0):
    """Tiles of 8 x 8 nested pixels; u is a neighbour of t when some pixel
    centre of u lies closer than adj_px pixel widths (chord) to one of t.
    Colours: greedy in tile order, each tile the smallest colour none of its
    already coloured neighbours has.  Returns (nbptr, nbs, color), the
    neighbour lists ascending."""
    nt = 12 * (nside // K) ** 2
    v = unit_vectors(nside)[tile_pixels(nside, nt, K2)]          # [nt, 64, 3]
    px = np.sqrt(4.0 * np.pi / (12.0 * nside * nside))
    flat = v.reshape(-1, 3)
    nbs, nbptr = [], [0]
    for t in range(nt):
        cos = (v[t] @ flat.T).max(axis=0).reshape(nt, K2).max(axis=1)    # nearest pair per tile
        dmin = np.sqrt(np.maximum(2.0 - 2.0 * cos, 0.0))                   # its chord
        near = [u for u in range(nt) if u != t and dmin[u] / px < adj_px]
        nbs += near
        nbptr.append(len(nbs))
    nbptr = np.array(nbptr, dtype=np.int64)
    nbs = np.array(nbs, dtype=np.int64)
    color = np.full(nt, -1, dtype=np.int64)
    for t in range(nt):
        used = {int(color[u]) for u in nbs[nbptr[t]: nbptr[t + 1]] if color[u] >= 0}
        c = 0
        while c in used:
            c += 1
        color[t] = c
    return nbptr, nbs, color


def tile_pixels(nside: int, ntiles: int, per: int) -> np.ndarray:
    """RING indices of the pixels of each tile (nested blocks of `per`)."""
    return nest_to_ring(nside, np.arange(ntiles * per)).reshape(ntiles, per)


def tile_blocks(M, tiles, nbptr, nbs):
    """(diag [nt][64][64], off [nslots][64][64]) of a dense level matrix."""
    nt = tiles.shape[0]
    diag = np.stack([M[np.ix_(tiles[t], tiles[t])] for t in range(nt)])
    off = np.stack([M[np.ix_(tiles[t], tiles[nbs[s]])]
                    for t in range(nt) for s in range(nbptr[t], nbptr[t + 1])]) \
        if nbptr[nt] > 0 else np.zeros((0, K2, K2))
    return diag, off


def _pattern(t, nbptr, nbs):
    return {t} | set(int(v) for v in nbs[nbptr[t]: nbptr[t + 1]])


def no_fill_product(Bhat, ninv_obs, obs_tiles, lev_tiles, nbptr, nbs):
    """Blocks of B_hat^T N^-1 B_hat without fill-in: block (t, u) sums over
    the tiles T in pattern(t) and pattern(u) only."""
    nt = lev_tiles.shape[0]
    ninv_obs = np.asarray(ninv_obs, dtype=np.float64)

    def block(t, u):
        acc = np.zeros((K2, K2))
        for T in sorted(_pattern(t, nbptr, nbs) & _pattern(u, nbptr, nbs)):
            o = obs_tiles[T]
            bt = Bhat[np.ix_(o, lev_tiles[t])]
            bu = Bhat[np.ix_(o, lev_tiles[u])]
            acc += bt.T @ (ninv_obs[o][:, None] * bu)
        return acc

    diag = np.stack([block(t, t) for t in range(nt)])
    off = np.stack([block(t, int(nbs[s])) for t in range(nt) for s in range(nbptr[t], nbptr[t + 1])]) \
        if nbptr[nt] > 0 else np.zeros((0, K2, K2))
    return diag, off


def block_icc(diag, off, nbptr, nbs, color, shift: float = 0.0):
    """Block incomplete Cholesky with no fill-in: A ~ L L^T with L lower in
    the order of increasing colour (tiles of one colour share no block), and
    L_ut nonzero only where A_ut is in the pattern.  Returns
    (L_tt [nt][64][64], L [nslots][64][64]) with L[slot t -> u] = L_tu when
    colour(u) < colour(t) and L_ut^T when colour(u) > colour(t), or None if a
    pivot fails."""
    from scipy.linalg import cholesky, solve_triangular

    nt = diag.shape[0]
    slot = {}
    for t in range(nt):
        for s in range(nbptr[t], nbptr[t + 1]):
            slot[(t, int(nbs[s]))] = s
    Ltt = np.zeros_like(diag)
    Lb = {}                          # (u, t) -> L_ut for colour(u) > colour(t)
    for c in range(int(np.max(color)) + 1):
        for t in np.nonzero(np.asarray(color) == c)[0]:
            t = int(t)
            S = diag[t] + shift * np.eye(K2)
            earlier = [k for k in _pattern(t, nbptr, nbs) - {t} if color[k] < c]
            for k in earlier:
                S = S - Lb[(t, k)] @ Lb[(t, k)].T
            try:
                Ltt[t] = cholesky(S, lower=True)
            except np.linalg.LinAlgError:
                return None
            for u in _pattern(t, nbptr, nbs) - {t}:
                if color[u] <= c:
                    continue
                R = off[slot[(u, t)]].copy()
                for k in earlier:
                    if (u, k) in Lb:
                        R = R - Lb[(u, k)] @ Lb[(t, k)].T
                # L_ut = R L_tt^-T
                Lb[(u, t)] = solve_triangular(Ltt[t], R.T, lower=True).T
    L = np.zeros_like(off)
    for (t, u), s in slot.items():
        L[s] = Lb[(t, u)] if color[u] < color[t] else Lb[(u, t)].T
    return Ltt, L
