"""torch.autograd wrappers: every forward and backward step runs in libmlcr.

* ``SHTSynth`` / ``SHTAdjoint``: y = Y x and its transpose (Sec. 2.1); the
  backward of each is the other transform.
* ``ApplyA``: y = A x (Sec. 2.3); A is symmetric, so the backward is A again.
* ``CRSolve``: x = A^-1 b by W-cycles (Fig. code:mg).  For a loss L(x) the
  backward solves the adjoint system A lam = dL/dx with the same solver (A is
  symmetric) and returns dL/db = lam.  With the prior split into bands,
  C_l = q_beta C_fid_l for l in band beta, dA/dq_beta = -(1/q_beta^2) S_fid^-1
  on the band, so dL/dq_beta = sum_{l in beta, m} lam_lm x_lm / (q_beta^2 C_fid_l)
  (b held fixed); the library's mlcr_prior_band_grad forms that sum on the
  device from the operator's current C_l = q_beta C_fid_l.  The solver's
  operator must hold C = q C_fid.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class SHTSynth(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm, geom, lmax, prec):
        ctx.geom, ctx.lmax, ctx.prec = geom, lmax, prec
        return api.sht_synth(geom, alm.contiguous(), lmax=lmax, prec=prec)

    @staticmethod
    def backward(ctx, gmap):
        return api.sht_adjoint(ctx.geom, gmap.contiguous(), lmax=ctx.lmax, prec=ctx.prec), None, None, None


class SHTAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, maps, geom, lmax, prec):
        ctx.geom, ctx.lmax, ctx.prec = geom, lmax, prec
        return api.sht_adjoint(geom, maps.contiguous(), lmax=lmax, prec=prec)

    @staticmethod
    def backward(ctx, galm):
        return api.sht_synth(ctx.geom, galm.contiguous(), lmax=ctx.lmax, prec=ctx.prec), None, None, None


class ApplyA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op, level, prec):
        ctx.op, ctx.level, ctx.prec = op, level, prec
        return api.apply_A(op, x.contiguous(), level=level, prec=prec)

    @staticmethod
    def backward(ctx, gy):
        return api.apply_A(ctx.op, gy.contiguous(), level=ctx.level, prec=ctx.prec), None, None, None


def band_index(lmax: int, edges) -> np.ndarray:
    """Band of every multipole (-1 outside all bands) for band edges e_0 < ... < e_B."""
    band = np.full(lmax + 1, -1, dtype=np.int64)
    for b in range(len(edges) - 1):
        band[edges[b]: edges[b + 1]] = b
    return band


def log_bands(lmax: int, nbands: int = 64) -> list[int]:
    """Log-spaced band edges on [2, lmax]: e_0 = 2,
    e_b = max(e_{b-1} + 1, round(2 (lmax / 2)^(b / nbands))), e_nbands = lmax + 1."""
    e = [2]
    for b in range(1, nbands):
        e.append(max(e[-1] + 1, int(round(2.0 * (lmax / 2.0) ** (b / nbands)))))
    e.append(lmax + 1)
    # drop bands squeezed out at the top
    out = [e[0]]
    for v in e[1:]:
        if v > out[-1] and out[-1] <= lmax:
            out.append(min(v, lmax + 1))
    return out


class CRSolve(torch.autograd.Function):
    """x = A^-1 b with a ``Solver``; q holds the band multipliers the solver
    was built with (C_l = q_beta C_fid_l), or None when not differentiated."""

    @staticmethod
    def forward(ctx, b, q, solver, cl_fid, edges, rtol, max_cycles, prec):
        x, _ = solver.solve(b.contiguous(), rtol=rtol, max_cycles=max_cycles, prec=prec)
        ctx.solver, ctx.rtol, ctx.max_cycles, ctx.prec = solver, rtol, max_cycles, prec
        ctx.cl_fid, ctx.edges = cl_fid, edges
        ctx.save_for_backward(x, q if q is not None else torch.empty(0, device=b.device))
        ctx.has_q = q is not None
        return x

    @staticmethod
    def backward(ctx, gx):
        x, q = ctx.saved_tensors
        lam, _ = ctx.solver.solve(gx.contiguous(), rtol=ctx.rtol, max_cycles=ctx.max_cycles,
                                  prec=ctx.prec)
        gq = None
        if ctx.has_q:
            # dL/dq_beta = sum_{l in beta, m} lam x / (q_beta C_l), reduced in the library
            op = ctx.solver.op
            band = band_index(op.lmax, ctx.edges)
            g = api.prior_band_grad(op, lam, x, band, q.detach().cpu().numpy())
            gq = torch.from_numpy(g).to(x.device)
        return lam, gq, None, None, None, None, None, None


def cr_solve(b, solver, q=None, cl_fid=None, edges=None, rtol=1e-10, max_cycles=60, prec=api.FP64):
    return CRSolve.apply(b, q, solver, cl_fid, edges, rtol, max_cycles, prec)
