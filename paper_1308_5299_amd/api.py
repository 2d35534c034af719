"""Python front end of the C ABI (include/mlcr.h).

Tensors are float64 CUDA (HIP) tensors: harmonic vectors [nrhs, (lmax+1)^2]
in real packed m-major order, maps [nrhs, 12 nside^2] in RING order.  Work
is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, load

FP64 = 0
FP32 = 1
BF16X3 = 2


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _batch(t: torch.Tensor, per: int, name: str) -> int:
    if t.numel() % per != 0 or t.numel() == 0:
        raise ValueError(f"{name} has {t.numel()} elements, not a positive multiple of {per}")
    return t.numel() // per


class Geometry:
    """HEALPix RING grid (or, via ``Geometry.gauss_legendre``, a Gauss-Legendre
    grid) plus Legendre and FFT tables up to lmax."""

    def __init__(self, nside: int, lmax: int, _gl: tuple | None = None):
        lib = load()
        h = ctypes.c_void_p()
        if _gl is None:
            check(lib.mlcr_geom_create(int(nside), int(lmax), ctypes.byref(h)))
            self.nside = int(nside)
            self.npix = 12 * self.nside * self.nside
            self.nrings = 4 * self.nside - 1
        else:
            nrings, nphi = _gl
            check(lib.mlcr_geom_create_gl(int(lmax), int(nrings), int(nphi), ctypes.byref(h)))
            self.nside = 0
            self.npix = int(nrings) * int(nphi)
            self.nrings = int(nrings)
            self.nphi = int(nphi)
        self._h = h
        self.lmax = int(lmax)

    @classmethod
    def gauss_legendre(cls, lmax: int, nrings: int, nphi: int) -> "Geometry":
        return cls(0, lmax, _gl=(nrings, nphi))

    def weights(self) -> np.ndarray:
        """Quadrature weight of one pixel of each ring."""
        w = np.empty(self.nrings, dtype=np.float64)
        check(load().mlcr_geom_weights(self._h, w.ctypes.data))
        return w

    def set_tuning(self, prec: int, adjoint_waves: int, synth_chains: int,
                   ring_threads: int) -> None:
        """Launch shapes of one arithmetic path on this geometry
        (mlcr_geom_set_tuning): adjoint_waves 4 or 8, synth_chains 2 or 4,
        ring_threads 512 or 1024."""
        check(load().mlcr_geom_set_tuning(self._h, int(prec), int(adjoint_waves),
                                          int(synth_chains), int(ring_threads)))

    def get_tuning(self, prec: int) -> dict:
        """The current launch shapes of one arithmetic path."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(load().mlcr_geom_get_tuning(self._h, int(prec), ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(c)))
        return {"adjoint_waves": a.value, "synth_chains": b.value, "ring_threads": c.value}

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().mlcr_geom_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def packed_ell(lmax: int) -> np.ndarray:
    """Multipole l of every entry of a real packed harmonic vector (m = 0 block,
    then a cosine and a sine block per m >= 1, l = m .. lmax)."""
    parts = [np.arange(lmax + 1)]
    for m in range(1, lmax + 1):
        ls = np.arange(m, lmax + 1)
        parts += [ls, ls]
    return np.concatenate(parts).astype(np.int64)


def nalm(lmax: int) -> int:
    return (lmax + 1) ** 2


def sht_synth(geom: Geometry, alm: torch.Tensor, lmax: int | None = None, prec: int = FP64,
              out: torch.Tensor | None = None) -> torch.Tensor:
    lmax = geom.lmax if lmax is None else int(lmax)
    _dev(alm, "alm")
    nrhs = _batch(alm, nalm(lmax), "alm")
    if out is None:
        out = torch.empty((nrhs, geom.npix), dtype=torch.float64, device=alm.device)
    _dev(out, "out")
    check(load().sht_synth(geom.handle, lmax, nrhs, ctypes.c_void_p(alm.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()), prec, _stream()))
    return out


def sht_adjoint(geom: Geometry, maps: torch.Tensor, lmax: int | None = None, prec: int = FP64,
                out: torch.Tensor | None = None) -> torch.Tensor:
    lmax = geom.lmax if lmax is None else int(lmax)
    _dev(maps, "maps")
    nrhs = _batch(maps, geom.npix, "maps")
    if out is None:
        out = torch.empty((nrhs, nalm(lmax)), dtype=torch.float64, device=maps.device)
    _dev(out, "out")
    check(load().sht_adjoint(geom.handle, lmax, nrhs, ctypes.c_void_p(maps.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), prec, _stream()))
    return out


class Operator:
    """A = S^-1 + B Y^T N^-1 Y B on the observation geometry (plus levels)."""

    def __init__(self, geom: Geometry, cl, bl, ninv: torch.Tensor, max_nrhs: int = 1,
                 lmax: int | None = None):
        lib = load()
        self.geom = geom
        self.lmax = geom.lmax if lmax is None else int(lmax)
        cl = np.ascontiguousarray(np.asarray(cl, dtype=np.float64)[: self.lmax + 1])
        bl = np.ascontiguousarray(np.asarray(bl, dtype=np.float64)[: self.lmax + 1])
        if cl.size != self.lmax + 1 or bl.size != self.lmax + 1:
            raise ValueError("cl and bl need lmax+1 entries")
        self.ninv = _dev(ninv, "ninv")
        if ninv.numel() != geom.npix:
            raise ValueError("ninv must have 12 nside^2 entries")
        self.cl, self.bl = cl, bl
        self.max_nrhs = int(max_nrhs)
        h = ctypes.c_void_p()
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib.mlcr_op_create(geom.handle, self.lmax, cl.ctypes.data_as(dp), bl.ctypes.data_as(dp),
                                 ctypes.c_void_p(ninv.data_ptr()), self.max_nrhs, ctypes.byref(h)))
        self._h = h
        self.level_lmax = {0: self.lmax}

    @property
    def handle(self):
        return self._h

    def set_level(self, h: int, lmax_h: int, fl) -> None:
        fl = np.ascontiguousarray(np.asarray(fl, dtype=np.float64)[: lmax_h + 1])
        check(load().mlcr_op_set_level(self._h, int(h), int(lmax_h),
                                       fl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self.level_lmax[int(h)] = int(lmax_h)

    def set_prior(self, cl) -> None:
        """Replace C_l (mlcr_op_set_prior): > 0 exactly where the current C_l is."""
        cl = np.ascontiguousarray(np.asarray(cl, dtype=np.float64)[: self.lmax + 1])
        if cl.size != self.lmax + 1:
            raise ValueError("cl needs lmax+1 entries")
        check(load().mlcr_op_set_prior(self._h, cl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self.cl = cl

    def set_level_gl(self, h: int, lmax_h: int, fl) -> None:
        """Level h with Y^T N^-1 Y on a Gauss-Legendre grid (downgraded N^-1)."""
        fl = np.ascontiguousarray(np.asarray(fl, dtype=np.float64)[: lmax_h + 1])
        check(load().mlcr_op_set_level_gl(self._h, int(h), int(lmax_h),
                                          fl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self.level_lmax[int(h)] = int(lmax_h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().mlcr_op_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cr_rhs(op: Operator, d: torch.Tensor, w1: torch.Tensor | None = None,
           w2: torch.Tensor | None = None) -> torch.Tensor:
    """b = B Y^T (N^-1 d + N^-1/2 w2) + S^-1/2 w1 (Sec. 2.3); w1 = w2 = None
    gives the Wiener-filter (maximum-likelihood) right-hand side."""
    _dev(d, "d")
    npix = int(op.ninv.numel())
    nrhs = _batch(d, npix, "d")
    b = torch.empty((nrhs, nalm(op.lmax)), dtype=torch.float64, device=d.device)
    for t, n, name in ((w1, nalm(op.lmax), "w1"), (w2, npix, "w2")):
        if t is not None:
            _dev(t, name)
            if _batch(t, n, name) != nrhs:
                raise ValueError(f"{name} must have the batch size of d")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()
    check(load().mlcr_cr_rhs(op.handle, nrhs, ptr(d), ptr(w1), ptr(w2), ptr(b), _stream()))
    return b


def apply_A(op: Operator, x: torch.Tensor, level: int = 0, prec: int = FP64,
            out: torch.Tensor | None = None) -> torch.Tensor:
    lmax = op.level_lmax[level]
    _dev(x, "x")
    nrhs = _batch(x, nalm(lmax), "x")
    if out is None:
        out = torch.empty((nrhs, nalm(lmax)), dtype=torch.float64, device=x.device)
    _dev(out, "out")
    check(load().apply_A(op.handle, int(level), nrhs, ctypes.c_void_p(x.data_ptr()),
                         ctypes.c_void_p(out.data_ptr()), prec, _stream()))
    return out


class KernelTimer:
    """Per-kernel HIP-event timing inside the library (context manager).

    with KernelTimer() as kt: ...; kt.result -> {name: (total_ms, calls)}
    """

    def __enter__(self):
        lib = load()
        check(lib.mlcr_timing_reset())
        check(lib.mlcr_timing_enable(1))
        self.result = {}
        return self

    def __exit__(self, *exc):
        lib = load()
        check(lib.mlcr_timing_enable(0))
        n = lib.mlcr_timing_count()
        buf = ctypes.create_string_buffer(64)
        for i in range(n):
            ms = ctypes.c_double()
            calls = ctypes.c_longlong()
            check(lib.mlcr_timing_get(i, buf, 64, ctypes.byref(ms), ctypes.byref(calls)))
            self.result[buf.value.decode()] = (ms.value, calls.value)
        return False


class Ladder:
    """A solver ladder (mlcr_ladder_desc): pixel levels finest first, each with
    N_side^h, lmax^h, n_rec^h and its cumulative filter f~^h_l; the top
    level's recursion count, the dense bottom's band limit, an optional top
    high-pass and whether coarse levels may use Gauss-Legendre grids."""

    def __init__(self, nside, lmax, nrec, filters, nrec_top: int = 1, lmax_dense: int = 40,
                 highpass=None, gl_levels: bool = True, smoother: int = 0, ridge_max: float = 1.0,
                 ridge_min: float = 1e-4,
                 keep_blocks: bool = False):
        self.nside = [int(v) for v in nside]
        self.lmax = [int(v) for v in lmax]
        self.nrec = [int(v) for v in nrec]
        self.filters = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in filters]
        self.nrec_top = int(nrec_top)
        self.lmax_dense = int(lmax_dense)
        self.highpass = None if highpass is None else np.ascontiguousarray(np.asarray(highpass, dtype=np.float64))
        self.gl_levels = bool(gl_levels)
        self.smoother = int(smoother)
        self.ridge_max = float(ridge_max)
        self.ridge_min = float(ridge_min)
        self.keep_blocks = bool(keep_blocks)
        n = len(self.nside)
        if not (len(self.lmax) == len(self.nrec) == len(self.filters) == n) or n > 8:
            raise ValueError("one nside, lmax, nrec and filter per level, at most 8 levels")
        for f, lm in zip(self.filters, self.lmax):
            if f.size < lm + 1:
                raise ValueError("a filter needs lmax^h + 1 entries")

    @classmethod
    def default(cls, nside: int, lmax: int) -> "Ladder":
        """The ladder the library uses when given none (mlcr_ladder_default)."""
        from ._lib import LadderDesc
        d = LadderDesc()
        buf = np.zeros(8 * (lmax + 1), dtype=np.float64)
        check(load().mlcr_ladder_default(int(nside), int(lmax), ctypes.byref(d), buf.ctypes.data))
        n = d.nlevels
        filt = [buf[h * (lmax + 1): h * (lmax + 1) + d.lmax[h] + 1].copy() for h in range(n)]
        return cls(list(d.nside[:n]), list(d.lmax[:n]), list(d.nrec[:n]), filt, d.nrec_top,
                   d.lmax_dense, None, bool(d.gl_levels), d.smoother, d.ridge_max, d.ridge_min,
                   bool(d.keep_blocks))

    def desc(self):
        """The C descriptor; its filter pointers point into this object's arrays."""
        from ._lib import LadderDesc
        dp = ctypes.POINTER(ctypes.c_double)
        d = LadderDesc()
        d.nlevels = len(self.nside)
        for h in range(d.nlevels):
            d.nside[h], d.lmax[h], d.nrec[h] = self.nside[h], self.lmax[h], self.nrec[h]
            d.filter[h] = self.filters[h].ctypes.data_as(dp)
        d.nrec_top = self.nrec_top
        d.lmax_dense = self.lmax_dense
        d.highpass = self.highpass.ctypes.data_as(dp) if self.highpass is not None else dp()
        d.gl_levels = 1 if self.gl_levels else 0
        d.smoother = self.smoother
        d.ridge_max = self.ridge_max
        d.ridge_min = self.ridge_min
        d.keep_blocks = 1 if self.keep_blocks else 0
        return d

    def check(self, nside_obs: int, lmax: int) -> None:
        """mlcr_ladder_check: raises MLCRError with the reason if invalid."""
        d = self.desc()
        check(load().mlcr_ladder_check(int(nside_obs), int(lmax), ctypes.byref(d)))


class Solver:
    """Multi-level CR solver (W-cycle) for an Operator; see include/mlcr.h."""

    def __init__(self, op: Operator, max_nrhs: int = 1, ladder: Ladder | None = None):
        lib = load()
        self.op = op
        self.max_nrhs = int(max_nrhs)
        self.ladder = ladder
        h = ctypes.c_void_p()
        d = ladder.desc() if ladder is not None else None
        check(lib.mlcr_solver_create(op.handle, ctypes.byref(d) if d is not None else None,
                                     self.max_nrhs, ctypes.byref(h)))
        self._h = h

    def set_profile(self, on: bool = True) -> None:
        """Per-level profile of the cycles (mlcr_solver_set_profile); clears it."""
        check(load().mlcr_solver_set_profile(self._h, 1 if on else 0))

    def profile(self) -> dict:
        """{"ms": [levels][4], "calls": [levels][4]}: kinds = A_h applications,
        level transforms, smoother, transfers; levels = top, pixel levels,
        dense bottom."""
        lib = load()
        n = lib.mlcr_solver_profile(self._h, 0, None, None)
        if n < 0:
            check(n)
        ms = np.zeros(4 * n)
        calls = np.zeros(4 * n, dtype=np.int64)
        r = lib.mlcr_solver_profile(self._h, n, ms.ctypes.data, calls.ctypes.data)
        if r < 0:
            check(r)
        return {"ms": ms.reshape(n, 4), "calls": calls.reshape(n, 4)}

    def info(self) -> dict:
        nl, lb, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rg = ctypes.c_float()
        check(load().mlcr_solver_info(self._h, ctypes.byref(nl), ctypes.byref(lb), ctypes.byref(nb),
                                      ctypes.byref(rg)))
        return {"nlevels": nl.value, "lmax_bottom": lb.value, "n_bottom": nb.value,
                "max_ridge": rg.value}

    def level_blocks(self, level: int, which: int = 0):
        """Smoother blocks of pixel level `level` (incomplete-Cholesky smoother):
        (diag [ntiles, 64, 64], off [nslots, 64, 64]) float32 tensors, stored
        column-major per block (entry (i, j) at [j, i]); which 0 = assembled
        approximant, 1 = factor (see mlcr_solver_level_blocks)."""
        lib = load()
        nt, ns = ctypes.c_int(), ctypes.c_longlong()
        check(lib.mlcr_solver_level_blocks(self._h, int(level), int(which), ctypes.byref(nt),
                                           ctypes.byref(ns), None, None))
        dev = self.op.ninv.device
        dg = torch.empty((nt.value, 64, 64), dtype=torch.float32, device=dev)
        of = torch.empty((max(ns.value, 1), 64, 64), dtype=torch.float32, device=dev)
        check(lib.mlcr_solver_level_blocks(self._h, int(level), int(which), ctypes.byref(nt),
                                           ctypes.byref(ns), ctypes.c_void_p(dg.data_ptr()),
                                           ctypes.c_void_p(of.data_ptr())))
        return dg, of[: ns.value]

    def bottom(self):
        """(A_B as an [n, n] float64 tensor, packed positions of its modes)."""
        n = ctypes.c_int()
        check(load().mlcr_solver_bottom(self._h, ctypes.byref(n), None, None))
        A = torch.empty((n.value, n.value), dtype=torch.float64, device=self.op.ninv.device)
        idx = np.zeros(n.value, dtype=np.int32)
        check(load().mlcr_solver_bottom(self._h, ctypes.byref(n), ctypes.c_void_p(A.data_ptr()),
                                        idx.ctypes.data))
        return A, idx

    def top_dinv(self) -> torch.Tensor:
        out = torch.empty((nalm(self.op.lmax),), dtype=torch.float64, device=self.op.ninv.device)
        check(load().mlcr_solver_top_dinv(self._h, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def solve(self, b: torch.Tensor, x0: torch.Tensor | None = None, rtol: float = 1e-8,
              max_cycles: int = 50, prec: int = FP64, raise_on_noconv: bool = True):
        """Returns (x, infos); infos is a list of dicts, one per RHS."""
        from ._lib import MLCRError, SolveInfo

        _dev(b, "b")
        nrhs = _batch(b, nalm(self.op.lmax), "b")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        infos = (SolveInfo * nrhs)()
        rc = load().wcycle_solve(self._h, nrhs, ctypes.c_void_p(b.data_ptr()),
                                 ctypes.c_void_p(x.data_ptr()), float(rtol), int(max_cycles),
                                 int(prec), ctypes.cast(infos, ctypes.c_void_p), _stream())
        out = [{k: getattr(i, k) for k, _ in SolveInfo._fields_} for i in infos]
        if rc != 0 and not (rc == -5 and not raise_on_noconv):
            check(rc)
        return x, out

    def set_graph(self, on: bool = True) -> None:
        """Replay the cycles of each solve from a captured HIP graph."""
        check(load().mlcr_solver_set_graph(self._h, 1 if on else 0))

    def graph_stats(self) -> dict:
        r, f = ctypes.c_longlong(), ctypes.c_longlong()
        check(load().mlcr_solver_graph_stats(self._h, ctypes.byref(r), ctypes.byref(f)))
        return {"replays": r.value, "fallbacks": f.value}

    def solve_pcg(self, b: torch.Tensor, x0: torch.Tensor | None = None, rtol: float = 1e-8,
                  max_iter: int = 50, prec: int = FP64, raise_on_noconv: bool = True):
        """Conjugate gradients with one CR-Cycle as the preconditioner;
        returns (x, infos) like solve()."""
        from ._lib import SolveInfo

        _dev(b, "b")
        nrhs = _batch(b, nalm(self.op.lmax), "b")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        infos = (SolveInfo * nrhs)()
        rc = load().pcg_solve(self._h, nrhs, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                              float(rtol), int(max_iter), int(prec), ctypes.cast(infos, ctypes.c_void_p),
                              _stream())
        out = [{k: getattr(i, k) for k, _ in SolveInfo._fields_} for i in infos]
        if rc != 0 and not (rc == -5 and not raise_on_noconv):
            check(rc)
        return x, out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().mlcr_solver_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prior_band_grad(op: Operator, lam: torch.Tensor, x: torch.Tensor, band, q=None) -> np.ndarray:
    """dL/dq_beta = sum_{l in beta, m} lam_lm x_lm / (q_beta C_l) over RHS and the
    operator's active modes (mlcr_prior_band_grad); band[l] = -1 or 0..B-1."""
    _dev(lam, "lam")
    _dev(x, "x")
    nrhs = _batch(lam, nalm(op.lmax), "lam")
    if _batch(x, nalm(op.lmax), "x") != nrhs:
        raise ValueError("lam and x must have the same batch size")
    band = np.ascontiguousarray(np.asarray(band, dtype=np.int32)[: op.lmax + 1])
    if band.size != op.lmax + 1:
        raise ValueError("band needs lmax+1 entries")
    nb = int(band.max()) + 1 if q is None else len(q)
    qa = None if q is None else np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    out = np.zeros(max(nb, 1), dtype=np.float64)
    check(load().mlcr_prior_band_grad(op.handle, nrhs, ctypes.c_void_p(lam.data_ptr()),
                                      ctypes.c_void_p(x.data_ptr()), band.ctypes.data, max(nb, 1),
                                      qa.ctypes.data if qa is not None else None, out.ctypes.data,
                                      _stream()))
    return out


def _ptrs(seq) -> "ctypes.Array":
    return (ctypes.c_void_p * len(seq))(*[ctypes.c_void_p(v) for v in seq])


def apply_A_grouped(ops, xs, prec: int = FP64, outs=None):
    """Top-level y_p = A_p x_p for a mixed batch (one operator per problem),
    run concurrently in the library; see include/mlcr.h."""
    n = len(ops)
    if n < 1 or len(xs) != n:
        raise ValueError("need one x per operator")
    ys = outs if outs is not None else [None] * n
    nr = (ctypes.c_int * n)()
    for p, (op, x) in enumerate(zip(ops, xs)):
        _dev(x, "x")
        nr[p] = _batch(x, nalm(op.lmax), "x")
        if nr[p] > op.max_nrhs:
            raise ValueError("nrhs exceeds the operator's max_nrhs")
        if ys[p] is None:
            ys[p] = torch.empty_like(x)
    check(load().apply_A_grouped(n, _ptrs([op.handle.value for op in ops]), ctypes.cast(nr, ctypes.c_void_p),
                                 _ptrs([x.data_ptr() for x in xs]), _ptrs([y.data_ptr() for y in ys]),
                                 int(prec), _stream()))
    return ys


def solve_grouped(solvers, bs, rtol: float = 1e-8, max_cycles: int = 50, prec: int = FP64,
                  raise_on_noconv: bool = True):
    """wcycle_solve for a mixed batch (one solver per problem, each at most
    once); returns (xs, infos) with infos[p] a list of dicts per RHS."""
    from ._lib import SolveInfo
    n = len(solvers)
    if n < 1 or len(bs) != n:
        raise ValueError("need one b per solver")
    nr = (ctypes.c_int * n)()
    xs = []
    for p, (S, b) in enumerate(zip(solvers, bs)):
        _dev(b, "b")
        nr[p] = _batch(b, nalm(S.op.lmax), "b")
        xs.append(torch.zeros_like(b))
    infos = (SolveInfo * sum(nr))()
    rc = load().wcycle_solve_grouped(n, _ptrs([S._h.value for S in solvers]), ctypes.cast(nr, ctypes.c_void_p),
                                     _ptrs([b.data_ptr() for b in bs]), _ptrs([x.data_ptr() for x in xs]),
                                     float(rtol), int(max_cycles), int(prec),
                                     ctypes.cast(infos, ctypes.c_void_p), _stream())
    flat = [{k: getattr(i, k) for k, _ in SolveInfo._fields_} for i in infos]
    out, o = [], 0
    for p in range(n):
        out.append(flat[o: o + nr[p]])
        o += nr[p]
    if rc != 0 and not (rc == -5 and not raise_on_noconv):
        check(rc)
    return xs, out


def nest2ring(nside: int, nest) -> np.ndarray:
    nest = np.ascontiguousarray(np.asarray(nest, dtype=np.int64))
    out = np.empty_like(nest)
    check(load().mlcr_nest2ring(int(nside), nest.size, nest.ctypes.data, out.ctypes.data))
    return out


def tile_graph(nside: int, max_nb: int = 12) -> dict:
    """Neighbour lists and sweep/probe colourings of the 8 x 8 nested tiles."""
    nt = 12 * (nside // 8) ** 2
    nb = np.empty((nt, max_nb), dtype=np.int32)
    sc = np.empty(nt, dtype=np.int32)
    pc = np.empty(nt, dtype=np.int32)
    ns, npr = ctypes.c_int(), ctypes.c_int()
    check(load().mlcr_tile_graph(int(nside), int(max_nb), nb.ctypes.data, sc.ctypes.data,
                                 pc.ctypes.data, ctypes.byref(ns), ctypes.byref(npr)))
    return {"nb": nb, "sweep_color": sc, "probe_color": pc, "n_sweep": ns.value,
            "n_probe": npr.value}


def ladder_plan(nside: int, lmax: int) -> dict:
    nl, nt, lb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ns = np.zeros(8, dtype=np.int32)
    lm = np.zeros(8, dtype=np.int32)
    nr = np.zeros(8, dtype=np.int32)
    check(load().mlcr_ladder_plan(int(nside), int(lmax), ctypes.byref(nl), ns.ctypes.data,
                                  lm.ctypes.data, nr.ctypes.data, ctypes.byref(nt), ctypes.byref(lb)))
    n = nl.value
    return {"nlevels": n, "nside": ns[:n].tolist(), "lmax": lm[:n].tolist(),
            "nrec": nr[:n].tolist(), "nrec_top": nt.value, "lmax_bottom": lb.value}


def cycle_counts(nrec, nrec_top: int, ncycles: int = 1) -> np.ndarray:
    nrec = np.ascontiguousarray(np.asarray(nrec, dtype=np.int32))
    nl = nrec.size
    out = np.zeros(4 * (nl + 2), dtype=np.int64)
    check(load().mlcr_cycle_counts(nl, nrec.ctypes.data, int(nrec_top), int(ncycles), out.ctypes.data))
    return out.reshape(nl + 2, 4)
