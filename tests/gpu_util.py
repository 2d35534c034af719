"""Helpers for GPU tests (torch device memory around the C ABI)."""
import numpy as np
import torch


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel2(a, b) -> float:
    """||a - b||_2 / ||b||_2 over the whole array."""
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b) -> float:
    """max |a - b| / max |b|: the per-element bar, so that one wrong ring,
    order or pixel cannot hide under the 2-norm of a large output."""
    a = np.asarray(a); b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def parity(a, b) -> float:
    """The larger of the relative 2-norm and the per-element relative error;
    every parity bar applies to both."""
    return max(rel2(a, b), maxrel(a, b))


def elem_bar(tol: float, lmax: int, fp64: bool) -> float:
    """Per-element bar that goes with a 2-norm bar `tol`.  On the float64 path
    both sides generate lambda_lm by a forward three-term recurrence whose
    rounding error grows about linearly with the number of steps, so one output
    value (a 4-pixel polar ring, say) can differ by ~lmax u: the bar, met per
    element at lmax <= 512, scales with lmax / 512.  On the mixed paths the
    contraction's own rounding dominates and the bar is the path's tolerance."""
    return tol * (max(1.0, lmax / 512.0) if fp64 else 1.0)


def check(got, want, tol: float, lmax: int = 0, fp64: bool = False, slack: float = 1.0):
    """(ok, (rel2, maxrel)) against the 2-norm bar tol and its per-element bar."""
    e2, em = rel2(got, want), maxrel(got, want)
    return e2 <= slack * tol and em <= slack * elem_bar(tol, lmax, fp64), (e2, em)
