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
