"""Autotuner for the launch shapes of the transform kernels.

For one workload (geometry, band limit, right-hand sides per launch,
arithmetic path) the tuner times every value of each tunable of
``mlcr_geom_set_tuning`` on full operator applies with the library's kernel
timers, keeps the fastest, and caches the choice in a JSON file keyed by
workload and device.  The tunables act on separate kernels -- adjoint waves
per workgroup on the Legendre adjoint and on the unpack step that adds its
split-K chunks (fewer waves, more chunks), recurrence chains per lane on the
Legendre synthesis, threads per workgroup on the ring step -- so each is
chosen by the time of the kernels it acts on, with the others held at their
current values (a coordinate search; ties keep the current value).

The tuner only selects among launch shapes the library already provides;
every choice computes the same result up to rounding order.
"""
from __future__ import annotations

import json
import os
import tempfile
from typing import Callable

# value lists: the library's default first
CANDIDATES = {
    "adjoint_waves": (8, 4),
    "synth_chains": (4, 2),
    "ring_threads": (1024, 512),
}
# the library timers each tunable is judged by (their sum)
KERNEL = {
    "adjoint_waves": ("legendre_adjoint", "unpack"),
    "synth_chains": ("legendre_synth",),
    "ring_threads": ("ring_apply",),
}
PREC_NAMES = {0: "fp64", 1: "fp32", 2: "bf16x3"}


def cache_key(nside: int, lmax: int, nrhs: int, prec: int, device: str = "") -> str:
    """Key of one workload in the cache file."""
    return (f"nside={int(nside)},lmax={int(lmax)},nrhs={int(nrhs)},"
            f"prec={PREC_NAMES.get(int(prec), str(prec))},device={device}")


def load_cache(path: str | None) -> dict:
    """The cache file as a dict ({} if absent or unreadable)."""
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return {}
    return d if isinstance(d, dict) else {}


def save_cache(path: str, cache: dict) -> None:
    """Write the cache file atomically (temporary file, then rename)."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def valid(cfg: dict) -> bool:
    """Whether a cached entry names one candidate for every tunable."""
    return (isinstance(cfg, dict) and set(cfg) == set(CANDIDATES)
            and all(cfg[k] in CANDIDATES[k] for k in CANDIDATES))


def choose(current: dict, measure: Callable[[dict], dict]) -> tuple[dict, dict]:
    """Coordinate search over CANDIDATES.

    measure(cfg) -> {timer name: ms per launch} for one configuration.
    Returns (best configuration, {tunable: {value: ms}})."""
    best = {k: current[k] for k in CANDIDATES}
    timings = {}
    for name, values in CANDIDATES.items():
        order = [best[name]] + [v for v in values if v != best[name]]
        res = {}
        for v in order:
            cfg = dict(best)
            cfg[name] = v
            ms = measure(cfg)
            res[v] = float(sum(ms[k] for k in KERNEL[name]))
        best[name] = min(order, key=lambda v: res[v])     # first of equal times: current
        timings[name] = res
    return best, timings


def tune(op, nrhs: int, prec: int, reps: int = 3, cache_path: str | None = None,
         device: str | None = None, seed: int = 0) -> dict:
    """Tune the launch shapes of ``op``'s geometry for applies of ``nrhs``
    right-hand sides in arithmetic path ``prec`` and leave them set.

    With ``cache_path``, a cached choice for the same workload and device is
    set without timing, and a new choice is stored.  Returns
    {"tuning": cfg, "cached": bool, "timings_ms": {...}}.
    """
    g = op.geom
    if device is None:
        import torch
        device = torch.cuda.get_device_name(0) if torch.cuda.is_available() else ""
    key = cache_key(g.nside, op.lmax, nrhs, prec, device)
    cache = load_cache(cache_path)
    if key in cache and valid(cache[key]):
        cfg = cache[key]
        g.set_tuning(prec, **cfg)
        return {"tuning": dict(cfg), "cached": True, "timings_ms": {}}

    import torch
    from .api import KernelTimer, apply_A
    gen = torch.Generator(device="cuda").manual_seed(int(seed))
    x = torch.randn(int(nrhs), (op.lmax + 1) ** 2, dtype=torch.float64, device="cuda",
                    generator=gen)
    y = torch.empty_like(x)

    def measure(cfg: dict) -> dict:
        g.set_tuning(prec, **cfg)
        apply_A(op, x, prec=prec, out=y)               # warm-up: tables and workspaces
        torch.cuda.synchronize()
        with KernelTimer() as kt:
            for _ in range(int(reps)):
                apply_A(op, x, prec=prec, out=y)
            torch.cuda.synchronize()
        return {k: v[0] / v[1] for k, v in kt.result.items()}

    best, timings = choose(g.get_tuning(prec), measure)
    g.set_tuning(prec, **best)
    if cache_path:
        cache[key] = best
        save_cache(cache_path, cache)
    return {"tuning": best, "cached": False,
            "timings_ms": {k: {str(v): round(t, 4) for v, t in r.items()}
                           for k, r in timings.items()}}
