"""The benchmark's reporting arithmetic, on the host: work counts, the
roofline of the dominant kernel, the method's minimum bytes, the counter
tables it quotes, and the one-GPU guard.  No GPU and no library needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads  # noqa: E402


def test_useful_flops_full_triangle():
    # 4 flops per (l, m, ring pair, RHS) over 0 <= m <= l <= lmax, 2 N_side pairs
    nside, lmax, R = 2048, 4096, 8
    ntri = sum(lmax - m + 1 for m in range(lmax + 1))
    assert bench.legendre_useful_flops(nside, lmax, R) == 4.0 * ntri * 2 * nside * R
    assert bench.legendre_useful_flops(nside, lmax, R) == 1100317065216.0
    # one recurrence pass (a multiply and an FMA per step) per chunk of 8 RHS
    assert bench.recurrence_flops(nside, lmax, 8) == bench.recurrence_flops(nside, lmax, 1)
    assert bench.recurrence_flops(nside, lmax, 9) == 2 * bench.recurrence_flops(nside, lmax, 8)


def test_min_bytes_two_stage_round_trip():
    nside, lmax, R = 2048, 4096, 8
    nrings, npix, nalm = 4 * nside - 1, 12 * nside * nside, (lmax + 1) ** 2
    f32 = 8.0 * nrings * (lmax + 1) * R
    assert bench.min_bytes("legendre_synth", nside, lmax, R, "fp32") == 8.0 * nalm * R + f32
    assert bench.min_bytes("legendre_adjoint", nside, lmax, R, "bf16x3") == f32 + 16.0 * nalm * R
    assert bench.min_bytes("ring_apply", nside, lmax, R, "fp64") == 4 * f32 + 8.0 * npix
    assert bench.min_bytes("unpack", nside, lmax, R, "fp32") is None


@pytest.mark.parametrize("path", ["fp32", "fp64", "bf16x3"])
def test_roofline_of_the_dominant_kernel(path):
    cfg = workloads.get_config("c5")
    kernels = {"pack": 0.45, "legendre_synth": 12.0, "ring_apply": 5.3,
               "legendre_adjoint": 14.0, "unpack": 1.5}
    roof = bench.roofline(kernels, cfg, 8, path)
    assert roof["kernel"] == "legendre_adjoint"
    useful = bench.legendre_useful_flops(cfg.nside, cfg.lmax, 8)
    if path == "bf16x3":
        assert roof["bound"] == "alu" and roof["peak"] == 78.6
        assert roof["achieved"] == pytest.approx(
            bench.recurrence_flops(cfg.nside, cfg.lmax, 8) / 14e-3 / 1e12)
        assert roof["useful_frac_of_bf16_peak"] == pytest.approx(useful / 14e-3 / 2.5e15)
    else:
        assert roof["bound"] == "mfma"
        assert roof["peak"] == (78.6 if path == "fp64" else 157.3)
        assert roof["achieved"] == pytest.approx(useful / 14e-3 / 1e12)
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"])
    # the quoted counters belong to this kernel, path and workload, and are
    # at least the method's minimum bytes
    assert roof["traffic"] is not None and roof["traffic"] >= roof["min_bytes"]
    assert 0.0 < roof["mfma_busy_counters"] < 1.0


def test_roofline_hbm_bound_kernel():
    cfg = workloads.get_config("c5")
    roof = bench.roofline({"ring_apply": 5.0, "pack": 0.4}, cfg, 8, "fp32")
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    mb = bench.min_bytes("ring_apply", cfg.nside, cfg.lmax, 8, "fp32")
    assert roof["achieved"] == pytest.approx(mb / 5e-3 / 1e9)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0)


def test_counter_tables_cover_the_benchmarked_kernels():
    for (name, path, wl, R), v in bench.MEASURED_TRAFFIC.items():
        assert wl == "c5" and R == 8
        assert v >= bench.min_bytes(name, 2048, 4096, R, path)
    for key, busy in bench.MEASURED_MFMA_BUSY.items():
        assert key in bench.MEASURED_TRAFFIC and 0.0 < busy < 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
