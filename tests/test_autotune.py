"""Host logic of the launch-shape autotuner (no GPU): the coordinate search,
the cache file and the cache-hit path."""
import json

from paper_1308_5299_amd import autotune as at

DEFAULT = {"adjoint_waves": 8, "synth_chains": 4, "ring_threads": 1024}


def test_choose_picks_the_fastest_value_of_each_tunable():
    calls = []

    def measure(cfg):
        calls.append(dict(cfg))
        return {"legendre_adjoint": 10.0 if cfg["adjoint_waves"] == 8 else 7.0,
                "legendre_synth": 5.0 if cfg["synth_chains"] == 4 else 6.0,
                "ring_apply": 3.0 if cfg["ring_threads"] == 1024 else 2.0,
                "unpack": 1.0 if cfg["adjoint_waves"] == 8 else 2.0}

    best, timings = at.choose(DEFAULT, measure)
    assert best == {"adjoint_waves": 4, "synth_chains": 4, "ring_threads": 512}
    assert len(calls) == 6
    # a choice is carried into the measurements of the later tunables
    assert all(c["adjoint_waves"] == 4 for c in calls[2:])
    # the adjoint's waves are judged with the unpack step that sums its chunks
    assert timings["adjoint_waves"] == {8: 11.0, 4: 9.0}


def test_choose_counts_the_unpack_against_more_chunks():
    def measure(cfg):
        four = cfg["adjoint_waves"] == 4
        return {"legendre_adjoint": 11.8 if four else 11.9, "unpack": 2.3 if four else 1.5,
                "legendre_synth": 8.0, "ring_apply": 6.0}

    best, _ = at.choose(DEFAULT, measure)
    assert best["adjoint_waves"] == 8


def test_choose_keeps_the_current_value_on_ties():
    current = {"adjoint_waves": 4, "synth_chains": 2, "ring_threads": 512}
    names = {n for ks in at.KERNEL.values() for n in ks}
    best, _ = at.choose(current, lambda cfg: {k: 1.0 for k in names})
    assert best == current


def test_cache_roundtrip_and_validation(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    key = at.cache_key(2048, 4096, 8, 2, "MI355X")
    assert key == "nside=2048,lmax=4096,nrhs=8,prec=bf16x3,device=MI355X"
    assert at.load_cache(path) == {}
    at.save_cache(path, {key: DEFAULT})
    assert at.load_cache(path) == {key: DEFAULT}
    assert at.valid(DEFAULT)
    assert not at.valid({"adjoint_waves": 6, "synth_chains": 4, "ring_threads": 1024})
    assert not at.valid({"adjoint_waves": 8})
    with open(path, "w") as f:
        f.write("{not json")
    assert at.load_cache(path) == {}


class _Geom:
    nside = 64

    def __init__(self):
        self.set = []

    def set_tuning(self, prec, **cfg):
        self.set.append((prec, cfg))


class _Op:
    lmax = 128

    def __init__(self):
        self.geom = _Geom()


def test_tune_sets_a_cached_choice_without_timing(tmp_path):
    path = str(tmp_path / "tune.json")
    cfg = {"adjoint_waves": 4, "synth_chains": 2, "ring_threads": 512}
    with open(path, "w") as f:
        json.dump({at.cache_key(64, 128, 8, 1, "dev"): cfg}, f)
    op = _Op()
    r = at.tune(op, 8, 1, cache_path=path, device="dev")
    assert r["cached"] and r["tuning"] == cfg
    assert op.geom.set == [(1, cfg)]
