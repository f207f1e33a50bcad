"""Host logic of the launch-shape autotuner (no device needed)."""
from paper_2601_12941_amd import autotune


def test_default_tile_matches_the_library_rule():
    # N + 9: the 3-sample reach of the taps and 3 samples of drift room per side
    assert autotune.default_tile(21) == 30
    assert autotune.default_tile(31) == 40
    assert autotune.default_tile(41) == 50
    assert autotune.default_tile(51) == 60


def test_candidates_respect_the_window_and_wavefront_limits():
    for N in (15, 21, 31, 41, 51, 63):
        c = autotune.candidates(N)
        assert c, N
        for tps, ts in c:
            assert tps in (16, 32, 64, 128, 256) and tps >= N
            assert tps >= 64 or N <= 16     # packed subsets only for N <= 16
            assert N + 5 <= ts <= 96
    assert {t for t, _ in autotune.candidates(15)} == {16, 32, 64, 128, 256}
    assert {t for t, _ in autotune.candidates(15, shape=12)} == {64, 128, 256}
    assert sorted({s for _, s in autotune.candidates(31)}) == [36, 40, 48]
    assert sorted({s for _, s in autotune.candidates(63)}) == [68, 72, 80]


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "c.json"))
    assert autotune._load() == {}
    autotune._store({"k": {"threads_per_subset": 64}})
    assert autotune._load()["k"]["threads_per_subset"] == 64
