"""Host-side checks of the autotuner's candidate set and cache file (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1308_3290_amd import autotune  # noqa: E402


def test_candidates_start_with_the_reference_and_cover_the_tile_shapes():
    plain = autotune.candidates(False)
    full = autotune.candidates(True)
    assert plain[0] == autotune.REFERENCE and full[0] == autotune.REFERENCE
    assert len(plain) == 2 and all(c["launch"]["mode"] == 0 for c in plain)
    pers = [c["launch"] for c in full if c["launch"]["mode"] == 1]
    assert {p["b_tile"] for p in pers} == {1, 2, 4, 8}
    assert {p["f_tile"] for p in pers} == {1, 2, 4}
    assert {p["wg_per_cu"] for p in pers} == {0, 1}


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune._load(path) == {}
    autotune._store(path, {"k": {"setting": autotune.REFERENCE}})
    assert json.load(open(path))["k"]["setting"] == autotune.REFERENCE
    os.environ["CGP_TUNE_CACHE"] = path
    try:
        assert autotune.cache_path() == path
    finally:
        del os.environ["CGP_TUNE_CACHE"]
