"""Host logic of the autotuner: the JSON cache round trip and candidate records (no GPU)."""
import json

from paper_2603_25834_amd.autotune import Candidate, THREADS, _Cache


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    c = _Cache(path)
    assert c.get("k") is None
    c.put("k", {"best": {"threads": 512, "band_rows": 0, "grid": 0, "form": 1}, "us_per_step": 1.5})
    again = _Cache(path)
    assert again.get("k")["best"]["threads"] == 512
    assert Candidate(**again.get("k")["best"]) == Candidate(512)
    with open(path) as fh:
        assert "k" in json.load(fh)


def test_thread_set_matches_the_library():
    # the library instantiates the fused kernels for exactly these workgroup sizes
    assert THREADS == (128, 192, 256, 384, 512)
