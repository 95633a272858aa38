"""Host logic of the autotuner's cache: keys separate what changes the
choice (device, N rounded to a power of two, precision, periodicity, theta,
r_cut / r_s, curve), entries survive round trips and updates, and a broken
file reads as empty."""
from paper_2609_17658_amd import tune


def test_problem_key_buckets_and_fields():
    p = {"r_s": 1.25 / 256, "r_cut": 0.0, "theta": 0.5, "periodic": 1}
    k = tune.problem_key(2_097_152, p, "mixed")
    assert k == tune.problem_key(2_000_000, p, "mixed")          # same power-of-two bucket
    assert k != tune.problem_key(4_194_304, p, "mixed")
    assert k != tune.problem_key(2_097_152, p, "fp64")
    assert k != tune.problem_key(2_097_152, dict(p, theta=0.7), "mixed")
    assert k != tune.problem_key(2_097_152, dict(p, r_cut=6 * p["r_s"]), "mixed")
    assert k != tune.problem_key(2_097_152, dict(p, curve=1), "mixed")
    assert "rc/rs4.50" in k


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.cache_get("a", path) is None
    tune.cache_put("a", {"best": {"group_max": 64}}, path)
    tune.cache_put("b", {"best": {"group_max": 32}}, path)
    assert tune.cache_get("a", path) == {"best": {"group_max": 64}}
    tune.cache_put("a", {"best": {"group_max": 16}}, path)
    assert tune.cache_get("a", path)["best"]["group_max"] == 16
    assert tune.cache_get("b", path)["best"]["group_max"] == 32


def test_broken_cache_reads_empty(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert tune.cache_get("a", str(path)) is None
    tune.cache_put("a", {"x": 1}, str(path))
    assert tune.cache_get("a", str(path)) == {"x": 1}


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("OG_TUNE_CACHE", str(tmp_path / "t.json"))
    assert tune.cache_path() == str(tmp_path / "t.json")
