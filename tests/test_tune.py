"""Autotuner bookkeeping on the CPU: candidate grids, size classes and the
JSON cache (no GPU; timing runs are in test_gpu_tune.py)."""
import json

from paper_1910_05971_amd import tune


def test_candidates_cover_the_grid():
    small = tune.csr_candidates(1000, 5000)
    assert len(small) == len(tune.TAUS)  # no binned layout: thresholds only
    assert {c["frontier_tau"] for c in small} == set(tune.TAUS)
    big = tune.csr_candidates(1 << 24, 1 << 29)
    assert len(big) == len(tune.TAUS) * len(tune.BIN_CHOICES)
    assert len(tune.csr_candidates(1000, 5000, all_bins=True)) == len(big)
    for c in big:
        assert c["bin_span"] in (0, 8, 16, 32) and c["bin_shift"] in (0, 14, 15)


def test_size_class():
    assert tune.size_class(1 << 24, 536_865_336) == "n2^24_e2^29"
    assert tune.size_class(65536, 524_280) == "n2^16_e2^19"
    assert tune.size_class(0, 0) == "n2^0_e2^0"


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "t.json")
    rec = {"n": 10, "nnz": 20, "best": {"opts": {"frontier_tau": 0.1}, "ms": 1.0}}
    tune.store("csr", "devA", "n2^4_e2^5", rec, p)
    tune.store("csr", "devA", "n2^5_e2^5", rec, p)
    tune.store("batch", "devB", "n2^4_e2^5", rec, p)
    db = json.load(open(p))
    assert set(db) == {"devA", "devB"} and set(db["devA"]["csr"]) == {"n2^4_e2^5", "n2^5_e2^5"}
    assert tune.load(p)["devB"]["batch"]["n2^4_e2^5"]["best"]["opts"] == {"frontier_tau": 0.1}
    assert tune.load(str(tmp_path / "missing.json")) == {}
    (tmp_path / "bad.json").write_text("{not json")
    assert tune.load(str(tmp_path / "bad.json")) == {}
