"""The autotuning cache (paper_2605_28684_amd/tuning.py) on the host: keys,
round trip through the JSON file, cached choices applied without timing,
out-of-range entries re-tuned, single-candidate targets skipped."""
import json
import types

import pytest

from paper_2605_28684_amd import romhip as R
from paper_2605_28684_amd import tuning as T


class FakeHandle:
    """Stands in for RomBatch: counts autotune calls, records set_tuning."""

    def __init__(self, ncand, best):
        self.cfg = types.SimpleNamespace(problem=1)
        self.precision, self.total_dof, self.r = 0, 3 * 262144, 10
        self.ncand, self.best = ncand, best
        self.tuned, self.set = [], {}

    def set_tuning(self, t, c):
        if c >= 0:
            assert c < self.ncand[t]
            self.set[t] = c
        return self.ncand[t]

    def autotune(self, t, q):
        self.tuned.append(t)
        self.set[t] = self.best[t]
        return self.best[t]


def test_key_buckets_and_fields():
    k = T.cache_key(R.TUNE_BT_PART, 1, 0, 786432, 10, "gfx950")
    assert k == "bt_part|p1|f0|n2^19|r10|gfx950"
    assert T.cache_key(R.TUNE_BT_PART, 1, 0, 1048575, 10, "gfx950") == k
    assert T.cache_key(R.TUNE_BT_PART, 1, 0, 1048576, 10, "gfx950") != k


def test_round_trip_cached_choices_skip_timing(tmp_path):
    path = str(tmp_path / "tune.json")
    ncand = {R.TUNE_RESIDUAL: 12, R.TUNE_DEIM_PASS: 3, R.TUNE_BT_PART: 3}
    best = {R.TUNE_RESIDUAL: 8, R.TUNE_DEIM_PASS: 2, R.TUNE_BT_PART: 1}
    h = FakeHandle(ncand, best)
    done = T.TuningCache(path).apply(h, q=object(), arch="gfx950")
    assert sorted(h.tuned) == sorted(ncand) and all(v[1] == "tuned" for v in done.values())
    data = json.load(open(path))
    assert data["version"] == 1 and len(data["choices"]) == 3
    h2 = FakeHandle(ncand, best)
    done2 = T.TuningCache(path).apply(h2, q=object(), arch="gfx950")
    assert h2.tuned == [] and h2.set == best
    assert all(v[1] == "cache" for v in done2.values())


def test_out_of_range_entry_is_retuned_and_single_candidates_skipped(tmp_path):
    path = str(tmp_path / "tune.json")
    c = T.TuningCache(path)
    key = T.cache_key(R.TUNE_RESIDUAL, 1, 0, 3 * 262144, 10, "gfx950")
    c.entries[key] = 99
    h = FakeHandle({R.TUNE_RESIDUAL: 12, R.TUNE_DEIM_PASS: 1, R.TUNE_BT_PART: 1},
                   {R.TUNE_RESIDUAL: 5, R.TUNE_DEIM_PASS: 0, R.TUNE_BT_PART: 0})
    done = c.apply(h, q=object(), arch="gfx950")
    assert h.tuned == [R.TUNE_RESIDUAL] and done == {"residual": (5, "tuned")}
    assert T.TuningCache(path).entries[key] == 5


def test_targets_that_need_q_are_skipped_without_it(tmp_path):
    h = FakeHandle({R.TUNE_RESIDUAL: 12, R.TUNE_DEIM_PASS: 3, R.TUNE_BT_PART: 3},
                   {R.TUNE_RESIDUAL: 1, R.TUNE_DEIM_PASS: 1, R.TUNE_BT_PART: 1})
    done = T.TuningCache(str(tmp_path / "t.json")).apply(h, q=None, arch="gfx950")
    assert list(done) == ["deim_pass"]


def test_wrong_version_is_rejected(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text(json.dumps({"version": 7, "choices": {}}))
    with pytest.raises(ValueError):
        T.TuningCache(str(p))
