"""Host-side logic of bench.py (no GPU): the committed HBM counters apply only to
the kernel sources and workload they were taken on, and the all-cores oracle
baseline runs the oracle in worker processes over disjoint systems."""
import json
import os

import numpy as np

import bench


def test_traffic_counters_apply_only_to_their_sources(tmp_path, monkeypatch):
    digest = bench.source_digest()
    assert len(digest) == 64 and digest == bench.source_digest()
    rec = {"source_sha256": digest, "systems": 4096, "p": 1,
           "kernels": {"d32": {"hbm_bytes_per_launch": 123}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("d32", 1, 4096) == 123
    assert bench.measured_traffic("d16", 1, 4096) is None        # another class
    assert bench.measured_traffic("d32", 2, 4096) is None        # other segment counts
    assert bench.measured_traffic("d32", -1, 4096) is None       # mixed segment counts
    assert bench.measured_traffic("d32", 1, 1024) is None        # another workload
    f.write_text(json.dumps(dict(rec, source_sha256="0" * 64)))
    assert bench.measured_traffic("d32", 1, 4096) is None        # other kernel sources
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("d32", 1, 4096) is None


def test_committed_traffic_record_is_well_formed():
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    assert t["systems"] == 4096 and t["p"] == 1 and len(t["source_sha256"]) == 64
    for k in t["kernels"].values():
        assert k["hbm_bytes_per_launch"] > 0


def test_all_cores_oracle_covers_the_sample_once():
    csamp = np.random.default_rng(2).choice(4096, size=12, replace=False)
    sps, n = bench.oracle_all_cores(4096, csamp, max_workers=3)
    assert 1 <= n <= 3 and sps > 0
    parts = [list(csamp[w::n]) for w in range(n)]
    assert sorted(int(i) for p in parts for i in p) == sorted(int(i) for i in csamp)
