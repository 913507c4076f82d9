"""The batched sweep's instances are a seeded draw; the committed table
(workloads/sweep64_instances.json) records them, so a change to the
generator or to NumPy's generator streams shows up here rather than as a
silently different benchmark workload (not GPU)."""
import json
import os

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sweep_instances_match_the_recorded_table():
    rec = json.load(open(os.path.join(ROOT, "workloads", "sweep64_instances.json")))
    assert rec["instances"] == W.batch_instance_table()
    sizes = [r["n"] for r in rec["instances"]]
    assert len(sizes) == 64 and set(sizes) <= {128, 192, 256, 384, 512}
    for r in rec["instances"]:
        assert 1.0 <= r["Gc"] <= 5.0
        assert r["l"] * r["n"] in (2.0, 4.0)
        assert 0.3 - 1.0 / r["n"] <= r["notch_end"] <= 0.6
