"""The stored oracle sample the benchmark's error report uses
(tests/golden/bench_reference.json) is what the oracle gives on the benchmark
workloads' initial states: the small workload's entry is recomputed here."""
import json
import os

import numpy as np

import misa_workloads as w
import oracle

REF = os.path.join(os.path.dirname(__file__), "golden", "bench_reference.json")


def test_reference_matches_oracle_on_c1():
    ref = json.load(open(REF))
    e = ref["c1"]
    x, v, box, rec = w.make_state(w.CONFIGS["c1"])
    assert e["atoms"] == len(x) and e["workload"] == w.CONFIGS["c1"].name
    sample = np.asarray(e["sample"])
    got = oracle.eam_sampled(oracle.Potential(oracle.TABLE, tables=w.potential_samples()), x, box, sample)
    assert np.array_equal(got["F"], np.asarray(e["F"]))
    assert np.array_equal(got["rho"], np.asarray(e["rho"]))
    assert np.array_equal(got["npairs"], np.asarray(e["npairs"]))


def test_reference_covers_the_workloads():
    ref = json.load(open(REF))
    for key in ("c2", "c3"):
        cfg = w.CONFIGS[key]
        assert ref[key]["workload"] == cfg.name and ref[key]["atoms"] == 2 * cfg.n_cells ** 3
        assert len(ref[key]["F"]) == len(ref[key]["sample"]) == len(ref[key]["far"])
    boxes = w.make_batch(w.BATCH_CONFIGS["c4"], n_boxes=len(ref["c4"]))
    for e, b in zip(ref["c4"], boxes):
        assert e["cells"] == b[0] and max(e["sample"]) < len(b[1])
