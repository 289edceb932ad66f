"""Writes bench_reference.json: oracle values on the initial states of the benchmark
workloads, for the benchmark's force-error report (which thereby never runs the
oracle itself).  Calls only the oracle and the seeded input generators:

    python tests/golden/make_bench_reference.py

Per workload, a seeded sample of atoms of the initial state (the state each timed
run starts from) with the oracle's exact cell-binned FP64 density, F'(rho), force
and in-range neighbour count (Eqs. eam_base and eam_force_ij, tables of Sec. 4.1),
and whether the atom lies farther than 2 rc from every recoil atom (the thermal
sub-sample).  C4: the same for three of its boxes."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import misa_workloads as w  # noqa: E402
import oracle  # noqa: E402

SAMPLE = {"c1": 200, "c2": 300, "c3": 1000}
C4_BOXES, C4_SAMPLE = 3, 150


def _entry(pot, x, box, sample, recoils):
    ref = oracle.eam_sampled(pot, x, box, sample)
    L = np.asarray(box)
    far = np.ones(len(sample), bool)
    for i in recoils:
        d = x[sample] - x[int(i)]
        d -= L * np.rint(d / L)
        far &= np.einsum("ij,ij->i", d, d) > (2 * w.RC) ** 2
    return {"sample": [int(i) for i in sample], "rho": ref["rho"].tolist(), "fp": ref["fp"].tolist(),
            "F": ref["F"].tolist(), "npairs": [int(k) for k in ref["npairs"]], "far": far.tolist()}


def main():
    pot = oracle.Potential(oracle.TABLE, tables=w.potential_samples())
    out = {"about": "oracle values on the initial states of the benchmark workloads; "
                    "written by tests/golden/make_bench_reference.py"}
    for name, m in SAMPLE.items():
        cfg = w.CONFIGS[name]
        x, v, box, rec = w.make_state(cfg)
        sample = np.random.default_rng(7).choice(len(x), size=min(m, len(x)), replace=False)
        out[name] = dict(workload=cfg.name, atoms=int(len(x)), **_entry(pot, x, box, sample, rec))
        print(name, len(x), "atoms", flush=True)
        del x, v
    boxes = w.make_batch(w.BATCH_CONFIGS["c4"], n_boxes=C4_BOXES)
    out["c4"] = []
    for k, (n, x, v, box, rec, _) in enumerate(boxes):
        sample = np.random.default_rng(k).choice(len(x), size=min(C4_SAMPLE, len(x)), replace=False)
        out["c4"].append(dict(box=k, cells=int(n), **_entry(pot, x, box, sample, rec)))
    with open(os.path.join(HERE, "bench_reference.json"), "w") as fh:
        json.dump(out, fh, separators=(",", ":"))


if __name__ == "__main__":
    main()
