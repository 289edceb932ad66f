"""Run-away capacity overflow (Algorithm 2: atoms that leave their sites go to the
clash set; the handle's capacity bounds it).  A step whose leavers do not fit is
undone: misa_step returns MISA_EOVERFLOW with the state exactly as at the start of
the failing step, bit for bit equal to a run of that many steps on a handle with
room, so the caller can move the state to a larger handle and go on."""
import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, MASS = w.A_FE, w.RC, w.DELTA, w.MASS_FE
TABLES = w.potential_samples()
N = 10
DT_MAX, DX_MAX = 1.0, 0.05


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _say(msg):
    print(msg, flush=True)


def _state(seed=3):
    """A 10^3-cell box with four 1 keV recoils: they leave their sites together,
    after about a dozen adaptive steps (0.05 A each)."""
    x, v, box = w.thermal_state(N, seed=seed)
    rec = w.add_recoils(x, v, box, 4, 1000.0, False, seed=seed)
    return x, v, rec


def _lattice(precision, cap, x, v, graph=False):
    from paper_2107_07866_amd import Lattice
    lat = Lattice(N, A, RC, DELTA, MASS, precision, runaway_capacity=cap)
    lat.set_tables(TABLES)
    lat.set_state(x, v)
    if graph:
        lat.set_graph(True)
    return lat


def _snapshot(lat):
    xg, vg = lat.get_state()
    return dict(x=xg, v=vg, F=lat.forces(), rho=lat.rho(), slots=lat.slots())


def _equal(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("precision,graph", [("fp64", False), ("fp32", False), ("fp32", True)])
def test_overflow_leaves_start_of_failing_step(torch_cuda, precision, graph):
    from paper_2107_07866_amd.misa import MisaError, MISA_EOVERFLOW
    x, v, rec = _state()
    small = _lattice(precision, 2, x, v, graph)
    with pytest.raises(MisaError) as ei:
        small.step(40, DT_MAX, DX_MAX)
    assert ei.value.code == MISA_EOVERFLOW
    st = ei.value.stats
    s = st["failed_step"]
    _say(f"{precision} graph={graph}: overflow at step {s}, {st['n_runaway']} run-aways, steps {st['steps']}")
    assert 0 < s < 40 and st["overflow"] == 1 and st["steps"] == s
    got = _snapshot(small)
    ref = _lattice(precision, 0, x, v, graph)
    rst = ref.step(s, DT_MAX, DX_MAX) if s > 0 else None
    want = _snapshot(ref)
    _equal(got, want, f"{precision} after {s} steps")
    for key in ("dt", "dt_next", "time", "vmax", "e_emb", "e_pair", "n_runaway"):
        assert st[key] == rst[key], (key, st[key], rst[key])
    # recounted from the state after the call (another summation order than the step's)
    assert abs(st["e_kin"] - rst["e_kin"]) <= 1e-12 * rst["e_kin"]
    # the next step of the reference is the one that overflowed: more leavers than 2
    rst2 = ref.step(1, DT_MAX, DX_MAX)
    assert rst2["n_runaway"] > 2
    # a second call on the small handle fails at its first step, state unchanged
    with pytest.raises(MisaError) as ei2:
        small.step(3, DT_MAX, DX_MAX)
    assert ei2.value.stats["failed_step"] == 0 and ei2.value.stats["steps"] == s
    _equal(_snapshot(small), want, "after the second call")
    # the state moves to a handle with room and goes on as the reference did
    big = _lattice(precision, 0, got["x"], got["v"], graph)
    big.step(1, DT_MAX, DX_MAX)
    ref_x, _ = ref.get_state()
    bx, _ = big.get_state()
    assert np.max(np.abs(bx - ref_x)) < 1e-9  # reloaded: forces recomputed from the same positions
    for lat in (small, ref, big):
        lat.close()


def test_batch_overflow_stops_only_its_box(torch_cuda):
    """In a batch, the box that overflows stops at the start of its failing step; the
    others run every step, each equal to its own single-box run."""
    from paper_2107_07866_amd import Batch
    from paper_2107_07866_amd.misa import MisaError
    states = [_state(seed) for seed in (3, 4, 5)]
    batch = Batch([N, N, N], A, RC, DELTA, MASS, runaway_capacity=[64, 2, 64])
    batch.set_tables(TABLES)
    for k, (x, v, _) in enumerate(states):
        batch.boxes[k].set_state(x, v)
    with pytest.raises(MisaError) as ei:
        batch.step(30, DT_MAX, DX_MAX)
    sts = ei.value.stats
    assert [st["overflow"] for st in sts] == [0, 1, 0]
    s = sts[1]["failed_step"]
    _say(f"batch box 1 stopped after {s} steps")
    assert 0 < s < 30 and sts[1]["steps"] == s and sts[0]["steps"] == 30
    for k, (x, v, _) in enumerate(states):
        ref = _lattice("fp32", 64, x, v)
        rst = ref.step(s if k == 1 else 30, DT_MAX, DX_MAX)
        _equal(_snapshot(batch.boxes[k]), _snapshot(ref), f"box {k}")
        for key in ("dt", "dt_next", "time", "n_runaway", "vmax"):
            assert sts[k][key] == rst[key], (k, key)
        assert abs(sts[k]["e_kin"] - rst["e_kin"]) <= 1e-12 * rst["e_kin"], k
        ref.close()
    batch.close()
