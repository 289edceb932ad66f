"""GPU tests of graph replay (misa_set_graph): steps replayed from one captured
HIP graph equal launched steps bit for bit, across repeated replays with eager
work and synchronisations between them, a change of dt_max (a new capture),
new tables (the graph is dropped), run-away atoms, and each pair form."""
import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, M = w.A_FE, w.RC, w.DELTA, w.MASS_FE
TABLES = w.potential_samples()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _say(msg):
    print(msg, flush=True)


def _pair(n, precision, schedule, x, v):
    from paper_2107_07866_amd import Lattice
    lats = []
    for graph in (False, True):
        lat = Lattice(n, A, RC, DELTA, M, precision, runaway_capacity=512)
        lat.set_tables(TABLES)
        if schedule != "gather":
            lat.set_pair_schedule(schedule)
        lat.set_state(x, v)
        lat.set_graph(graph)
        lats.append(lat)
    return lats


@pytest.mark.parametrize("precision,schedule", [("fp64", "gather"), ("fp32", "gather"), ("fp32", "half")])
def test_graph_replay_equals_launched_steps(torch_cuda, precision, schedule):
    torch = torch_cuda
    n = 16
    x, v, box, _ = w.make_state(w.CONFIGS["c2"], n_cells=n)  # 1 keV recoil at the centre
    eager, graph = _pair(n, precision, schedule, x, v)
    plan = [(10, 1.0, 0.05), (7, 1.0, 0.05), (5, 0.5, 0.05), (1, 1.0, 0.05), (6, 1.0, 0.05), (12, 1.0, 0.05)]
    for rnd, (nsteps, dt_max, dx_max) in enumerate(plan):
        if rnd == 4:  # new tables drop the captured step
            for lat in (eager, graph):
                lat.set_tables(TABLES)
        st = [lat.step(nsteps, dt_max, dx_max) for lat in (eager, graph)]
        torch.cuda.synchronize()
        xe, ve = eager.get_state()
        xg, vg = graph.get_state()
        assert np.array_equal(xe, xg) and np.array_equal(ve, vg), (precision, schedule, rnd)
        for key in ("dt", "dt_next", "time", "e_kin", "e_emb", "e_pair", "n_runaway", "vmax", "steps"):
            assert st[0][key] == st[1][key], (precision, schedule, rnd, key, st[0][key], st[1][key])
        # eager work between the replays: a force evaluation on the current state
        e = [lat.compute() for lat in (eager, graph)]
        torch.cuda.synchronize()
        assert np.array_equal(eager.forces(), graph.forces())
        assert np.array_equal(e[0].cpu().numpy(), e[1].cpu().numpy())
        _say(f"{precision} {schedule} round {rnd}: {nsteps} steps equal, run-aways {st[1]['n_runaway']}")
    assert st[1]["n_runaway"] >= 1
    for lat in (eager, graph):
        lat.close()


def test_batch_graph_replay_equals_launched_steps(torch_cuda):
    """Batched steps replayed from a graph equal launched batched steps, also after
    tile shapes change (a new capture) and with eager work between the calls."""
    torch = torch_cuda
    from paper_2107_07866_amd import Batch
    cfg = w.BATCH_CONFIGS["c4"]
    boxes = w.make_batch(cfg, 5)
    cells = [b[0] for b in boxes]
    bats = []
    for graph in (False, True):
        bt = Batch(cells, A, RC, DELTA, M)
        bt.set_tables(TABLES)
        for k, b in enumerate(boxes):
            bt.boxes[k].set_state(b[1], b[2])
        bt.set_graph(graph)
        bats.append(bt)
    for rnd, nsteps in enumerate((8, 5, 1, 9)):
        if rnd == 2:
            for bt in bats:
                bt.set_tile_shape(1, 3)
        st = [bt.step(nsteps, cfg.dt_max, cfg.dx_max) for bt in bats]
        torch.cuda.synchronize()
        for k in range(len(cells)):
            xe, ve = bats[0].boxes[k].get_state()
            xg, vg = bats[1].boxes[k].get_state()
            assert np.array_equal(xe, xg) and np.array_equal(ve, vg), (rnd, k)
            for key in ("dt", "time", "e_kin", "e_emb", "e_pair", "n_runaway"):
                assert st[0][k][key] == st[1][k][key], (rnd, k, key)
        for bt in bats:  # eager work between the calls
            bt.boxes[0].forces()
        _say(f"batch round {rnd}: {nsteps} steps equal")
    for bt in bats:
        bt.close()
