"""GPU tests of batched replicas: misa_batch_step on many uneven boxes gives, bit for
bit, what misa_step gives on each box alone (the single-box path is itself checked
against the oracle in test_gpu_parity.py), and the batch's own energies agree with
the oracle on a sampled box."""
import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, MASS = w.A_FE, w.RC, w.DELTA, w.MASS_FE
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


def _cases():
    cfg = w.BATCH_CONFIGS["c4"]
    boxes = w.make_batch(cfg, 6)
    # plus a ragged, non-cubic box with a hot 2 keV recoil
    x, v, box = w.thermal_state((13, 11, 9), seed=77)
    rec = w.add_recoils(x, v, box, 1, 2000.0, True, seed=77)
    boxes.append(((13, 11, 9), x, v, box, rec, 2000.0))
    return cfg, boxes


def test_batch_equals_single_boxes(torch_cuda):
    torch = torch_cuda
    from paper_2107_07866_amd import Batch, Lattice
    cfg, boxes = _cases()
    cells = [b[0] for b in boxes]
    _say(f"batch of {len(cells)} boxes: {cells}")
    batch = Batch(cells, A, RC, DELTA, MASS)
    batch.set_tables(TABLES)
    for k, (_, x, v, _, _, _) in enumerate(boxes):
        batch.boxes[k].set_state(x, v)
    singles = []
    for (n, x, v, _, _, _) in boxes:
        lat = Lattice(n, A, RC, DELTA, MASS, "fp32")
        lat.set_tables(TABLES)
        lat.set_state(x, v)
        singles.append(lat)
    for rnd, nsteps in enumerate((1, 12, 7)):
        st_b = batch.step(nsteps, cfg.dt_max, cfg.dx_max)
        torch.cuda.synchronize()
        for k, lat in enumerate(singles):
            st = lat.step(nsteps, cfg.dt_max, cfg.dx_max)
            xb, vb = batch.boxes[k].get_state()
            xs, vs = lat.get_state()
            assert np.array_equal(xb, xs) and np.array_equal(vb, vs), (rnd, k)
            assert np.array_equal(batch.boxes[k].forces(), lat.forces()), (rnd, k)
            assert np.array_equal(batch.boxes[k].slots(), lat.slots()), (rnd, k)
            for key in ("dt", "dt_next", "time", "e_kin", "e_emb", "e_pair", "n_runaway", "vmax"):
                assert st_b[k][key] == st[key], (rnd, k, key, st_b[k][key], st[key])
        _say(f"round {rnd}: {nsteps} steps equal; run-aways {[s['n_runaway'] for s in st_b]}")
    for lat in singles:
        lat.close()
    batch.close()


def test_batch_energy_matches_oracle(torch_cuda, orc):
    """After a few batched steps, one box's energy and sampled forces against the oracle."""
    torch = torch_cuda
    from paper_2107_07866_amd import Batch
    cfg, boxes = _cases()
    boxes = boxes[:3]
    batch = Batch([b[0] for b in boxes], A, RC, DELTA, MASS)
    batch.set_tables(TABLES)
    for k, (_, x, v, _, _, _) in enumerate(boxes):
        batch.boxes[k].set_state(x, v)
    st = batch.step(5, cfg.dt_max, cfg.dx_max)
    torch.cuda.synchronize()
    pot = orc.Potential(orc.TABLE, tables=TABLES)
    for k in range(3):
        x, _ = batch.boxes[k].get_state()
        box = boxes[k][3]
        ref = orc.eam(pot, x, box, cells=True)
        F = batch.boxes[k].forces()
        ferr = np.abs(F - ref["F"]).max() / np.sqrt(np.mean(ref["F"] ** 2))
        e = st[k]["e_emb"] + st[k]["e_pair"]
        eerr = abs(e - (ref["e_emb"] + ref["e_pair"])) / len(x)
        _say(f"box {k}: force {ferr:.2e} energy/atom {eerr:.2e}")
        assert ferr < 1e-3 and eerr < 1e-5
    batch.close()


def test_batch_tile_shapes_keep_per_atom_results(torch_cuda):
    """Boxes on every tile shape (ragged sizes included): positions, velocities,
    forces and slots equal the single-box run bit for bit (each atom sums its
    stencil in the same order whatever the tiling); energies agree to rounding."""
    torch = torch_cuda
    from paper_2107_07866_amd import Batch, Lattice
    from paper_2107_07866_amd import misa as M
    cfg, boxes = _cases()
    cells = [b[0] for b in boxes]
    batch = Batch(cells, A, RC, DELTA, MASS)
    batch.set_tables(TABLES)
    for k, (_, x, v, _, _, _) in enumerate(boxes):
        batch.boxes[k].set_state(x, v)
        batch.set_tile_shape(k, k % len(M.MISA_TILE_SHAPES))
    _say("shapes " + str([M.MISA_TILE_SHAPES[batch.tile_shape(k)] for k in range(len(cells))]))
    singles = []
    for (n, x, v, _, _, _) in boxes:
        lat = Lattice(n, A, RC, DELTA, MASS, "fp32")
        lat.set_tables(TABLES)
        lat.set_state(x, v)
        singles.append(lat)
    for rnd, nsteps in enumerate((1, 9)):
        st_b = batch.step(nsteps, cfg.dt_max, cfg.dx_max)
        torch.cuda.synchronize()
        for k, lat in enumerate(singles):
            st = lat.step(nsteps, cfg.dt_max, cfg.dx_max)
            xb, vb = batch.boxes[k].get_state()
            xs, vs = lat.get_state()
            assert np.array_equal(xb, xs) and np.array_equal(vb, vs), (rnd, k)
            assert np.array_equal(batch.boxes[k].forces(), lat.forces()), (rnd, k)
            assert np.array_equal(batch.boxes[k].slots(), lat.slots()), (rnd, k)
            for key in ("dt", "dt_next", "time", "n_runaway", "vmax"):
                assert st_b[k][key] == st[key], (rnd, k, key)
            for key in ("e_kin", "e_emb", "e_pair"):
                assert abs(st_b[k][key] - st[key]) <= 1e-12 * abs(st[key]), (rnd, k, key, st_b[k][key], st[key])
        _say(f"round {rnd}: {nsteps} steps equal on every tile shape")
    for lat in singles:
        lat.close()
    batch.close()


def test_batch_autotune(torch_cuda):
    """The autotuner times both policies, keeps one, reports the steps it took, and
    the batch goes on matching single boxes advanced by the same steps."""
    torch = torch_cuda
    from paper_2107_07866_amd import Batch, Lattice
    cfg, boxes = _cases()
    boxes = boxes[:4]
    cells = [b[0] for b in boxes]
    batch = Batch(cells, A, RC, DELTA, MASS)
    batch.set_tables(TABLES)
    for k, (_, x, v, _, _, _) in enumerate(boxes):
        batch.boxes[k].set_state(x, v)
    rep = batch.autotune(3, cfg.dt_max, cfg.dx_max)
    _say(f"autotune: {rep}, shapes {[batch.tile_shape(k) for k in range(len(cells))]}")
    assert rep["policy"] in (0, 1) and rep["steps_done"] in (4, 8)
    assert all(m > 0 for m in rep["ms_per_step"])
    batch.step(4, cfg.dt_max, cfg.dx_max)
    torch.cuda.synchronize()
    for k, (n, x, v, _, _, _) in enumerate(boxes):
        lat = Lattice(n, A, RC, DELTA, MASS, "fp32")
        lat.set_tables(TABLES)
        lat.set_state(x, v)
        for _ in range(rep["steps_done"] // 4):  # per policy tried: 1 untimed step, then 3 timed
            lat.step(1, cfg.dt_max, cfg.dx_max)
            lat.step(3, cfg.dt_max, cfg.dx_max)
        lat.step(4, cfg.dt_max, cfg.dx_max)
        xb, vb = batch.boxes[k].get_state()
        xs, vs = lat.get_state()
        assert np.array_equal(xb, xs) and np.array_equal(vb, vs), k
        lat.close()
    batch.close()
