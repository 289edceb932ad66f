"""Checkpoint and resume: a run stopped, saved, loaded into a fresh handle and
continued equals the uninterrupted run bit for bit (positions, velocities, forces,
slots, run-away list, statistics).  Through misa_get_state / misa_set_state the
continuation agrees within rounding only: positions travel as absolute
coordinates and the site-relative displacements come back to ~1e-15 A."""
import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, MASS = w.A_FE, w.RC, w.DELTA, w.MASS_FE
TABLES = w.potential_samples()
N = 12
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


def _lattice(precision, tables=TABLES):
    from paper_2107_07866_amd import Lattice
    lat = Lattice(N, A, RC, DELTA, MASS, precision)
    lat.set_tables(tables)
    return lat


def _snapshot(lat):
    xg, vg = lat.get_state()
    return dict(x=xg, v=vg, F=lat.forces(), slots=lat.slots())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_resume_bit_identical(torch_cuda, precision):
    x, v, box = w.thermal_state(N, seed=9)
    w.add_recoils(x, v, box, 1, 1000.0, True, seed=9)  # run-away atoms in the saved state
    ref = _lattice(precision)
    ref.set_state(x, v)
    ref.step(15, DT_MAX, DX_MAX)  # odd: the current copy of u, v is the second one
    ref.step(5, DT_MAX, DX_MAX)
    want_st = ref.step(10, DT_MAX, DX_MAX)
    want = _snapshot(ref)

    run = _lattice(precision)
    run.set_state(x, v)
    run.step(15, DT_MAX, DX_MAX)
    st_mid = run.step(5, DT_MAX, DX_MAX)
    buf = run.save_checkpoint()
    run.close()
    _say(f"{precision}: checkpoint of {buf.nbytes} bytes after 20 steps, {st_mid['n_runaway']} run-aways")
    assert st_mid["n_runaway"] >= 1
    back = _lattice(precision)
    back.load_checkpoint(buf)
    got_st = back.step(10, DT_MAX, DX_MAX)
    got = _snapshot(back)
    for k in want:
        assert np.array_equal(got[k], want[k]), (precision, k)
    for k in ("dt", "dt_next", "time", "steps", "n_runaway", "vmax", "e_emb", "e_pair"):
        assert got_st[k] == want_st[k], (precision, k, got_st[k], want_st[k])

    # through positions and velocities: equal within rounding
    via = _lattice(precision)
    via.set_state(*_snapshot_state_at(precision, x, v, 20))
    via.step(10, DT_MAX, DX_MAX)
    xv, _ = via.get_state()
    d = xv - want["x"]
    d -= np.asarray(box) * np.rint(d / np.asarray(box))
    _say(f"  via get_state/set_state: max |dx| {np.max(np.abs(d)):.1e} A after 10 more steps")
    assert np.max(np.abs(d)) < 1e-8
    for lat in (ref, back, via):
        lat.close()


def _snapshot_state_at(precision, x, v, nsteps):
    lat = _lattice(precision)
    lat.set_state(x, v)
    lat.step(nsteps, DT_MAX, DX_MAX)
    out = lat.get_state()
    lat.close()
    return out


def test_checkpoint_refusals(torch_cuda):
    from paper_2107_07866_amd import Lattice
    from paper_2107_07866_amd.misa import MisaError
    x, v, box = w.thermal_state(N, seed=9)
    lat = _lattice("fp32")
    lat.set_state(x, v)
    buf = lat.save_checkpoint()
    other = Lattice(N + 1, A, RC, DELTA, MASS, "fp32")  # another box
    other.set_tables(TABLES)
    with pytest.raises(MisaError):
        other.load_checkpoint(buf)
    fp64 = _lattice("fp64")  # another precision
    with pytest.raises(MisaError):
        fp64.load_checkpoint(buf)
    shifted = _lattice("fp32", tables=w.potential_samples(variant="shifted"))  # other tables
    with pytest.raises(MisaError):
        shifted.load_checkpoint(buf)
    bad = buf.copy()
    bad[:8] = 0
    with pytest.raises(MisaError):
        lat.load_checkpoint(bad)
    for h in (lat, other, fp64, shifted):
        h.close()
