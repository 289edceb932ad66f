"""misa_set_state_noalloc (placement scratch in a static device array, no
allocation) against misa_set_state, through the C ABI: slot tables, positions,
velocities and forces bit for bit, on two calls in a row on one handle, the
second with fewer atoms; the size limit and a non-finite input are refused."""
import ctypes as C

import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, M_FE = w.A_FE, w.RC, w.DELTA, w.MASS_FE
TABLES = w.potential_samples()
N_CELLS = 12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _say(msg):
    print(msg, flush=True)


def _states():
    """A thermal 12^3 box with an interstitial and two atoms far off their sites, then
    a smaller state of the same box: 300 atoms removed (vacancies), one moved off site."""
    x, v, box = w.thermal_state(N_CELLS, sigma=0.05, seed=31)
    x1 = np.vstack([x, [[2.5 * A + 0.03, 2.0 * A - 0.02, 3.0 * A + 0.01]]])
    v1 = np.vstack([v, [[0.01, -0.02, 0.005]]])
    x1[10] += [0.9, 0.1, -0.2]
    x1[400] += [-0.7, 0.6, 0.1]
    keep = np.ones(len(x), bool)
    keep[np.random.default_rng(5).choice(len(x), 300, replace=False)] = False
    x2, v2 = x[keep].copy(), v[keep].copy()
    x2[7] += [0.0, 0.8, 0.8]
    return [(x1, v1), (x2, v2)]


def _result(lat):
    import torch
    lat.compute()
    torch.cuda.synchronize()
    xg, vg = lat.get_state()
    return lat.slots(), xg, vg, lat.forces(), lat.rho()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_placement_equals_set_state(torch_cuda, precision):
    torch = torch_cuda
    from paper_2107_07866_amd import Lattice, misa as M
    lat = Lattice(N_CELLS, A, RC, DELTA, M_FE, precision)  # the no-alloc handle: both calls on it
    lat.set_tables(TABLES)
    for call, (x, v) in enumerate(_states()):
        _say(f"noalloc {precision} call {call}: {len(x)} atoms")
        ref = Lattice(N_CELLS, A, RC, DELTA, M_FE, precision)
        ref.set_tables(TABLES)
        ref.set_state(x, v)
        want = _result(ref)
        ref.close()
        xt = torch.tensor(x, dtype=torch.float64, device="cuda")
        vt = torch.tensor(v, dtype=torch.float64, device="cuda")
        M.misa_set_state_noalloc(lat.h, xt, vt)
        got = _result(lat)
        assert M.misa_atom_count(lat.h) == len(x)
        for name, a, b in zip(("slots", "x", "v", "F", "rho"), got, want):
            assert np.array_equal(a, b), (precision, call, name)
        # the off-site atoms (three, then one) went through the run-away list
        assert (got[0] < 0).sum() >= (3, 1)[call]
    lat.close()


def test_noalloc_refusals(torch_cuda):
    torch = torch_cuda
    from paper_2107_07866_amd import Lattice, misa as M
    lat = Lattice(N_CELLS, A, RC, DELTA, M_FE, "fp32")
    lat.set_tables(TABLES)
    x, v = _states()[1]
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    vt = torch.tensor(v, dtype=torch.float64, device="cuda")
    # beyond the scratch size: refused before any memory is touched
    rc = M.lib.misa_set_state_noalloc(lat.h, C.c_void_p(xt.data_ptr()), C.c_void_p(vt.data_ptr()),
                                      M.MISA_NOALLOC_MAX_ATOMS + 1)
    assert rc == M.MISA_EINVAL
    assert b"MISA_NOALLOC_MAX_ATOMS" in M.lib.misa_last_error(lat.h)
    bad = xt.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(Exception):
        M.misa_set_state_noalloc(lat.h, bad, vt)
    M.misa_set_state_noalloc(lat.h, xt, vt)  # the next call loads normally
    ref = Lattice(N_CELLS, A, RC, DELTA, M_FE, "fp32")
    ref.set_tables(TABLES)
    ref.set_state(x, v)
    assert np.array_equal(lat.slots(), ref.slots())
    ref.close()
    lat.close()
