"""GPU Wigner-Seitz defect counts (misa_defects) against the oracle's count of the
same positions: exact integers, on placed defect states and after a cascade."""
import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, MASS = w.A_FE, w.RC, w.DELTA, w.MASS_FE


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _lattice(n, precision="fp32"):
    from paper_2107_07866_amd import Lattice
    lat = Lattice(n, A, RC, DELTA, MASS, precision)
    lat.set_tables(w.potential_samples())
    return lat


def _check(lat, orc, n, tag):
    x, _ = lat.get_state()
    got = lat.defects()
    vac, inter, _ = orc.wigner_seitz(n, A, x)
    print(f"{tag}: gpu {got} oracle vacancies {vac} interstitials {inter}", flush=True)
    assert (got["vacancies"], got["interstitials"]) == (vac, inter)
    return got


def test_defects_of_placed_states(torch_cuda, orc):
    n = (9, 8, 10)
    x, v, _ = w.thermal_state(n, seed=21)
    rng = np.random.default_rng(21)
    L = np.array(n) * A
    cases = {
        "thermal": (x, v),
        "vacancies": (np.delete(x, [1, 50, 999], 0), np.delete(v, [1, 50, 999], 0)),
        "interstitials": (np.vstack([x, rng.uniform(0, 1, (7, 3)) * L]), np.vstack([v, np.zeros((7, 3))])),
    }
    y = x.copy()
    y[[5, 6, 700]] = rng.uniform(0, 1, (3, 3)) * L  # three atoms moved anywhere: Frenkel pairs or shuffles
    cases["frenkel"] = (y, v)
    for tag, (xx, vv) in cases.items():
        lat = _lattice(n)
        lat.set_state(xx, vv)
        _check(lat, orc, n, tag)
        lat.close()


def test_defects_after_a_cascade(torch_cuda, orc):
    n = (14, 14, 14)
    x, v, box = w.thermal_state(n, seed=22)
    w.add_recoils(x, v, box, 1, 1500.0, True, seed=22)
    lat = _lattice(n)
    lat.set_state(x, v)
    for k in range(4):
        lat.step(60, 1.0, 0.05)
        got = _check(lat, orc, n, f"after {60 * (k + 1)} steps")
    assert got["runaway"] > 0
    lat.close()
