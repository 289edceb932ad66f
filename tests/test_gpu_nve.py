"""GPU NVE checks on the shifted-force tables (continuous energy at the cut-off):
total energy of the FP64 and FP32 forms over 400 steps of 1 fs stays within the
velocity-Verlet fluctuation the oracle shows on the same trajectory, without
drift, and the FP64 form's energies follow the oracle's step by step."""
import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, M = w.A_FE, w.RC, w.DELTA, w.MASS_FE


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _energies(lat, chunks, per):
    out = []
    for _ in range(chunks):
        st = lat.step(per, 1.0)
        out.append(st["e_kin"] + st["e_emb"] + st["e_pair"])
    return np.array(out)


def test_nve_energy_conservation(torch_cuda, orc):
    from paper_2107_07866_amd import Lattice
    tabs = w.potential_samples(variant="shifted")
    n = 6
    x, v, box = w.thermal_state(n, sigma=0.02, seed=31)
    N = len(x)
    chunks, per = 20, 20
    # oracle: the same 400 steps, energies logged every step
    p = orc.Potential(orc.TABLE, tables=tabs)
    _, _, _, log = orc.run(p, x, v, box, M, chunks * per, 1.0)
    e_orc = log[:, 1] + log[:, 2] + log[:, 3]
    fluct = float(np.max(np.abs(e_orc - e_orc[0])))
    print(f"oracle: max |E - E0| {fluct / N:.2e} eV/atom over {chunks * per} steps", flush=True)
    for prec in ("fp64", "fp32"):
        lat = Lattice(n, A, RC, DELTA, M, prec)
        lat.set_tables(tabs)
        lat.set_state(x, v)
        e = _energies(lat, chunks, per)
        torch_cuda.cuda.synchronize()
        ref = e_orc[per - 1::per]
        dev = float(np.max(np.abs(e - e[0])))
        drift = abs(float(np.mean(e[-5:]) - np.mean(e[:5])))
        diff = float(np.max(np.abs(e - ref)))
        print(f"{prec}: max |E - E0| {dev / N:.2e} eV/atom, drift {drift / N:.2e} eV/atom, "
              f"max |E - E_oracle| {diff / N:.2e} eV/atom", flush=True)
        assert dev <= 2.0 * fluct + 1e-6 * N, prec
        assert drift <= fluct + 1e-6 * N, prec
        if prec == "fp64":
            assert diff <= 1e-9 * N, diff
        else:
            assert diff <= 1e-5 * N, diff
        lat.close()
