"""GPU tests of the half-stencil pair schedule (Newton's third law, Sec. 4.2: each
pair evaluated once, tiles run in 8 colours, partner writes in phases): forces,
densities and energies against the CPU oracle, agreement with the gather
schedule to float32 rounding, bit-reproducibility, a recoil trajectory with
run-away atoms, and the calls it must refuse."""
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


def _lattice(n, schedule, precision="fp32", cap=0):
    from paper_2107_07866_amd import Lattice
    lat = Lattice(n, A, RC, DELTA, M, precision, runaway_capacity=cap)
    lat.set_tables(TABLES)
    lat.set_pair_schedule(schedule)
    return lat


def _ferr(F, ref):
    scale = max(float(np.sqrt(np.mean(ref ** 2))), 1e-3)
    return float(np.max(np.abs(F - ref))) / scale


def _states():
    """Cubic C1 box (one tile per colour), a non-cubic box with several tiles per
    colour, and the latter with a vacancy, an interstitial and a close pair."""
    x1, v1, box1, _ = w.make_state(w.CONFIGS["c1"])
    n2 = (32, 16, 48)
    x2, v2, box2 = w.thermal_state(n2, sigma=0.08, seed=11)
    L = np.asarray(box2)
    keep = np.ones(len(x2), bool)
    keep[[3, 4100]] = False  # two vacancies
    xd = np.vstack([x2[keep], [[0.25 * A, 0.25 * A, 0.5 * A]], [(x2[9] + [0.9, 0.0, 0.0]) % L]])
    vd = np.vstack([v2[keep], np.zeros((2, 3))])
    return [("c1", 16, x1, v1, box1), ("non-cubic", n2, x2, v2, box2), ("defects", n2, xd, vd, box2)]


def test_half_state_against_oracle_and_gather(torch_cuda, orc):
    import torch
    pot = orc.Potential(orc.TABLE, tables=TABLES)
    for name, n, x, v, box in _states():
        _say(f"half schedule, {name} box {n}, {len(x)} atoms")
        out = {}
        for sched in ("gather", "half"):
            lat = _lattice(n, sched, cap=64)
            lat.set_state(x, v)
            e = lat.compute()
            torch.cuda.synchronize()
            out[sched] = (lat.forces(), lat.rho(), lat.fprime(), e.cpu().numpy())
            lat.close()
        ref = orc.eam(pot, x, box)
        F, rho, fp, e = out["half"]
        nz = ref["rho"] > 0
        ferr = _ferr(F, ref["F"])
        rerr = float(np.max(np.abs(rho[nz] - ref["rho"][nz]) / ref["rho"][nz]))
        eerr = abs(float(e.sum()) - ref["e_emb"] - ref["e_pair"]) / len(x)
        gerr = _ferr(F, out["gather"][0])
        grho = float(np.max(np.abs(rho[nz] - out["gather"][1][nz]) / ref["rho"][nz]))
        _say(f"  vs oracle: force {ferr:.2e} rho {rerr:.2e} energy/atom {eerr:.2e}; "
             f"vs gather: force {gerr:.2e} rho {grho:.2e}")
        assert ferr < 1e-3 and rerr < 1e-5 and eerr < 1e-5, (name, ferr, rerr, eerr)
        assert gerr < 1e-4 and grho < 1e-5, (name, gerr, grho)
        # Newton's third law holds term by term in the half schedule
        assert np.max(np.abs(F.sum(axis=0))) <= 1e-5 * np.abs(F).sum(), name


def test_half_is_bit_reproducible(torch_cuda):
    import torch
    _say("half schedule reproducibility")
    x, v, box = w.thermal_state((32, 16, 16), sigma=0.06, seed=21)
    runs = []
    for _ in range(2):
        lat = _lattice((32, 16, 16), "half")
        lat.set_state(x, v)
        lat.compute()
        F1 = lat.forces()
        st = lat.step(8, 1.0)
        xg, vg = lat.get_state()
        torch.cuda.synchronize()
        runs.append((F1, xg, vg, st["e_emb"] + st["e_pair"]))
        lat.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    assert runs[0][3] == runs[1][3]


def test_half_recoil_trajectory(torch_cuda, orc):
    """1 keV recoil on a 16^3 box: run-away atoms, adaptive dt and the separate
    final kick of the half schedule against the FP64 oracle."""
    _say("half schedule recoil trajectory")
    pot = orc.Potential(orc.TABLE, tables=TABLES)
    n = 16
    x, v, box, _ = w.make_state(w.CONFIGS["c2"], n_cells=n)
    lat = _lattice(n, "half", cap=256)
    lat.set_state(x, v)
    st = lat.step(30, 1.0, 0.05)
    xg, vg = lat.get_state()
    xo, vo, _, log = orc.run(pot, x, v, box, M, 30, 1.0, dx_max=0.05, cells=True)
    L = np.asarray(box)
    d = xg - xo
    d -= L * np.rint(d / L)
    _say(f"  max |dx| {np.max(np.abs(d)):.2e} A, dt {st['dt']:.6f} vs {log[-1, 0]:.6f}, "
         f"run-aways {st['n_runaway']}, e_kin {st['e_kin']:.6f} vs {log[-1, 1]:.6f}")
    assert st["n_runaway"] >= 1
    assert np.max(np.abs(d)) < 1e-4
    assert abs(st["dt"] - log[-1, 0]) < 1e-5 * log[-1, 0]
    assert abs(st["e_kin"] - log[-1, 1]) < 1e-5 * abs(log[-1, 1])
    epot = st["e_emb"] + st["e_pair"]
    assert abs(epot - log[-1, 2] - log[-1, 3]) < 1e-5 * abs(log[-1, 2] + log[-1, 3])
    ke = 0.5 * M * float(np.sum(vg * vg)) / w.ACC_A_FS2
    assert abs(st["e_kin"] - ke) < 1e-10 * ke
    lat.close()


def test_half_schedule_refusals(torch_cuda):
    from paper_2107_07866_amd import Lattice
    _say("half schedule refusals")
    for n, prec in (((16, 16, 16), "fp64"), ((13, 11, 9), "fp32"), ((16, 16, 24), "fp32")):
        lat = Lattice(n, A, RC, DELTA, M, prec)
        with pytest.raises(RuntimeError):
            lat.set_pair_schedule("half")
        lat.set_pair_schedule("gather")
        lat.close()
    with pytest.raises(ValueError):
        lat = Lattice(16, A, RC, DELTA, M, "fp32")
        try:
            lat.set_pair_schedule("third")
        finally:
            lat.close()
