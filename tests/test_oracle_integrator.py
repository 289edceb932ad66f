"""Pins of the oracle's time loop (Sec. 2.1, Fig. 1, read as velocity Verlet)."""
import numpy as np

import misa_workloads as w

A = w.A_FE


def _state(n=4, seed=21, sigma=0.05, T=300.0):
    return w.thermal_state(n, sigma=sigma, temperature=T, seed=seed)


def test_unit_constant(orc):
    assert abs(orc.acc_unit() - 9.648533215665326e-3) < 1e-17
    assert abs(orc.acc_unit() - w.ACC_A_FS2) < 1e-18


def test_time_reversibility(orc):
    P = orc.Potential(orc.ANALYTIC_SF)
    x0, v0, box = _state()
    x1, v1, F1, _ = orc.run(P, x0, v0, box, w.MASS_FE, 100, 1.0)
    x2, v2, F2, _ = orc.run(P, x1, -v1, box, w.MASS_FE, 100, 1.0, F=F1)
    assert np.max(np.abs(x2 - x0)) < 1e-9
    assert np.max(np.abs(v2 + v0)) < 1e-9


def test_energy_error_scales_as_dt_squared(orc):
    P = orc.Potential(orc.ANALYTIC_SF)
    x0, v0, box = _state(T=600.0, sigma=0.08)

    def max_err(dt, steps):
        _, _, _, log = orc.run(P, x0, v0, box, w.MASS_FE, steps, dt)
        e = log[:, 1] + log[:, 2] + log[:, 3]
        r0 = orc.eam(P, x0, box)
        e0 = orc.kinetic(v0, w.MASS_FE) + r0["e_emb"] + r0["e_pair"]
        return np.max(np.abs(e - e0))

    e1 = max_err(2.0, 50)
    e2 = max_err(1.0, 100)
    assert 3.5 < e1 / e2 < 4.5


def test_momentum_conservation(orc):
    P = orc.Potential(orc.ANALYTIC)
    x0, v0, box = _state(n=5, T=300.0)
    p0 = v0.sum(axis=0) * w.MASS_FE
    _, v1, _, _ = orc.run(P, x0, v0, box, w.MASS_FE, 20, 1.0)
    p1 = v1.sum(axis=0) * w.MASS_FE
    assert np.max(np.abs(p1 - p0)) <= 1e-12 * np.abs(v0).sum() * w.MASS_FE


def test_adaptive_dt_rule(orc):
    P = orc.Potential(orc.ANALYTIC)
    x0, v0, box = _state(n=5, T=300.0)
    v0 = v0.copy()
    v0[3] = [0.3, -0.4, 0.0]  # |v| = 0.5 A/fs
    _, _, _, log = orc.run(P, x0, v0, box, w.MASS_FE, 3, 1.0, dx_max=0.05)
    assert abs(log[0, 4] - 0.5) < 1e-15
    assert abs(log[0, 0] - 0.1) < 1e-15
    for dt, vmax in log[:, [0, 4]]:
        assert abs(dt - min(1.0, 0.05 / vmax)) < 1e-15
    # fixed step when dx_max = 0
    _, _, _, log2 = orc.run(P, x0, v0, box, w.MASS_FE, 2, 1.0, dx_max=0.0)
    assert (log2[:, 0] == 1.0).all()


def test_free_flight(orc):
    # two atoms farther apart than rc move ballistically: x(t) = x0 + v t exactly in the limit
    P = orc.Potential(orc.ANALYTIC)
    x0 = np.array([[5.0, 5.0, 5.0], [25.0, 25.0, 25.0]])
    v0 = np.array([[0.01, 0.0, -0.02], [0.0, 0.005, 0.0]])
    x1, v1, F, _ = orc.run(P, x0, v0, (60.0, 60.0, 60.0), w.MASS_FE, 10, 0.5)
    assert np.allclose(x1, x0 + 5.0 * v0, atol=1e-14)
    assert np.array_equal(v1, v0)


def test_thermal_state_temperature():
    x, v, box = w.thermal_state(6, temperature=300.0, seed=5)
    N = len(x)
    ke = 0.5 * w.MASS_FE * np.sum(v * v) / w.ACC_A_FS2
    T = 2 * ke / (3 * (N - 1) * w.KB_EV)
    assert abs(T - 300.0) < 1e-9
    assert np.max(np.abs(v.sum(axis=0))) < 1e-12
