"""Pins of the oracle's EAM densities, energies and forces (Sec. 2.2).

Closed forms (perfect-lattice shell sums, a two-atom cluster), invariants
(inversion symmetry, Newton's third law), finite differences of the energy and
an exact cell-binned re-derivation of the brute-force pair set.
"""
import numpy as np
import pytest

import misa_workloads as w

A = w.A_FE
# BCC shells within rc = 5.0: (|d|/a, multiplicity)
SHELLS = [(np.sqrt(3) / 2, 8), (1.0, 6), (np.sqrt(2), 12), (np.sqrt(11) / 2, 24), (np.sqrt(3), 8)]


def _closed_form(f, phi, F):
    rho0 = sum(m * f(s * A) for s, m in SHELLS)
    e = F(rho0) + 0.5 * sum(m * phi(s * A) for s, m in SHELLS)
    return rho0, e


def _analytic_numpy(shifted=False):
    f = lambda r: np.exp(-3 * (r / 2.47 - 1))
    df = lambda r: -(3 / 2.47) * np.exp(-3 * (r / 2.47 - 1))
    phi = lambda r: 0.4 * (np.exp(-3.2 * (r - 2.5)) - 2 * np.exp(-1.6 * (r - 2.5)))
    dphi = lambda r: 0.4 * (-3.2 * np.exp(-3.2 * (r - 2.5)) + 3.2 * np.exp(-1.6 * (r - 2.5)))
    if shifted:
        f0, phi0 = f, phi
        f = lambda r: f0(r) - f0(5.0) - (r - 5.0) * df(5.0)
        phi = lambda r: phi0(r) - phi0(5.0) - (r - 5.0) * dphi(5.0)
    F = lambda rho: -np.sqrt(rho)
    return f, phi, F


@pytest.mark.parametrize("n", [4, 5, 6])
def test_perfect_lattice_closed_form(orc, n):
    x = w.bcc_positions(n)
    box = (n * A,) * 3
    for mode, shifted in ((orc.ANALYTIC, False), (orc.ANALYTIC_SF, True)):
        P = orc.Potential(mode)
        r = orc.eam(P, x, box, want_pairs=True)
        rho0, ec = _closed_form(*_analytic_numpy(shifted))
        assert np.max(np.abs(r["rho"] - rho0)) < 1e-12 * rho0
        assert abs((r["e_emb"] + r["e_pair"]) / len(x) - ec) < 1e-12
        assert (r["npairs"] == 58).all()
        assert np.max(np.abs(r["F"])) < 1e-12  # inversion symmetry
    # the printed reference values
    rho0, ec = _closed_form(*_analytic_numpy(False))
    assert abs(rho0 - 15.4520271188193) < 1e-12 and abs(ec - (-7.22334604804693)) < 1e-12


def test_table_mode_perfect_lattice(orc):
    x = w.bcc_positions(5)
    box = (5 * A,) * 3
    Pt = orc.Potential(orc.TABLE, tables=w.potential_samples())
    r = orc.eam(Pt, x, box)
    rho0, ec = _closed_form(*_analytic_numpy(False))
    assert np.max(np.abs(r["rho"] - rho0)) < 1e-9
    assert abs((r["e_emb"] + r["e_pair"]) / len(x) - ec) < 1e-9
    assert np.max(np.abs(r["F"])) < 1e-12


def test_two_atom_cluster(orc):
    P = orc.Potential(orc.ANALYTIC)
    f, phi, F = _analytic_numpy(False)
    x = np.array([[10.0, 10.0, 10.0], [12.1, 11.3, 9.4]])
    box = (40.0, 40.0, 40.0)
    res = orc.eam(P, x, box)
    d = x[1] - x[0]
    r = np.linalg.norm(d)
    rho = f(r)
    dF = -0.5 / np.sqrt(rho)
    df = -(3 / 2.47) * f(r)
    dphi = 0.4 * (-3.2 * np.exp(-3.2 * (r - 2.5)) + 3.2 * np.exp(-1.6 * (r - 2.5)))
    F1 = (2 * dF * df + dphi) * d / r  # force on atom 0 points along +d when s > 0
    assert np.allclose(res["rho"], rho, rtol=1e-14)
    assert abs(res["e_emb"] + res["e_pair"] - (2 * F(rho) + phi(r))) < 1e-14
    assert np.allclose(res["F"][0], F1, rtol=1e-13)
    assert np.allclose(res["F"][1], -F1, rtol=1e-13)


def test_isolated_atom(orc):
    P = orc.Potential(orc.ANALYTIC)
    x = np.array([[1.0, 1.0, 1.0], [20.0, 20.0, 20.0]])
    r = orc.eam(P, x, (40.0, 40.0, 40.0))
    assert (r["rho"] == 0).all() and (r["fp"] == 0).all() and (r["F"] == 0).all()
    assert r["e_emb"] == 0.0 and r["e_pair"] == 0.0


def _energy(orc, P, x, box):
    r = orc.eam(P, x, box)
    return r["e_emb"] + r["e_pair"]


@pytest.mark.parametrize("mode", ["analytic", "shifted", "table"])
def test_force_is_minus_energy_gradient(orc, mode):
    rng = np.random.default_rng(7)
    n = 4
    x = w.bcc_positions(n) + rng.normal(0, 0.05, size=(2 * n ** 3, 3))
    box = (n * A,) * 3
    P = {"analytic": orc.Potential(orc.ANALYTIC), "shifted": orc.Potential(orc.ANALYTIC_SF),
         "table": orc.Potential(orc.TABLE, tables=w.potential_samples())}[mode]
    F = orc.eam(P, x, box)["F"]
    h = 1e-5
    for i in (0, 17, 64, 101):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(_energy(orc, P, xp, box) - _energy(orc, P, xm, box)) / (2 * h)
            scale = max(np.sqrt(np.mean(F ** 2)), 1e-3)
            assert abs(fd - F[i, a]) / scale < 1e-6, (i, a, fd, F[i, a])


def test_three_atom_cluster_gradient(orc):
    P = orc.Potential(orc.ANALYTIC)
    x = np.array([[10.0, 10.0, 10.0], [12.3, 10.4, 9.9], [11.1, 12.2, 10.7]])
    box = (30.0, 30.0, 30.0)
    F = orc.eam(P, x, box)["F"]
    h = 1e-6
    for i in range(3):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(_energy(orc, P, xp, box) - _energy(orc, P, xm, box)) / (2 * h)
            assert abs(fd - F[i, a]) < 1e-7 * max(1.0, abs(F[i, a]))


def test_newton_third_law_sum_of_forces(orc):
    x, v, box = w.thermal_state(6, sigma=0.1, seed=3)
    P = orc.Potential(orc.ANALYTIC)
    F = orc.eam(P, x, box)["F"]
    assert np.max(np.abs(F.sum(axis=0))) <= 1e-10 * np.abs(F).sum()


def test_minimum_image_translation_invariance(orc):
    x, v, box = w.thermal_state(5, sigma=0.1, seed=4)
    P = orc.Potential(orc.ANALYTIC)
    r0 = orc.eam(P, x, box)
    r1 = orc.eam(P, x + np.array([3.3, -7.1, 100.0]), box)
    assert np.max(np.abs(r0["F"] - r1["F"])) < 1e-11
    assert abs(r0["e_pair"] - r1["e_pair"]) < 1e-9


def test_cell_binned_pair_set_equals_brute_force(orc):
    x, v, box = w.thermal_state(16, sigma=0.02, seed=1000)
    P = orc.Potential(orc.ANALYTIC)
    rb = orc.eam(P, x, box, want_pairs=True)
    rc = orc.eam(P, x, box, cells=True, want_pairs=True)
    assert np.array_equal(rb["npairs"], rc["npairs"])
    for i in (0, 1, 4095, 8191, 5000):
        assert np.array_equal(orc.neighbours(x, box, 5.0, i, cells=False),
                              orc.neighbours(x, box, 5.0, i, cells=True))
    assert np.max(np.abs(rb["F"] - rc["F"])) < 1e-12
    assert np.max(np.abs(rb["rho"] - rc["rho"])) < 1e-12
    # sampled exact mode reproduces the full evaluation on its sample
    s = np.array([3, 77, 2048, 8000])
    rs = orc.eam_sampled(P, x, box, s)
    assert np.max(np.abs(rs["F"] - rb["F"][s])) < 1e-12
    assert np.max(np.abs(rs["rho"] - rb["rho"][s])) < 1e-12
    assert np.array_equal(rs["npairs"], rb["npairs"][s])


def test_small_box_cell_dedup(orc):
    # 3x3x3 cells: fewer than 3 cut-off-wide cells per axis, neighbour cells must not double count
    x, v, box = w.thermal_state(3, sigma=0.05, seed=9)
    P = orc.Potential(orc.ANALYTIC)
    rb = orc.eam(P, x, box, want_pairs=True)
    rc = orc.eam(P, x, box, cells=True, want_pairs=True)
    assert np.array_equal(rb["npairs"], rc["npairs"])
    assert np.max(np.abs(rb["F"] - rc["F"])) < 1e-12
