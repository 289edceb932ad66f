"""Pins of the oracle's Wigner-Seitz defect count (the direct defect analysis the
paper names in Sec. 1 and applies to cascades in Sec. 5.1): closed cases and a
brute-force nearest-site cross-check -- no GPU."""
import numpy as np

import misa_workloads as w

A = w.A_FE


def test_perfect_and_thermal_lattice_have_no_defects(orc):
    n = (5, 6, 4)
    x = w.bcc_positions(n, A)
    assert orc.wigner_seitz(n, A, x)[:2] == (0, 0)
    xt, _, _ = w.thermal_state(n, seed=3)  # sigma 0.02 A: every atom stays in its own cell
    v, i, occ = orc.wigner_seitz(n, A, xt)
    assert (v, i) == (0, 0) and (occ == 1).all()


def test_removed_atoms_are_vacancies(orc):
    n = (5, 5, 5)
    x = w.bcc_positions(n, A)
    keep = np.ones(len(x), bool)
    keep[[0, 17, 123, 249]] = False
    assert orc.wigner_seitz(n, A, x[keep])[:2] == (4, 0)


def test_added_atom_is_an_interstitial_and_a_moved_atom_a_frenkel_pair(orc):
    n = (5, 5, 5)
    x = w.bcc_positions(n, A)
    extra = np.array([[0.5 * A + 0.11, 0.2 * A, 0.05 * A]])
    assert orc.wigner_seitz(n, A, np.concatenate([x, extra]))[:2] == (0, 1)
    y = x.copy()
    y[7] = extra[0]  # the atom of site 7 leaves for an interstitial position elsewhere
    assert orc.wigner_seitz(n, A, y)[:2] == (1, 1)


def test_occupancy_matches_brute_force_nearest_site(orc):
    """Random positions: the per-site counts equal an exhaustive nearest-site search."""
    n = (4, 4, 5)
    rng = np.random.default_rng(5)
    L = np.array(n) * A
    x = rng.uniform(0, 1, (300, 3)) * L
    vac, inter, occ = orc.wigner_seitz(n, A, x)
    ref = np.zeros(2 * n[0] * n[1] * n[2], dtype=np.int32)
    for p in x:
        s, _ = orc.nearest_site_brute(n, A, p)
        ref[s] += 1
    assert np.array_equal(occ, ref)
    assert vac == int((ref == 0).sum()) and inter == int(np.maximum(ref - 1, 0).sum())
    assert len(x) - inter + vac == len(ref)  # atoms - extra + empty = sites
