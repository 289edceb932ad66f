"""Pins of the oracle's lattice list, neighbour offset index and hash (Sec. 3).

Every expectation here comes from the paper's worked example, from textbook
BCC crystallography, or from exhaustive search -- never from the oracle's own
formulas retyped.
"""
import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
A = 2.855


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                out.append([float(t) for t in line.split()])
    return out


def test_lattice_id_paper_example(orc):
    # Sec. 3, Hash Initialization: (3, 4) -> 43 with box_x = 5
    for bx, by, x, y, expect in _rows("lattice_id_2d_example.txt"):
        assert orc.lattice_id(int(bx), int(by), int(x), int(y), 0) == int(expect)


def test_lattice_id_3d_is_a_bijection(orc):
    nx, ny, nz = 5, 4, 3
    seen = set()
    for Z, Y, X in itertools.product(range(nz), range(ny), range(2 * nx)):
        i = orc.lattice_id(nx, ny, X, Y, Z)
        assert 0 <= i < 2 * nx * ny * nz
        assert orc.lattice_coords(nx, ny, i) == (X, Y, Z)
        seen.add(i)
    assert len(seen) == 2 * nx * ny * nz
    # consecutive X in a row are consecutive ids; rows of 2*box_x, planes of 2*box_x*box_y
    assert orc.lattice_id(nx, ny, 1, 0, 0) - orc.lattice_id(nx, ny, 0, 0, 0) == 1
    assert orc.lattice_id(nx, ny, 0, 1, 0) - orc.lattice_id(nx, ny, 0, 0, 0) == 2 * nx
    assert orc.lattice_id(nx, ny, 0, 0, 1) - orc.lattice_id(nx, ny, 0, 0, 0) == 2 * nx * ny


def test_site_positions_form_bcc(orc):
    # odd X are body centres shifted by half a cell in y and z (Sec. 3 figure of the 2-D lattice)
    nx = ny = nz = 3
    pos = np.array([orc.site_position(A, X, Y, Z)
                    for Z, Y, X in itertools.product(range(nz), range(ny), range(2 * nx))])
    ref = set()
    for i, j, k in itertools.product(range(nx), range(ny), range(nz)):
        ref.add((round(i * A, 9), round(j * A, 9), round(k * A, 9)))
        ref.add((round((i + .5) * A, 9), round((j + .5) * A, 9), round((k + .5) * A, 9)))
    got = {tuple(np.round(p, 9)) for p in pos}
    assert got == ref
    assert np.allclose(orc.site_position(A, 1, 0, 0), [0.5 * A, 0.5 * A, 0.5 * A])


def _shell_counts(R):
    """Cartesian enumeration of BCC points (integer and half-integer) strictly within R."""
    cnt = {}
    w = int(np.ceil(R / A)) + 1
    for i, j, k in itertools.product(range(-w, w + 1), repeat=3):
        for off in (0.0, 0.5):
            d2q = 4 * ((i + off) ** 2 + (j + off) ** 2 + (k + off) ** 2)  # 4 |d/a|^2, an integer
            if d2q == 0:
                continue
            if d2q * (A / 2) ** 2 < R * R:
                cnt[int(round(d2q))] = cnt.get(int(round(d2q)), 0) + 1
    return cnt


@pytest.mark.parametrize("R,expected", [(5.0 + 2 * 0.3, 58), (5.0 + 2 * 0.6, 64), (5.0 + 2 * 0.65, 88)])
def test_stencil_sizes(orc, R, expected):
    for parity in (0, 1):
        st = orc.stencil(A, R, parity)
        assert len(st) == expected
        assert len({tuple(r) for r in st}) == expected
    golden = {int(a): int(b) for a, b in _rows("bcc_shells.txt")}
    counts = _shell_counts(R)
    assert sum(counts.values()) == expected
    for s, m in counts.items():
        assert golden[s] == m


def test_stencil_shells_and_parity_symmetry(orc):
    R = 6.2
    for parity in (0, 1):
        st = orc.stencil(A, R, parity)
        X0 = parity
        base = orc.site_position(A, X0 + 40, 20, 20)
        d2 = []
        for dX, dY, dZ in st:
            p = orc.site_position(A, X0 + 40 + dX, 20 + dY, 20 + dZ)
            d2.append(int(round(4 * np.sum((p - base) ** 2) / A ** 2)))
        vals, mult = np.unique(d2, return_counts=True)
        golden = {int(a): int(b) for a, b in _rows("bcc_shells.txt")}
        for v, m in zip(vals, mult):
            assert golden[v] == m
    even = {tuple(r) for r in orc.stencil(A, R, 0)}
    odd = {tuple(r) for r in orc.stencil(A, R, 1)}
    assert odd == {(-a, -b, -c) for a, b, c in even}
    # first-shell offsets of a corner site: X +-1, Y and Z in {0, -1}
    first = {(dx, dy, dz) for dx, dy, dz in even if dx in (-1, 1) and dy in (0, -1) and dz in (0, -1)}
    assert len(first) == 8


def test_hash_matches_exhaustive_nearest_site(orc):
    rng = np.random.default_rng(5)
    n = (5, 4, 6)
    L = np.array(n) * A
    for _ in range(400):
        x = rng.uniform(-0.3, 1.3, size=3) * L  # includes points outside the box
        s_rule, u, u2 = orc.hash_site(n, A, x)
        s_brute, d2 = orc.nearest_site_brute(n, A, x)
        assert s_rule == s_brute
        assert abs(u2 - d2) < 1e-9
        # u is x minus the site, up to a lattice translation
        X, Y, Z = orc.lattice_coords(n[0], n[1], s_rule)
        p = orc.site_position(A, X, Y, Z)
        d = x - u - p
        assert np.allclose(d / L - np.rint(d / L), 0.0, atol=1e-12)


def test_place_perfect_and_defects(orc):
    import misa_workloads as w
    n = (5, 5, 5)
    x = w.bcc_positions(n)
    slot = orc.place(n, A, 0.6, x)
    assert (slot >= 0).all()
    assert len(np.unique(slot)) == len(slot)
    # an interstitial at the octahedral site (a/2, 0, 0) of cell (2,2,2) stays out of the array
    extra = np.array([[2.5 * A, 2.0 * A, 2.0 * A]])
    slot2 = orc.place(n, A, 0.6, np.vstack([x, extra]))
    assert slot2[-1] == -1 and (slot2[:-1] >= 0).all()
    # two atoms near one site: the lower id keeps the slot
    y = np.vstack([x, x[7] + [0.1, 0.0, 0.0]])
    slot3 = orc.place(n, A, 0.6, y)
    assert slot3[7] >= 0 and slot3[-1] == -1
    y2 = np.vstack([x[7] + [0.1, 0.0, 0.0], x])
    slot4 = orc.place(n, A, 0.6, y2)
    assert slot4[0] >= 0 and slot4[8] == -1


def test_rehash_invariants(orc):
    """The three guarantees listed under Algorithm 2, with the slot tolerance."""
    import misa_workloads as w
    n = (6, 5, 5)
    L = np.array(n) * A
    rng = np.random.default_rng(11)
    x = w.bcc_positions(n) + rng.normal(0, 0.3, size=(2 * 150, 3))
    slot = orc.place(n, A, 0.6, x)
    for it in range(4):
        x = x + rng.normal(0, 0.2, size=x.shape)
        slot = orc.rehash(n, A, 0.6, x, slot)
        used = slot[slot >= 0]
        assert len(np.unique(used)) == len(used)  # (1) one atom per slot
        for i in np.nonzero(slot >= 0)[0]:  # (2) an occupied slot holds an atom within delta of its site
            X, Y, Z = orc.lattice_coords(n[0], n[1], slot[i])
            d = x[i] - orc.site_position(A, X, Y, Z)
            d -= L * np.rint(d / L)
            assert d @ d <= 0.36 + 1e-12
        free = set(range(2 * np.prod(n))) - set(used.tolist())
        for i in np.nonzero(slot < 0)[0]:  # (3) no clash atom is left next to an empty site within delta
            s, _, u2 = orc.hash_site(n, A, x[i])
            assert not (u2 <= 0.36 and s in free)
