"""Pins of the oracle's table interpolation (Sec. 4.1: per-segment cubic S_k and S_k').

The segment rule (cubic Hermite with fourth-order difference slopes) is a
reading of the paper; these tests fix what any correct implementation of it
must satisfy: it passes through the samples, reproduces cubics exactly where
the five-point slopes are exact, is C1 at the nodes and converges as h^4.
"""
import numpy as np

import misa_workloads as w


def test_interpolates_the_samples(orc):
    rng = np.random.default_rng(0)
    y = rng.normal(size=40)
    h = 0.125  # power of two: (k h) / h == k exactly, so each node is hit with t == 0
    v, d, ext = orc.spline_eval(0.0, h, y, np.arange(39) * h)
    assert np.array_equal(v, y[:39])
    assert not ext.any()


def test_reproduces_cubics_on_interior_segments(orc):
    h, n = 0.05, 60
    xs = np.arange(n) * h
    c = [0.3, -1.2, 0.7, 0.25]
    p = np.polynomial.Polynomial(c)
    y = p(xs)
    q = np.linspace(2 * h, (n - 3) * h, 997)
    v, d, _ = orc.spline_eval(0.0, h, y, q)
    assert np.max(np.abs(v - p(q))) < 1e-12
    assert np.max(np.abs(d - p.deriv()(q))) < 1e-10
    # a quartic is not reproduced: the rule is not an exact-polynomial fit
    y4 = xs ** 4
    v4, _, _ = orc.spline_eval(0.0, h, y4, q)
    assert np.max(np.abs(v4 - q ** 4)) > 1e-9


def test_c1_continuity_at_nodes(orc):
    rng = np.random.default_rng(3)
    y = np.cumsum(rng.normal(size=50))
    h = 0.2
    k = np.arange(2, 47)
    eps = 1e-9
    vl, dl, _ = orc.spline_eval(0.0, h, y, k * h - eps)
    vr, dr, _ = orc.spline_eval(0.0, h, y, k * h + eps)
    assert np.max(np.abs(vl - vr)) < 1e-7
    assert np.max(np.abs(dl - dr)) < 1e-6


def test_fourth_order_convergence_against_analytic(orc):
    P = orc.Potential(orc.ANALYTIC)
    errs = []
    for n in (500, 1000, 2000):
        h = 5.0 / (n - 1)
        r = np.arange(n) * h
        fy, _ = P.f(r)
        q = np.linspace(1.5, 4.9, 401)
        v, d, _ = orc.spline_eval(0.0, h, fy, q)
        fv, fd = P.f(q)
        errs.append(np.max(np.abs(v - fv)))
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


def test_production_tables_match_analytic(orc):
    P = orc.Potential(orc.ANALYTIC)
    tabs = w.potential_samples()
    Pt = orc.Potential(orc.TABLE, tables=tabs)
    r = np.linspace(1.0, 4.999, 3001)
    for g, gt in ((P.f, Pt.f), (P.phi, Pt.phi)):
        (v, d), (vt, dt) = g(r), gt(r)
        assert np.max(np.abs(vt - v) / np.maximum(np.abs(v), 1e-3)) < 1e-9
        assert np.max(np.abs(dt - d) / np.maximum(np.abs(d), 1e-3)) < 1e-6
    rho = np.linspace(5.0, 40.0, 501)
    (v, d), (vt, dt) = P.emb(rho), Pt.emb(rho)
    assert np.max(np.abs(vt - v)) < 1e-9 and np.max(np.abs(dt - d)) < 1e-7


def test_extrapolation_beyond_last_node(orc):
    y = np.arange(10, dtype=float) ** 2
    v, d, ext = orc.spline_eval(0.0, 1.0, y, [9.0, 10.5])
    assert not ext[0] and ext[1]
    # linear continuation from the last node value with the last node slope (y9 - y8)
    assert v[1] == 81.0 + (81.0 - 64.0) * 1.5
    assert d[1] == 17.0


def test_analytic_derivatives_match_central_differences(orc):
    for mode in (orc.ANALYTIC, orc.ANALYTIC_SF):
        P = orc.Potential(mode)
        h = 1e-6
        r = np.linspace(1.2, 4.95, 37)
        for g in (P.f, P.phi):
            vp, _ = g(r + h)
            vm, _ = g(r - h)
            _, d = g(r)
            assert np.max(np.abs((vp - vm) / (2 * h) - d)) < 1e-7
        rho = np.linspace(1.0, 50.0, 23)
        vp, _ = P.emb(rho + h)
        vm, _ = P.emb(rho - h)
        _, d = P.emb(rho)
        assert np.max(np.abs((vp - vm) / (2 * h) - d)) < 1e-7
    # shifted-force variant vanishes with zero slope at the cut-off
    P = orc.Potential(orc.ANALYTIC_SF)
    for g in (P.f, P.phi):
        v, d = g([5.0])
        assert abs(v[0]) < 1e-15 and abs(d[0]) < 1e-15


def test_end_segments_closed_form(orc):
    """The slope rules next to the ends (one-sided at nodes 0 and n-1, second-order
    central at nodes 1 and n-2) against the Hermite segment they must produce on a
    polynomial, written out by hand.  With y = s^2 or s^3 sampled at s = x / h = 0..n-1:
      segment 0,   y = s^2: slopes (1, 2) vs exact (0, 2)       -> S = t^2 + (t^3 - 2t^2 + t)
      segment 1,   y = s^3: slopes (4, 12) vs exact (3, 12)     -> S = s^3 + (t^3 - 2t^2 + t)
      segment n-3, y = s^3: slope at n-2 is 3(n-2)^2 + 1        -> S = s^3 + (t^3 - t^2)
      segment n-2, y = s^2: slopes (2(n-2), 2n-3) vs (.., 2n-2) -> S = s^2 - (t^3 - t^2)
    (t3 - 2t2 + t and t3 - t2 are the Hermite weights of the left and right slope)."""
    h, n = 0.5, 12
    s = np.arange(n, dtype=float)
    t = np.linspace(0.05, 0.95, 19)
    h10, h11 = t ** 3 - 2 * t ** 2 + t, t ** 3 - t ** 2
    dh10, dh11 = 3 * t ** 2 - 4 * t + 1, 3 * t ** 2 - 2 * t
    cases = [(0, s ** 2, t ** 2 + h10, 2 * t + dh10),
             (1, s ** 3, (1 + t) ** 3 + h10, 3 * (1 + t) ** 2 + dh10),
             (n - 3, s ** 3, (n - 3 + t) ** 3 + h11, 3 * (n - 3 + t) ** 2 + dh11),
             (n - 2, s ** 2, (n - 2 + t) ** 2 - h11, 2 * (n - 2 + t) - dh11)]
    for k, y, want, dwant in cases:
        v, d, ext = orc.spline_eval(0.0, h, y, (k + t) * h)
        assert not ext.any()
        assert np.max(np.abs(v - want)) < 1e-12, k
        assert np.max(np.abs(d * h - dwant)) < 1e-11, k  # d/dx = (d/dt) / h
