"""Pins of the oracle's surrogate-network arithmetic (learned form) against
finite differences, closed forms and library routines -- no GPU."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as O

oracle.build(force=False)

H = O.H


def rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(O.MLP_PARAMS)
    p[:H] = rng.normal(0, 1.5, H) * scale
    p[H:2 * H] = rng.normal(0, 0.5, H)
    p[2 * H:2 * H + H * H] = rng.normal(0, 1 / np.sqrt(H), H * H)
    p[2 * H + H * H:3 * H + H * H] = rng.normal(0, 0.3, H)
    p[3 * H + H * H:4 * H + H * H] = rng.normal(0, 1 / np.sqrt(H), H)
    p[-1] = 0.7
    return p


def test_tangent_matches_finite_differences():
    """dy/dt carried by the forward pass equals the central difference of y."""
    p = rand_params(1)
    t = np.linspace(-1.2, 1.2, 41)
    h = 1e-6
    y, dy = O.forward_t(p, t)
    yp, _ = O.forward_t(p, t + h)
    ym, _ = O.forward_t(p, t - h)
    assert np.allclose(dy, (yp - ym) / (2 * h), rtol=1e-7, atol=1e-8)


def test_evaluate_scaling_and_derivative():
    """g(x) = shift + scale y((x - c) s) and g'(x) = scale s dy/dt (chain rule by FD)."""
    p = rand_params(2)
    net = (1.6, 5.0, -0.3, 2.5, p)
    x = np.linspace(1.7, 4.9, 17)
    g, dg = O.evaluate(net, x)
    h = 1e-6
    gp, _ = O.evaluate(net, x + h)
    gm, _ = O.evaluate(net, x - h)
    assert np.allclose(dg, (gp - gm) / (2 * h), rtol=1e-7, atol=1e-8)
    c, s = O.scaling(1.6, 5.0)
    y, _ = O.forward_t(p, (x - c) * s)
    assert np.allclose(g, -0.3 + 2.5 * y, rtol=0, atol=1e-14)


def test_single_path_network_closed_form():
    """Only W1[0], W2[0][0], w3[0] non-zero: y = b3 + w3 silu(W2 silu(W1 t) + b2[0])
    plus the constant contributions of the other units (silu(b2[n]) w3[n] = 0 here)."""
    p = np.zeros(O.MLP_PARAMS)
    a, b, c, b2, b3 = 1.7, -0.8, 1.3, 0.25, 0.4
    p[0] = a
    p[2 * H] = b          # W2[0][0]
    p[2 * H + H * H] = b2  # b2[0]
    p[3 * H + H * H] = c   # w3[0]
    p[-1] = b3
    t = np.linspace(-1, 1, 9)
    sil = lambda z: z / (1 + np.exp(-z))
    dsil = lambda z: (1 + np.exp(-z) + z * np.exp(-z)) / (1 + np.exp(-z)) ** 2
    inner = b * sil(a * t) + b2
    y_ref = b3 + c * sil(inner)
    dy_ref = c * dsil(inner) * b * dsil(a * t) * a
    y, dy = O.forward_t(p, t)
    assert np.allclose(y, y_ref, rtol=0, atol=1e-15)
    assert np.allclose(dy, dy_ref, rtol=0, atol=1e-15)


def test_silu_derivatives_match_finite_differences():
    z = np.linspace(-8, 8, 101)
    h = 1e-5
    assert np.allclose(O.dsilu(z), (O.silu(z + h) - O.silu(z - h)) / (2 * h), atol=1e-9)
    assert np.allclose(O.d2silu(z), (O.dsilu(z + h) - O.dsilu(z - h)) / (2 * h), atol=1e-9)


@pytest.mark.parametrize("seed", [3, 4])
def test_param_grad_matches_finite_differences(seed):
    """Reverse pass (through the tangent, with silu'') against central differences
    of L(p) = sum_b c_val y + c_der dy/dt, for every parameter."""
    rng = np.random.default_rng(seed)
    p = rand_params(seed)
    t = rng.uniform(-1, 1, 7)
    cv = rng.normal(size=7)
    cd = rng.normal(size=7)

    def L(q):
        y, dy = O.forward_t(q, t)
        return float(cv @ y + cd @ dy)

    g = O.param_grad(p, t, cv, cd)
    h = 1e-6
    fd = np.empty_like(p)
    for j in range(len(p)):
        e = np.zeros_like(p)
        e[j] = h
        fd[j] = (L(p + e) - L(p - e)) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_c_oracle_network_matches_numpy():
    """The C oracle's own evaluation of a network agrees with the numpy one."""
    p = rand_params(5)
    net = (1.6, 5.0, 0.1, 1.9, p)
    x = np.linspace(1.6, 5.0, 33)
    v, d = oracle.mlp_eval(net, x)
    g, dg = O.evaluate(net, x)
    assert np.allclose(v, g, rtol=1e-13, atol=1e-14)
    assert np.allclose(d, dg, rtol=1e-13, atol=1e-14)


def test_adam_first_step_closed_form():
    """With zero moments the first Adam step moves each weight by lr g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    p = rng.normal(size=20)
    g = rng.normal(size=20)
    lr = 1e-2
    p1, m, v = O.adam_step(p, g, np.zeros(20), np.zeros(20), 1, lr)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-6, 6, 1000), [0.0, 1.0, -2.5, 1.00390625]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.round_bf16(x), ref)


def test_force_match_coefficients_are_the_loss_gradient():
    """The per-pair coefficients fed to param_grad reproduce d(loss)/d(weights) of the
    force-matching loss (finite differences over a subset of f and phi weights)."""
    rng = np.random.default_rng(9)
    n, K = 3, 6
    r = rng.uniform(2.0, 4.8, (n, K))
    r[0, 5] = 0.0  # an empty slot
    dh = rng.normal(size=(n, K, 3))
    dh /= np.linalg.norm(dh, axis=2, keepdims=True)
    fpi = rng.normal(-0.13, 0.01, n)
    fpj = rng.normal(-0.13, 0.01, (n, K))
    fref = rng.normal(size=(n, 3))
    nf = (1.6, 5.0, 0.5, 0.6, rand_params(10))
    npf = (1.6, 5.0, -0.1, 0.4, rand_params(11))
    F, loss, cf, cp = O.force_match(nf, npf, r, dh, fpi, fpj, fref)
    m = r > 0
    c, s = O.scaling(1.6, 5.0)
    gf = O.param_grad(nf[4], ((r - c) * s)[m], np.zeros(m.sum()), cf[m])
    gp = O.param_grad(npf[4], ((r - c) * s)[m], np.zeros(m.sum()), cp[m])
    h = 1e-6
    for which, g in ((0, gf), (1, gp)):
        for j in rng.choice(O.MLP_PARAMS, 25, replace=False):
            def L(dw):
                nets = [list(nf), list(npf)]
                q = nets[which][4].copy()
                q[j] += dw
                nets[which][4] = q
                return O.force_match(tuple(nets[0]), tuple(nets[1]), r, dh, fpi, fpj, fref)[1]
            fd = (L(h) - L(-h)) / (2 * h)
            assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (which, j, fd, g[j])


def test_force_match_force_is_the_pair_sum():
    rng = np.random.default_rng(12)
    r = rng.uniform(2.0, 4.8, (2, 4))
    dh = rng.normal(size=(2, 4, 3))
    dh /= np.linalg.norm(dh, axis=2, keepdims=True)
    fpi, fpj = np.array([-0.1, -0.2]), rng.normal(-0.1, 0.01, (2, 4))
    nf = (1.6, 5.0, 0.5, 0.6, rand_params(13))
    npf = (1.6, 5.0, -0.1, 0.4, rand_params(14))
    F, _, _, _ = O.force_match(nf, npf, r, dh, fpi, fpj, np.ones((2, 3)))
    for i in range(2):
        ref = np.zeros(3)
        for k in range(4):
            _, df = O.evaluate(nf, [r[i, k]])
            _, dp = O.evaluate(npf, [r[i, k]])
            ref += ((fpi[i] + fpj[i, k]) * df[0] + dp[0]) * dh[i, k]
        assert np.allclose(F[i], ref, rtol=1e-13, atol=1e-15)


def _constant_net(lo, hi, value):
    p = np.zeros(O.MLP_PARAMS)
    p[-1] = 1.0  # y = b3 + sum_n w3[n] silu(b2[n]) = 1
    return (lo, hi, value - 1.0, 1.0, p)


def test_oracle_mlp_mode_wiring_closed_form():
    """Networks that are constants inside their ranges: on a perfect lattice whose
    58 neighbours all lie inside the f range, rho = 58 c_f exactly, every force is
    zero, and the energy per atom is the F constant plus 29 times the phi constant."""
    a, rc = 2.855, 5.0
    n = 6
    from misa_workloads import synth
    x = synth.bcc_positions((n, n, n), a)
    box = (n * a,) * 3
    pot = oracle.Potential(oracle.MLP, rc=rc, tables=synth.potential_samples(),
                           mlp={"f": _constant_net(2.0, rc, 0.7), "phi": _constant_net(2.0, rc, -0.05),
                                "F": _constant_net(10.0, 60.0, -3.0)})
    res = oracle.eam(pot, x, box, cells=True)
    assert np.allclose(res["rho"], 58 * 0.7, rtol=0, atol=1e-12)
    assert np.abs(res["F"]).max() < 1e-12
    e = (res["e_emb"] + res["e_pair"]) / len(x)
    assert abs(e - (-3.0 + 29 * -0.05)) < 1e-12


def test_oracle_mlp_mode_falls_back_to_the_table_outside_the_range():
    """f network range ending below the fifth shell (sqrt(3) a = 4.945 A): the 50
    inner neighbours take the network constant, the 8 fifth-shell ones the table."""
    a, rc, n = 2.855, 5.0, 6
    from misa_workloads import synth
    tabs = synth.potential_samples()
    x = synth.bcc_positions((n, n, n), a)
    pot = oracle.Potential(oracle.MLP, rc=rc, tables=tabs,
                           mlp={"f": _constant_net(2.0, 4.9, 0.7), "phi": _constant_net(2.0, rc, -0.05),
                                "F": _constant_net(10.0, 60.0, -3.0)})
    res = oracle.eam(pot, x, (n * a,) * 3, cells=True)
    f5, _, _ = oracle.spline_eval(*tabs["f"], [np.sqrt(3.0) * a])
    assert np.allclose(res["rho"], 50 * 0.7 + 8 * f5[0], rtol=0, atol=1e-12)
