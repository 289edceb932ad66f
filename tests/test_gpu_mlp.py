"""GPU parity of the learned form (surrogate networks) through the C ABI against
the oracle: both forward paths, the backward pass, Adam, the table targets, the
force-matching data, training gains, and lattice forces of the MISA_MLP form
against the oracle's MLP potential mode.

Tolerances (float32 kernels against float64 references):
  * float32 forward pass: 2e-5 of the largest |value| (32-term sums of O(1) terms
    in float32);
  * matrix-core forward pass: activations enter as two bfloat16 terms (relative
    representation error <= 2^-17), float32 accumulation: 3e-4 of the largest |value|;
  * gradients: float32 sums over the samples of a block, float64 across blocks:
    2e-4 of the largest |component|;
  * lattice forces of the learned form: float32 pair geometry (the float32 form's
    ~1e-5) plus the matrix-core evaluation: 2e-3 of the rms force.
"""
import numpy as np
import pytest

import misa_workloads as w
from oracle import mlp as O

pytestmark = pytest.mark.gpu

A, RC, DELTA, MASS = w.A_FE, w.RC, w.DELTA, w.MASS_FE
TABLES = w.potential_samples()
FNS = (0, 1, 2)
RANGES = {0: (1.6, RC), 1: (1.6, RC), 2: (4.0, 36.0)}
ORC_KEYS = {0: "f", 1: "phi", 2: "F"}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def M(torch_cuda):
    from paper_2107_07866_amd import misa
    return misa


@pytest.fixture(scope="module")
def trainer(M, torch_cuda):
    t = M.misa_mlp_trainer_create(torch_cuda.cuda.current_stream().cuda_stream)
    yield t
    M.misa_mlp_trainer_destroy(t)


def _say(msg):
    print(msg, flush=True)


def rand_net(seed, fn):
    rng = np.random.default_rng(seed)
    H = O.H
    p = np.zeros(O.MLP_PARAMS)
    p[:H] = rng.normal(0, 1.5, H)
    p[H:2 * H] = rng.normal(0, 0.5, H)
    p[2 * H:2 * H + H * H] = rng.normal(0, 1 / np.sqrt(H), H * H)
    p[2 * H + H * H:3 * H + H * H] = rng.normal(0, 0.3, H)
    p[3 * H + H * H:4 * H + H * H] = rng.normal(0, 1 / np.sqrt(H), H)
    p[-1] = 0.2
    p = O.round_bf16(p)
    lo, hi = RANGES[fn]
    return {"x_lo": lo, "x_hi": hi, "y_shift": 0.3, "y_scale": 1.7, "params": p.astype(np.float32)}


def as_tuple(net):
    return (net["x_lo"], net["x_hi"], net["y_shift"], net["y_scale"], np.asarray(net["params"], dtype=np.float64))


def _lattice(n, precision, tables=TABLES):
    from paper_2107_07866_amd import Lattice
    lat = Lattice(n, A, RC, DELTA, MASS, precision)
    lat.set_tables(tables)
    return lat


@pytest.mark.parametrize("path", [0, 1])
def test_forward_paths_match_oracle(M, trainer, torch_cuda, path):
    torch = torch_cuda
    for fn in FNS:
        _say(f"forward path {path} fn {fn}")
        net = rand_net(100 + fn, fn)
        M.misa_mlp_trainer_set(trainer, fn, net)
        lo, hi = RANGES[fn]
        xs = np.random.default_rng(fn).uniform(lo, hi, 1037)  # ragged: not a multiple of 64 or 256
        x = torch.tensor(xs, dtype=torch.float64, device="cuda")
        y, dy = torch.empty_like(x), torch.empty_like(x)
        M.misa_mlp_eval(trainer, fn, path, x, y, dy)
        g, dg = O.evaluate(as_tuple(net), xs)
        tol = 2e-5 if path == 0 else 3e-4
        ey = np.abs(y.cpu().numpy() - g).max() / np.abs(g).max()
        ed = np.abs(dy.cpu().numpy() - dg).max() / np.abs(dg).max()
        _say(f"  value {ey:.2e} derivative {ed:.2e}")
        assert ey <= tol and ed <= tol


def test_backward_pass_matches_oracle(M, trainer, torch_cuda):
    torch = torch_cuda
    for fn in FNS:
        _say(f"backward fn {fn}")
        net = rand_net(200 + fn, fn)
        M.misa_mlp_trainer_set(trainer, fn, net)
        rng = np.random.default_rng(300 + fn)
        lo, hi = RANGES[fn]
        n = 777
        xs = rng.uniform(lo, hi, n)
        cv, cd = rng.normal(size=n), rng.normal(size=n)
        dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
        grad = torch.empty(O.MLP_PARAMS, dtype=torch.float64, device="cuda")
        M.misa_mlp_grad(trainer, fn, dev(xs), dev(cv), dev(cd), grad)
        c, s = O.scaling(lo, hi)
        ref = O.param_grad(as_tuple(net)[4], (xs - c) * s, cv, cd)
        err = np.abs(grad.cpu().numpy() - ref).max() / np.abs(ref).max()
        _say(f"  gradient {err:.2e}")
        assert err <= 2e-4


def test_adam_step_matches_oracle(M, trainer, torch_cuda):
    torch = torch_cuda
    net = rand_net(400, 0)
    M.misa_mlp_trainer_set(trainer, 0, net)
    g = np.random.default_rng(401).normal(size=O.MLP_PARAMS)
    lr = 3e-3
    p0 = np.asarray(net["params"], dtype=np.float64)
    ref1, m1, v1 = O.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    ref2, _, _ = O.adam_step(ref1, 0.5 * g, m1, v1, 2, lr)
    gd = torch.tensor(g, dtype=torch.float64, device="cuda")
    M.misa_mlp_adam(trainer, 0, gd, lr)
    M.misa_mlp_adam(trainer, 0, 0.5 * gd, lr)
    got, master = M.misa_mlp_trainer_get(trainer, 0)
    assert np.abs(master - ref2).max() <= 1e-6 * np.abs(ref2).max()
    # the network handed out is the bfloat16 rounding of the float32 master
    assert np.array_equal(got["params"].astype(np.float64), O.round_bf16(master.astype(np.float64)))


def test_table_targets_match_oracle_spline(M, torch_cuda, orc):
    torch = torch_cuda
    lat = _lattice(6, "fp64")
    for fn in FNS:
        key = ORC_KEYS[fn]
        lo, hi = (0.3, RC) if fn < 2 else (0.0, 70.0)  # F: beyond the last node too
        xs = np.random.default_rng(fn).uniform(lo, hi, 2001)
        x = torch.tensor(xs, dtype=torch.float64, device="cuda")
        y, dy = torch.empty_like(x), torch.empty_like(x)
        M.misa_table_eval(lat.h, fn, x, y, dy)
        v, d, _ = orc.spline_eval(*TABLES[key], xs)
        assert np.allclose(y.cpu().numpy(), v, rtol=1e-12, atol=1e-13)
        assert np.allclose(dy.cpu().numpy(), d, rtol=1e-11, atol=1e-12)
    lat.close()


def _quick_fit(M, torch, trainer, lat, iters=20000, seed=21):
    from paper_2107_07866_amd import surrogate as S
    nets, losses, samples = {}, {}, {}
    rng = np.random.default_rng(seed)
    for fn in FNS:
        lo, hi = RANGES[fn]
        x, y, dy = S.table_samples(lat.h, fn, lo, hi, 200_000, rng)
        net = {"x_lo": lo, "x_hi": hi, "y_shift": float(y.mean()), "y_scale": float(y.std()),
               "params": S.init_params(rng)}
        M.misa_mlp_trainer_set(trainer, fn, net)
        init = dict(net)
        losses[fn] = M.misa_mlp_fit(trainer, fn, x, y, dy, dict(iters=iters, batch=4096, quantize=1, lr=1e-2,
                                                                   lr_final=1e-5, seed=seed + fn))
        nets[fn], _ = M.misa_mlp_trainer_get(trainer, fn)
        samples[fn] = (x, y, dy, init)
    return nets, losses, samples


def test_training_gain(M, trainer, torch_cuda, orc):
    """What training buys: the fitted networks track the tables' f' / phi' / F' two
    orders of magnitude better than the same networks before training, and well
    enough for forces (max error of the derivative below 1 % of its range)."""
    torch = torch_cuda
    lat = _lattice(6, "fp64")
    nets, losses, samples = _quick_fit(M, torch, trainer, lat)
    for fn in FNS:
        lo, hi = RANGES[fn]
        xs = np.linspace(lo, hi, 4001)
        _, d_ref, _ = orc.spline_eval(*TABLES[ORC_KEYS[fn]], xs)
        init = samples[fn][3]
        _, d_init = O.evaluate(as_tuple(dict(init, params=O.round_bf16(init["params"]))), xs)
        _, d_fit = O.evaluate(as_tuple(nets[fn]), xs)
        span = np.abs(d_ref).max()
        e0 = np.abs(d_init - d_ref).max() / span
        e1 = np.abs(d_fit - d_ref).max() / span
        _say(f"fn {fn}: loss {losses[fn]:.2e}; derivative error before {e0:.2e} after {e1:.2e}")
        assert e1 < 1e-2 and e1 * 100 < e0
    lat.close()


def test_mlp_form_forces_match_oracle(M, trainer, torch_cuda, orc):
    """Lattice forces, densities and energy of the MISA_MLP form against the oracle's
    MLP potential mode (same bfloat16 weights, float64), on thermal states with
    vacancies and a ragged box; no run-away atoms (pairs with those take the tables)."""
    torch = torch_cuda
    lat64 = _lattice(6, "fp64")
    nets, _, _ = _quick_fit(M, torch, trainer, lat64, iters=8000, seed=31)
    lat64.close()
    pot = orc.Potential(orc.MLP, tables=TABLES, mlp={ORC_KEYS[fn]: as_tuple(nets[fn]) for fn in FNS})
    for n, nvac, seed in (((8, 8, 8), 0, 1), ((9, 7, 10), 5, 2)):
        _say(f"mlp form box {n} vacancies {nvac}")
        x, v, _ = w.thermal_state(n, seed=seed)
        keep = np.ones(len(x), bool)
        keep[np.random.default_rng(seed).choice(len(x), nvac, replace=False)] = False
        x, v = x[keep], v[keep]
        box = tuple(k * A for k in n)
        lat = _lattice(n, "mlp")
        lat.set_mlp(nets)
        lat.set_state(x, v)
        e = lat.compute(energies=True)
        torch.cuda.synchronize()
        assert (lat.slots() >= 0).all()  # no run-away atoms
        ref = orc.eam(pot, x, box, cells=True)
        F = lat.forces()
        scale = float(np.sqrt(np.mean(ref["F"] ** 2)))
        ferr = np.abs(F - ref["F"]).max() / scale
        rerr = np.abs(lat.rho() - ref["rho"]).max() / np.abs(ref["rho"]).max()
        et = e.cpu().numpy().sum()
        eerr = abs(et - (ref["e_emb"] + ref["e_pair"])) / len(x)
        _say(f"  force {ferr:.2e} rho {rerr:.2e} energy/atom {eerr:.2e} eV")
        assert ferr <= 2e-3 and rerr <= 1e-4 and eerr <= 1e-4
        lat.close()


def test_mlp_form_half_schedule(M, trainer, torch_cuda, orc):
    """The learned form on the half-stencil schedule (each owned pair through the
    networks once, 8 colours of tiles): forces, densities and energy against the
    gather schedule (float32 rounding apart) and the oracle's MLP mode, on a thermal
    box with vacancies (no run-away atoms: their pairs take the tables); then 10
    steps of both schedules."""
    torch = torch_cuda
    lat64 = _lattice(6, "fp64")
    nets, _, _ = _quick_fit(M, torch, trainer, lat64, iters=8000, seed=33)
    lat64.close()
    pot = orc.Potential(orc.MLP, tables=TABLES, mlp={ORC_KEYS[fn]: as_tuple(nets[fn]) for fn in FNS})
    n = (16, 16, 32)
    x, v, _ = w.thermal_state(n, seed=5)
    keep = np.ones(len(x), bool)
    keep[[7, 900, 4000]] = False
    x, v = x[keep], v[keep]
    box = tuple(k * A for k in n)
    out = {}
    for sched in ("gather", "half"):
        _say(f"mlp form box {n}, {sched} schedule")
        lat = _lattice(n, "mlp")
        lat.set_mlp(nets)
        lat.set_pair_schedule(sched)
        lat.set_state(x, v)
        e = lat.compute(energies=True)
        torch.cuda.synchronize()
        out[sched] = (lat.forces(), lat.rho(), lat.fprime(), float(e.cpu().numpy().sum()))
        lat.close()
    ref = orc.eam(pot, x, box, cells=True)
    scale = float(np.sqrt(np.mean(ref["F"] ** 2)))
    F, rho, fp, et = out["half"]
    ferr = np.abs(F - ref["F"]).max() / scale
    rerr = np.abs(rho - ref["rho"]).max() / np.abs(ref["rho"]).max()
    eerr = abs(et - (ref["e_emb"] + ref["e_pair"])) / len(x)
    gf = np.abs(F - out["gather"][0]).max() / scale
    gr = np.abs(rho - out["gather"][1]).max() / np.abs(ref["rho"]).max()
    gp = np.abs(fp - out["gather"][2]).max() / np.abs(out["gather"][2]).max()
    ge = abs(et - out["gather"][3]) / len(x)
    _say(f"  half vs oracle: force {ferr:.2e} rho {rerr:.2e} energy/atom {eerr:.2e} eV; "
         f"vs gather: force {gf:.2e} rho {gr:.2e} F' {gp:.2e} energy/atom {ge:.2e}")
    assert ferr <= 2e-3 and rerr <= 1e-4 and eerr <= 1e-4
    assert gf <= 1e-4 and gr <= 1e-6 and gp <= 1e-5 and ge <= 1e-6
    assert np.max(np.abs(F.sum(axis=0))) <= 1e-5 * np.abs(F).sum()  # pair terms cancel in pairs
    traj = {}
    for sched in ("gather", "half"):
        lat = _lattice(n, "mlp")
        lat.set_mlp(nets)
        lat.set_pair_schedule(sched)
        lat.set_state(x, v)
        st = lat.step(10, 1.0, 0.05)
        traj[sched] = (lat.get_state()[0], st)
        lat.close()
    L = np.asarray(box)
    d = traj["half"][0] - traj["gather"][0]
    d -= L * np.rint(d / L)
    _say(f"  10 steps: max |dx| half vs gather {np.max(np.abs(d)):.2e} A")
    assert np.max(np.abs(d)) < 1e-5
    assert abs(traj["half"][1]["dt"] - traj["gather"][1]["dt"]) < 1e-6 * traj["gather"][1]["dt"]


def test_mlp_half_schedule_recoil(M, trainer, torch_cuda):
    """A 1 keV recoil in the learned form on both schedules: the recoil leaves its slot
    (its pairs then take the float64 tables of the run-away path, lattice pairs the
    networks); trajectories, run-away counts and step lengths agree to float32
    rounding over 30 adaptive steps."""
    torch = torch_cuda
    lat64 = _lattice(6, "fp64")
    nets, _, _ = _quick_fit(M, torch, trainer, lat64, iters=4000, seed=35)
    lat64.close()
    n = (16, 16, 16)
    x, v, box = w.thermal_state(n, seed=9)
    w.add_recoils(x, v, box, 1, 1000.0, True, seed=9)
    out = {}
    for sched in ("gather", "half"):
        lat = _lattice(n, "mlp")
        lat.set_mlp(nets)
        lat.set_pair_schedule(sched)
        lat.set_state(x, v)
        st = lat.step(30, 1.0, 0.05)
        out[sched] = (lat.get_state()[0], st, lat.slots())
        lat.close()
    L = np.asarray(box)
    d = out["half"][0] - out["gather"][0]
    d -= L * np.rint(d / L)
    _say(f"mlp recoil, 30 steps: run-aways {out['half'][1]['n_runaway']} / {out['gather'][1]['n_runaway']}, "
         f"max |dx| half vs gather {np.max(np.abs(d)):.2e} A")
    assert out["half"][1]["n_runaway"] >= 1
    assert out["half"][1]["n_runaway"] == out["gather"][1]["n_runaway"]
    assert np.array_equal(out["half"][2], out["gather"][2])
    assert np.max(np.abs(d)) < 1e-5
    assert abs(out["half"][1]["dt"] - out["gather"][1]["dt"]) < 1e-6 * out["gather"][1]["dt"]


def test_collect_matches_oracle(M, torch_cuda, orc):
    """Force-matching data: per sampled atom, the pair list and the reference force
    (the float64 table force; with no run-away atoms it is the atom's whole force)."""
    torch = torch_cuda
    from paper_2107_07866_amd import surrogate as S
    n = (8, 8, 8)
    x, v, _ = w.thermal_state(n, seed=5)
    keep = np.ones(len(x), bool)
    keep[[3, 100, 777]] = False  # vacancies
    x, v = x[keep], v[keep]
    lat = _lattice(n, "fp64")
    lat.set_state(x, v)
    lat.compute(energies=False)
    slots = lat.slots()
    ids = np.array([0, 1, 2, 50, 99, 500, 1000, 1020])
    sites = slots[ids]
    vacant = np.setdiff1d(np.arange(2 * n[0] * n[1] * n[2]), slots)[:1]  # an empty lattice site
    assert len(vacant) == 1
    r, dhat, fpj, fpi, fref = S.collect(lat.h, np.concatenate([sites, vacant]))
    torch.cuda.synchronize()
    pot = orc.Potential(orc.TABLE, tables=TABLES)
    ref = orc.eam(pot, x, tuple(k * A for k in n), want_pairs=True)
    fr = fref.cpu().numpy().reshape(-1, 3)
    rr = r.cpu().numpy().reshape(-1, M.MISA_FM_SLOTS)
    assert np.allclose(fr[:-1], ref["F"][ids], rtol=0, atol=1e-10 * np.abs(ref["F"]).max())
    assert np.allclose(fpi.cpu().numpy()[:-1], ref["fp"][ids], rtol=1e-12)
    assert ((rr[:-1] > 0).sum(1) == ref["npairs"][ids]).all()
    assert (rr[-1] == 0).all() and (fr[-1] == 0).all()
    lat.close()


def test_force_matching_loss_and_descent(M, trainer, torch_cuda):
    """Full-batch force matching: the loss the kernels report before the first update
    equals the oracle's force-matching loss of the same networks and data, and
    small full-batch steps lower it."""
    torch = torch_cuda
    from paper_2107_07866_amd import surrogate as S
    lat = _lattice(8, "fp64")
    _quick_fit(M, torch, trainer, lat, iters=4000, seed=41)
    x, v, _ = w.thermal_state((8, 8, 8), seed=6, temperature=900.0)
    lat.set_state(x, v)
    lat.compute(energies=False)
    sites = lat.slots()
    sites = sites[sites >= 0][:300]
    data = S.collect(lat.h, sites)
    nets = {fn: M.misa_mlp_trainer_get(trainer, fn)[0] for fn in (0, 1)}
    K = M.MISA_FM_SLOTS
    r, dhat, fpj, fpi, fref = (d.cpu().numpy() for d in data)
    n = len(sites)
    _, ref_loss, _, _ = O.force_match(as_tuple(nets[0]), as_tuple(nets[1]), r.reshape(n, K),
                                      dhat.reshape(n, K, 3), fpi, fpj.reshape(n, K), fref.reshape(n, 3))
    base = dict(batch=n, quantize=1, seed=3)
    l0 = M.misa_mlp_force_match(trainer, *data, dict(base, iters=1, lr=1e-12, lr_final=1e-12))
    _say(f"force-matching loss {l0:.6e} oracle {ref_loss:.6e}")
    assert abs(l0 - ref_loss) <= 1e-4 * ref_loss
    l1 = M.misa_mlp_force_match(trainer, *data, dict(base, iters=300, lr=1e-4, lr_final=1e-5))
    _say(f"after 300 full-batch steps {l1:.6e}")
    assert l1 < l0
    lat.close()


def test_mlp_form_runaway_pairs_use_the_tables(M, trainer, torch_cuda, orc):
    """With run-away atoms present, their pairs take the float64 tables in the learned form
    too: a run-away atom's force equals the float32 table form's up to the networks' F'
    error of its lattice partners (the run-away kernels are shared by both forms)."""
    torch = torch_cuda
    lat64 = _lattice(6, "fp64")
    nets, _, _ = _quick_fit(M, torch, trainer, lat64, iters=8000, seed=51)
    lat64.close()
    n = (8, 8, 8)
    x, v, _ = w.thermal_state(n, seed=9)
    extra = np.array([[2.5 * A + 0.05, 2.0 * A - 0.03, 2.0 * A + 0.02], [5.3 * A, 4.6 * A, 1.2 * A]])
    x = np.vstack([x, extra])
    v = np.vstack([v, np.zeros((2, 3))])
    out = {}
    for form in ("mlp", "fp32"):
        lat = _lattice(n, form)
        if form == "mlp":
            lat.set_mlp(nets)
        lat.set_state(x, v)
        lat.compute(energies=False)
        torch.cuda.synchronize()
        slots = lat.slots()
        out[form] = (lat.forces(), np.nonzero(slots < 0)[0])
        lat.close()
    F_mlp, run = out["mlp"]
    F_tab, run_t = out["fp32"]
    assert len(run) >= 2 and np.array_equal(run, run_t)
    err = np.abs(F_mlp[run] - F_tab[run]).max() / np.abs(F_tab[run]).max()
    print(f"run-away forces, learned vs table form: {err:.2e} ({len(run)} run-away atoms)", flush=True)
    assert err < 1e-3


def test_learned_vs_table_side_by_side(M, trainer, torch_cuda, orc):
    """What the learned form gains over the method without it (the spline tables of
    Sec. 4.1), on one thermal state: the bytes that hold f, phi and F, the force error
    against the oracle's table potential, and the stepping rate, side by side.  The
    networks hold the three functions in ~1/17 of the bytes of the tables' float64
    samples (and ~1/60 of the float32 records the table form reads), at a force error
    near 1e-3 against ~1e-5; they step slower (their SiLU evaluations cost more than
    the table look-ups they replace)."""
    import time
    torch = torch_cuda
    lat64 = _lattice(6, "fp64")
    nets, _, _ = _quick_fit(M, torch, trainer, lat64, iters=8000, seed=41)
    lat64.close()
    n = 24
    x, v, box = w.thermal_state(n, seed=5)
    pot = orc.Potential(orc.TABLE, tables=TABLES)
    ref = orc.eam(pot, x, box)
    rms = np.sqrt(np.mean(np.sum(ref["F"] ** 2, axis=1)))
    rows = {}
    for form in ("fp32", "mlp"):
        lat = _lattice(n, form)
        if form == "mlp":
            lat.set_mlp(nets)
        lat.set_state(x, v)
        lat.compute()
        torch.cuda.synchronize()
        err = float(np.max(np.linalg.norm(lat.forces() - ref["F"], axis=1)) / rms)
        lat.step(3, 1.0, 0.05)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(20, 1.0, 0.05)
        torch.cuda.synchronize()
        rate = len(x) * 20 / (time.perf_counter() - t0)
        lat.close()
        rows[form] = (err, rate)
    n_tab = sum(len(TABLES[k][2]) for k in ("f", "phi", "F"))
    table_bytes = 8 * n_tab                                  # float64 samples of the three tables
    records = 3 * (n_tab // 3 - 1) * 16 + 4095 * (16 + 24)    # float32 cubic records + the q-window
    weight_bytes = 3 * O.MLP_PARAMS * 2                      # bfloat16 weights of three networks
    _say(f"table form:   {table_bytes} B of samples ({records} B of float32 records), force error "
         f"{rows['fp32'][0]:.2e}, {rows['fp32'][1]:.3e} atom-steps/s")
    _say(f"learned form: {weight_bytes} B of weights, force error {rows['mlp'][0]:.2e}, "
         f"{rows['mlp'][1]:.3e} atom-steps/s")
    assert weight_bytes * 15 < table_bytes
    assert rows["fp32"][0] < 1e-4
    assert rows["mlp"][0] < 2e-2


def _splitmix64(z):
    z = (z + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def test_fused_fit_step_matches_oracle(M, trainer, torch_cuda, orc):
    """Two steps of misa_mlp_fit (the fused launch: partial gradients, their sum and
    the Adam update) against the oracle: the same SplitMix64 mini-batches, the
    Sobolev loss coefficients, the parameter gradient and two Adam updates."""
    torch = torch_cuda
    fn, n, batch, lr, lam, seed = 1, 3000, 200, 2e-3, 1.0, 77
    lo, hi = RANGES[fn]
    net = rand_net(500, fn)
    M.misa_mlp_trainer_set(trainer, fn, net)
    rng = np.random.default_rng(501)
    x = rng.uniform(lo, hi, n)
    y, dy, _ = orc.spline_eval(*TABLES[ORC_KEYS[fn]], x)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    M.misa_mlp_fit(trainer, fn, dev(x), dev(y), dev(dy),
                   dict(iters=2, batch=batch, quantize=0, lr=lr, lr_final=lr, seed=seed, **{"lambda": lam}))
    _, master = M.misa_mlp_trainer_get(trainer, fn)
    c, s = O.scaling(lo, hi)
    p = np.asarray(net["params"], dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(2):
        idx = np.array([_splitmix64(seed ^ _splitmix64((step * 0x100000001B3 + i) & 0xFFFFFFFFFFFFFFFF)) % n
                        for i in range(batch)])
        t = (x[idx] - c) * s
        yn, dyn = O.forward_t(p.astype(np.float32).astype(np.float64), t)
        cv, cd, _ = O.sobolev_coefs(yn, dyn, (y[idx] - net["y_shift"]) / net["y_scale"],
                                    dy[idx] / (net["y_scale"] * s), lam)
        g = O.param_grad(p.astype(np.float32).astype(np.float64), t, cv, cd)
        p, m, v = O.adam_step(p, g, m, v, step + 1, lr)
        p = p.astype(np.float32).astype(np.float64)  # float32 master weights
    err = np.abs(master - p)
    _say(f"fused fit, two steps: max |w - w_oracle| {err.max():.2e} (steps of size {lr})")
    # Adam's first steps move each weight by about lr whatever the gradient's size, so a
    # weight agrees to float32 rounding unless its gradient is too small to fix a sign
    assert np.sum(err > 1e-6 * np.abs(p).max()) <= 3
    assert err.max() <= 2.5 * lr


def test_fit_many_equals_separate_fits(M, torch_cuda):
    """misa_mlp_fit_many of three networks gives network fn bit for bit the weights of
    a misa_mlp_fit call of its own with the seed raised by fn."""
    torch = torch_cuda
    opts = dict(iters=40, batch=512, quantize=1, lr=5e-3, lr_final=1e-4, seed=3)
    rng = np.random.default_rng(602)
    data = {}
    for fn in FNS:
        lo, hi = RANGES[fn]
        x = rng.uniform(lo, hi, 5000)
        y, dy = np.sin(x), np.cos(x)
        data[fn] = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (x, y, dy)]
    got = {}
    for together in (True, False):
        t = M.misa_mlp_trainer_create(torch.cuda.current_stream().cuda_stream)
        for fn in FNS:
            M.misa_mlp_trainer_set(t, fn, rand_net(610 + fn, fn))
        if together:
            losses = M.misa_mlp_fit_many(t, FNS, *[[data[f][k] for f in FNS] for k in range(3)], opts)
        else:
            losses = [M.misa_mlp_fit(t, fn, *data[fn], dict(opts, seed=opts["seed"] + fn)) for fn in FNS]
        got[together] = ([M.misa_mlp_trainer_get(t, fn)[1] for fn in FNS], losses)
        M.misa_mlp_trainer_destroy(t)
    for fn in FNS:
        assert np.array_equal(got[True][0][fn], got[False][0][fn]), fn
    assert np.allclose(got[True][1], got[False][1], rtol=1e-12)
