"""GPU parity at full workload sizes, in the launch configuration the benchmark
times: the 320^3-cell box (65.5 M atoms, five 2 keV recoils) and the 128^3-cell
box (4.2 M atoms, one 1 keV recoil at the centre) with the default 5000-point
tables (FP32: persistent LDS kernels with the fused final half-kick; FP64: the
tiled gather kernels), and the 256-box batch of uneven cascades.

The oracle cannot evaluate these boxes whole in test time, so it computes
sampled atoms one by one (exact, cell-binned, float64): random atoms plus the
recoil atoms and every atom within rc of them, which takes the run-away path.
Beside the samples go properties that hold at any size: sum of forces, the
kinetic energy and max |v| recounted from the returned state, the adaptive step
rule, the whole-box energy (4.2 M atoms) and a 10-step trajectory (4.2 M atoms).

Bars: FP64 forces within 1e-6 of the rms force (max |dF| / rms |F|), densities
and F' within 1e-12 relative; FP32 pair arithmetic within the loose bounds
derived for float32 sums (force 1e-3, density 1e-5 relative).  Beside the rms
measure, which the 25-50 eV/A forces next to the recoils inflate, every sampled
atom farther than 2 rc from all recoil atoms is held to a per-atom bound,
|dF_i| / max(|F_i|, rms over those atoms): 1e-9 (FP64), 1e-4 (FP32).  The
per-atom neighbour counts of the density pass equal the oracle's on the sample.
"""
import numpy as np
import pytest

import misa_workloads as w

pytestmark = pytest.mark.gpu

A, RC, DELTA, M = w.A_FE, w.RC, w.DELTA, w.MASS_FE
TABLES = w.potential_samples()
BARS = {"fp64": dict(F=1e-6, rho=1e-12, fp=1e-11, sumF=1e-9, Fth=1e-9),
        "fp32": dict(F=1e-3, rho=1e-5, fp=1e-5, sumF=1e-5, Fth=1e-4)}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def pot(orc):
    return orc.Potential(orc.TABLE, tables=TABLES)


def _say(msg):
    print(msg, flush=True)


def _sample(orc, x, box, rec, n_random, seed):
    """Random atoms, the recoil atoms and all atoms within rc of each recoil atom."""
    rng = np.random.default_rng(seed)
    picks = [rng.choice(len(x), size=n_random, replace=False), np.asarray(rec, dtype=np.int64)]
    for i in rec:
        picks.append(orc.neighbours(x, box, RC, int(i), cells=True))
    return np.unique(np.concatenate(picks))


def thermal_mask(x, box, sample, hot):
    """Sampled atoms farther than 2 rc from every atom of `hot` (minimum image)."""
    L = np.asarray(box)
    far = np.ones(len(sample), bool)
    for i in hot:
        d = x[sample] - x[int(i)]
        d -= L * np.rint(d / L)
        far &= np.einsum("ij,ij->i", d, d) > (2 * RC) ** 2
    return far


def _check_sampled(orc, pot, lat, box, sample, form, what, hot=()):
    """Per-atom rho, F', forces and neighbour counts of the lattice's current state on
    the sample; hot: the recoil atoms (their surroundings are excluded from the
    per-atom thermal measure)."""
    xg, vg = lat.get_state()
    F, rho, fp = lat.forces(), lat.rho(), lat.fprime()
    ref = orc.eam_sampled(pot, xg, box, sample)
    scale = max(float(np.sqrt(np.mean(ref["F"] ** 2))), 1e-3)
    ferr = float(np.max(np.abs(F[sample] - ref["F"]))) / scale
    nz = ref["rho"] > 0
    rerr = float(np.max(np.abs(rho[sample][nz] - ref["rho"][nz]) / ref["rho"][nz]))
    fperr = float(np.max(np.abs(fp[sample][nz] - ref["fp"][nz]) / np.abs(ref["fp"][nz])))
    th = thermal_mask(xg, box, sample, hot)
    fth = np.linalg.norm(ref["F"][th], axis=1)
    rms_th = float(np.sqrt(np.mean(fth ** 2)))
    dth = np.linalg.norm(F[sample][th] - ref["F"][th], axis=1)
    therr = float(np.max(dth / np.maximum(fth, rms_th)))
    _say(f"  {form} {what}: {len(sample)} sampled atoms, force {ferr:.2e} rho {rerr:.2e} F' {fperr:.2e}; "
         f"{int(th.sum())} thermal atoms, per-atom force {therr:.2e}")
    b = BARS[form]
    assert ferr <= b["F"] and rerr <= b["rho"] and fperr <= b["fp"], (form, what, ferr, rerr, fperr)
    assert therr <= b["Fth"], (form, what, therr)
    cnt = lat.neighbour_counts()[sample]
    assert np.array_equal(cnt, ref["npairs"]), (form, what, np.nonzero(cnt != ref["npairs"])[0][:8])
    lat.compute()  # the count export rebuilt the tables: densities and forces of this state again
    assert np.all(rho[sample][~nz] == 0.0)
    # Newton's third law over the whole box
    assert np.max(np.abs(F.sum(axis=0))) <= b["sumF"] * float(np.abs(F).sum()), (form, what)
    return xg, vg


def _check_stats(st, vg, dt_max, dx_max, what):
    """Statistics of a step call against a recount from the returned state."""
    ke = 0.5 * M * float(np.sum(vg * vg)) / w.ACC_A_FS2
    vmax = float(np.sqrt(np.max(np.sum(vg * vg, axis=1))))
    _say(f"  {what}: dt {st['dt']:.6f} fs, next {st['dt_next']:.6f} fs, run-aways {st['n_runaway']}, "
         f"e_kin {st['e_kin']:.6f} eV")
    assert abs(st["e_kin"] - ke) <= 1e-10 * ke, (what, st["e_kin"], ke)
    assert abs(st["vmax"] - vmax) <= 1e-12 * vmax, (what, st["vmax"], vmax)
    assert abs(st["dt_next"] - min(dt_max, dx_max / vmax)) <= 1e-12 * st["dt_next"], what
    assert st["overflow"] == 0 and st["range_violations"] == 0, what


@pytest.mark.parametrize("form", ["fp32", "fp64"])
def test_c3_full_box_sampled_parity(torch_cuda, orc, pot, form):
    """65,536,000 atoms: the state as placed, then after 20 adaptive steps in
    which the 2 keV recoils leave their sites."""
    torch = torch_cuda
    from paper_2107_07866_amd import Lattice
    cfg = w.CONFIGS["c3"]
    x, v, box, rec = w.make_state(cfg)
    _say(f"full 320^3 box, {form}: {len(x)} atoms, recoils {list(rec)}")
    sample = _sample(orc, x, box, rec, 2000, seed=7)
    lat = Lattice(cfg.n_cells, A, RC, DELTA, M, form)
    lat.set_tables(TABLES)
    lat.set_state(x, v)
    lat.compute()
    torch.cuda.synchronize()
    _check_sampled(orc, pot, lat, box, sample, form, "placed state", rec)
    st = lat.step(20, cfg.dt_max, cfg.dx_max)
    torch.cuda.synchronize()
    _, vg = _check_sampled(orc, pot, lat, box, sample, form, "after 20 steps", rec)
    _check_stats(st, vg, cfg.dt_max, cfg.dx_max, f"{form} 20 steps")
    assert st["n_runaway"] >= len(rec)
    d = lat.defects()
    assert d["runaway"] == st["n_runaway"] and d["vacancies"] == d["interstitials"], d
    lat.close()
    del lat
    torch.cuda.empty_cache()


def test_c2_full_box_trajectory_and_energy(torch_cuda, orc, pot):
    """4,194,304 atoms, 1 keV recoil at the centre: FP64 positions, velocities, dt
    and energies against the oracle's own 10-step trajectory over the whole box;
    then both forms sampled after 40 steps, when the recoil runs away."""
    torch = torch_cuda
    from paper_2107_07866_amd import Lattice
    cfg = w.CONFIGS["c2"]
    x, v, box, rec = w.make_state(cfg)
    L = np.asarray(box)
    _say(f"full 128^3 box: {len(x)} atoms, recoil {list(rec)}")
    lat = Lattice(cfg.n_cells, A, RC, DELTA, M, "fp64")
    lat.set_tables(TABLES)
    lat.set_state(x, v)
    st = lat.step(10, cfg.dt_max, cfg.dx_max)
    torch.cuda.synchronize()
    xg, vg = lat.get_state()
    _say("  oracle: 10-step cell-binned trajectory of the whole box")
    xo, vo, _, log = orc.run(pot, x, v, box, M, 10, cfg.dt_max, dx_max=cfg.dx_max, cells=True)
    d = xg - xo
    d -= L * np.rint(d / L)
    dv = float(np.max(np.abs(vg - vo)))
    _say(f"  fp64 10 steps: max |dx| {np.max(np.abs(d)):.2e} A, max |dv| {dv:.2e} A/fs, "
         f"dt {st['dt']:.9f} vs {log[-1, 0]:.9f}")
    assert np.max(np.abs(d)) < 1e-8 and dv < 1e-8
    assert abs(st["dt"] - log[-1, 0]) <= 1e-12 * log[-1, 0]
    assert abs(st["e_kin"] - log[-1, 1]) <= 1e-10 * log[-1, 1]
    ref = orc.eam(pot, xg, box, cells=True)
    etot = ref["e_emb"] + ref["e_pair"]
    _say(f"  fp64 energy {st['e_emb'] + st['e_pair']:.9f} vs oracle {etot:.9f} eV")
    assert abs(st["e_emb"] + st["e_pair"] - etot) <= 1e-12 * abs(etot)
    _check_stats(st, vg, cfg.dt_max, cfg.dx_max, "fp64 10 steps")
    lat.close()

    sample = _sample(orc, x, box, rec, 10000, seed=8)
    for form in ("fp64", "fp32"):
        _say(f"full 128^3 box, {form}: 40 steps")
        lat = Lattice(cfg.n_cells, A, RC, DELTA, M, form)
        lat.set_tables(TABLES)
        lat.set_state(x, v)
        st = lat.step(40, cfg.dt_max, cfg.dx_max)
        torch.cuda.synchronize()
        xg, vg = _check_sampled(orc, pot, lat, box, sample, form, "after 40 steps", rec)
        _check_stats(st, vg, cfg.dt_max, cfg.dx_max, f"{form} 40 steps")
        assert st["n_runaway"] >= 1
        ref = orc.eam(pot, xg, box, cells=True)
        eerr = abs(st["e_emb"] + st["e_pair"] - ref["e_emb"] - ref["e_pair"]) / len(x)
        _say(f"  {form} energy error {eerr:.2e} eV/atom")
        assert eerr <= (1e-12 if form == "fp64" else 1e-5)
        lat.close()
    torch.cuda.empty_cache()


def test_c4_full_batch_sampled_parity(torch_cuda, orc, pot):
    """All 256 uneven boxes in one batch after the tile autotuner and 10 steps:
    every box's statistics against its returned state, sampled forces of six
    boxes against the oracle, and the largest box bit-identical to a run of its
    own handle."""
    torch = torch_cuda
    from paper_2107_07866_amd import Batch, Lattice
    cfg = w.BATCH_CONFIGS["c4"]
    boxes = w.make_batch(cfg)
    _say(f"full batch: {len(boxes)} boxes, {sum(len(b[1]) for b in boxes)} atoms")
    batch = Batch([b[0] for b in boxes], A, RC, DELTA, M, runaway_capacity=4096)
    batch.set_tables(TABLES)
    for k, b in enumerate(boxes):
        batch.boxes[k].set_state(b[1], b[2])
    tune = batch.autotune(2, cfg.dt_max, cfg.dx_max)
    _say(f"  autotune {tune}")
    sts = batch.step(10, cfg.dt_max, cfg.dx_max)
    torch.cuda.synchronize()
    steps = tune["steps_done"] + 10
    for k in range(len(boxes)):
        _, vg = batch.boxes[k].get_state()
        ke = 0.5 * M * float(np.sum(vg * vg)) / w.ACC_A_FS2
        assert abs(sts[k]["e_kin"] - ke) <= 1e-10 * ke, k
        assert sts[k]["steps"] == steps and sts[k]["overflow"] == 0, k
    sizes = [len(b[1]) for b in boxes]
    big, small = int(np.argmax(sizes)), int(np.argmin(sizes))
    rng = np.random.default_rng(9)
    pick = [big, small] + [int(k) for k in rng.choice(len(boxes), 4, replace=False)]
    for k in pick:
        n, _, _, box, rec, e_rec = boxes[k]
        xg, _ = batch.boxes[k].get_state()
        sample = _sample(orc, xg, box, rec, min(300, len(xg)), seed=k)
        ref = orc.eam_sampled(pot, xg, box, sample)
        F = batch.boxes[k].forces()
        ferr = float(np.max(np.abs(F[sample] - ref["F"]))) / float(np.sqrt(np.mean(ref["F"] ** 2)))
        _say(f"  box {k} {n} cells, {e_rec:.0f} eV: force {ferr:.2e} on {len(sample)} atoms, "
             f"run-aways {sts[k]['n_runaway']}")
        assert ferr <= BARS["fp32"]["F"], k
    # the largest box alone, same number of steps and the same step arguments
    n, x, v, _, _, _ = boxes[big]
    lat = Lattice(n, A, RC, DELTA, M, "fp32", runaway_capacity=4096)
    lat.set_tables(TABLES)
    lat.set_state(x, v)
    for _ in range(tune["steps_done"]):
        lat.step(1, cfg.dt_max, cfg.dx_max)
    st = lat.step(10, cfg.dt_max, cfg.dx_max)
    xs, vs = lat.get_state()
    xb, vb = batch.boxes[big].get_state()
    assert np.array_equal(xs, xb) and np.array_equal(vs, vb)
    assert st["dt"] == sts[big]["dt"] and st["n_runaway"] == sts[big]["n_runaway"]
    lat.close()
    batch.close()
    torch.cuda.empty_cache()
