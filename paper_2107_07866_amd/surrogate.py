"""Training pipeline of the learned form (orchestration over the C ABI).

Every numeric step runs in the library's HIP kernels: targets come from the
handle's float64 spline tables (misa_table_eval), the fit and the force matching
are misa_mlp_fit / misa_mlp_force_match, and force-matching data are collected
from a lattice state by misa_mlp_collect.  This module only draws the seeded
sample points and the initial weights and moves arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from . import misa as M

H = M.MISA_MLP_HIDDEN


def default_ranges(rc):
    """Input ranges served by the networks: pair distances from 1.6 A to the
    cut-off (lattice pairs sit far above 1.6 A; closer pairs take the tables) and
    densities 4 .. 36 around the perfect-lattice value 15.45."""
    return {M.MISA_FN_F: (1.6, rc), M.MISA_FN_PHI: (1.6, rc), M.MISA_FN_EMB: (4.0, 36.0)}


def init_params(rng):
    """Initial weights: W1 ~ N(0, 1), W2, w3 ~ N(0, 1/32), biases 0."""
    p = np.zeros(M.MISA_MLP_PARAMS, dtype=np.float64)
    p[0:H] = rng.normal(0.0, 1.0, H)
    p[2 * H:2 * H + H * H] = rng.normal(0.0, 1.0 / np.sqrt(H), H * H)
    p[3 * H + H * H:4 * H + H * H] = rng.normal(0.0, 1.0 / np.sqrt(H), H)
    return p.astype(np.float32)


def table_samples(h, fn, lo, hi, n, rng, device="cuda"):
    """n points uniform in [lo, hi] with the handle's table value and derivative (device tensors)."""
    x = torch.as_tensor(rng.uniform(lo, hi, n), dtype=torch.float64, device=device)
    y = torch.empty_like(x)
    dy = torch.empty_like(x)
    M.misa_table_eval(h, fn, x, y, dy)
    return x, y, dy


DEFAULT_FIT = dict(iters=120000, batch=4096, quantize=1, lr=5e-3, lr_final=1e-6, seed=7)


def fit_surrogates(h, rc, n_samples=1_000_000, seed=11, fit=None, ranges=None, trainer=None, device="cuda"):
    """Fit the three networks to n_samples table samples each.

    Returns (trainer, {fn: net dict}, {fn: final loss}, samples); samples keep the
    device arrays alive (the trainer keeps pointers to them for force matching)."""
    fit = dict(DEFAULT_FIT, **(fit or {}))
    ranges = ranges or default_ranges(rc)
    rng = np.random.default_rng(seed)
    t = trainer or M.misa_mlp_trainer_create(torch.cuda.current_stream().cuda_stream)
    nets, losses, samples = {}, {}, {}
    fns = (M.MISA_FN_F, M.MISA_FN_PHI, M.MISA_FN_EMB)
    for fn in fns:
        lo, hi = ranges[fn]
        x, y, dy = table_samples(h, fn, lo, hi, n_samples, rng, device)
        ys = y.double()
        net = {"x_lo": lo, "x_hi": hi, "y_shift": float(ys.mean()), "y_scale": float(ys.std()),
               "params": init_params(rng)}
        M.misa_mlp_trainer_set(t, fn, net)
        samples[fn] = (x, y, dy)
    # the three networks step together (one launch per optimiser step for all of them);
    # network fn draws its mini-batches with seed fit["seed"] + fn
    fitted = M.misa_mlp_fit_many(t, fns, [samples[f][0] for f in fns], [samples[f][1] for f in fns],
                                 [samples[f][2] for f in fns], fit)
    for fn, loss in zip(fns, fitted):
        losses[fn] = loss
        nets[fn], _ = M.misa_mlp_trainer_get(t, fn)
    return t, nets, losses, samples


def collect(h, sites, device="cuda"):
    """Force-matching data of the given lattice ids from the handle's current state."""
    n = len(sites)
    S = M.MISA_FM_SLOTS
    r = torch.empty(n * S, dtype=torch.float64, device=device)
    dhat = torch.empty(n * S * 3, dtype=torch.float64, device=device)
    fpj = torch.empty(n * S, dtype=torch.float64, device=device)
    fpi = torch.empty(n, dtype=torch.float64, device=device)
    fref = torch.empty(n * 3, dtype=torch.float64, device=device)
    M.misa_mlp_collect(h, np.asarray(sites, dtype=np.int64), r, dhat, fpj, fpi, fref)
    return r, dhat, fpj, fpi, fref


DEFAULT_FM = dict(iters=2000, batch=256, quantize=1, lr=1e-3, lr_final=1e-6, seed=13)


def force_match(trainer, data, fm=None):
    """Tune the f and phi networks on collected data; returns (loss, {fn: net})."""
    fm = dict(DEFAULT_FM, **(fm or {}))
    loss = M.misa_mlp_force_match(trainer, *data, fm)
    nets = {fn: M.misa_mlp_trainer_get(trainer, fn)[0] for fn in (M.MISA_FN_F, M.MISA_FN_PHI)}
    return loss, nets


def cascade_snapshots(cfg, n_env=10_000, snapshots=5, steps_between=200, seed=17, device="cuda"):
    """Force-matching data from a cascade run of a workload (float64 table form).

    The run starts from the workload's seeded initial state; after every
    steps_between steps (and at step 0) n_env / snapshots slotted atoms are
    sampled, half of them the closest to the first recoil atom and half uniformly,
    and their pair lists and table forces collected.  Returns the five device
    tensors of misa_mlp_collect, concatenated, and a short record of the run."""
    import misa_workloads as w
    from .lattice import Lattice

    x, v, box, rec = w.make_state(cfg)
    lat = Lattice(cfg.n_cells, w.A_FE, w.RC, w.DELTA, w.MASS_FE, "fp64")
    lat.set_tables(w.potential_samples())
    lat.set_state(x, v)
    rng = np.random.default_rng(seed)
    per = n_env // snapshots
    parts, info = [], {"steps": [], "n_runaway": []}
    L = np.asarray(box)
    for k in range(snapshots):
        if k:
            st = lat.step(steps_between, cfg.dt_max, cfg.dx_max)
            info["n_runaway"].append(int(st["n_runaway"]))
        info["steps"].append(k * steps_between)
        lat.compute(energies=False)
        xg, _ = lat.get_state()
        slots = lat.slots()
        ok = np.nonzero(slots >= 0)[0]
        centre = xg[rec[0]] if len(rec) else L / 2
        d = xg[ok] - centre
        d -= L * np.round(d / L)
        near = ok[np.argsort((d * d).sum(1))[: per // 2]]
        rest = np.setdiff1d(ok, near)
        far = rng.choice(rest, per - len(near), replace=False)
        parts.append(collect(lat.h, slots[np.concatenate([near, far])], device))
    lat.close()
    data = tuple(torch.cat([p[i] for p in parts]) for i in range(5))
    return data, info
