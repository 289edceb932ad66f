#!/usr/bin/env python3
"""Benchmark of the EAM lattice MD step (the MISA-MD hot path) on one MI355X.

Prints ONE JSON line.  `value` is atom-steps/s of the headline form (the first
of --forms) on the chosen workload; every form's atom-steps/s, per-kernel times
and errors go under "forms".  The errors are those of the initial state (the state
the run starts from) against a stored sample of FP64 oracle values
(tests/golden/bench_reference.json, written by make_bench_reference.py beside it):
the benchmark itself runs the oracle only for the cpu_baseline figure.

Workloads (synthetic, seeded; the recipe lives in misa_workloads.synth):
  c3: 320^3 BCC cells = 65,536,000 atoms, 300 K + 5 recoils at 2 keV, adaptive dt
      (0.05 A per step, at most 1 fs), FP32 pair arithmetic (one GPU's share at
      real shape);
  c2: 128^3 cells = 4,194,304 atoms, 1 recoil at 1 keV, adaptive dt;
  c1: 16^3 cells = 8,192 atoms, fixed dt = 1 fs.
Inputs are resident in HBM before the timed region; the timed region is
exactly --steps steps of misa_step between two synchronisations.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s + HBM GB/s: FP64-table vs FP32 vs MLP forms at stated force error"

# Algorithmic arithmetic per in-range pair (directed, i <- j), the figures the roofline is
# priced with: separation and distance, table index, spline value or derivatives, the
# force combination and its accumulation; square root and reciprocal not counted.
FLOP_RHO_PAIR = 22
FLOP_FORCE_PAIR = 34
# A second, instruction-level model, reported beside it: every stencil candidate pays the
# separation and squared distance (8); an in-range pair then pays index and cubic (10) in
# the density pass, index, both derivatives, combination and accumulation (21) in the
# force pass (the kernels work on r^2, so no square root or division is executed).
ALT_FLOP_CANDIDATE = 8
ALT_FLOP_RHO_PAIR = 10
ALT_FLOP_FORCE_PAIR = 21
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "mlp": 2500.0}  # mlp: dense bf16 matrix cores
# learned form: per network evaluation, the 1-32-32-1 layers' multiply-adds (2 flops each);
# the rho pass evaluates f (values), the force pass f and phi (values and input tangents)
FLOP_MLP_VALUE = 2 * (32 + 32 * 32 + 32)
FLOP_MLP_TANGENT = 2 * FLOP_MLP_VALUE
HBM_PEAK_GBS = 8000.0
# bytes each pass must move per atom (each datum once): u, v, F, rho, F' as stored per form.
# The FP32 form fuses the final half-kick into the force pass (it also reads and writes v).
BYTES_PER_ATOM_STEP = {
    "fp64": {"kick_drift": 120, "rho": 40, "force": 104, "final_kick": 0},
    "fp32": {"kick_drift": 108, "rho": 32, "force": 88, "final_kick": 0},
    "mlp": {"kick_drift": 108, "rho": 32, "force": 40, "final_kick": 60},
}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def train_learned_form(seed=11):
    """The learned form's networks: fit to 1e6 table samples each, then force matching
    on 1e4 atoms sampled from a C2 cascade run (outside every timed region)."""
    import torch

    import misa_workloads as w
    from paper_2107_07866_amd import Lattice, misa as M, surrogate as S

    info = {}
    t0 = time.time()
    lat = Lattice(8, w.A_FE, w.RC, w.DELTA, w.MASS_FE, "fp64")
    lat.set_tables(w.potential_samples())
    trainer, nets, losses, samples = S.fit_surrogates(lat.h, w.RC, n_samples=1_000_000, seed=seed)
    torch.cuda.synchronize()
    lat.close()
    info["fit_loss"] = {["f", "phi", "F"][k]: v for k, v in losses.items()}
    info["fit_s"] = round(time.time() - t0, 2)
    _log(f"[bench] mlp: fitted to table samples in {info['fit_s']} s, losses {info['fit_loss']}")
    t1 = time.time()
    data, run = S.cascade_snapshots(w.CONFIGS["c2"], n_env=10_000, snapshots=5, steps_between=200, seed=seed)
    n_env = data[3].numel()
    full = dict(batch=n_env, quantize=1, seed=seed)
    before = M.misa_mlp_force_match(trainer, *data, dict(full, iters=1, lr=1e-12, lr_final=1e-12))
    M.misa_mlp_force_match(trainer, *data, dict(iters=3000, batch=1024, quantize=1, lr=2e-4, lr_final=1e-6,
                                                seed=seed))
    after = M.misa_mlp_force_match(trainer, *data, dict(full, iters=1, lr=1e-12, lr_final=1e-12))
    nets = {fn: M.misa_mlp_trainer_get(trainer, fn)[0] for fn in (M.MISA_FN_F, M.MISA_FN_PHI, M.MISA_FN_EMB)}
    M.misa_mlp_trainer_destroy(trainer)
    del samples
    info.update(force_match_loss_before=before, force_match_loss_after=after, force_match_atoms=n_env,
                c2_snapshot_steps=run["steps"], force_match_s=round(time.time() - t1, 2),
                weights_bytes=3 * M.MISA_MLP_PARAMS * 2, table_bytes_fp64=3 * (w.N_TABLE - 1) * 4 * 8)
    _log(f"[bench] mlp: force matching on {n_env} atoms from C2 snapshots: loss {before:.3e} -> {after:.3e} "
         f"({info['force_match_s']} s)")
    return nets, info


REFERENCE = os.path.join(ROOT, "tests", "golden", "bench_reference.json")


def bench_reference(key):
    """Oracle values on the initial state of workload key (tests/golden/make_bench_reference.py
    writes them), or None."""
    try:
        with open(REFERENCE) as fh:
            return json.load(fh).get(key)
    except (OSError, ValueError):
        return None


def initial_state_errors(lat, ref, table_form):
    """Errors of the handle's rho, F' and forces on the stored oracle sample of its
    initial state (call right after set_state)."""
    import numpy as np
    import torch
    lat.compute()
    torch.cuda.synchronize()
    sample = np.asarray(ref["sample"], dtype=np.int64)
    Fr, rr, fpr = np.asarray(ref["F"]), np.asarray(ref["rho"]), np.asarray(ref["fp"])
    Fg, rg = lat.forces()[sample], lat.rho()[sample]
    out = {}
    scale = float(np.sqrt(np.mean(Fr ** 2)))
    out["force_err_max_rel_rms"] = float(np.max(np.abs(Fg - Fr))) / max(scale, 1e-3)
    # per atom, on sampled atoms farther than 2 rc from every recoil atom:
    # |dF_i| / max(|F_i|, rms |F| over those atoms)
    far = np.asarray(ref["far"], dtype=bool)
    if far.any():
        fth = np.linalg.norm(Fr[far], axis=1)
        rms_th = float(np.sqrt(np.mean(fth ** 2)))
        dth = np.linalg.norm(Fg[far] - Fr[far], axis=1)
        out["force_err_per_atom_thermal"] = float(np.max(dth / np.maximum(fth, rms_th)))
    out["thermal_sample"] = int(far.sum())
    nz = rr > 0
    out["rho_err_max_rel"] = float(np.max(np.abs(rg[nz] - rr[nz]) / rr[nz])) if nz.any() else 0.0
    # embedding energy per sampled atom: |F'| |d rho| to first order, so the density error bounds it
    out["emb_energy_err_max_eV"] = float(np.max(np.abs(fpr * (rg - rr))))
    out["force_err_sample"] = int(len(sample))
    out["mean_pairs_per_atom"] = float(np.mean(ref["npairs"]))
    if table_form:  # the pair set of the density pass, atom by atom
        out["pair_counts_equal_oracle"] = bool(np.array_equal(lat.neighbour_counts()[sample],
                                                              np.asarray(ref["npairs"])))
    return out


def run_form(form, x, v, box, cfg, steps, warmup, ref, nets=None, graph=False):
    import numpy as np
    import torch

    import misa_workloads as w
    from paper_2107_07866_amd import Lattice

    tabs = w.potential_samples()
    t0 = time.time()
    # fp32-half / mlp-half: the form with each pair evaluated once (coloured tiles)
    half = form in ("fp32-half", "mlp-half")
    lat = Lattice(cfg.n_cells, w.A_FE, w.RC, w.DELTA, w.MASS_FE, {"fp32-half": "fp32", "mlp-half": "mlp"}.get(form, form))
    lat.set_tables(tabs)
    if half:
        lat.set_pair_schedule("half")
    if nets is not None:
        lat.set_mlp(nets)
    lat.set_state(x, v)
    torch.cuda.synchronize()
    _log(f"[bench] {form}: state loaded in {time.time() - t0:.1f} s ({lat.state_bytes / 1e9:.2f} GB)")
    errs = {}
    if ref is not None:  # the initial state against the stored oracle sample (outside the timed region)
        errs = initial_state_errors(lat, ref, form not in ("mlp", "mlp-half"))
        _log(f"[bench] {form}: initial state: force error {errs['force_err_max_rel_rms']:.2e} (per atom, thermal "
             f"{errs.get('force_err_per_atom_thermal', float('nan')):.2e}), rho error {errs['rho_err_max_rel']:.2e}, "
             f"pair counts equal {errs.get('pair_counts_equal_oracle')} (oracle sample of {errs['force_err_sample']})")
    dx_max = cfg.dx_max
    if graph:  # steps replay a captured HIP graph (per-kernel event timing would disable it)
        lat.set_graph(True)
    if warmup > 0:
        lat.step(warmup, cfg.dt_max, dx_max)
    torch.cuda.synchronize()
    lat.set_timing(not graph)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = lat.step(steps, cfg.dt_max, dx_max)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    timing = lat.timing() if not graph else {}
    lat.set_timing(False)
    wall = t2 - t1
    n = x.shape[0]
    out = {
        "atom_steps_per_s": n * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "kernel_ms_per_step": {k: ms / max(steps, 1) for k, (ms, cnt) in timing.items()},
        "kernel_launches": {k: cnt for k, (ms, cnt) in timing.items()},
        "graph_replay": bool(graph),
        "last_dt_fs": st["dt"],
        "simulated_fs": st["time"],
        "n_runaway": st["n_runaway"],
        "range_violations": st["range_violations"],
        "e_kin_eV": st["e_kin"],
        "e_pot_eV": st["e_emb"] + st["e_pair"],
        "defects": lat.defects(),
    }
    _log(f"[bench] {form}: {out['atom_steps_per_s']:.3e} atom-steps/s, {out['ms_per_step']:.3f} ms/step, "
         f"run-aways {st['n_runaway']}")
    out.update(errs)
    out["K"] = int(lat.stencil().shape[1])
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def run_batch(cfg, steps, warmup, ref, seq_steps=20, graph=False):
    """Batched replicas: every box stepped by misa_batch_step; beside it the same boxes
    stepped one handle at a time (seq_steps steps each) for the gain of batching."""
    import numpy as np
    import torch

    import misa_workloads as w
    from paper_2107_07866_amd import Batch, Lattice, misa as M

    t0 = time.time()
    boxes = w.make_batch(cfg)
    n_atoms = sum(b[1].shape[0] for b in boxes)
    _log(f"[bench] {cfg.name}: {len(boxes)} boxes, {n_atoms} atoms generated in {time.time() - t0:.1f} s")
    tabs = w.potential_samples()
    t0 = time.time()
    # capacity = every atom of the largest box: the synthetic crystal loses its order after ~0.5 ps
    cap = max(2 * b[0] ** 3 for b in boxes)
    batch = Batch([b[0] for b in boxes], w.A_FE, w.RC, w.DELTA, w.MASS_FE, runaway_capacity=cap)
    _log(f"[bench] batch: {len(boxes)} handles created in {time.time() - t0:.1f} s")
    batch.set_tables(tabs)
    for k, b in enumerate(boxes):
        batch.boxes[k].set_state(b[1], b[2])
    torch.cuda.synchronize()
    _log(f"[bench] batch: tables and states loaded, {time.time() - t0:.1f} s")
    errs = []
    for e in (ref or []):  # stored oracle samples of the first boxes' initial states
        r = initial_state_errors(batch.boxes[e["box"]], e, True)
        errs.append(r)
    batch_err = {}
    if errs:
        batch_err["force_err_max_rel_rms"] = max(r["force_err_max_rel_rms"] for r in errs)
        batch_err["pair_counts_equal_oracle"] = all(r["pair_counts_equal_oracle"] for r in errs)
        batch_err["force_err_boxes"] = len(errs)
        _log(f"[bench] batch: initial states of {len(errs)} boxes: force error "
             f"{batch_err['force_err_max_rel_rms']:.2e}, pair counts equal {batch_err['pair_counts_equal_oracle']}")
    # tile shapes: the autotuner times both policies on the initial states, which are
    # then loaded again so that the warm-up and the timed steps start where they would
    tune = batch.autotune(max(2, warmup), cfg.dt_max, cfg.dx_max)
    shapes = [M.MISA_TILE_SHAPES[batch.tile_shape(k)] for k in range(len(boxes))]
    tune["boxes_off_8x8x8"] = int(sum(1 for s_ in shapes if s_ != (8, 8, 8)))
    _log(f"[bench] batch: tile autotune {tune}")
    for k, b in enumerate(boxes):
        batch.boxes[k].set_state(b[1], b[2])
    if graph:  # batched steps replay a captured HIP graph (per-kernel timing would disable it)
        batch.set_graph(True)
    if warmup > 0:
        batch.step(warmup, cfg.dt_max, cfg.dx_max, want_stats=False)
    torch.cuda.synchronize()
    _log(f"[bench] batch: {warmup} warm-up steps done, {time.time() - t0:.1f} s")
    M.misa_set_timing(batch.boxes[0].h, not graph)
    torch.cuda.synchronize()
    chunk = max(1, min(steps, 200))
    wall, done, st = 0.0, 0, None
    while done < steps:  # timed in chunks so that progress shows; the chunks' walls are summed
        k = min(chunk, steps - done)
        t1 = time.perf_counter()
        st = batch.step(k, cfg.dt_max, cfg.dx_max, want_stats=(done + k == steps))
        torch.cuda.synchronize()
        wall += time.perf_counter() - t1
        done += k
        _log(f"[bench] batch: {done}/{steps} steps, {1e3 * wall / done:.3f} ms/step")
    timing = M.misa_get_timing(batch.boxes[0].h)
    M.misa_set_timing(batch.boxes[0].h, False)
    out = {"atom_steps_per_s": n_atoms * steps / wall, "ms_per_step": 1e3 * wall / steps,
           "kernel_ms_per_step": {k: ms / steps for k, (ms, cnt) in timing.items()} if not graph else {},
           "graph_replay": bool(graph),
           "boxes": len(boxes), "atoms": n_atoms, "tile_autotune": tune,
           "n_runaway_total": int(sum(s["n_runaway"] for s in st)),
           "frenkel_pairs_total": int(sum(M.misa_defects(bx.h)["vacancies"] for bx in batch.boxes)),
           "simulated_fs_min": min(s["time"] for s in st), "simulated_fs_max": max(s["time"] for s in st),
           **batch_err}
    _log(f"[bench] batch: {out['atom_steps_per_s']:.3e} atom-steps/s, {out['ms_per_step']:.3f} ms/step, "
         f"run-aways {out['n_runaway_total']}")
    batch.close()
    del batch
    torch.cuda.empty_cache()
    # the same boxes, one handle and one misa_step call at a time
    seq = 0.0
    for b in boxes:
        lat = Lattice(b[0], w.A_FE, w.RC, w.DELTA, w.MASS_FE, "fp32")
        lat.set_tables(tabs)
        lat.set_state(b[1], b[2])
        lat.step(2, cfg.dt_max, cfg.dx_max)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        lat.step(seq_steps, cfg.dt_max, cfg.dx_max)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t2
        lat.close()
    out["one_box_at_a_time_atom_steps_per_s"] = n_atoms * seq_steps / seq
    _log(f"[bench] the same boxes one at a time: {out['one_box_at_a_time_atom_steps_per_s']:.3e} atom-steps/s")
    return out


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "k_force_lds_c3_fp32_hbm_counters.txt")
CSRC = os.path.join(ROOT, "paper_2107_07866_amd", "csrc")


STEP_SOURCES = ("integrate_kernels.hip", "lattice_lds_kernels.hip", "misa_internal.h")


def kernel_source_sha256():
    """sha256 over the sources of the kernels that move the C3 FP32 step's bytes (the
    persistent pair passes and the kick-drift; name and bytes, in this order)."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def counted_traffic():
    """From the committed rocprofv3 counter summary of the C3 FP32 step (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain-copy calibration): HBM bytes per launch of k_force_lds
    and per step, or None when a kernel source has changed since the counters were taken."""
    try:
        kv = {}
        for line in open(COUNTER_SUMMARY):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") != kernel_source_sha256():
            return None
        return {"dominant": float(kv["dominant_traffic_bytes"]), "step": float(kv["step_traffic_bytes"])}
    except (OSError, KeyError, ValueError):
        return None


def roofline(form, res, n_atoms):
    """Dominant lattice kernel (by measured time) against the ALU peak of its precision."""
    kms = res["kernel_ms_per_step"]
    if not kms:  # graph replay: no per-kernel timing
        return None
    dom = "force" if kms["force"] >= kms["rho"] else "rho"
    pairs = res.get("mean_pairs_per_atom", 58.0)
    avg_ms = kms[dom]
    peak = PEAK_TFLOPS[form]
    alt = None
    if form == "mlp":  # every stencil candidate runs the networks (the whole wave takes part)
        per_atom = res["K"] * (2 * FLOP_MLP_TANGENT if dom == "force" else FLOP_MLP_VALUE)
        model = "1-32-32-1 layer multiply-adds per stencil candidate"
    else:
        per_atom = pairs * (FLOP_FORCE_PAIR if dom == "force" else FLOP_RHO_PAIR)
        model = f"{FLOP_FORCE_PAIR if dom == 'force' else FLOP_RHO_PAIR} flops per in-range pair"
        alt_atom = res["K"] * ALT_FLOP_CANDIDATE + pairs * (ALT_FLOP_FORCE_PAIR if dom == "force"
                                                             else ALT_FLOP_RHO_PAIR)
        alt_ach = n_atoms * alt_atom / (avg_ms * 1e-3) / 1e12
        alt = {"flop_model": f"{ALT_FLOP_CANDIDATE} per candidate + "
                             f"{ALT_FLOP_FORCE_PAIR if dom == 'force' else ALT_FLOP_RHO_PAIR} per in-range pair",
               "flop_per_atom": round(alt_atom, 1), "achieved": round(alt_ach, 3), "frac": round(alt_ach / peak, 4)}
    achieved = n_atoms * per_atom / (avg_ms * 1e-3) / 1e12
    kname = {"fp32": f"k_{dom}_lds", "fp64": f"k_{dom}_lds64", "mlp": f"k_{dom}_mlp"}[form]
    counted = counted_traffic() if (form == "fp32" and dom == "force" and n_atoms == 65536000) else None
    out = {"kernel": kname, "bound": "mfma" if form == "mlp" else "alu",
           "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
           "traffic": counted["dominant"] if counted else None, "traffic_unit": "B/launch",
           "avg_launch_ms": round(avg_ms, 4), "flop_model": model, "algorithmic_flop_per_atom": round(per_atom, 1),
           "algorithmic_bytes_per_launch": n_atoms * (BYTES_PER_ATOM_STEP[form][dom])}
    if alt:
        out["instruction_model"] = alt
    return out


def cpu_baseline(cfg, x, v, box, budget_s=15.0):
    """The oracle (exact cell-binned FP64 EAM + velocity Verlet) on the workload's own
    state. A box of more than 2e6 atoms gets one step, its starting forces computed
    first and not timed; a smaller one as many steps as fit in budget_s."""
    import misa_workloads as w
    import oracle
    pot = oracle.Potential(oracle.TABLE, tables=w.potential_samples())
    N = x.shape[0]
    if N > 2_000_000:
        F = oracle.eam(pot, x, box, cells=True)["F"]
        t0 = time.perf_counter()
        oracle.run(pot, x, v, box, w.MASS_FE, 1, cfg.dt_max, dx_max=cfg.dx_max, cells=True, F=F)
        steps = 1
    else:
        steps, F = 0, None
        t0 = time.perf_counter()
        while True:
            x, v, F, _ = oracle.run(pot, x, v, box, w.MASS_FE, 5, cfg.dt_max, dx_max=cfg.dx_max, cells=True, F=F)
            steps += 5
            if time.perf_counter() - t0 > budget_s or steps >= 5000:
                break
    dt = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": N * steps / dt, "unit": "atom-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"{cfg.name}: the timed box itself ({N} atoms), {steps} step(s) from its start, exact "
                      f"cell-binned FP64 EAM from the same spline tables, {dt:.1f} s"
                      + (" (starting forces computed first, untimed)" if N > 2_000_000 else "")}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--graph", action="store_true",
                    help="replay each step from a captured HIP graph (no per-kernel breakdown then)")
    ap.add_argument("--forms", default=None,
                    help="comma list of fp32,fp64,fp32-half,mlp,mlp-half; first is the headline value (fp32 or fp64)")
    ap.add_argument("--mlp-steps", type=int, default=5, help="timed steps of the learned form (it is slower)")
    ap.add_argument("--no-error-check", dest="error_check", action="store_false",
                    help="skip the error report against the stored oracle sample of the initial state")
    ap.add_argument("--error-sample", type=int, default=None, help="0: the same as --no-error-check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (scale for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.error_sample == 0:
        args.error_check = False
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 1 << 30, "copy_calibration_bytes_written": 1 << 30}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only (spreading a box over GPUs by halo exchange is not implemented); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import misa_workloads as w

    if args.workload == "c4":
        cfg = w.BATCH_CONFIGS["c4"]
        # the recipe names 2000 steps; the synthetic BCC crystal stays ordered for ~0.5 ps only,
        # so the default times the first 400 steps (about 0.3 ps of dynamics)
        steps = args.steps if args.steps is not None else 400
        torch.cuda.set_device(0)
        res = run_batch(cfg, steps, args.warmup, bench_reference("c4") if args.error_check else None,
                        graph=args.graph)
        head = {"kernel_ms_per_step": res["kernel_ms_per_step"], "K": 64, "mean_pairs_per_atom": 58.0}
        line = {"metric": METRIC, "value": res["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1,
                "steps": steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": cfg.name, "boxes": res["boxes"], "atoms": res["atoms"],
                           "cells_per_axis": [cfg.n_min, cfg.n_max], "recoil_eV": [cfg.e_min, cfg.e_max],
                           "pair_precision": "fp32", "integration": "f64", "dt_max_fs": cfg.dt_max,
                           "dx_max_A": cfg.dx_max},
                "roofline": roofline("fp32", head, res["atoms"]), "forms": {"fp32": res},
                "cpu_baseline": None}
        print(json.dumps(line), flush=True)
        return
    cfg = w.CONFIGS[args.workload]
    steps = args.steps if args.steps is not None else cfg.steps
    forms = (args.forms or (cfg.precision + "," + ("fp64" if cfg.precision == "fp32" else "fp32")
                            + ",fp32-half,mlp,mlp-half")).split(",")
    if forms[0] not in ("fp32", "fp64"):
        raise SystemExit("the first form is the headline value: fp32 or fp64")
    torch.cuda.set_device(0)
    t0 = time.time()
    x, v, box, rec = w.make_state(cfg)
    _log(f"[bench] {cfg.name}: {x.shape[0]} atoms generated in {time.time() - t0:.1f} s; recoils {rec}")
    ref = bench_reference(args.workload) if args.error_check else None
    if ref is not None and ref.get("atoms") != x.shape[0]:
        raise SystemExit("stored oracle sample does not match the workload; rerun tests/golden/make_bench_reference.py")

    results = {}
    trained = None
    for form in forms:
        if form in ("mlp", "mlp-half"):
            if trained is None:
                trained = train_learned_form()
            nets, info = trained
            k = min(steps, args.mlp_steps)
            results[form] = run_form(form, x, v, box, cfg, k, min(args.warmup, 2), ref, nets=nets)
            results[form]["training"] = info
            results[form]["timed_steps"] = k
        else:
            results[form] = run_form(form, x, v, box, cfg, steps, args.warmup, ref, graph=args.graph)
    head = results[forms[0]]
    n = x.shape[0]
    bpa = sum(BYTES_PER_ATOM_STEP[forms[0]].values())
    line = {
        "metric": METRIC,
        "value": head["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if forms[0] == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "atoms": n, "cells": [cfg.n_cells] * 3,
                   "pair_precision": forms[0], "integration": "f64", "dt_max_fs": cfg.dt_max,
                   "dx_max_A": cfg.dx_max, "recoils": cfg.n_recoils, "recoil_eV": cfg.recoil_ev,
                   "temperature_K": cfg.temperature, "table_points": w.N_TABLE},
        "roofline": roofline(forms[0], head, n),
        "hbm_model": {"bytes_per_atom_step": bpa,
                      "achieved_GBps": round(head["atom_steps_per_s"] * bpa / 1e9, 1),
                      "frac": round(head["atom_steps_per_s"] * bpa / 1e9 / HBM_PEAK_GBS, 4)},
        "forms": results,
    }
    learned = [f for f in ("mlp-half", "mlp") if f in results]
    table = [f for f in ("fp32", "fp32-half", "fp64") if f in results]
    if learned and table:
        # what the learned form gains over the tables: bytes holding f, phi, F; force error; rate
        tabs = w.potential_samples()
        sample_bytes = 8 * sum(len(tabs[k][2]) for k in ("f", "phi", "F"))
        from paper_2107_07866_amd import misa as M
        weight_bytes = 3 * M.MISA_MLP_PARAMS * 2
        line["learned_vs_table"] = {
            "table": {"form": table[0], "bytes": sample_bytes, "bytes_of": "float64 samples of f, phi, F",
                      "atom_steps_per_s": results[table[0]]["atom_steps_per_s"],
                      "force_err_max_rel_rms": results[table[0]].get("force_err_max_rel_rms")},
            "learned": {"form": learned[0], "bytes": weight_bytes, "bytes_of": "bfloat16 weights of 3 networks",
                        "atom_steps_per_s": results[learned[0]]["atom_steps_per_s"],
                        "force_err_max_rel_rms": results[learned[0]].get("force_err_max_rel_rms")},
        }
    counted = counted_traffic() if (forms[0] == "fp32" and n == 65536000) else None
    line["hbm_model"]["counted_GBps"] = (round(counted["step"] / (head["ms_per_step"] * 1e-3) / 1e9, 1)
                                         if counted else None)
    line["hbm_model"]["counted_bytes_per_step"] = counted["step"] if counted else None
    # the paper's own figure, as context only: one SW26010 core group (1 MPE + 64 CPEs), FP64, 20,480,000
    # BCC Fe atoms, 10 steps in 21.29 s (Sec. 5.2, single core group evaluation), assuming all of it stepping
    line["paper_context"] = {"value": 20.48e6 * 10 / 21.2939, "unit": "atom-steps/s",
                             "hardware": "1 SW26010 core group (1 MPE + 64 CPEs)", "dtype": "f64",
                             "workload": "20,480,000-atom BCC Fe, 10 steps (derived from the run time)"}
    if not args.no_cpu_baseline:
        _log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(cfg, x, v, box)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
