#!/usr/bin/env python3
"""Throughput of the coupled per-step update on one MI355X.

Headline workload: the electrified jet, 128 x 128 x 512 nodes (8.4 M), two
Shan-Chen components injected through a nozzle of radius 8 (1 % azimuthal
perturbation, Poiseuille inflow 0.02) towards a collector plane held at a
potential difference giving a mean E_z = 2e-3, generator-connected charge,
Carreau fluid (n = 0.4), FP32 populations, FP64 entropic alpha, 8 red-black
SOR sweeps of the Poisson equation every step.  One step = every stage of
the update (pull, densities, curvature and charge, Poisson, electric field,
forces, alpha, Carreau, collision) over the whole box.

The jet is first formed: `--form` steps (default 10000, the configured run
length) from the initial state, then checkpointed (populations and
potential).  Each alpha starter (series root, learned network, plain Newton
from 2) restarts from that checkpoint: one recorded step gives its alpha on
the checkpoint state (compared with plain Newton's), the autotuner picks the
launch mapping, then W warm-up steps and K timed steps replayed as captured
step graphs (wall clock between device synchronisations).  `value` is the
series starter's MLUPS; the learned and plain ones sit beside it.  A further
instance times every phase of the same window with HIP events (phases in
order on one stream): the per-kernel rooflines come from those times.

Also reported: the batched ensemble (256 boxes, learned starter), and the
CPU oracle timed on a bounded sample on the host.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS coupled step, % of HBM roofline; learned-α vs plain Newton, same accuracy"
HBM_PEAK_GBS = 8000.0
COPY_MIB = 256


def alpha_bytes_per_node(storage_bytes: int, ncomp: int) -> int:
    """Algorithmic HBM bytes of k_alpha per node: the 19 pulled populations of
    each component read once, alpha * beta (FP64) written per component, and
    the node's type byte."""
    return ncomp * 19 * storage_bytes + ncomp * 8 + 1


def collide_bytes_per_node(storage_bytes: int, field_bytes: int, ncomp: int) -> int:
    """Algorithmic HBM bytes of k_collide per node: the 19 pulled populations
    of each component read once and written once, alpha * beta read, the
    neighbour fields read once (psi per component, phi, |E|^2), the node's
    charge and component densities, and its type byte."""
    pops = 2 * ncomp * 19 * storage_bytes
    fields = (ncomp + 2 + 1 + ncomp) * field_bytes
    return pops + ncomp * 8 + fields + 1


def step_bytes_per_node(storage_bytes: int, ncomp: int, sor_sweeps: float) -> float:
    """Algorithmic bytes of a whole step per node: one read and one write of
    every population, the density/charge/potential fields materialised once
    (10 scalar fields written or read), 4 scalar fields per SOR sweep."""
    return 2 * ncomp * 19 * storage_bytes + 10 * storage_bytes + 4 * storage_bytes * sor_sweeps


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(inputs, budget_s: float = 12.0):
    """The FP64 oracle on the host: all threads on the headline jet (whole
    steps from its initial state, within the budget), one thread on the same
    jet geometry reduced to 48 x 48 x 128 (the full box takes tens of seconds
    per step on one thread)."""
    import oracle
    oracle.build(force=False)

    def run(wl, nthreads, budget, max_steps=50):
        o = oracle.Oracle(wl.params, wl.boxes[0], nthreads=nthreads)
        used = oracle.lib().ora_threads()
        t0 = time.perf_counter()
        n = 0
        while n < max_steps:
            o.step(1)
            n += 1
            if time.perf_counter() - t0 >= budget:
                break
        dt = time.perf_counter() - t0
        del o
        return wl.nodes * n / dt / 1e6, n, dt, used

    full = inputs.jet()
    v, n, dt, used = run(full, 0, budget_s)
    small = inputs.jet(nx=48, ny=48, nz=128, r_noz=8.0)
    v1, n1, dt1, _ = run(small, 1, 0.5 * budget_s)
    b = full.boxes[0]
    return {"value": round(v, 4), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"{n} steps of the {b.nx}x{b.ny}x{b.nz} jet from its initial state, FP64 oracle, "
                      f"{used} OpenMP threads, {dt:.1f} s",
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "single_thread": {"value": round(v1, 4), "unit": "MLUPS",
                              "sample": f"{n1} steps of the jet geometry reduced to 48x48x128, 1 thread, "
                                        f"{dt1:.1f} s"}}


# steps the autotuner advances the state (22 trials of 32 steps and 60 graph
# warm-up steps; elbm_autotune)
AUTOTUNE_STEPS = 22 * 32 + 60


def _ensemble_run(elbm, learned, wl, guess, launch, warm, steps):
    """One starter on the ensemble from its initial state: `warm` untimed
    steps at `launch` (None: the autotuner chooses it, its trials being the
    warm-up), then `steps` timed steps; returns the mapping, the autotuner's
    times, ms per step and the Newton updates per solved node-component."""
    import torch
    lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess=guess)
    if guess == "mlp":
        lat.mlp_set_weights(learned.load_weights())
    if launch:
        lat.set_launch(**launch)
        lat.step(warm, record=False)
        best, ms = launch, {}
    else:
        best, ms = lat.autotune(32)
    lat.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.step(steps, record=False)
    lat.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    lat.step(1, record=True)
    diags = [lat.diagnostics(i) for i in range(len(wl.boxes))]
    ncol = sum(d["n_collisions"] for d in diags)
    iters = sum(d["mean_newton_iters"] * (d["n_collisions"] - d["n_fallback"]) for d in diags)
    nfb = sum(d["n_fallback"] for d in diags)
    lat.close()
    return best, ms, dt / steps * 1e3, iters / max(ncol - nfb, 1)


def ensemble_leg(elbm, inputs, learned, steps: int, trial: int, launch=None, compare=("series", "standard")):
    """The batched ensemble: 256 independent periodic drop boxes (edges 24 to
    64, own radius, charge, field and Carreau exponent), FP32 populations,
    learned starter; the autotuner's trials serve as warm-up (or a given
    launch mapping and `trial` warm-up steps), then `steps` steps replayed as
    captured graphs of the chosen mapping.  Each starter in `compare` then
    runs the same number of steps from the same initial state at that
    mapping and is timed over the same window."""
    t0 = time.perf_counter()
    wl = inputs.ensemble()
    mode = "mlp" if os.path.exists(learned.WEIGHTS) else "series"
    print(f"[bench] ensemble: {len(wl.boxes)} boxes, {wl.nodes} nodes, guess {mode} "
          f"(inputs {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    warm = trial if launch else AUTOTUNE_STEPS
    best, ms, ms_step, iters = _ensemble_run(elbm, learned, wl, mode, launch, trial, steps)
    sb = step_bytes_per_node(4, wl.params.ncomp, wl.params.sor_sweeps)

    def rate(t):
        return wl.nodes / (t * 1e-3) / 1e6

    runs = {mode: {"mlups": round(rate(ms_step), 3), "ms_per_step": round(ms_step, 4),
                   "mean_newton_iters": round(iters, 4)}}
    for g in compare:
        if not g or g == mode:
            continue
        print(f"[bench] ensemble: starter {g}, {warm} + {steps} steps", file=sys.stderr, flush=True)
        _, _, t, it = _ensemble_run(elbm, learned, wl, g, best, warm, steps)
        runs[g] = {"mlups": round(rate(t), 3), "ms_per_step": round(t, 4), "mean_newton_iters": round(it, 4)}
    edges = sorted({b.nx for b in wl.boxes})
    return {
        "workload": f"ensemble: {len(wl.boxes)} periodic drop boxes, edges {edges}, FP32 populations, FP64 alpha",
        "nodes": wl.nodes,
        "steps": steps,
        "start_step": warm + 1,
        "mlups": round(rate(ms_step), 3),
        "ms_per_step": round(ms_step, 4),
        "hbm_frac": round(sb * rate(ms_step) * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
        "alpha_guess": mode,
        "mean_newton_iters": round(iters, 4),
        "starters": runs,
        "autotune": {"best": best, "ms_per_step": dict(
            [(f"tile{t}", round(float(ms[t]), 4)) for t in range(4)]
            + [(f"remap{r}", round(float(ms[4 + r]), 4)) for r in range(2)]
            + [(f"prio{r}", round(float(ms[6 + r]), 4)) for r in range(2)]
            + [(f"graph{g}", round(float(ms[8 + k]), 4)) for k, g in enumerate((2, 4, 8))]) if len(ms) else None},
    }


def parse_launch(text):
    v = [int(x) for x in text.split(",")]
    if len(v) not in (3, 4, 5):
        sys.exit(f"--launch takes remap,graph_steps,tile[,sweep_priority[,stencil_lds]], got {text!r}")
    return {"xcd_remap": v[0], "graph_steps": v[1], "tile": v[2], "sweep_priority": v[3] if len(v) >= 4 else 0,
            "stencil_lds": v[4] if len(v) == 5 else 0}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed steps after the warm-up (default 500)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps after the checkpoint and the autotuner")
    ap.add_argument("--form", type=int, default=10000,
                    help="steps that form the jet before the checkpoint (default 10000, the configured run)")
    ap.add_argument("--starters", default="series,mlp,standard",
                    help="alpha starters to time (the first is the reported value)")
    ap.add_argument("--launch", default=None,
                    help="launch mapping remap,graph_steps,tile[,sweep_priority[,stencil_lds]] for every starter "
                         "(no autotuner)")
    ap.add_argument("--phase-steps", type=int, default=50, help="steps of the per-phase event timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--ensemble-steps", type=int, default=100)
    ap.add_argument("--ensemble-starters", default="series,standard",
                    help="starters timed beside the learned one on the ensemble ('' for none)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the batched-ensemble leg (with --launch: that mapping, no autotuner)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              f"the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1612_05404_amd import elbm, inputs, learned

    # A plain device copy of known size (read + write of COPY_MIB each): the
    # reference that scales HBM traffic counters taken over this program.
    src = torch.ones(COPY_MIB << 18, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    if args.ensemble_only:
        launch = parse_launch(args.launch) if args.launch else None
        print(json.dumps({"ensemble": ensemble_leg(elbm, inputs, learned, args.ensemble_steps, trial=32,
                                                   launch=launch, compare=args.ensemble_starters.split(","))}),
              flush=True)
        return

    t0 = time.perf_counter()
    wl = inputs.jet()
    box = wl.boxes[0]
    nodes = wl.nodes
    have_net = os.path.exists(learned.WEIGHTS)
    starters = [m for m in args.starters.split(",") if m and (m != "mlp" or have_net)]
    if not starters:
        sys.exit("no alpha starter to time")
    print(f"[bench] jet {box.nx}x{box.ny}x{box.nz} (inputs {time.perf_counter() - t0:.1f} s), forming "
          f"{args.form} steps", file=sys.stderr, flush=True)

    def make(mode, launch=None):
        lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess=mode)
        if mode == "mlp":
            lat.mlp_set_weights(learned.load_weights())
        if launch:
            lat.set_launch(**launch)
        return lat

    # ---- formation run and checkpoint (series starter: the converged state
    # does not depend on the starter)
    t1 = time.perf_counter()
    lat = make("series")
    lat.step(args.form, record=True)
    lat.sync()
    f_ck = lat.get_populations(0)
    phi_ck = lat.read_potential(0)
    rho_ck, _ = lat.read_moments(0)
    form_diag = lat.diagnostics(0)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    liquid = int((rho_ck[0] > wl.params.rho_th).sum())
    print(f"[bench] formed in {time.perf_counter() - t1:.1f} s: {liquid} liquid nodes", file=sys.stderr, flush=True)

    def restore(mode, launch=None):
        lat = make(mode, launch)
        lat.set_populations(0, f_ck)
        lat.set_potential(0, phi_ck)
        return lat

    results, alphas = {}, {}
    ref_mode = "standard"
    for mode in starters + ([ref_mode] if ref_mode not in starters else []):
        timed = mode in starters
        print(f"[bench] starter {mode}", file=sys.stderr, flush=True)
        lat = restore(mode)
        lat.step(1, record=True)                 # alpha of every node on the checkpoint state
        al, it = lat.read_alpha(0)
        alphas[mode] = (al, it)
        if not timed:
            lat.close()
            continue
        launch = parse_launch(args.launch) if args.launch else None
        if launch:
            lat.set_launch(**launch)
        else:
            launch, _ = lat.autotune(16)
        lat.step(args.warmup, record=False)
        d0 = lat.diagnostics(0)
        lat.sync()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        lat.step(args.steps, record=False)
        lat.sync()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        lat.step(1, record=True)                 # solver statistics (outside the timed region)
        d1 = lat.diagnostics(0)
        lat.close()
        del lat
        torch.cuda.empty_cache()
        ncol = d1["n_collisions"] - d0["n_collisions"]
        nfb = d1["n_fallback"] - d0["n_fallback"]
        results[mode] = dict(dt=tb - ta, launch=launch, d1=d1, ncol=ncol, nfb=nfb,
                             neg=d1["n_negative"] - d0["n_negative"])

    # alpha of each starter against plain Newton on the checkpoint state
    a_ref, i_ref = alphas[ref_mode]
    fluid = ((box.node_type & 3) == inputs.FLUID)[None]
    for mode, (al, it) in alphas.items():
        if mode not in results:
            continue
        both = (it >= 0) & (i_ref >= 0) & fluid
        err = np.abs(al - a_ref)[both] / a_ref[both]
        results[mode]["alpha_err"] = float(err.max()) if err.size else 0.0
        results[mode]["same_fallbacks"] = bool(np.array_equal(it < 0, i_ref < 0))
        # mean updates of that one recorded step (the checkpoint state)
        results[mode]["ck_iters"] = float(it[(it >= 0) & fluid].mean())
    del alphas

    # ---- per-phase device time of the same window (phases in order on one stream)
    head = starters[0]
    r = results[head]
    lat = restore(head, r["launch"])
    lat.step(1, record=False)
    lat.set_timing(True)
    lat.step(args.phase_steps, record=False)
    ph = lat.timing()
    lat.close()
    del lat, f_ck
    torch.cuda.empty_cache()
    nph = max(ph["steps"], 1)
    phase_ms = {k: v / nph for k, v in ph.items() if k != "steps"}

    esz = 4
    mlups = nodes * args.steps / r["dt"] / 1e6
    ms_step = r["dt"] / args.steps * 1e3
    sb = step_bytes_per_node(esz, wl.params.ncomp, wl.params.sor_sweeps)
    step_gbs = sb * nodes / (ms_step * 1e-3) / 1e9
    ab_ = alpha_bytes_per_node(esz, wl.params.ncomp)
    cb = collide_bytes_per_node(esz, 8, wl.params.ncomp)
    kernels = {}
    for k, nbytes in (("alpha", ab_), ("collide", cb)):
        ms = phase_ms[k]
        gbs = nbytes * nodes / (ms * 1e-3) / 1e9
        kernels["k_" + k] = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_node": nbytes,
                             "avg_ms": round(ms, 5)}
    starters_out = {}
    for mode, v in results.items():
        starters_out[mode] = {
            "mlups": round(nodes * args.steps / v["dt"] / 1e6, 3),
            "ms_per_step": round(v["dt"] / args.steps * 1e3, 4),
            "mean_newton_iters": round(v["d1"]["mean_newton_iters"], 4),
            "checkpoint_step_updates": round(v["ck_iters"], 4),
            "alpha_max_rel_err_vs_plain": v["alpha_err"],
            "same_fallback_nodes_as_plain": v["same_fallbacks"],
            "window_fallback_frac": round(v["nfb"] / max(v["ncol"], 1), 7),
            "window_negative_pop_frac": round(v["neg"] / max(19 * v["ncol"], 1), 8),
            "window_end_sor_residual_rel": round(v["d1"]["sor_residual"] / max(v["d1"]["sor_scale"], 1e-300), 6),
            "launch": v["launch"],
        }
    out = {
        "metric": METRIC,
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"jet: {box.nx}x{box.ny}x{box.nz} charged leaky-dielectric jet, nozzle radius 8, "
                        f"E_z 2e-3, Carreau n 0.4, generator charge, FP32 populations / FP64 fields, "
                        f"FP64 alpha, {wl.params.sor_sweeps} SOR sweeps/step",
            "nodes": nodes,
            "start_step": args.form + 1 + args.warmup,
            "formed_steps": args.form,
            "liquid_nodes_at_checkpoint": liquid,
            "sor_sweeps": wl.params.sor_sweeps,
            "alpha_guess": head,
            "alpha_precision": "f64",
            "launch": r["launch"],
        },
        "roofline": {
            "kernel": "coupled step (all kernels of one step)",
            "bound": "hbm",
            "achieved": round(step_gbs, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(step_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_node": sb,
            "avg_ms": round(ms_step, 5),
        },
        "roofline_kernels": kernels,
        "phase_ms_per_step": {k: round(v, 5) for k, v in phase_ms.items()},
        "phase_steps": args.phase_steps,
        "starters": starters_out,
        "formation": {"steps": args.form, "mean_newton_iters": round(form_diag["mean_newton_iters"], 4),
                      "fallback_frac": round(form_diag["n_fallback"] / max(form_diag["n_collisions"], 1), 7),
                      "sor_residual_rel": round(form_diag["sor_residual"] / max(form_diag["sor_scale"], 1e-300), 6)},
    }
    if not args.no_ensemble:
        out["ensemble"] = ensemble_leg(elbm, inputs, learned, args.ensemble_steps, trial=32,
                                       compare=args.ensemble_starters.split(","))
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inputs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
