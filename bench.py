#!/usr/bin/env python3
"""Throughput of the coupled per-step update on one MI355X.

Default workload: a charged drop between two fixed-potential electrodes
(64 x 64 x 128 nodes, two Shan-Chen components, uniform E_z = 1e-3, Carreau
fluid, FP32 populations and fields, FP64 entropic alpha, 8 red-black SOR
sweeps of the Poisson equation every step).  One step = every stage of the
update (pull, densities, curvature and charge, Poisson, electric field,
forces, alpha, Carreau, collision) over the whole box.

Prints one JSON line: MLUPS (million lattice-node updates per second) over K
steps (default 2000, the whole configured run, after W warm-up steps from the
initial state) replayed as captured step graphs, in the launch mapping the
autotuner chose on a separate instance; the per-phase breakdown of the same
W + K steps from HIP events on the library's stream (second instance, phases
in order on one stream); the rooflines of the two collision kernels from their
event-timed launches over steps 251..266, the window their hardware counters
are taken on (third instance): k_alpha, the dominant one, bound by FP64
arithmetic (its HBM roofline beside it), and k_collide against HBM; and the
CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS coupled step, % of HBM roofline; learned-α vs plain Newton, same accuracy"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
COPY_MIB = 256
ROOF_AT, ROOF_STEPS = 250, 16  # the roofline window: steps 251..266

# Counted with rocprofv3 --pmc on the default workload with the series
# starter and the autotuner's mapping, over the launches of steps 251..266
# (early steps need more Newton updates): FP64 operations per node of one
# k_alpha launch (64 lanes x (2 FMA + ADD + MUL + TRANS) wave instructions),
# and the HBM bytes of one launch of each kernel (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0, the factors a plain 256 MiB copy gives for the same
# counters).  None: not counted for the current kernels.
ALPHA_FP64_FLOP_PER_NODE = 10954
ALPHA_TRAFFIC_BYTES = 377_100_296
COLLIDE_TRAFFIC_BYTES = 216_229_999


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


def step_bytes_per_node(storage_bytes: int, ncomp: int, sor_sweeps: int) -> int:
    """Algorithmic bytes of a whole step per node: one read and one write of
    every population, the density/charge/potential fields materialised once
    (10 scalar fields written or read), 4 scalar fields per SOR sweep."""
    return 2 * ncomp * 19 * storage_bytes + 10 * storage_bytes + 4 * storage_bytes * sor_sweeps


def cpu_baseline(wl, budget_s: float = 15.0, max_steps: int = 200):
    import oracle
    oracle.build(force=False)
    box = wl.boxes[0]
    o = oracle.Oracle(wl.params, box, nthreads=0)
    threads = oracle.lib().ora_threads()
    t0 = time.perf_counter()
    n = 0
    while n < max_steps:
        o.step(1)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": box.n * n / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of the same {box.nx}x{box.ny}x{box.nz} box, FP64 oracle, "
                      f"{threads} OpenMP threads, {dt:.1f} s"}


def ensemble_leg(elbm, inputs, learned, steps: int, trial: int):
    """The batched ensemble: 256 independent periodic drop boxes (edges 24 to
    64, own radius, charge, field and Carreau exponent), FP32 populations,
    learned starter; the autotuner's trials serve as warm-up, then `steps`
    steps replayed as captured graphs of the chosen mapping."""
    import torch
    t0 = time.perf_counter()
    wl = inputs.ensemble()
    mode = "mlp" if os.path.exists(learned.WEIGHTS) else "series"
    print(f"[bench] ensemble: {len(wl.boxes)} boxes, {wl.nodes} nodes, guess {mode} "
          f"(inputs {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess=mode)
    if mode == "mlp":
        lat.mlp_set_weights(learned.load_weights())
    best, ms = lat.autotune(trial)
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
    edges = sorted({b.nx for b in wl.boxes})
    return {
        "workload": f"ensemble: {len(wl.boxes)} periodic drop boxes, edges {edges}, FP32 populations, FP64 alpha",
        "nodes": wl.nodes,
        "steps": steps,
        "mlups": round(wl.nodes * steps / dt / 1e6, 3),
        "ms_per_step": round(dt / steps * 1e3, 4),
        "alpha_guess": mode,
        "mean_newton_iters": round(iters / max(ncol - nfb, 1), 4),
        "autotune": {"best": best, "ms_per_step": dict(
            [(f"tile{t}", round(float(ms[t]), 4)) for t in range(4)]
            + [(f"remap{r}", round(float(ms[4 + r]), 4)) for r in range(2)]
            + [(f"graph{g}", round(float(ms[6 + k]), 4)) for k, g in enumerate((2, 4, 8))])},
    }


def jet_leg(elbm, inputs, learned, warmup: int, steps: int):
    """The jet (128x128x512, FP32, inlet disk and collector, Carreau, generator
    charge): after `warmup` steps and the autotuner, `steps` graph-replayed
    steps with each starter; MLUPS and mean Newton updates at identical alpha."""
    import torch
    t0 = time.perf_counter()
    wl = inputs.jet()
    b = wl.boxes[0]
    print(f"[bench] jet {b.nx}x{b.ny}x{b.nz} (inputs {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    out = {"workload": f"jet: {b.nx}x{b.ny}x{b.nz}, inlet disk r 8, E_z 2e-3, Carreau n 0.4, FP32 populations, "
                       f"FP64 alpha, {wl.params.sor_sweeps} SOR sweeps/step",
           "nodes": wl.nodes, "warmup": warmup, "steps": steps, "starters": {}}
    for mode in ("standard", "series", "mlp"):
        if mode == "mlp" and not os.path.exists(learned.WEIGHTS):
            continue
        lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess=mode)
        if mode == "mlp":
            lat.mlp_set_weights(learned.load_weights())
        lat.step(warmup, record=False)
        launch, _ = lat.autotune(16)
        lat.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat.step(steps, record=False)
        lat.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        lat.step(1, record=True)
        d = lat.diagnostics(0)
        out["starters"][mode] = {"mlups": round(wl.nodes * steps / dt / 1e6, 3),
                                 "mean_newton_iters": round(d["mean_newton_iters"], 4),
                                 "fallback_frac": round(d["n_fallback"] / max(d["n_collisions"], 1), 6),
                                 "launch": launch}
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000,
                    help="timed steps (default: the field drop's configured run length)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="efield_drop", choices=["efield_drop", "jet", "drop32", "ensemble"],
                    help="ensemble only with --roofline-only (the default run times it in its own leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--alpha-guess", default="series", choices=["series", "standard", "mlp"],
                    help="initial guess of the alpha Newton iteration for the reported value")
    ap.add_argument("--single-mode", action="store_true",
                    help="time only the reported guess (no comparison run)")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--ensemble-steps", type=int, default=100)
    ap.add_argument("--no-jet", action="store_true", help="skip the jet leg (three starters)")
    ap.add_argument("--jet-warmup", type=int, default=200)
    ap.add_argument("--jet-steps", type=int, default=100)
    ap.add_argument("--launch", default=None,
                    help="launch mapping remap,graph_steps,tile[,sweep_priority] (skips the autotuner)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the collision's roofline window (for counter runs)")
    args = ap.parse_args()
    if args.workload == "ensemble" and not args.roofline_only:
        ap.error("--workload ensemble serves --roofline-only counter runs; the default run times the ensemble itself")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              f"the update has no multi-GPU path in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1612_05404_amd import elbm, inputs

    # A plain device copy of known size (read + write of COPY_MIB each): the
    # reference that scales HBM traffic counters taken over this program.
    src = torch.ones(COPY_MIB << 18, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    wl = inputs.WORKLOADS[args.workload]()
    box = wl.boxes[0]
    nodes = wl.nodes
    esz = 8 if wl.dtype == "f64" else 4
    from paper_1612_05404_amd import learned
    have_net = os.path.exists(learned.WEIGHTS)
    if args.alpha_guess == "mlp" and not have_net:
        sys.exit(f"--alpha-guess mlp needs the stored network {learned.WEIGHTS}")
    modes = [args.alpha_guess] + [m for m in ("standard", "series", "mlp")
                                  if m != args.alpha_guess and (m != "mlp" or have_net)]
    def make(mode, launch=None):
        lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess=mode)
        if mode == "mlp":
            lat.mlp_set_weights(learned.load_weights())
        if launch:
            lat.set_launch(**launch)
        return lat

    def tuned_launch(mode):
        if args.launch:
            v = [int(x) for x in args.launch.split(",")]
            if len(v) not in (3, 4):
                sys.exit(f"--launch takes remap,graph_steps,tile[,sweep_priority], got {args.launch!r}")
            return {"xcd_remap": v[0], "graph_steps": v[1], "tile": v[2], "sweep_priority": v[3] if len(v) == 4 else 0}
        # tuned on a throw-away instance: the timed runs start from the initial state
        lat = make(mode)
        lat.step(args.warmup, record=False)
        launch, _ = lat.autotune(32)
        lat.close()
        return launch

    def roofline_window(mode, launch):
        # k_alpha and k_collide times over the window where the counters are taken
        lat = make(mode, launch)
        lat.step(ROOF_AT, record=False)
        lat.set_timing(True)
        lat.step(ROOF_STEPS, record=False)
        ph = lat.timing()
        lat.close()
        n = max(ph["steps"], 1)
        return ph["alpha"] / n, ph["collide"] / n

    if args.roofline_only:
        launch = tuned_launch(args.alpha_guess)
        ams, cms = roofline_window(args.alpha_guess, launch)
        print(json.dumps({"roofline_window": {"steps": [ROOF_AT + 1, ROOF_AT + ROOF_STEPS], "alpha_ms": round(ams, 5),
                                              "collide_ms": round(cms, 5), "launch": launch}}), flush=True)
        return

    results = {}
    for mode in modes:
        print(f"[bench] workload {wl.name} {box.nx}x{box.ny}x{box.nz} dtype {wl.dtype} sor_sweeps "
              f"{wl.params.sor_sweeps} alpha guess {mode}", file=sys.stderr, flush=True)
        launch = tuned_launch(mode)
        # timed region: W warm-up steps, then K steps as replayed step graphs,
        # wall clock between device-wide synchronisations
        lat = make(mode, launch)
        lat.step(args.warmup, record=False)
        lat.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(args.steps, record=False)
        lat.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # one recorded step for the solver statistics (outside the timed region)
        lat.step(1, record=True)
        diag = lat.diagnostics(0)
        lat.close()
        res = dict(dt=t1 - t0, diag=diag, launch=launch)
        if mode == args.alpha_guess:
            # the same W + K steps again with HIP events around every phase
            # (direct launches): the per-phase breakdown of the timed run
            lat = make(mode, launch)
            lat.step(args.warmup, record=False)
            lat.set_timing(True)
            lat.step(args.steps, record=False)
            res["ph"] = lat.timing()
            lat.close()
            res["roof_ms"] = roofline_window(mode, launch)
        results[mode] = res
        torch.cuda.empty_cache()
        if args.single_mode:
            break
    r = results[args.alpha_guess]
    dt, ph, diag = r["dt"], r["ph"], r["diag"]
    mlups = nodes * args.steps / dt / 1e6
    steps_timed = max(ph["steps"], 1)
    al_ms, co_ms = r["roof_ms"]
    fesz = 4 if wl.dtype == "f32all" else 8
    ab_ = alpha_bytes_per_node(esz, wl.params.ncomp)
    cb = collide_bytes_per_node(esz, fesz, wl.params.ncomp)
    al_gbs = ab_ * nodes / (al_ms * 1e-3) / 1e9
    co_gbs = cb * nodes / (co_ms * 1e-3) / 1e9
    counted = wl.name == "efield_drop" and args.alpha_guess == "series"
    flop = ALPHA_FP64_FLOP_PER_NODE if counted else None
    tflops = flop * nodes / (al_ms * 1e-3) / 1e12 if flop else None
    sb = step_bytes_per_node(esz, wl.params.ncomp, wl.params.sor_sweeps)
    comparison = {
        m: {"mlups": round(nodes * args.steps / v["dt"] / 1e6, 3),
            "mean_newton_iters": round(v["diag"]["mean_newton_iters"], 4),
            "launch": v["launch"]}
        for m, v in results.items()
    }
    out = {
        "metric": METRIC,
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {box.nx}x{box.ny}x{box.nz} two-component charged drop, "
                        f"FP32 populations, FP64 alpha, Carreau, {wl.params.sor_sweeps} SOR sweeps/step"
            if wl.name == "efield_drop" else f"{wl.name}: {box.nx}x{box.ny}x{box.nz}",
            "nodes": nodes,
            "sor_sweeps": wl.params.sor_sweeps,
            "alpha_guess": args.alpha_guess,
            "alpha_precision": "f64",
            "launch": r["launch"],
        },
        "roofline": {
            "kernel": "k_alpha",
            "bound": "alu",
            "achieved": round(tflops, 3) if tflops else None,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(tflops / FP64_PEAK_TFLOPS, 4) if tflops else None,
            "traffic": ALPHA_TRAFFIC_BYTES if counted else None,
            "fp64_flop_per_node": flop,
            "avg_ms": round(al_ms, 5),
            "window_steps": [ROOF_AT + 1, ROOF_AT + ROOF_STEPS],
        },
        "roofline_hbm": {
            "kernel": "k_alpha",
            "bound": "hbm",
            "achieved": round(al_gbs, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(al_gbs / HBM_PEAK_GBS, 4),
            "traffic": ALPHA_TRAFFIC_BYTES if counted else None,
            "bytes_per_node": ab_,
            "avg_ms": round(al_ms, 5),
        },
        "roofline_collide": {
            "kernel": "k_collide",
            "bound": "hbm",
            "achieved": round(co_gbs, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(co_gbs / HBM_PEAK_GBS, 4),
            "traffic": COLLIDE_TRAFFIC_BYTES if counted else None,
            "bytes_per_node": cb,
            "avg_ms": round(co_ms, 5),
        },
        "step_effective_gbs": round(sb * mlups * 1e6 / 1e9, 2),
        "step_bytes_per_node": sb,
        "phase_ms_per_step": {k: round(v / steps_timed, 5) for k, v in ph.items() if k != "steps"},
        "mean_newton_iters": round(diag["mean_newton_iters"], 4),
        "alpha_fallback_frac": round(diag["n_fallback"] / max(diag["n_collisions"], 1), 6),
        "alpha_guess_comparison": comparison,
    }
    if not args.no_ensemble and args.workload == "efield_drop":
        out["ensemble"] = ensemble_leg(elbm, inputs, learned, args.ensemble_steps, trial=32)
    if not args.no_jet and args.workload == "efield_drop":
        out["jet"] = jet_leg(elbm, inputs, learned, args.jet_warmup, args.jet_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
