#!/usr/bin/env python3
"""Throughput of the coupled per-step update on one MI355X.

Default workload: a charged drop between two fixed-potential electrodes
(64 x 64 x 128 nodes, two Shan-Chen components, uniform E_z = 1e-3, Carreau
fluid, FP32 populations and fields, FP64 entropic alpha, 8 red-black SOR
sweeps of the Poisson equation every step).  One step = every stage of the
update (pull, densities, curvature and charge, Poisson, electric field,
forces, alpha, Carreau, collision) over the whole box.

Prints one JSON line: MLUPS (million lattice-node updates per second) over K
steps replayed as captured step graphs, the roofline of the dominant kernel
(the collision) from HIP events on the library's stream over the next K
steps, and the CPU oracle timed on a bounded sample.
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


def collide_bytes_per_node(storage_bytes: int, ncomp: int) -> int:
    """Algorithmic HBM bytes of one collision per node: the 19 pulled
    populations of each component read once and written once, plus the
    neighbour fields read once (psi per component, phi, |E|^2) and the node's
    own charge, liquid density and type byte."""
    pops = 2 * ncomp * 19 * storage_bytes
    fields = (ncomp + 4) * storage_bytes + 1
    return pops + fields


def step_bytes_per_node(storage_bytes: int, ncomp: int, sor_sweeps: int) -> int:
    """Algorithmic bytes of a whole step per node: one read and one write of
    every population, the density/charge/potential fields materialised once
    (10 scalar fields written or read), 4 scalar fields per SOR sweep."""
    return 2 * ncomp * 19 * storage_bytes + 10 * storage_bytes + 4 * storage_bytes * sor_sweeps


def cpu_baseline(wl, budget_s: float = 12.0, max_steps: int = 20):
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="efield_drop", choices=["efield_drop", "jet", "drop32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--alpha-guess", default="series", choices=["series", "standard", "mlp"],
                    help="initial guess of the alpha Newton iteration for the reported value")
    ap.add_argument("--single-mode", action="store_true",
                    help="time only the reported guess (no comparison run)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              f"the update has no multi-GPU path in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1612_05404_amd import elbm, inputs

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
    results = {}
    for mode in modes:
        print(f"[bench] workload {wl.name} {box.nx}x{box.ny}x{box.nz} dtype {wl.dtype} sor_sweeps "
              f"{wl.params.sor_sweeps} alpha guess {mode}", file=sys.stderr, flush=True)
        lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess=mode)
        if mode == "mlp":
            lat.mlp_set_weights(learned.load_weights())
        lat.step(args.warmup, record=False)
        lat.sync()
        # timed region: K steps as replayed step graphs, wall clock between
        # device-wide synchronisations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(args.steps, record=False)
        lat.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # the next K steps with HIP events around every phase (direct
        # launches) for the per-kernel durations of the roofline
        lat.set_timing(True)
        lat.step(args.steps, record=False)
        ph = lat.timing()
        lat.set_timing(False)
        # one recorded step for the solver statistics (outside the timed region)
        lat.step(1, record=True)
        diag = lat.diagnostics(0)
        results[mode] = dict(dt=t1 - t0, ph=ph, diag=diag)
        lat.close()
        del lat
        torch.cuda.empty_cache()
        if args.single_mode:
            break
    r = results[args.alpha_guess]
    dt, ph, diag = r["dt"], r["ph"], r["diag"]
    mlups = nodes * args.steps / dt / 1e6
    steps_timed = max(ph["steps"], 1)
    coll_ms = ph["collide"] / steps_timed
    cb = collide_bytes_per_node(esz, wl.params.ncomp)
    achieved = cb * nodes / (coll_ms * 1e-3) / 1e9
    sb = step_bytes_per_node(esz, wl.params.ncomp, wl.params.sor_sweeps)
    comparison = {
        m: {"mlups": round(nodes * args.steps / v["dt"] / 1e6, 3),
            "collide_ms": round(v["ph"]["collide"] / max(v["ph"]["steps"], 1), 5),
            "mean_newton_iters": round(v["diag"]["mean_newton_iters"], 4)}
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
        },
        "roofline": {
            "kernel": "k_collide",
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_node": cb,
            "avg_ms": round(coll_ms, 5),
        },
        "step_effective_gbs": round(sb * mlups * 1e6 / 1e9, 2),
        "step_bytes_per_node": sb,
        "phase_ms_per_step": {k: round(v / steps_timed, 5) for k, v in ph.items() if k != "steps"},
        "mean_newton_iters": round(diag["mean_newton_iters"], 4),
        "alpha_fallback_frac": round(diag["n_fallback"] / max(diag["n_collisions"], 1), 6),
        "alpha_guess_comparison": comparison,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
