"""Throughput of the compact-WENO SSP-RK3 step on one MI355X.

Workload: 2D Euler, periodic [0,2]^2 on 2048 x 2048 cells, smooth density
wave rho = 1 + 0.2 sin(pi (x + y)), u = v = 0.7, p = 1 (exact cell averages,
seeded-free closed form), CFL-rule dt (w1 = 1/12) computed on the device every
step.  One bench step = one SSP-RK3 step: 3 stages x (x-lines, y-lines,
combine) over the whole grid.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
BYTES_PER_CELL_UPDATE = 544.0   # algorithmic bytes of one 2D SSP-RK3 cell-update
BYTES_PER_SWEEP_CELL = 64.0     # line kernel: read the stage input, write L


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=4)
    return ap.parse_args()


def cpu_baseline(n, steps):
    """The CPU oracle (unchanged, OpenMP over lines) on a bounded sample of the
    same workload: `steps` SSP-RK3 steps of the full grid."""
    import oracle
    import workloads as W
    U = W.density_wave_2d(n, n)
    dx = 2.0 / n
    t0 = time.perf_counter()
    oracle.run_2d(U, (0, 0, 0, 0), dx, dx, 1e30, cfl=1.0 / 12.0, max_steps=steps)
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt, "unit": "cell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of the full {n}x{n} grid ({dt:.1f} s, FP64)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is design-only here)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1402_5618_amd as pp
    import workloads as W

    n = args.n
    dx = 2.0 / n
    U0 = torch.tensor(W.density_wave_2d(n, n), device="cuda")
    cfl = 1.0 / 12.0
    cells = n * n

    def measure(precision):
        solver = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=(0, 0, 0, 0), precision=precision)
        U = U0.clone()
        if args.warmup > 0:
            solver.run(U, 1e30, args.warmup, cfl)
        U.copy_(U0)
        torch.cuda.synchronize()
        solver.set_timing(True)
        t0 = time.perf_counter()
        t_reached, steps = solver.run(U, 1e30, args.steps, cfl)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        timing = solver.get_timing()
        solver.set_timing(False)
        assert steps == args.steps, (steps, args.steps)
        code, flags = solver.status()
        solver.close()
        ex = W.density_wave_2d(n, n, t=t_reached)
        Uh = U.cpu().numpy()
        return dict(wall=wall, steps=steps, t=t_reached, timing=timing, flags=flags, U=Uh,
                    l1=W.error_norms(Uh[0], ex[0], dx * dx)[0])

    r64 = measure(pp.PP_FP64)
    rmx = measure(pp.PP_MIXED)
    steps = r64["steps"]
    value = cells * steps / r64["wall"]
    ms_step = 1e3 * r64["wall"] / steps
    timing = r64["timing"]
    value_mx = cells * steps / rmx["wall"]
    l1_mx_vs_fp64 = float(np.abs(rmx["U"][0] - r64["U"][0]).sum() / np.abs(r64["U"][0]).sum())
    mass_drift = float(abs(rmx["U"][0].sum() - W.density_wave_2d(n, n)[0].sum())
                       / W.density_wave_2d(n, n)[0].sum())

    # dominant kernel of the step and its roofline (algorithmic bytes / launch)
    dom = max(timing, key=lambda k: timing[k][0])
    ms_tot, launches = timing[dom]
    avg_ms = ms_tot / max(launches, 1)
    if dom == "combine":
        bytes_launch = cells * (160.0 + 192.0 + 192.0) / 3.0
    else:
        bytes_launch = cells * BYTES_PER_SWEEP_CELL
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9

    line = {
        "metric": "cell-updates/s, 2D 2048^2 FP64 vs mixed-FP32 at fixed L1 error; % HBM BW",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D Euler smooth density wave, periodic {n}x{n}, SSP-RK3, "
                        f"CFL-rule dt (w1=1/12), {steps} steps; value = FP64 form",
            "nx": n, "ny": n, "precision": "fp64",
            "pct_hbm_algorithmic": 100.0 * value * BYTES_PER_CELL_UPDATE / (HBM_PEAK_GBS * 1e9),
            "l1_rho_vs_exact": r64["l1"],
            "t_reached": r64["t"],
            "status_flags": r64["flags"],
            "kernel_ms_per_launch": {k: (v[0] / max(v[1], 1)) for k, v in timing.items()},
            "mixed": {
                "value": value_mx,
                "ms_per_step": 1e3 * rmx["wall"] / steps,
                "speedup_vs_fp64": value_mx / value,
                "pct_hbm_algorithmic": 100.0 * value_mx * BYTES_PER_CELL_UPDATE / (HBM_PEAK_GBS * 1e9),
                "l1_rho_vs_exact": rmx["l1"],
                "l1_rho_rel_vs_fp64": l1_mx_vs_fp64,
                "mass_drift_rel": mass_drift,
                "status_flags": rmx["flags"],
                "kernel_ms_per_launch": {k: (v[0] / max(v[1], 1)) for k, v in rmx["timing"].items()},
            },
        },
        "roofline": {
            "bound": "hbm",
            "kernel": {"x": "line_kernel x-lines", "y": "line_kernel y-lines",
                       "combine": "combine2d_kernel"}[dom],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
