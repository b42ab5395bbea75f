"""Throughput of the compact-WENO SSP-RK3 step on one MI355X.

Workload: 2D Euler, periodic [0,2]^2 on 2048 x 2048 cells, smooth density
wave rho = 1 + 0.2 sin(pi (x + y)), u = v = 0.7, p = 1 (exact cell averages,
seeded-free closed form), CFL-rule dt (w1 = 1/12) computed on the device every
step.  One bench step = one SSP-RK3 step: 3 stages x (x-lines, y-lines,
combine) over the whole grid.  Prints one JSON line.

Other workloads (one JSON line each, bounded runs):
  --workload sedov2d      quarter-plane near-vacuum blast, 1024^2, reflective
                          x=0 / y=0, transmissive far sides, mixed precision
                          (--precision fp64, --fv gauss, --full to t = 1 with
                          --checkpoint / --resume across runs)
  --workload ensemble     4096 seeded 1D Riemann problems, N in [256, 4096],
                          mixed precision, one persistent launch per stage,
                          hipGraph replay, per-problem dt
  --workload wave1d       Example 3.1 at N = 200, dt = w1 h^(5/3)/S, to t = 2
  --workload rarefaction1d / blast1d   the 1D positivity configurations, N = 4000
  --workload char1d       cost of the characteristic-wise against the component-wise
                          reconstruction (Tables 2-3: density wave, CFL 0.16, t = 2,
                          N = 28..224; and the N = 4000 double rarefaction per step)
  --workload char2d       the same on the 2D density wave (4x4 blocks per line):
                          ms per step of both reconstructions, N = 256..2048
  --dt-rule cfl|pp|restart   time-step rule of ensemble / rarefaction1d / blast1d
  --recon cweno|char      reconstruction of ensemble (FP64) / wave1d / rarefaction1d / blast1d
  --workload gauss2d      Gauss-node 2D operator against the line operator: error of L
                          on a smooth nonlinear flow and cost per step, N = 128..2048
  --workload copy         plain device copy of a known size (counter calibration)
  --workload accuracy     wall time against L1 error, FP64 and mixed, N = 128..2048

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--no-cpu] [--workload W]
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
FP64_PEAK_TFLOPS = 78.6         # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
BYTES_PER_CELL_UPDATE = 544.0   # algorithmic bytes of one 2D SSP-RK3 cell-update
BYTES_PER_SWEEP_CELL = 64.0     # line kernel: read the stage input, write L
# combine, averaged over the three stages: reads U0 (not in stage 1), Us, Lx,
# Ly and writes both layouts, 32 B per cell each: (160 + 192 + 192) / 3
BYTES_PER_COMBINE_CELL = 544.0 / 3.0
# Algorithmic FP64 operations of one line sweep per 2D cell (4 components),
# counted from the scheme's formulas (+ - * / sqrt = 1 each): indicators shared
# by the two sides 4 x 33, WENO-Z weights 4 x 2 x 23, rows 4 x 2 x 22,
# Thomas 4 x 2 x 8, limiter test (smooth data) 44, HLLC 108, flux difference 8.
FLOPS_PER_SWEEP_CELL = 716.0

# HBM traffic of the FP64 line kernels from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, 2048^2 density wave), scaled by the copy
# calibration: a 1 GiB device copy reads FETCH_SIZE 524300 KiB (x 2.0) and
# WRITE_SIZE 1048576 KiB (x 1.0).  Valid only for the kernel sources whose
# hash is recorded (profiles/line_kernel_2d_density_wave_2048_fp64.md);
# otherwise traffic is reported null.
TRAFFIC_RECORD = {
    "src_sha256": "c799dec158d8fbb4dbb4399ae5a1334a007458ef6a59c4d3a16c401b26ee4f43",
    "fetch_scale": 2.0, "write_scale": 1.0,
    "x": {"fetch_kib": 66010.0, "write_kib": 163970.0},
    "y": {"fetch_kib": 66310.9, "write_kib": 163840.0},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=12,
                    help="oracle steps of the full grid for cpu_baseline (about 10 s on 16 threads)")
    ap.add_argument("--workload", default="density2d",
                    choices=["density2d", "sedov2d", "ensemble", "wave1d", "rarefaction1d",
                             "blast1d", "copy", "accuracy", "char1d", "char2d", "gauss2d"])
    ap.add_argument("--dt-rule", default="cfl", choices=["cfl", "pp", "restart"],
                    help="ensemble / rarefaction1d / blast1d: averages' CFL, interface-state "
                         "bound, or the averages' CFL with a step redone at half dt")
    ap.add_argument("--recon", default="cweno", choices=["cweno", "char"],
                    help="wave1d / rarefaction1d / blast1d: component-wise or characteristic-wise")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--fv", default="line", choices=["line", "gauss"],
                    help="sedov2d: the 2D operator (one state pair per face, or Gauss nodes)")
    ap.add_argument("--full", action="store_true",
                    help="sedov2d / ensemble: run to the configuration's end time")
    ap.add_argument("--checkpoint", default=None,
                    help="sedov2d: write the state, t and step count to this .npz at the end")
    ap.add_argument("--resume", default=None,
                    help="sedov2d: continue from a --checkpoint file")
    ap.add_argument("--max-wall", type=float, default=240.0,
                    help="--full runs stop after this many seconds (sedov2d: the near-vacuum "
                         "centre makes t = 1 take ~1e7 steps; the FP64 ensemble under the "
                         "restart rule takes ~275 s, and a near-vacuum problem can keep the "
                         "CFL-rule run stepping past any cap)")
    return ap.parse_args()


def other_workload(args):
    """Bounded throughput runs of the other configurations (one JSON line)."""
    import numpy as np
    import torch

    import paper_1402_5618_amd as pp
    import workloads as W
    prec_name = args.precision or ("mixed" if args.workload in ("sedov2d", "ensemble") else "fp64")
    prec = pp.PP_MIXED if prec_name == "mixed" else pp.PP_FP64
    rule_id = {"cfl": pp.PP_DT_CFL, "pp": pp.PP_DT_PP, "restart": pp.PP_DT_RESTART}[args.dt_rule]
    recon_id = {"cweno": pp.PP_RECON_CWENO, "char": pp.PP_RECON_CHAR}[args.recon]
    out = {"unit": "cell-updates/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if prec_name == "fp64" else "f32+f64",
           "data": "synthetic", "warmup": 0}
    if args.workload == "copy":
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.update(metric="device copy GB/s (read + write)", unit="GB/s",
                   value=2 * nbytes * args.steps / dt / 1e9, steps=args.steps,
                   config={"workload": f"copy of {nbytes} bytes x {args.steps}"})
    elif args.workload == "accuracy":
        # cost against L1 error (the paper's Table 2 / Fig. 1 methodology) for
        # both forms of the compact scheme and the explicit WENO-JS / WENO-Z
        # schemes it is compared with: the 2D density wave to a fixed time on
        # N^2 grids
        T = 0.05
        rows = []
        forms = (("fp64", pp.PP_FP64, pp.PP_RECON_CWENO), ("mixed", pp.PP_MIXED, pp.PP_RECON_CWENO),
                 ("wenojs", pp.PP_FP64, pp.PP_RECON_WENOJS), ("wenoz", pp.PP_FP64, pp.PP_RECON_WENOZ))
        for n in (128, 256, 512, 1024, 2048):
            dx = 2.0 / n
            U0 = W.density_wave_2d(n, n)
            for name, pr, rc in forms:
                U = torch.tensor(U0, device="cuda")
                s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=(0, 0, 0, 0), precision=pr,
                              recon=rc)
                warm = U.clone()
                s.run(warm, T, 3, 1.0 / 12.0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t, k = s.run(U, T, 10 ** 7, 1.0 / 12.0)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                s.close()
                Uh = U.cpu().numpy()
                l1 = W.error_norms(Uh[0], W.density_wave_2d(n, n, t=t)[0], dx * dx)[0]
                rows.append({"n": n, "form": name, "steps": k, "wall_s": wall, "l1_rho": l1,
                             "cell_updates_per_s": n * n * k / wall})
                print(f"accuracy: n={n} {name} steps={k} wall={wall:.3f}s L1={l1:.3e}",
                      file=sys.stderr, flush=True)
        def equal_accuracy(other):
            # for each compact FP64 point, the cheapest `other` run with an L1
            # at least as small, if any, and the compact run's speedup over it
            eq = []
            for r in rows:
                if r["form"] != "fp64":
                    continue
                cands = [m for m in rows if m["form"] == other and m["l1_rho"] <= r["l1_rho"]]
                m = min(cands, key=lambda m: m["wall_s"]) if cands else None
                eq.append({"l1_fp64": r["l1_rho"], "n_fp64": r["n"],
                           "n_" + other: m["n"] if m else None,
                           "fp64_speedup": (m["wall_s"] / r["wall_s"]) if m else None})
            return eq
        eq = equal_accuracy("mixed")
        for e in eq:   # the mixed form's speedup over FP64 at equal accuracy
            sp = e.pop("fp64_speedup")
            e["mixed_speedup"] = 1.0 / sp if sp else None
        out.update(metric="wall time against L1 error, 2D density wave to t=0.05",
                   value=None, steps=None,
                   config={"workload": "2D density wave, periodic [0,2]^2, CFL 1/12, t = 0.05, "
                                       "N = 128..2048; compact scheme in FP64 and mixed, "
                                       "explicit WENO-JS and WENO-Z in FP64", "table": rows,
                           "equal_accuracy": eq,
                           "compact_vs_wenojs": equal_accuracy("wenojs"),
                           "compact_vs_wenoz": equal_accuracy("wenoz")})
    elif args.workload == "gauss2d":
        # the Gauss-node operator against the line operator on a smooth,
        # nonlinear 2D flow: the error of L against the exact cell average of
        # -div(f, g), and the cost of an SSP-RK3 step (timed over --steps
        # steps, per-sweep kernel times from HIP events), N = 128..2048
        rows = []
        for n in (128, 256, 512, 1024, 2048):
            U0 = W.smooth_flow_2d(n, n, quad=4)
            ex = W.smooth_flow_2d_divergence(n, n, quad=4)
            for fv, name in ((pp.PP_FV_LINE, "line"), (pp.PP_FV_GAUSS, "gauss")):
                s = pp.Solver(ndim=2, nx=n, ny=n, dx=1.0 / n, dy=1.0 / n, bc=(0, 0, 0, 0), fv=fv)
                U = torch.tensor(U0, device="cuda")
                L = torch.empty_like(U)
                s.rhs(U, L)
                torch.cuda.synchronize()
                l1 = float(np.abs(L.cpu().numpy() - ex).mean())
                s.run(U.clone(), 1e30, 2, 1.0 / 12.0)
                torch.cuda.synchronize()
                s.set_timing(True)
                t0 = time.perf_counter()
                _, k = s.run(U, 1e30, args.steps, 1.0 / 12.0)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                tm = s.get_timing()
                s.set_timing(False)
                s.close()
                rows.append({"n": n, "operator": name, "l1_L": l1, "steps": k,
                             "ms_per_step": 1e3 * wall / k, "cell_updates_per_s": n * n * k / wall,
                             "kernel_ms_per_launch": {q: v[0] / max(v[1], 1) for q, v in tm.items()}})
                print(f"gauss2d: n={n} {name} L1(L)={l1:.3e} {1e3 * wall / k:.3f} ms/step",
                      file=sys.stderr, flush=True)
        # cheapest line-operator grid whose L error is at least as small as
        # each Gauss-node grid's, and the cost ratio of their steps
        eq = []
        for r in rows:
            if r["operator"] != "gauss":
                continue
            c = [m for m in rows if m["operator"] == "line" and m["l1_L"] <= r["l1_L"]]
            m = min(c, key=lambda m: m["ms_per_step"]) if c else None
            eq.append({"n_gauss": r["n"], "l1_gauss": r["l1_L"], "n_line": m["n"] if m else None,
                       "gauss_step_speedup": (m["ms_per_step"] / r["ms_per_step"]) if m else None})
        g = [r for r in rows if r["operator"] == "gauss" and r["n"] == 2048][0]
        out.update(metric="cell-updates/s, 2D Gauss-node operator (3 nodes per face), FP64, 2048^2",
                   value=g["cell_updates_per_s"], steps=g["steps"], ms_per_step=g["ms_per_step"],
                   config={"workload": "smooth nonlinear 2D flow, periodic [0,1]^2, CFL 1/12, "
                                       f"{args.steps} steps per grid; N = 128..2048; Gauss-node "
                                       "and line (dimension-by-dimension) operators, FP64",
                           "table": rows, "equal_L_error": eq})
    elif args.workload == "sedov2d":
        n = 1024
        dx = 1.1 / n
        t_done, steps, flags, min_rho, min_p = 0.0, 0, 0, math.inf, math.inf
        steps_before, wall_before = 0, 0.0
        if args.resume:
            ck = np.load(args.resume)
            U = torch.tensor(ck["U"], device="cuda")
            t_done, steps_before = float(ck["t"]), int(ck["steps"])
            min_rho, min_p, wall_before = float(ck["min_rho"]), float(ck["min_p"]), float(ck["wall"])
        else:
            U = torch.tensor(W.sedov_corner_2d(n), device="cuda")
        fv_id = pp.PP_FV_GAUSS if args.fv == "gauss" else pp.PP_FV_LINE
        s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=(2, 1, 2, 1), precision=prec, fv=fv_id)
        torch.cuda.synchronize()
        # --full: to t = 1 in chunks of --steps steps (the state advances in
        # place; each chunk restarts the clock at the chunk's start), with the
        # status word and the minima checked after every chunk; otherwise one
        # chunk
        t0 = time.perf_counter()
        while True:
            try:
                t, k = s.run(U, 1.0 - t_done, args.steps, 1.0 / 12.0)
            except pp.PPError as e:
                flags = e.code
                break
            t_done += t
            steps += k
            Uh = U.cpu().numpy()
            min_rho = min(min_rho, float(Uh[0].min()))
            min_p = min(min_p, float(W.pressure(Uh).min()))
            if args.full:
                print(f"sedov2d: {steps_before + steps} steps, t = {t_done:.4f}, min rho {min_rho:.3e}, "
                      f"min p {min_p:.3e}, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
            if not args.full or t_done >= 1.0 - 1e-12 or k == 0 or \
                    time.perf_counter() - t0 > args.max_wall:
                break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        Uh = U.cpu().numpy()
        if args.checkpoint:
            np.savez(args.checkpoint, U=Uh, t=t_done, steps=steps_before + steps, min_rho=min_rho,
                     min_p=min_p, wall=wall_before + wall)
        out.update(metric="cell-updates/s, 2D Sedov-type blast 1024^2",
                   value=n * n * steps / wall if steps else None,
                   steps=steps, ms_per_step=1e3 * wall / steps if steps else None,
                   config={"workload": f"quarter-plane blast 1024^2 on [0,1.1]^2, {prec_name}, "
                                       f"{args.fv} operator, {steps} steps (t = {t_done:.4e} of 1.0)",
                           "steps_total": steps_before + steps, "wall_total_s": wall_before + wall,
                           "min_rho_over_run": min_rho, "min_p_over_run": min_p,
                           "final_min_rho": float(Uh[0].min()),
                           "final_min_p": float(W.pressure(Uh).min()), "status": flags,
                           "symmetry_rel": float(np.abs(Uh[0] - Uh[0].T).max() / Uh[0].max()),
                           "note": "minima sampled after each chunk of steps"})
        s.close()
    elif args.workload == "ensemble":
        ens = W.riemann_ensemble()
        nb = len(ens.lengths)
        U = torch.tensor(ens.U, device="cuda")
        s = pp.Solver(ndim=1, lengths=ens.lengths, dxs=ens.dx, bcs=[1] * (2 * nb), precision=prec,
                      batch_rule=rule_id, recon=recon_id)
        plan, plan_ms = s.batch_tune(U, 1.0 / 12.0)       # launch plan (length classes)
        s.batch_run(U.clone(), ens.t_end, 2, 1.0 / 12.0)   # warm-up (graph, kernels)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flags = 0
        t_min = None
        if args.full:
            # to t_end in pieces of `chunk` steps per problem (pp_cweno_batch_continue
            # resumes exactly), one progress line per piece on stderr
            chunk, cap = 2000, 2000
            try:
                prev = s.batch_run(U, ens.t_end, cap, 1.0 / 12.0)
            except pp.PPError as e:
                flags, prev = e.code, s.last_batch_steps()
            while True:
                cap += chunk
                try:
                    steps, ts = s.batch_continue(U, ens.t_end, cap, 1.0 / 12.0)
                except pp.PPError as e:
                    flags = e.code
                    steps, ts = s.last_batch_steps(), s.last_batch_times()
                t_min = min(ts)
                # a problem short of t_end that took no step in this piece was
                # retired with a non-finite dt (it left the admissible set)
                running = sum(1 for a, b in zip(steps, prev) if a > b)
                print(f"ensemble: {running} problems advanced, t_min {t_min:.4g} of {ens.t_end}, "
                      f"max steps {max(steps)}, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
                if running == 0 or time.perf_counter() - t0 > args.max_wall:
                    break
                prev = steps
        else:
            try:
                steps = s.batch_run(U, ens.t_end, args.steps, 1.0 / 12.0)
            except pp.PPError as e:
                steps, flags = s.last_batch_steps(), e.code
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        cu = float(np.dot(np.asarray(steps, dtype=np.float64), ens.lengths))
        Uh = U.cpu().numpy()
        p = W.pressure(Uh)
        out.update(metric="cell-updates/s, 4096-problem 1D Riemann ensemble",
                   value=cu / wall, steps=int(max(steps)), ms_per_step=1e3 * wall / max(steps),
                   config={"workload": f"{nb} Riemann problems, N in [256,4096] (sum "
                                       f"{int(ens.lengths.sum())} cells), {prec_name}, "
                                       f"{args.recon} reconstruction, " +
                                       (f"to t_end {ens.t_end} (problems at t_end: "
                                        f"{sum(1 for t in ts if t >= ens.t_end)}; slowest at "
                                        f"t = {t_min})" if args.full else
                                          f"{args.steps} steps per problem (bounded; t_end "
                                          f"{ens.t_end} not reached)"),
                           "launch_plan": plan, "plan_ms_per_step": plan_ms,
                           "dt_rule": args.dt_rule, "restarts": s.restarts(),
                           "short_of_t_end": ([(i, float(ts[i]), int(steps[i])) for i in range(nb)
                                               if ts[i] < ens.t_end][:16] if args.full else None),
                           "problems_out_of_G": int(sum(1 for i in range(nb) if
                                                        p[ens.offsets[i]:ens.offsets[i + 1]].min() <= 0
                                                        or Uh[0, ens.offsets[i]:ens.offsets[i + 1]].min() <= 0)),
                           "status": flags})
        s.close()
    elif args.workload == "char1d":
        # the paper's Tables 2-3 on the GPU: wall time and L1 of the density
        # wave for the component-wise and the characteristic-wise
        # reconstruction at lambda max(|u|+a) = 0.16 to t = 2, and the cost
        # per step of both on a 4000-cell line
        rows = []
        for n in (28, 56, 112, 224):
            h = 2.0 / n
            for name, rc in (("component-wise", pp.PP_RECON_CWENO), ("characteristic", pp.PP_RECON_CHAR)):
                s = pp.Solver(ndim=1, nx=n, dx=h, bc=(0, 0, 0, 0), recon=rc)
                U = torch.tensor(W.density_wave_1d(n), device="cuda")
                s.run(U.clone(), 2.0, 3, 0.16)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t, k = s.run(U, 2.0, 10 ** 8, 0.16)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                s.close()
                Uh = U.cpu().numpy()
                l1 = W.error_norms(Uh[0], W.density_wave_1d(n, t=t)[0], h)[0]
                rows.append({"n": n, "recon": name, "steps": k, "wall_s": wall, "l1_rho": l1,
                             "us_per_step": 1e6 * wall / k})
                print(f"char1d: n={n} {name} steps={k} wall={wall:.3f}s L1={l1:.3e}",
                      file=sys.stderr, flush=True)
        per_step = {}
        for name, rc in (("component-wise", pp.PP_RECON_CWENO), ("characteristic", pp.PP_RECON_CHAR)):
            s = pp.Solver(ndim=1, nx=4000, dx=2.0 / 4000, bc=(1, 1, 0, 0), recon=rc)
            U = torch.tensor(W.double_rarefaction_1d(4000), device="cuda")
            s.run(U.clone(), 0.6, 5, 1.0 / 12.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t, k = s.run(U, 0.6, 200, 1.0 / 12.0)
            torch.cuda.synchronize()
            per_step[name] = 1e6 * (time.perf_counter() - t0) / k
            s.close()
        ratio = [r2["wall_s"] / r1["wall_s"] for r1, r2 in zip(rows[0::2], rows[1::2])]
        out.update(metric="wall time of the characteristic against the component-wise "
                          "reconstruction, 1D density wave to t=2",
                   value=None, steps=None,
                   config={"workload": "1D density wave (Example 3.1), periodic [0,2], "
                                       "lambda max(|u|+a) = 0.16, t = 2, N = 28..224, FP64; "
                                       "double rarefaction N = 4000, 200 steps",
                           "table": rows, "char_over_component_wall": ratio,
                           "us_per_step_n4000": per_step,
                           "paper_char_over_component_cpu_n224": 29.22 / 8.86})
    elif args.workload == "char2d":
        # cost per step of the characteristic-wise against the component-wise
        # reconstruction on the 2D density wave (CFL 1/12), and their L1
        # after the timed steps (equal to roundoff: three fields are constant)
        rows = []
        for n in (256, 1024, 2048):
            h = 2.0 / n
            for name, rc in (("component-wise", pp.PP_RECON_CWENO), ("characteristic", pp.PP_RECON_CHAR)):
                s = pp.Solver(ndim=2, nx=n, ny=n, dx=h, dy=h, bc=(0, 0, 0, 0), recon=rc)
                U = torch.tensor(W.density_wave_2d(n, n), device="cuda")
                s.run(U.clone(), 10.0, 2, 1.0 / 12.0)
                torch.cuda.synchronize()
                k = 10
                t0 = time.perf_counter()
                t, k = s.run(U, 10.0, k, 1.0 / 12.0)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                s.close()
                Uh = U.cpu().numpy()
                l1 = float(np.abs(Uh[0] - W.density_wave_2d(n, n, t=t)[0]).mean())
                rows.append({"n": n, "recon": name, "steps": k, "ms_per_step": 1e3 * wall / k,
                             "l1_rho": l1})
                print(f"char2d: n={n} {name} {1e3 * wall / k:.3f} ms/step L1={l1:.3e}",
                      file=sys.stderr, flush=True)
        ratio = [r2["ms_per_step"] / r1["ms_per_step"] for r1, r2 in zip(rows[0::2], rows[1::2])]
        out.update(metric="ms per SSP-RK3 step of the characteristic against the component-wise "
                          "reconstruction, 2D density wave",
                   value=None, steps=None,
                   config={"workload": "2D density wave, periodic [0,2]^2, CFL 1/12, 10 steps, "
                                       "N = 256, 1024, 2048, FP64",
                           "table": rows, "char_over_component": ratio})
    else:
        if args.workload == "wave1d":
            n, h, U0, bc, T, rule = 200, 0.01, W.density_wave_1d(200), (0, 0), 2.0, pp.PP_DT_H53
        elif args.workload == "rarefaction1d":
            n, h, U0, bc, T, rule = 4000, 2.0 / 4000, W.double_rarefaction_1d(4000), (1, 1), 0.6, rule_id
        else:
            n, h, U0, bc, T, rule = 4000, 2.0 / 4000, W.vacuum_blast_1d(4000), (1, 1), 1e-3, rule_id
        U = torch.tensor(U0, device="cuda")
        s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0), precision=prec, recon=recon_id)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            t, steps = s.run(U, T, 10 ** 8, 1.0 / 12.0, rule)
            flags = 0
        except pp.PPError as e:
            t, steps, flags = T, -1, e.code
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        Uh = U.cpu().numpy()
        extra = {}
        if args.workload == "wave1d":
            extra["l1_rho_vs_exact"] = W.error_norms(Uh[0], W.density_wave_1d(n, t=t)[0], h)[0]
        out.update(metric=f"cell-updates/s, 1D {args.workload} N={n}",
                   value=(n * steps / wall) if steps > 0 else None, steps=steps,
                   ms_per_step=(1e3 * wall / steps) if steps > 0 else None,
                   config=dict(workload=f"1D {args.workload}, N={n}, to t={T}, {prec_name}, "
                                        f"{args.recon}, dt rule {args.dt_rule}",
                               min_rho=float(Uh[0].min()), min_p=float(W.pressure(Uh).min()),
                               status=flags, wall_s=wall, restarts=s.restarts(), **extra))
        s.close()
    print(json.dumps(out), flush=True)


def mixed_roofline(timing, cells):
    """The same algorithmic FP64-equivalent work per cell for the mixed form's
    dominant line kernel (its float and FP64 operations together), against
    the FP64 vector peak (non-packed FP32 issues at the same rate)."""
    dom = max(("x", "y"), key=lambda k: timing[k][0])
    avg_ms = timing[dom][0] / max(timing[dom][1], 1)
    tf = FLOPS_PER_SWEEP_CELL * cells / (avg_ms * 1e-3) / 1e12
    return {"kernel": dom, "avg_launch_ms": avg_ms, "achieved_TFLOPs": tf,
            "frac_of_78.6": tf / FP64_PEAK_TFLOPS,
            "hbm_algorithmic_GBs": BYTES_PER_SWEEP_CELL * cells / (avg_ms * 1e-3) / 1e9}


def kernel_source_hash():
    """sha256 of the HIP sources the traffic counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in ("ppcweno.hip", "ppc_device.h"):
        with open(os.path.join(ROOT, "paper_1402_5618_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def host_cpu():
    """Model name and clock of the host CPU (from /proc/cpuinfo)."""
    model, mhz = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if model is None and line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                if mhz is None and line.startswith("cpu MHz"):
                    mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return model, mhz


def cpu_baseline(n, steps):
    """The CPU oracle (unchanged, OpenMP over lines) on a bounded sample of the
    same workload: `steps` SSP-RK3 steps of the full grid on every host
    thread, and one step on a single thread."""
    import oracle
    import workloads as W
    U = W.density_wave_2d(n, n)
    dx = 2.0 / n
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.run_2d(U, (0, 0, 0, 0), dx, dx, 1e30, cfl=1.0 / 12.0, max_steps=steps)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.run_2d(U, (0, 0, 0, 0), dx, dx, 1e30, cfl=1.0 / 12.0, max_steps=1)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    model, mhz = host_cpu()
    return {"value": n * n * steps / dt, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of the full {n}x{n} grid ({dt:.1f} s, FP64)",
            "cpu_model": model, "cpu_mhz": mhz,
            "one_thread": {"value": n * n / dt1, "sample": f"1 step of the full grid ({dt1:.1f} s)"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is design-only here)", file=sys.stderr)
        sys.exit(2)
    if args.workload != "density2d":
        other_workload(args)
        return
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

    # dominant kernel of the step (a line kernel) and its roofline: it is
    # bound by FP64 VALU work, so the roofline is algorithmic FP64 operations
    # per launch over the measured launch time; its HBM rate is given beside
    dom = max(("x", "y"), key=lambda k: timing[k][0])
    ms_tot, launches = timing[dom]
    avg_ms = ms_tot / max(launches, 1)
    achieved_tflops = FLOPS_PER_SWEEP_CELL * cells / (avg_ms * 1e-3) / 1e12
    achieved_gbs = BYTES_PER_SWEEP_CELL * cells / (avg_ms * 1e-3) / 1e9
    traffic = None
    if TRAFFIC_RECORD is not None and TRAFFIC_RECORD["src_sha256"] == kernel_source_hash():
        rec = TRAFFIC_RECORD[dom]
        traffic = rec["fetch_kib"] * 1024 * TRAFFIC_RECORD["fetch_scale"] + \
            rec["write_kib"] * 1024 * TRAFFIC_RECORD["write_scale"]

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
            # the HBM-bound kernel of the step: algorithmic bytes per launch
            # (the stage average) over its HIP-event launch time
            "combine_hbm": {
                "achieved_GBs": BYTES_PER_COMBINE_CELL * n * n /
                (timing["combine"][0] / max(timing["combine"][1], 1) * 1e-3) / 1e9,
                "peak_GBs": HBM_PEAK_GBS,
            },
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
                "line_kernel_alu": mixed_roofline(rmx["timing"], cells),
            },
        },
        "roofline": {
            "bound": "alu",
            # what the counters show for this kernel: VALUBusy ~48 %, one
            # workgroup (2 waves per SIMD) per CU, 5.81e7 VALU wave
            # instructions per launch (a 95 us issue floor), so issue latency
            # rather than VALU throughput or HBM limits it
            "counters": "VALU issue latency: VALUBusy ~48 %, one workgroup per CU, "
                        "issue floor 95 us per launch",
            "kernel": {"x": "line_kernel x-lines", "y": "line_kernel y-lines"}[dom],
            "achieved": achieved_tflops,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "flops_per_cell": FLOPS_PER_SWEEP_CELL,
            "cells_per_launch": cells,
            "avg_launch_ms": avg_ms,
            "hbm_algorithmic_GBs": achieved_gbs,
            "hbm_frac": achieved_gbs / HBM_PEAK_GBS,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
