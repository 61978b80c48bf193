#!/usr/bin/env python3
"""Benchmark of the boundary-integral Poisson-Boltzmann hot path on one GPU.

One step = one complete solve of the workload through the C ABI: source
terms (Eq_Ss), restarted GMRES(10) on the direct-sum product
(eqdbef1)/(eqdbef2), and the solvation energy (solvation_energy), with the
inputs already resident on the device.  The headline solver is FP64
iterative refinement around FP32-pair GMRES cycles; the plain FP64 GMRES
solver is timed beside it on the same workload.

Printed (one JSON line on stdout):
  value      Gpair-kernels/s of the mixed solver over the whole step:
             (FP32 + FP64 products) x N(N-1) ordered pairs / wall time.
  roofline   the FP32-pair product kernel: 61 algorithmic FLOP per ordered
             pair x N(N-1) per launch / its average launch time (HIP events
             around every launch on the solver's stream, timed region only)
             against the published FP32 vector peak.
  cpu_baseline  the FP64 CPU oracle's product on the host cores.
  serving    solves/s and p50/p99 latency of the plain FP64 solver, the
             plain mixed solver and the served (batched, memory-admitted)
             mixed solver on a stream of uneven requests
             (paper_1301_5885_amd/serve.py).

Usage: python bench.py [--steps K] [--warmup W] [--workload kirkwood]
                       [--serve-requests 64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matvec Gpair-kernels/s + solves/s, mixed vs FP64 at <=1e-6 energy rel err"
FLOP_PER_PAIR = 61          # algorithmic count per ordered pair, FMA = 2
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}   # MI355X vector peaks
TOL = 1e-8                  # relative residual of every timed solve
WORKLOADS = {
    "kirkwood": "Kirkwood sphere: R=20 A, geodesic nu=32 (N=20480 flat triangles), "
                "Nc=200 charges uniform in r<=18 A, Q in {-1,+1}; eps1=1, eps2=80, "
                "kappa=0.1257/A; GMRES(10) to rel. residual 1e-8",
    "star": "Star-shaped surface R=30 A, nu=64 (N=81920), Nc=2000, Q~N(0,0.5^2); "
            "eps1=1, eps2=80, kappa=0.1257/A; GMRES(10) to rel. residual 1e-8",
    "born": "Born ion: sphere R=2 A, nu=8 (N=1280), one +1 charge at the centre; "
            "eps1=1, eps2=80, kappa=0.1257/A; GMRES(10) to rel. residual 1e-8",
    "large": "Large single solve: sphere R=40 A, nu=128 (N=327680), Nc=5000 charges in "
             "r<=36 A, Q~N(0,0.5^2); eps1=1, eps2=80, kappa=0.1257/A; GMRES(10) to rel. "
             "residual 1e-8",
}


SERVING_WORKLOAD = ("the first requests of a seeded 512-request stream: star-shaped surfaces, "
                    "N = 20 nu^2 log-uniform in [1280, 81920], Nc = N/40, Q~N(0,0.5^2) inside "
                    "0.8 r, kappa~U[0,0.3]; Poisson arrivals at 0.8 x the plain FP64 solver's "
                    "throughput, plus a saturation run")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("pair_math.h", "matvec.hip"):
        with open(os.path.join(ROOT, "paper_1301_5885_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key, workload):
    """HBM bytes per launch from a committed counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def valu_from_profiles(kernel_key, workload, avg_s):
    """Hardware VALU FLOPs per launch from the committed counter summary (if
    taken on the current kernel source), over this run's launch time."""
    path = os.path.join(ROOT, "profiles", f"valu_flops_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel_key)
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    tf = rec["hw_flop_per_launch"] / avg_s / 1e12
    return {"hw_flop_per_launch": rec["hw_flop_per_launch"], "tflops": round(tf, 3),
            "frac": round(tf / rec["peak"], 4),
            "source": f"rocprofv3 SQ_INSTS_VALU_FLOPS_* (profiles/valu_flops_{workload}.md)"}


def golden_energy(workload):
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_reference.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["energy_kcal_per_mol"]


def run_solver(ctx, gabi, torch, u, mode, steps, warmup, pairs):
    """Two timed passes of `steps` solves (each solve includes its energy):
    the first with kernel timing off gives the throughput; the second, the
    same solves with HIP events recorded around every pair-kernel launch
    (event-record nodes inside the replayed round graphs, which add about
    3 us per record), gives the kernel durations for the roofline."""
    for _ in range(warmup):
        ctx.solve_dev(u, tol=TOL, mode=mode)
        ctx.energy_dev(None)
    torch.cuda.synchronize()
    infos, energies = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(ctx.solve_dev(u, tol=TOL, mode=mode))
        energies.append(ctx.energy_dev(None))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for prec in (gabi.FP64, gabi.FP32_PAIR):
        ctx.kernel_time(prec, reset=True)
    ctx.set_kernel_timing(True)
    timed_infos = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        timed_infos.append(ctx.solve_dev(u, tol=TOL, mode=mode))
        ctx.energy_dev(None)
    torch.cuda.synchronize()
    elapsed_timed = time.perf_counter() - t1
    ctx.set_kernel_timing(False)
    kt = {}
    for prec, key in ((gabi.FP64, "fp64"), (gabi.FP32_PAIR, "fp32")):
        avg, cnt = ctx.kernel_time(prec, reset=True)
        kt[key] = (avg, cnt)
    p64 = sum(i["matvecs_fp64"] for i in infos)
    p32 = sum(i["matvecs_fp32"] for i in infos)
    return {
        "elapsed": elapsed, "infos": infos, "energies": energies,
        "products_fp64": p64, "products_fp32": p32,
        "gpairs_per_s": (p64 + p32) * pairs / elapsed / 1e9,
        "solves_per_s": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "timed_pass_ms_per_step": 1e3 * elapsed_timed / steps,
        "timed_products_fp64": sum(i["matvecs_fp64"] for i in timed_infos),
        "timed_products_fp32": sum(i["matvecs_fp32"] for i in timed_infos),
        "kernel_total_ms": {k: v[0] * v[1] for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
    }


def roofline(res, key, n, workload, gabi=None):
    products = res["timed_products_fp32" if key == "fp32" else "timed_products_fp64"]
    if products == 0:
        return None
    # every launch of the timed pass is timed; launches skipped after an early
    # stop of a cycle last a few microseconds and are charged to the real
    # products
    avg_s = res["kernel_total_ms"][key] / products / 1e3
    flop = FLOP_PER_PAIR * n * (n - 1)
    achieved = flop / avg_s / 1e12
    peak = PEAK_TFLOPS[key]
    t = traffic_from_profiles(f"pair_{key}", workload)
    bucket = n.bit_length() - 1
    scheme, R, blocks, tail = gabi.tune_get(gabi.FP32_PAIR if key == "fp32" else gabi.FP64,
                                            bucket)
    mixed = "true" if key == "fp32" else "false"
    kname = (f"gabi::sym_pair_kernel<{mixed}>" if scheme == gabi.SCHEME_SYMMETRIC
             else f"gabi::pair_kernel<{mixed}, {R}>")
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": t,
            "hw_valu": valu_from_profiles(key, workload, avg_s),
            "kernel": kname, "scheme": "symmetric" if scheme else "split",
            "target_blocks": blocks, "tail_pieces": tail,
            "avg_launch_ms": round(avg_s * 1e3, 5),
            "flop_per_launch": flop,
            "timing": "HIP events around every pair-kernel launch in a second timed pass "
                      f"of the same solves ({res['timed_pass_ms_per_step']:.3f} ms/step with "
                      "the event records)"}


def cpu_baseline(problem, seconds):
    """The FP64 oracle's product on the host cores: whole products when one
    takes at most `seconds` at about 1 Gpair/s, else rows of it (each row is
    a full sum over all sources, the same work per pair)."""
    import numpy as np
    import oracle
    el = oracle.mesh_elements(problem.V, problem.F)
    u = np.random.default_rng(0).normal(size=2 * el.n)
    args = (problem.eps1, problem.eps2, problem.kappa)
    full = el.n * (el.n - 1) <= seconds * 1e9
    if full:
        unit_pairs = el.n * (el.n - 1)
        run = lambda: oracle.matvec(el, u, *args)
        what = f"full FP64 products of the workload (N={el.n}, {unit_pairs} ordered pairs each)"
    else:
        nrows = int(max(64, min(2 * el.n, seconds * 1e9 / 4 / (el.n - 1))))
        rows = np.random.default_rng(1).choice(2 * el.n, nrows, replace=False)
        unit_pairs = nrows * (el.n - 1)
        run = lambda: oracle.matvec_rows(el, u, rows, *args)
        what = (f"samples of {nrows} random rows of the FP64 product (N={el.n}, "
                f"{unit_pairs} ordered pairs each)")
    reps, t0 = 0, time.perf_counter()
    while True:
        run()
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    elapsed = time.perf_counter() - t0
    out = {"value": round(reps * unit_pairs / elapsed / 1e9, 5), "unit": "Gpair-kernels/s",
           "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{reps} {what}, {elapsed:.1f} s wall"}
    # the same oracle on one core, to set beside single-core CPU figures
    cores = oracle.num_threads()
    nrows1 = int(max(16, min(2 * el.n, seconds * 0.25 * 0.08e9 / (el.n - 1))))
    rows1 = np.random.default_rng(2).choice(2 * el.n, nrows1, replace=False)
    oracle.set_num_threads(1)
    try:
        reps1, t1 = 0, time.perf_counter()
        while True:
            oracle.matvec_rows(el, u, rows1, *args)
            reps1 += 1
            if time.perf_counter() - t1 >= seconds * 0.25:
                break
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(cores)
    out["one_core"] = {"value": round(reps1 * nrows1 * (el.n - 1) / el1 / 1e9, 5),
                       "sample": f"{reps1} samples of {nrows1} random rows, {el1:.1f} s wall"}
    return out


def warm_sequence(ctx, gabi, p, steps):
    """Solves along a sequence of nearby problems, the many-solves use case:
    every charge moves by an N(0, (0.05 A)^2) step per solve.  Mixed IR at the
    bench tolerance, from zero against from the previous solution (kept on
    the device, gabi_solve_opts.x0_previous); wall time per solve includes
    the charge upload, the solve and the energy.  Not the headline."""
    import numpy as np
    rng = np.random.default_rng(77)
    P = [p.pos.copy()]
    for _ in range(steps):
        P.append(P[-1] + rng.normal(scale=0.05, size=p.pos.shape))
    runs = {}
    for key, previous in (("cold", 0), ("warm", 1)):
        ctx.set_charges(P[0], p.q)
        ctx.solve(tol=TOL, mode=gabi.SOLVE_MIXED_IR)
        its, energies, seconds = [], [], 0.0
        for Pk in P[1:]:
            t0 = time.perf_counter()
            ctx.set_charges(Pk, p.q)
            _, info = ctx.solve(tol=TOL, mode=gabi.SOLVE_MIXED_IR, x0_previous=previous)
            energies.append(ctx.energy())
            seconds += time.perf_counter() - t0
            if not info["converged"]:
                raise RuntimeError(f"{key} sequence solve did not converge: {info}")
            its.append(info["iterations"])
        runs[key] = (seconds, its, energies)
    (tc, ic, ec), (tw, iw, ew) = runs["cold"], runs["warm"]
    return {"steps": steps,
            "perturbation": "every charge moved by N(0, (0.05 A)^2) per solve",
            "cold_ms_per_solve": round(1e3 * tc / steps, 3),
            "warm_ms_per_solve": round(1e3 * tw / steps, 3),
            "cold_iterations_per_solve": sum(ic) / steps,
            "warm_iterations_per_solve": sum(iw) / steps,
            "max_energy_rel_diff_warm_vs_cold": max(abs(a / b - 1) for a, b in zip(ew, ec))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kirkwood", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the serving stream to serve after the single-solve "
                         "timing (0: skip; the stream has 512)")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--sequence-steps", type=int, default=8,
                    help="nearby problems solved cold and warm-started after the timing "
                         "(0: skip)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="before timing, run one device copy of this many MiB "
                         "(a kernel of known traffic for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not "
              "supported (the row-sharded multi-GPU product is a design only)",
              file=sys.stderr)
        sys.exit(2)

    from paper_1301_5885_amd import serve
    serve_problems = None
    if args.serve_requests > 0:
        # generated in a process pool, before anything touches the GPU
        log(f"[bench] generating {args.serve_requests} serving requests")
        serve_problems = serve.make_problems(args.serve_requests, 16)

    import torch
    from paper_1301_5885_amd import gabi
    from paper_1301_5885_amd.synth import config_problem

    p = config_problem(args.workload)
    n = p.n
    pairs = n * (n - 1)
    log(f"[bench] workload {args.workload} N={n} Nc={p.nc}")
    if args.copy_mb:
        a = torch.ones(args.copy_mb * 131072, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_mb} MiB read + written")
        del a, b
    ctx = gabi.Context(0)
    ctx.load_problem(p)
    u = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    E_ref = golden_energy(args.workload)

    results = {}
    for key, mode in (("mixed", gabi.SOLVE_MIXED_IR), ("fp64", gabi.SOLVE_FP64)):
        log(f"[bench] timing {key}: {args.warmup} warmup + {args.steps} steps")
        r = run_solver(ctx, gabi, torch, u, mode, args.steps, args.warmup, pairs)
        E = r["energies"][-1]
        r["energy"] = E
        r["energy_rel_err"] = abs(E / E_ref - 1) if E_ref else None
        results[key] = r
        log(f"[bench] {key}: {r['ms_per_step']:.3f} ms/step, "
            f"{r['gpairs_per_s']:.1f} Gpairs/s, E={E:.8f}, err={r['energy_rel_err']}")

    mixed, fp64 = results["mixed"], results["fp64"]
    line = {
        "metric": METRIC,
        "value": round(mixed["gpairs_per_s"], 3),
        "unit": "Gpair-kernels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair terms, f64 accumulation/Krylov/residual/energy",
        "data": "synthetic (seeded surface and charges)",
        "config": {"workload": WORKLOADS[args.workload], "N": n, "Nc": p.nc,
                   "eps1": p.eps1, "eps2": p.eps2, "kappa": p.kappa,
                   "restart": 10, "tol": TOL, "solver": "mixed IR (FP32-pair GMRES "
                   "cycles, FP64 residuals)", "parallelism": "single GPU"},
        "solves_per_s": round(mixed["solves_per_s"], 3),
        "energy_rel_err": mixed["energy_rel_err"],
        "products_per_solve": {"fp32": mixed["products_fp32"] / args.steps,
                               "fp64": mixed["products_fp64"] / args.steps},
        "roofline": roofline(mixed, "fp32", n, args.workload, gabi),
        "fp64_solver": {
            "value": round(fp64["gpairs_per_s"], 3), "unit": "Gpair-kernels/s",
            "solves_per_s": round(fp64["solves_per_s"], 3),
            "ms_per_step": round(fp64["ms_per_step"], 4),
            "energy_rel_err": fp64["energy_rel_err"],
            "products_per_solve": fp64["products_fp64"] / args.steps,
            "roofline": roofline(fp64, "fp64", n, args.workload, gabi),
        },
        "speedup_mixed_over_fp64": round(mixed["solves_per_s"] / fp64["solves_per_s"], 3),
    }
    if args.sequence_steps > 0:
        log(f"[bench] warm-started sequence: {args.sequence_steps} nearby problems")
        line["warm_sequence"] = warm_sequence(ctx, gabi, p, args.sequence_steps)
        log(f"[bench] sequence: {line['warm_sequence']}")
    ctx.close()
    if serve_problems is not None:
        log(f"[bench] serving {args.serve_requests} requests")
        line["serving"] = serve.run(args.serve_requests, args.serve_slots,
                                    problems=serve_problems)
        line["serving"]["workload"] = SERVING_WORKLOAD
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (oracle, ~{args.cpu_seconds:.0f} s)")
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
