#!/usr/bin/env python3
"""Benchmark of the boundary-integral Poisson-Boltzmann hot path on one GPU.

One step = one complete solve of the workload through the C ABI: source
terms (Eq_Ss), restarted GMRES(20) on the direct-sum product
(eqdbef1)/(eqdbef2), and the solvation energy (solvation_energy), with the
inputs already resident on the device.  The headline solver is FP64
iterative refinement around FP32-pair GMRES cycles; the plain FP64 GMRES
solver is timed beside it on the same workload.

The default workload is the largest single-GPU one (sphere, N = 327,680).

Printed (one JSON line on stdout):
  value      Gpair-kernels/s of the mixed solver over the whole step:
             (FP32 + FP64 products) x N(N-1) ordered pairs / wall time.
  energy_rel_err, potential_err
             error of the energy and of phi/psi against the oracle's tight
             solve stored under tests/golden/ (sampled elements where the
             whole vector is not stored).
  roofline   the FP32-pair product kernel: 61 algorithmic FLOP per ordered
             pair x N(N-1) per product / its time per product (HIP events
             around the product's pair launches in separate event-timed
             solves) against the published FP32 vector peak; executed_frac
             is the rocprofv3 VALU FLOP count over the same time.
  fp64_solver  the plain FP64 GMRES solver on the same workload.
  tree_ir_solver  the treecode refinement on the same workload: GMRES(20)
             cycles on the treecode product inside FP64 refinement (solves/s,
             errors, speedup over the mixed and FP64 solvers).
  secondary  the same figures on a smaller workload (default kirkwood).
  cpu_baseline  the FP64 CPU oracle on the host cores: product rate, an
             extrapolated solve time at the workload, a measured solve of
             the secondary workload.
  serving    solves/s and p50/p99 latency of the plain FP64 solver, the
             plain mixed solver and the served (batched, memory-admitted)
             mixed solver on a stream of uneven requests
             (paper_1301_5885_amd/serve.py).

Usage: python bench.py [--steps K] [--warmup W] [--workload large]
                       [--serve-requests 512]
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
RESTART = 20                # GMRES(m) of every solver: the top of Section 2.4's 10-20
WORKLOADS = {
    "kirkwood": "Kirkwood sphere: R=20 A, geodesic nu=32 (N=20480 flat triangles), "
                "Nc=200 charges uniform in r<=18 A, Q in {-1,+1}; eps1=1, eps2=80, "
                "kappa=0.1257/A; GMRES(20) to rel. residual 1e-8",
    "star": "Star-shaped surface R=30 A, nu=64 (N=81920), Nc=2000, Q~N(0,0.5^2); "
            "eps1=1, eps2=80, kappa=0.1257/A; GMRES(20) to rel. residual 1e-8",
    "born": "Born ion: sphere R=2 A, nu=8 (N=1280), one +1 charge at the centre; "
            "eps1=1, eps2=80, kappa=0.1257/A; GMRES(20) to rel. residual 1e-8",
    "large": "Large single solve: sphere R=40 A, nu=128 (N=327680), Nc=5000 charges in "
             "r<=36 A, Q~N(0,0.5^2); eps1=1, eps2=80, kappa=0.1257/A; GMRES(20) to rel. "
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


def golden(workload):
    """Stored oracle values of the workload (tests/golden/, written by
    make_golden.py from the CPU oracle alone), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_reference.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def potential_errors(u, ref, n):
    """Error of phi and psi (Section 3.1, eq. (eqerr1): relative error of the
    surface potential) against the oracle's tight solve: over the whole
    vector where it is stored, else over its seeded sampled elements."""
    import numpy as np
    if ref is None:
        return None
    full = ref.get("full_u")
    if full:
        path = os.path.join(ROOT, "tests", "golden", full)
        if os.path.exists(path):
            r = np.load(path, allow_pickle=False)
            out = {"over": f"all {n} elements"}
            for key, a, b in (("phi", u[:n], r[:n]), ("psi", u[n:], r[n:])):
                out[f"{key}_rel_err"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
                out[f"{key}_max_rel_err"] = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
            return out
    smp = ref.get("samples")
    if not smp:
        return None
    idx = np.asarray(smp["index"], dtype=np.int64)
    out = {"over": f"{idx.size} sampled elements (seed {smp['seed']})"}
    for key, a, b in (("phi", u[idx], np.asarray(smp["phi"])),
                      ("psi", u[n + idx], np.asarray(smp["psi"]))):
        out[f"{key}_rel_err"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        out[f"{key}_max_rel_err"] = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    return out


def run_solver(ctx, gabi, torch, u, mode, steps, warmup, event_solves, pairs):
    """`steps` timed solves (each with its energy) with kernel timing off give
    the throughput; then `event_solves` more solves of the same problem with
    HIP events recorded around every product's pair-kernel launches
    (event-record nodes inside the replayed round graphs, about 3 us per
    record) give the kernel durations for the roofline."""
    for _ in range(warmup):
        ctx.solve_dev(u, tol=TOL, mode=mode, restart=RESTART)
        ctx.energy_dev(None)
    torch.cuda.synchronize()
    infos, energies = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(ctx.solve_dev(u, tol=TOL, mode=mode, restart=RESTART))
        energies.append(ctx.energy_dev(None))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    u_host = u.cpu().numpy()
    for prec in (gabi.FP64, gabi.FP32_PAIR):
        ctx.kernel_time(prec, reset=True)
    ctx.set_kernel_timing(True)
    timed_infos = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(event_solves):
        timed_infos.append(ctx.solve_dev(u, tol=TOL, mode=mode, restart=RESTART))
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
    ptree = sum(i.get("matvecs_tree", 0) for i in infos)
    return {
        "steps": steps, "elapsed": elapsed, "infos": infos, "energies": energies,
        "u": u_host,
        "products_fp64": p64, "products_fp32": p32, "products_tree": ptree,
        "gpairs_per_s": (p64 + p32) * pairs / elapsed / 1e9,
        "solves_per_s": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "event_solves": event_solves,
        "timed_pass_ms_per_step": 1e3 * elapsed_timed / max(1, event_solves),
        "timed_products_fp64": sum(i["matvecs_fp64"] for i in timed_infos),
        "timed_products_fp32": sum(i["matvecs_fp32"] for i in timed_infos),
        "kernel_total_ms": {k: v[0] * v[1] for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
    }


def roofline(res, key, n, workload, gabi=None):
    products = res["timed_products_fp32" if key == "fp32" else "timed_products_fp64"]
    if products == 0:
        return None
    # every product of the event pass is timed (from before its first pair
    # launch to after its last); launches skipped after an early stop of a
    # cycle last a few microseconds and are charged to the real products
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
    hw = valu_from_profiles(key, workload, avg_s)
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": t,
            "executed_frac": hw["frac"] if hw else None,
            "hw_valu": hw,
            "kernel": kname, "scheme": "symmetric" if scheme else "split",
            "target_blocks": blocks, "tail_pieces": tail,
            "avg_launch_ms": round(avg_s * 1e3, 5),
            "flop_per_launch": flop,
            "flop_basis": "algorithmic: 61 FLOP per ordered pair x N(N-1) per product; "
                          "executed_frac is the rocprofv3 VALU FLOP count of the same "
                          "kernel over this duration",
            "timing": f"HIP events around the pair-kernel launches of every product in "
                      f"{res['event_solves']} further solves of the same problem "
                      f"({res['timed_pass_ms_per_step']:.3f} ms/solve with the event records)"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _rows_rate(oracle, el, u, args, seconds, rng_seed, threads=None):
    """Gpair-kernels/s of the oracle's product on random rows (each row a
    full sum over all sources)."""
    import numpy as np
    rate_guess = 1e9 if threads is None else 0.08e9 * threads
    nrows = int(max(16, min(2 * el.n, seconds * rate_guess / 3 / (el.n - 1))))
    rows = np.random.default_rng(rng_seed).choice(2 * el.n, nrows, replace=False)
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.matvec_rows(el, u, rows, *args)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return reps * nrows * (el.n - 1) / dt / 1e9, f"{reps} samples of {nrows} random rows, " \
                                                  f"{dt:.1f} s wall"


def cpu_baseline(problem, seconds, fp64_products, small=None):
    """The FP64 CPU oracle on the host cores.

    value: Gpair-kernels/s of its product (rows of the workload's product;
    each row is a full sum over all sources), built as the CPU-baseline plan
    says (-O3 -march=native, no contraction: bitwise the default build).
    solve: the oracle's time for one whole solve of the workload, extrapolated
    as (products of an FP64 GMRES(m) solve at the bench tolerance) x (product
    time) + the source-term and energy sums at the same pair rate; small: one
    measured oracle solve (rhs + GMRES + energy) of a smaller workload."""
    import numpy as np
    import oracle
    el = oracle.mesh_elements(problem.V, problem.F)
    u = np.random.default_rng(0).normal(size=2 * el.n)
    args = (problem.eps1, problem.eps2, problem.kappa)
    cores = oracle.num_threads()
    out = {"unit": "Gpair-kernels/s", "cores": cores, "kind": "oracle",
           "cpu_model": _cpu_model(), "nproc": os.cpu_count()}
    oracle.use_native_build(True)
    try:
        rate, what = _rows_rate(oracle, el, u, args, seconds * 0.5, 1)
        out["value"] = round(rate, 5)
        out["build"] = "gcc " + " ".join(oracle.NATIVE_FLAGS) + " -fopenmp"
        out["sample"] = f"{what} of the FP64 product (N={el.n})"
        oracle.set_num_threads(1)
        try:
            r1, w1 = _rows_rate(oracle, el, u, args, seconds * 0.15, 2, threads=1)
        finally:
            oracle.set_num_threads(cores)
        out["one_core"] = {"value": round(r1, 5), "sample": w1}
    finally:
        oracle.use_native_build(False)
    r2, w2 = _rows_rate(oracle, el, u, args, seconds * 0.2, 3)
    out["default_build"] = {"value": round(r2, 5), "build": "gcc -O2 -fopenmp", "sample": w2}
    pairs = el.n * (el.n - 1)
    src_pairs = 2 * el.n * problem.nc  # source terms + energy sums, about 1 pair each
    t_solve = (fp64_products * pairs + src_pairs) / (rate * 1e9)
    out["solve"] = {"kind": "extrapolated", "seconds_per_solve": round(t_solve, 3),
                    "solves_per_s": round(1.0 / t_solve, 6), "products": fp64_products,
                    "basis": f"products of the GPU FP64 GMRES({RESTART}) solve at the bench tolerance "
                             "(the oracle's count agrees within one at the stored workloads) "
                             "x the measured product rate"}
    if small is not None:
        ps = small
        els = oracle.mesh_elements(ps.V, ps.F)
        t0 = time.perf_counter()
        _, E, info = oracle.solve(els, ps.pos, ps.q, ps.eps1, ps.eps2, ps.kappa,
                                  restart=RESTART, tol=TOL, maxit=1000)
        ts = time.perf_counter() - t0
        out["small_solve"] = {"workload": f"N={els.n}, Nc={len(ps.q)}", "kind": "measured",
                              "seconds_per_solve": round(ts, 3),
                              "solves_per_s": round(1.0 / ts, 5),
                              "products": info["matvecs"], "build": "gcc -O2 -fopenmp"}
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
        ctx.solve(tol=TOL, mode=gabi.SOLVE_MIXED_IR, restart=RESTART)
        its, energies, seconds = [], [], 0.0
        for Pk in P[1:]:
            t0 = time.perf_counter()
            ctx.set_charges(Pk, p.q)
            _, info = ctx.solve(tol=TOL, mode=gabi.SOLVE_MIXED_IR, restart=RESTART, x0_previous=previous)
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


TREE_OPTS = (0.7, 5, 256)   # theta, degree, leaf size of the treecode timing


def tree_crossover(gabi, torch, nus=(16, 32, 40, 48, 56, 64, 96, 128), reps=3):
    """Direct-sum (FP64 and FP32-pair) against treecode (FP64) products on
    geodesic spheres of about 4 elements per square Angstrom: per-product
    device time (HIP events on the context's stream, averaged over `reps`)
    and the treecode's error against the direct FP64 product; the crossover
    is the smallest N measured at which the treecode is faster than the
    direct FP64 product."""
    import math
    import numpy as np
    from paper_1301_5885_amd.synth import icosphere
    theta, degree, leaf = TREE_OPTS
    rows = []
    for nu in nus:
        n = 20 * nu * nu
        V, F = icosphere(nu, math.sqrt(n / (16 * math.pi)))
        with gabi.Context(0) as ctx:
            ctx.set_surface_mesh(V, F)
            ctx.set_charges(np.zeros((1, 3)), np.ones(1))
            ctx.set_params(1.0, 80.0, 0.1257)
            u = torch.tensor(np.random.default_rng(nu).normal(size=2 * n), device="cuda")
            y = torch.empty_like(u)
            yt = torch.empty_like(u)
            ctx.set_stream()
            stream = torch.cuda.current_stream()

            def timed(fn):
                fn()                                   # warm-up (builds, uploads)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    fn()
                e1.record(stream)
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / reps

            t64 = timed(lambda: ctx.matvec_dev(u, y, gabi.FP64))
            t32 = timed(lambda: ctx.matvec_dev(u, yt, gabi.FP32_PAIR))
            t_tree = timed(lambda: ctx.tree_matvec_dev(u, yt, theta, degree, leaf))
            t_tree32 = timed(lambda: ctx.tree_matvec_dev(u, yt, theta, degree, leaf,
                                                         gabi.FP32_PAIR))
            info = ctx.tree_info(theta, degree, leaf)
            ctx.matvec_dev(u, y, gabi.FP64)
            ctx.tree_matvec_dev(u, yt, theta, degree, leaf)
            torch.cuda.synchronize()
            err = float(torch.linalg.norm(yt - y) / torch.linalg.norm(y))
            ctx.tree_matvec_dev(u, yt, theta, degree, leaf, gabi.FP32_PAIR)
            torch.cuda.synchronize()
            err32 = float(torch.linalg.norm(yt - y) / torch.linalg.norm(y))
        tree_pairs = info["far_pairs"] + info["near_pairs"]
        rows.append({"N": n, "direct_fp64_ms": round(t64, 4), "direct_fp32_pair_ms": round(t32, 4),
                     "tree_fp64_ms": round(t_tree, 4), "tree_rel_err_vs_direct": err,
                     "tree_fp32_ms": round(t_tree32, 4), "tree_fp32_rel_err_vs_direct": err32,
                     "tree_pairs_per_product": tree_pairs,
                     "tree_fp64_tflops": round(tree_pairs * FLOP_PER_PAIR / t_tree / 1e9, 2),
                     "tree_fp32_tflops": round(tree_pairs * FLOP_PER_PAIR / t_tree32 / 1e9, 2),
                     "tree_device_bytes": info["device_bytes"]})
        log(f"[bench] tree N={n}: direct {t64:.3f} ms (fp32-pair {t32:.3f}), tree {t_tree:.3f} "
            f"ms, err {err:.2e} (fp32 evaluation {t_tree32:.3f} ms, err {err32:.2e})")
    faster = [r["N"] for r in rows if r["tree_fp64_ms"] < r["direct_fp64_ms"]]
    faster32 = [r["N"] for r in rows if r["tree_fp64_ms"] < r["direct_fp32_pair_ms"]]
    faster3232 = [r["N"] for r in rows if r["tree_fp32_ms"] < r["direct_fp32_pair_ms"]]
    big = rows[-1]
    return {"opts": {"theta": theta, "degree": degree, "leaf_size": leaf},
            "roofline": {"bound": "alu", "achieved": big["tree_fp32_tflops"],
                         "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                         "frac": round(big["tree_fp32_tflops"] / PEAK_TFLOPS["fp32"], 4),
                         "N": big["N"],
                         "basis": "treecode product with FP32 sums: 61 algorithmic FLOP per "
                                  "evaluated pair (near element pairs and proxy pairs) over the "
                                  "product's device time (all its kernels)"},
            "method": "barycentric Lagrange treecode (particle-cluster, target batches), FP64 "
                      "sums, and FP32 sums (tree_fp32_*)",
            "rows": rows,
            "crossover_N_vs_fp64": faster[0] if faster else None,
            "crossover_N_vs_fp32_pair": faster32[0] if faster32 else None,
            "crossover_N_fp32_sums_vs_fp32_pair": faster3232[0] if faster3232 else None,
            "crossover_note": "smallest measured N with the treecode product (FP64 sums) faster "
                              "than the direct FP64 (FP32-pair) product, and with FP32 sums "
                              "faster than the direct FP32-pair product (None: not within the "
                              "sizes measured)"}


def measure(gabi, torch, name, steps, warmup, fp64_steps, event_solves, tree_steps=0):
    """Mixed and FP64 solves of one workload on one context (and, with
    tree_steps, the treecode refinement: inner cycles on treecode products,
    FP64 direct residuals; its products are not direct pairs, so it reports
    solves/s and its errors, not Gpair-kernels/s or a roofline)."""
    from paper_1301_5885_amd.synth import config_problem
    t0 = time.perf_counter()
    p = config_problem(name)
    n = p.n
    log(f"[bench] workload {name} N={n} Nc={p.nc} (generated in "
        f"{time.perf_counter() - t0:.1f} s)")
    ctx = gabi.Context(0)
    ctx.load_problem(p)
    u = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    ref = golden(name)
    E_ref = ref["energy_kcal_per_mol"] if ref else None
    results = {}
    runs = [("mixed", gabi.SOLVE_MIXED_IR, steps, warmup, event_solves),
            ("fp64", gabi.SOLVE_FP64, fp64_steps, min(warmup, 1), event_solves)]
    if tree_steps > 0:
        runs.append(("tree_ir", gabi.SOLVE_TREE_IR, tree_steps, 1, 0))
    for key, mode, k, w, ev in runs:
        log(f"[bench] {name} {key}: {w} warmup + {k} timed + {ev} event-timed solves")
        r = run_solver(ctx, gabi, torch, u, mode, k, w, ev, n * (n - 1))
        E = r["energies"][-1]
        r["energy"] = E
        r["energy_rel_err"] = abs(E / E_ref - 1) if E_ref else None
        r["potential_err"] = potential_errors(r["u"], ref, n)
        results[key] = r
        log(f"[bench] {name} {key}: {r['ms_per_step']:.3f} ms/solve, "
            f"{r['gpairs_per_s']:.1f} Gpairs/s, E={E:.8f}, err={r['energy_rel_err']}, "
            f"potential {r['potential_err']}")
    mixed, fp64 = results["mixed"], results["fp64"]
    tree = results.get("tree_ir")
    solver_line = lambda r, key: {
        "value": round(r["gpairs_per_s"], 3), "unit": "Gpair-kernels/s",
        "solves_per_s": round(r["solves_per_s"], 4), "ms_per_step": round(r["ms_per_step"], 4),
        "steps": r["steps"],
        "energy": r["energy"], "energy_rel_err": r["energy_rel_err"],
        "potential_err": r["potential_err"],
        "products_per_solve": {"fp32": r["products_fp32"] / r["steps"],
                               "fp64": r["products_fp64"] / r["steps"]},
        "roofline": roofline(r, key, n, name, gabi)}
    out = {"workload": WORKLOADS[name], "key": name, "N": n, "Nc": p.nc,
           "oracle_reference": (f"tests/golden/{name}_reference.json (oracle GMRES to "
                                f"{ref['tol']:g})") if ref else None,
           "mixed": solver_line(mixed, "fp32"), "fp64_solver": solver_line(fp64, "fp64"),
           "speedup_mixed_over_fp64": round(mixed["solves_per_s"] / fp64["solves_per_s"], 3)}
    if tree:
        dflt = gabi.default_opts()
        out["tree_ir_solver"] = {
            "method": f"FP64 iterative refinement around GMRES({RESTART}) cycles on the treecode "
                      f"product (theta {dflt.tree_theta:g}, degree {dflt.tree_degree}, leaves of "
                      f"{dflt.tree_leaf}, pair terms in FP32); residuals are FP64 direct products",
            "solves_per_s": round(tree["solves_per_s"], 4),
            "ms_per_step": round(tree["ms_per_step"], 4), "steps": tree["steps"],
            "energy": tree["energy"], "energy_rel_err": tree["energy_rel_err"],
            "potential_err": tree["potential_err"],
            "products_per_solve": {"tree": tree["products_tree"] / tree["steps"],
                                   "fp64": tree["products_fp64"] / tree["steps"]},
            "speedup_over_mixed": round(tree["solves_per_s"] / mixed["solves_per_s"], 3),
            "speedup_over_fp64": round(tree["solves_per_s"] / fp64["solves_per_s"], 3),
            "energy_rel_diff_vs_fp64_solver": abs(tree["energy"] / fp64["energy"] - 1)}
    return ctx, p, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed solves of the plain FP64 solver beside the headline "
                         "(at most --steps)")
    ap.add_argument("--tree-steps", type=int, default=5,
                    help="timed solves of the treecode refinement beside the headline "
                         "(0: skip)")
    ap.add_argument("--event-solves", type=int, default=2,
                    help="solves with HIP events around the pair kernels (roofline)")
    ap.add_argument("--secondary", default="kirkwood",
                    help="a second, smaller workload timed the same way ('none': skip)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving stream to serve after the single-solve "
                         "timing (0: skip; the stream has 512)")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-caps", default=None,
                    help="round caps of the served runs (serve.py --caps; default: "
                         "slack 0.5 and floor 32768, then none)")
    ap.add_argument("--sequence-steps", type=int, default=8,
                    help="nearby problems solved cold and warm-started after the timing, "
                         "on the secondary workload (0: skip)")
    ap.add_argument("--no-tree", action="store_true",
                    help="skip the direct-sum/treecode product timing")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="before timing, run one device copy of this many MiB "
                         "(a kernel of known traffic for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not "
              "supported (the row-sharded multi-GPU product is a design only)",
              file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()

    from paper_1301_5885_amd import serve
    serve_problems = None
    if args.serve_requests > 0:
        # generated in a process pool, before anything touches the GPU
        log(f"[bench] generating {args.serve_requests} serving requests")
        serve_problems = serve.make_problems(args.serve_requests, 16)

    import torch
    from paper_1301_5885_amd import gabi

    if args.copy_mb:
        a = torch.ones(args.copy_mb * 131072, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_mb} MiB read + written")
        del a, b

    fp64_steps = max(1, min(args.fp64_steps, args.steps))
    ctx, p, head = measure(gabi, torch, args.workload, args.steps, args.warmup, fp64_steps,
                           args.event_solves, tree_steps=args.tree_steps)
    ctx.close()
    mixed = head["mixed"]
    line = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "Gpair-kernels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair terms, f64 accumulation/Krylov/residual/energy",
        "data": "synthetic (seeded surface and charges)",
        "config": {"workload": head["workload"], "N": head["N"], "Nc": head["Nc"],
                   "eps1": p.eps1, "eps2": p.eps2, "kappa": p.kappa,
                   "restart": RESTART, "tol": TOL, "solver": "mixed IR (FP32-pair GMRES "
                   "cycles, FP64 residuals)", "parallelism": "single GPU"},
        "solves_per_s": mixed["solves_per_s"],
        "energy_rel_err": mixed["energy_rel_err"],
        "potential_err": mixed["potential_err"],
        "oracle_reference": head["oracle_reference"],
        "products_per_solve": mixed["products_per_solve"],
        "roofline": mixed["roofline"],
        "fp64_solver": head["fp64_solver"],
        "speedup_mixed_over_fp64": head["speedup_mixed_over_fp64"],
    }
    if "tree_ir_solver" in head:
        line["tree_ir_solver"] = head["tree_ir_solver"]
    small = None
    if args.secondary != "none" and args.secondary != args.workload:
        ctx2, small, sec = measure(gabi, torch, args.secondary, args.steps, args.warmup,
                                   args.steps, args.event_solves,
                                   tree_steps=args.steps if args.tree_steps > 0 else 0)
        line["secondary"] = sec
        if args.sequence_steps > 0:
            log(f"[bench] warm-started sequence: {args.sequence_steps} nearby problems")
            line["warm_sequence"] = warm_sequence(ctx2, gabi, small, args.sequence_steps)
            line["warm_sequence"]["workload"] = args.secondary
            log(f"[bench] sequence: {line['warm_sequence']}")
        ctx2.close()
    if not args.no_tree:
        log("[bench] direct-sum vs treecode products")
        line["treecode"] = tree_crossover(gabi, torch)
    if serve_problems is not None:
        log(f"[bench] serving {args.serve_requests} requests")
        line["serving"] = serve.run(
            args.serve_requests, args.serve_slots, problems=serve_problems,
            caps=serve.parse_caps(args.serve_caps or serve.DEFAULT_CAPS))
        line["serving"]["workload"] = SERVING_WORKLOAD
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (oracle, ~{args.cpu_seconds:.0f} s + a small solve)")
        line["cpu_baseline"] = cpu_baseline(
            p, args.cpu_seconds, head["fp64_solver"]["products_per_solve"]["fp64"], small)
    else:
        line["cpu_baseline"] = None
    line["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
