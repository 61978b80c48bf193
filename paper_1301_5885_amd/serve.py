"""Serving benchmark: a stream of solve requests of uneven size on one GPU.

The request mix: seeded star-shaped surfaces with N = 20 nu^2 log-uniform in
[1280, 81920], Nc = N/40 charges, kappa ~ U[0, 0.3] (`synth.serving_requests`).
Three ways of serving the same stream are measured:

  plain FP64    one solve at a time through a context, restarted GMRES(20)
                on the FP64 product (the paper's solver, kept on the device);
  plain mixed   the same with FP64 iterative refinement around FP32-pair
                GMRES cycles;
  served mixed  the serving loop (`gabi_server_*`): requests are admitted by
                device-memory footprint and slot count and join the running
                batch at cycle boundaries, so the products of all active
                molecules share one persistent launch.  A round cap keeps
                the oldest request's rounds from growing by more than a
                slack (the largest surfaces set the tail latency): run with
                the cap, then without it.

Every solve runs to the same relative residual.  The service time of a plain
solve is host clock from upload to energy.  Arrivals are Poisson at 0.8 x the
plain FP64 solver's throughput (measured first on the same stream); the
plain solvers' latencies under those arrivals follow exactly from their
measured service times (one solve at a time, first come first served), the
served latencies are measured live (result time minus scheduled arrival).  A
saturation run submits the whole stream at once and gives each solver's
capacity in solves/s.

    python -m paper_1301_5885_amd.serve [--requests 512] [--max-slots 32]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

TOL = 1e-8
ARRIVAL_SEED = 6000
LOAD = 0.8
# served runs: under the round cap slack 0.5, floor 32,768 elements (the
# reported figures), then without a cap for comparison
DEFAULT_CAPS = "0.5:32768,none"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _build(i):
    from .synth import serving_requests
    return serving_requests(i + 1)[i][2]()


def make_problems(count, workers):
    """The first `count` requests of the serving stream (generated on the host
    in a process pool; call before the GPU is used)."""
    workers = max(1, min(workers, count))
    if workers == 1:
        return [_build(i) for i in range(count)]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_build, range(count), chunksize=1)


def to_requests(problems, gabi):
    return [gabi.Request.from_mesh(p.V, p.F, p.pos, p.q, eps1=p.eps1, eps2=p.eps2,
                                   kappa=p.kappa, tag=i)
            for i, p in enumerate(problems)]


def pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def solo(reqs, gabi, torch, mode, tol):
    """One solve at a time; returns per-request service seconds, energies and
    iteration counts."""
    svc, energies, its = [], [], []
    with gabi.Context(0) as ctx:
        for r in reqs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.load_request(r)
            _, info = ctx.solve(tol=tol, mode=mode)
            e = ctx.energy()
            svc.append(time.perf_counter() - t0)
            energies.append(e)
            its.append(info["iterations"])
            if not info["converged"]:
                raise RuntimeError(f"request {r.c.tag} did not converge: {info}")
    return np.array(svc), np.array(energies), np.array(its)


def fifo_latencies(arrivals, service):
    """Latency of each request at a single first-come-first-served server."""
    done, lat = 0.0, []
    for a, s in zip(arrivals, service):
        start = max(a, done)
        done = start + s
        lat.append(done - a)
    return np.array(lat)


def served(reqs, gabi, arrivals, mode, tol, budget, max_slots, cap=None):
    """Live run of the serving loop; returns latencies, energies (by tag),
    makespan and server statistics.  cap: (slack, floor_elements) of the
    round cap (gabi_server_set_round_cap), or None for none."""
    results = {}
    with gabi.Server(device=0, budget_bytes=budget, max_slots=max_slots, tol=tol,
                     mode=mode) as s:
        if cap is not None:
            s.set_round_cap(cap[0], cap[1])
        t0 = s.clock()
        order = np.argsort(arrivals, kind="stable")
        for k in order:
            due = t0 + arrivals[k]
            while True:
                now = s.clock()
                if now >= due:
                    break
                for r in s.poll():
                    results[r["tag"]] = r
                time.sleep(min(0.002, due - now))
            s.submit(reqs[k])
        # wait for the rest, reporting completions; a minute without any
        # completion ends the run with an error
        last, t_last = -1, time.time()
        while not s.drain(10.0):
            st = s.stats()
            log(f"[serve]   completed {st['completed']}/{st['submitted']}, active {st['active']}, "
                f"queued {st['queued']}, rounds {st['rounds']}")
            if st["completed"] != last:
                last, t_last = st["completed"], time.time()
            elif time.time() - t_last > 60.0:
                raise RuntimeError(f"serving loop made no progress for 60 s: {st}")
        while True:
            got = s.poll()
            if not got:
                break
            for r in got:
                results[r["tag"]] = r
        st = s.stats()
    if len(results) != len(reqs):
        raise RuntimeError(f"{len(results)} of {len(reqs)} results returned")
    bad = [r for r in results.values() if r["status"] != gabi.OK]
    if bad:
        raise RuntimeError(f"{len(bad)} requests failed, e.g. {bad[0]}")
    lat = np.array([results[i]["t_done"] - (t0 + arrivals[i]) for i in range(len(reqs))])
    energies = np.array([results[i]["energy"] for i in range(len(reqs))])
    makespan = max(r["t_done"] for r in results.values()) - t0
    return lat, energies, makespan, st


def parse_caps(text):
    """'none,0.1:20480' -> [None, (0.1, 20480)]."""
    out = []
    for item in text.split(","):
        item = item.strip()
        if item in ("", "none"):
            out.append(None)
        else:
            slack, floor = item.split(":")
            out.append((float(slack), int(floor)))
    return out


def cap_name(cap):
    return "none" if cap is None else f"slack {cap[0]:g}, floor {cap[1]}"


def run(count=64, max_slots=32, budget_gib=16.0, tol=TOL, workers=16, problems=None,
        caps=(None,)):
    """The whole serving comparison; returns a JSON-ready dict.  The served
    runs are repeated for every round cap in `caps`; the first is reported as
    served_mixed, all of them under cap_sweep."""
    t_gen = time.perf_counter()
    if problems is None:
        problems = make_problems(count, workers)
    t_gen = time.perf_counter() - t_gen
    import torch
    from . import gabi
    reqs = to_requests(problems, gabi)
    ns = np.array([r.n for r in reqs])
    pairs = ns * (ns - 1.0)
    log(f"[serve] {count} requests generated in {t_gen:.1f} s; N median {int(np.median(ns))}, "
        f"max {ns.max()}")
    budget = int(budget_gib * (1 << 30))

    # warm-up: one small solve per mode (library load, first-launch costs)
    small = int(np.argmin(ns))
    solo([reqs[small]], gabi, torch, gabi.SOLVE_FP64, tol)
    solo([reqs[small]], gabi, torch, gabi.SOLVE_MIXED_IR, tol)

    out = {"requests": count, "tol": tol, "max_slots": max_slots,
           "budget_bytes": budget, "N_median": int(np.median(ns)), "N_max": int(ns.max()),
           "load": LOAD}
    log("[serve] plain FP64, one at a time")
    s64, e64, it64 = solo(reqs, gabi, torch, gabi.SOLVE_FP64, tol)
    log(f"[serve]   {count / s64.sum():.2f} solves/s")
    log("[serve] plain mixed, one at a time")
    smx, emx, itmx = solo(reqs, gabi, torch, gabi.SOLVE_MIXED_IR, tol)
    log(f"[serve]   {count / smx.sum():.2f} solves/s")

    rate = LOAD * count / s64.sum()
    gaps = np.random.default_rng(ARRIVAL_SEED).exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out["arrival_rate_per_s"] = round(rate, 4)

    sweep = []
    for cap in caps:
        log(f"[serve] served mixed (round cap: {cap_name(cap)}), Poisson arrivals at "
            f"{rate:.2f}/s")
        lat_p, e_sv, span_p, st_p = served(reqs, gabi, arrivals, gabi.SOLVE_MIXED_IR, tol,
                                           budget, max_slots, cap)
        log(f"[serve]   p50 {1e3 * pct(lat_p, 50):.1f} ms p99 {1e3 * pct(lat_p, 99):.1f} ms, "
            f"max active {st_p['max_active']}")
        log("[serve] served mixed, saturation (all requests at t=0)")
        lat_s, e_ss, span_s, st_s = served(reqs, gabi, np.zeros(count), gabi.SOLVE_MIXED_IR,
                                           tol, budget, max_slots, cap)
        log(f"[serve]   {count / span_s:.2f} solves/s, max active {st_s['max_active']}")
        sweep.append((cap, lat_p, e_sv, span_p, st_p, lat_s, e_ss, span_s, st_s))
    cap, lat_p, e_sv, span_p, st_p, lat_s, e_ss, span_s, st_s = sweep[0]

    def block(service, energies, lat_poisson, lat_sat, capacity, extra=None):
        d = {"solves_per_s": round(capacity, 3),
             "p50_ms": round(1e3 * pct(lat_poisson, 50), 2),
             "p99_ms": round(1e3 * pct(lat_poisson, 99), 2),
             "p50_ms_saturated": round(1e3 * pct(lat_sat, 50), 2),
             "p99_ms_saturated": round(1e3 * pct(lat_sat, 99), 2)}
        if service is not None:
            d["mean_service_ms"] = round(1e3 * float(np.mean(service)), 3)
        if extra:
            d.update(extra)
        return d

    rel = lambda e: np.abs(e / e64 - 1.0)
    out["plain_fp64"] = block(s64, e64, fifo_latencies(arrivals, s64),
                              fifo_latencies(np.zeros(count), s64), count / s64.sum(),
                              {"iterations_median": float(np.median(it64))})
    out["plain_mixed"] = block(smx, emx, fifo_latencies(arrivals, smx),
                               fifo_latencies(np.zeros(count), smx), count / smx.sum(),
                               {"energy_rel_err_vs_fp64_max": float(rel(emx).max())})
    out["served_mixed"] = block(None, e_sv, lat_p, lat_s, count / span_s, {
        "energy_rel_err_vs_fp64_max": float(max(rel(e_sv).max(), rel(e_ss).max())),
        "max_active_poisson": st_p["max_active"], "max_active_saturated": st_s["max_active"],
        "rounds_saturated": st_s["rounds"], "peak_bytes": st_s["peak_bytes"],
        "poisson_makespan_s": round(span_p, 3), "round_cap": cap_name(cap)})
    if len(sweep) > 1:
        out["cap_sweep"] = [
            {"round_cap": cap_name(c), "solves_per_s": round(count / ss, 3),
             "p50_ms": round(1e3 * pct(lp, 50), 2), "p90_ms": round(1e3 * pct(lp, 90), 2),
             "p99_ms": round(1e3 * pct(lp, 99), 2), "max_ms": round(1e3 * float(np.max(lp)), 2),
             "energy_rel_err_vs_fp64_max": float(max(rel(ep).max(), rel(es).max()))}
            for c, lp, ep, sp, stp, ls, es, ss, sts in sweep]
    out["speedup_served_over_plain_fp64"] = round(
        out["served_mixed"]["solves_per_s"] / out["plain_fp64"]["solves_per_s"], 3)
    out["p99_ratio_served_over_plain_fp64"] = round(
        out["served_mixed"]["p99_ms"] / out["plain_fp64"]["p99_ms"], 3)
    out["ordered_pairs_per_request_mean"] = float(pairs.mean())
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--max-slots", type=int, default=32)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--tol", type=float, default=TOL)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--caps", default=DEFAULT_CAPS,
                    help="round caps of the served runs, comma-separated: 'none' or "
                         "slack:floor_elements (the first is reported as served_mixed)")
    a = ap.parse_args(argv)
    res = run(a.requests, a.max_slots, a.budget_gib, a.tol, a.workers, caps=parse_caps(a.caps))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
