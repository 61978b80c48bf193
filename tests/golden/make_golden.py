"""Write oracle reference values for the full-size workloads.

Calls only the CPU oracle (oracle/) on the seeded synthetic inputs; nothing
here touches the HIP library.  Output: tests/golden/<name>_reference.json
with the tightly converged FP64 solve of the workload:

* the solvation energy (Section 2.3, eq. (solvation_energy)) and GMRES info;
* the norms of phi and psi, and phi/psi at seeded sampled elements, so that
  the potential error (Section 3.1, eq. (eqerr1)) of any GPU solve can be
  stated against the oracle;
* optionally (``--full-u``) the whole solution vector u = [phi; psi] as
  tests/golden/<name>_u.npy (float64, no pickle);
* unless ``--no-loose``, the energy and GMRES info of a second solve at
  tol 1e-8, the tolerance of the timed GPU runs.  With ``--no-loose`` an
  earlier file's loose entry is kept as it was.
* with ``--loose-first`` (for sizes where each oracle product takes
  minutes) the tol-1e-8 solve comes first, from x0 = 0, and is written out
  at once as both the loose entry and a provisional reference; the tight
  reference is then reached by restarted GMRES warm-started from that
  solution (same operator, same stopping rule ||b - Au|| / ||b|| <= tol)
  and the file is written again.

    python tests/golden/make_golden.py kirkwood --full-u
    python tests/golden/make_golden.py large --tol 1e-10 --loose-first
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1301_5885_amd.synth import config_problem  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE_SEED = 7001


def sample_index(n, count=2048, seed=SAMPLE_SEED):
    """Seeded, sorted element indices at which phi and psi are stored."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _record(a, p, u, E, info, tol, seconds):
    idx = sample_index(p.n, a.samples)
    return {
        "workload": a.name, "N": p.n, "Nc": p.nc, "eps1": p.eps1,
        "eps2": p.eps2, "kappa": p.kappa, "restart": 10,
        "tol": tol, "energy_kcal_per_mol": E, "gmres": info,
        "phi_norm": float(np.linalg.norm(u[:p.n])),
        "psi_norm": float(np.linalg.norm(u[p.n:])),
        "samples": {"seed": SAMPLE_SEED, "index": idx.tolist(),
                    "phi": u[idx].tolist(), "psi": u[p.n + idx].tolist()},
        "seconds": seconds,
        "threads": oracle.num_threads(), "cpu": _cpu_model(),
        "source": "oracle/ (FP64 CPU), tests/golden/make_golden.py",
    }


def _write(a, out, u):
    if a.full_u:
        np.save(os.path.join(HERE, f"{a.name}_u.npy"), u, allow_pickle=False)
        out["full_u"] = f"{a.name}_u.npy"
    with open(os.path.join(HERE, f"{a.name}_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    short = {k: v for k, v in out.items() if k != "samples"}
    print(json.dumps(short, indent=1), flush=True)


def loose_first(a):
    """tol-1e-8 solve from x0 = 0, written at once; then the tight solve
    warm-started from it, written over the provisional reference."""
    p = config_problem(a.name)
    el = oracle.mesh_elements(p.V, p.F)
    t0 = time.time()
    b = oracle.rhs(el, p.pos, p.q, p.eps1)
    u8, info8 = oracle.gmres(el, b, p.eps1, p.eps2, p.kappa, restart=10,
                             tol=1e-8, maxit=2000)
    E8 = oracle.energy(el, u8, p.pos, p.q, p.eps1, p.eps2, p.kappa)
    t8 = time.time() - t0
    print(f"{a.name}: tol 1e-8 solve E {E8!r} {info8} {t8:.0f} s", flush=True)
    out = _record(a, p, u8, E8, info8, 1e-8, t8)
    out["tol_1e-8"] = {"energy_kcal_per_mol": E8, "gmres": info8}
    _write(a, out, u8)
    if a.tol >= 1e-8:
        return
    u, info = oracle.gmres(el, b, p.eps1, p.eps2, p.kappa, restart=10,
                           tol=a.tol, maxit=2000, x0=u8)
    E = oracle.energy(el, u, p.pos, p.q, p.eps1, p.eps2, p.kappa)
    t = time.time() - t0
    print(f"{a.name}: tight solve tol {a.tol} E {E!r} {info} {t:.0f} s", flush=True)
    out = _record(a, p, u, E, info, a.tol, t)
    out["warm_start"] = "the tol-1e-8 solution below"
    out["tol_1e-8"] = {"energy_kcal_per_mol": E8, "gmres": info8}
    _write(a, out, u)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--no-loose", action="store_true")
    ap.add_argument("--full-u", action="store_true")
    ap.add_argument("--samples", type=int, default=2048)
    ap.add_argument("--loose-first", action="store_true")
    a = ap.parse_args(argv)
    if a.loose_first:
        return loose_first(a)

    path = os.path.join(HERE, f"{a.name}_reference.json")
    old = {}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)

    p = config_problem(a.name)
    el = oracle.mesh_elements(p.V, p.F)
    t0 = time.time()
    b = oracle.rhs(el, p.pos, p.q, p.eps1)
    u, info = oracle.gmres(el, b, p.eps1, p.eps2, p.kappa, restart=10,
                           tol=a.tol, maxit=2000)
    E = oracle.energy(el, u, p.pos, p.q, p.eps1, p.eps2, p.kappa)
    t_tight = time.time() - t0
    print(f"{a.name}: tight solve tol {a.tol} E {E!r} {info} "
          f"{t_tight:.0f} s", flush=True)
    idx = sample_index(p.n, a.samples)
    out = {
        "workload": a.name, "N": p.n, "Nc": p.nc, "eps1": p.eps1,
        "eps2": p.eps2, "kappa": p.kappa, "restart": 10,
        "tol": a.tol, "energy_kcal_per_mol": E, "gmres": info,
        "phi_norm": float(np.linalg.norm(u[:p.n])),
        "psi_norm": float(np.linalg.norm(u[p.n:])),
        "samples": {"seed": SAMPLE_SEED, "index": idx.tolist(),
                    "phi": u[idx].tolist(), "psi": u[p.n + idx].tolist()},
        "seconds": t_tight,
        "threads": oracle.num_threads(), "cpu": _cpu_model(),
        "source": "oracle/ (FP64 CPU), tests/golden/make_golden.py",
    }
    if a.no_loose:
        if "tol_1e-8" in old:
            out["tol_1e-8"] = old["tol_1e-8"]
    else:
        u8, info8 = oracle.gmres(el, b, p.eps1, p.eps2, p.kappa, restart=10,
                                 tol=1e-8, maxit=2000)
        E8 = oracle.energy(el, u8, p.pos, p.q, p.eps1, p.eps2, p.kappa)
        out["tol_1e-8"] = {"energy_kcal_per_mol": E8, "gmres": info8}
        out["seconds"] = time.time() - t0
    if a.full_u:
        np.save(os.path.join(HERE, f"{a.name}_u.npy"), u, allow_pickle=False)
        out["full_u"] = f"{a.name}_u.npy"
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    short = {k: v for k, v in out.items() if k != "samples"}
    print(json.dumps(short, indent=1), flush=True)


if __name__ == "__main__":
    main()
