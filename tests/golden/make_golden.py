"""Write oracle reference values for the full-size workloads.

Calls only the CPU oracle (oracle/) on the seeded synthetic inputs; nothing
here touches the HIP library.  Output: tests/golden/<name>_reference.json
with the tightly converged (tol 1e-12) FP64 solve of the workload.

    python tests/golden/make_golden.py kirkwood
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1301_5885_amd.synth import config_problem  # noqa: E402


def main(name):
    p = config_problem(name)
    el = oracle.mesh_elements(p.V, p.F)
    t0 = time.time()
    b = oracle.rhs(el, p.pos, p.q, p.eps1)
    u, info = oracle.gmres(el, b, p.eps1, p.eps2, p.kappa, restart=10,
                           tol=1e-12, maxit=2000)
    E = oracle.energy(el, u, p.pos, p.q, p.eps1, p.eps2, p.kappa)
    u8, info8 = oracle.gmres(el, b, p.eps1, p.eps2, p.kappa, restart=10,
                             tol=1e-8, maxit=2000)
    E8 = oracle.energy(el, u8, p.pos, p.q, p.eps1, p.eps2, p.kappa)
    out = {
        "workload": name, "N": p.n, "Nc": p.nc, "eps1": p.eps1, "eps2": p.eps2,
        "kappa": p.kappa, "restart": 10,
        "tol": 1e-12, "energy_kcal_per_mol": E, "gmres": info,
        "tol_1e-8": {"energy_kcal_per_mol": E8, "gmres": info8},
        "phi_norm": float(np.linalg.norm(u[:p.n])),
        "psi_norm": float(np.linalg.norm(u[p.n:])),
        "seconds": time.time() - t0,
        "source": "oracle/ (FP64 CPU), tests/golden/make_golden.py",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"{name}_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "kirkwood")
