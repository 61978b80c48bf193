"""The stored oracle reference solves (tests/golden/, written by
make_golden.py from the CPU oracle alone) are consistent with the workloads
they name and with themselves: sizes and parameters of the seeded problem,
a converged GMRES record at the stored tolerance, the sampled element
indices of the stated seed (the ones the bench and the GPU tests read),
the two tolerances' energies within what their residuals allow, and, where
the whole solution is stored, its norms and samples equal to the record's.
No GPU and no oracle solve is needed."""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
sys.path.insert(0, os.path.dirname(HERE))

import make_golden  # noqa: E402
from paper_1301_5885_amd.synth import config_problem  # noqa: E402

SIZES = {"kirkwood": (20480, 200), "star": (81920, 2000), "large": (327680, 5000)}


def load(name):
    path = os.path.join(HERE, "golden", f"{name}_reference.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored reference for {name}")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["kirkwood", "star", "large"])
def test_reference_record(name):
    ref = load(name)
    n, nc = SIZES[name]
    assert (ref["workload"], ref["N"], ref["Nc"]) == (name, n, nc)
    assert (ref["eps1"], ref["eps2"], ref["kappa"]) == (1.0, 80.0, 0.1257)
    g = ref["gmres"]
    assert g["converged"] and 0.0 < g["rel_residual"] <= ref["tol"] <= 1e-10
    assert g["matvecs"] >= g["iterations"] >= 1
    # the sampled elements are the seeded choice the readers recompute
    s = ref["samples"]
    idx = make_golden.sample_index(n, len(s["index"]), s["seed"])
    assert np.array_equal(idx, np.asarray(s["index"]))
    assert len(s["phi"]) == len(s["psi"]) == len(idx) == 2048
    assert np.all(np.isfinite(s["phi"])) and np.all(np.isfinite(s["psi"]))
    # the tol-1e-8 solve: converged, and its energy within what the two
    # residuals allow of the tight one (both are oracle GMRES(10) solves)
    loose = ref["tol_1e-8"]
    assert loose["gmres"]["converged"] and loose["gmres"]["rel_residual"] <= 1e-8
    e, e8 = ref["energy_kcal_per_mol"], loose["energy_kcal_per_mol"]
    assert e < 0 and abs(e8 / e - 1) <= 1e-7


def test_reference_sizes_match_the_generators():
    """N and Nc of every stored reference are those of the seeded workload
    (the small kirkwood and star are generated; large is the geodesic
    sphere of frequency 128, N = 20 nu^2)."""
    for name in ("kirkwood", "star"):
        p = config_problem(name)
        assert (p.n, p.nc) == SIZES[name]
    assert 20 * 128 ** 2 == SIZES["large"][0]


def test_kirkwood_full_solution_matches_its_record():
    ref = load("kirkwood")
    u = np.load(os.path.join(HERE, "golden", ref["full_u"]), allow_pickle=False)
    n = ref["N"]
    assert u.shape == (2 * n,) and u.dtype == np.float64
    assert np.linalg.norm(u[:n]) == pytest.approx(ref["phi_norm"], rel=1e-14)
    assert np.linalg.norm(u[n:]) == pytest.approx(ref["psi_norm"], rel=1e-14)
    idx = np.asarray(ref["samples"]["index"])
    assert np.array_equal(u[idx], np.asarray(ref["samples"]["phi"]))
    assert np.array_equal(u[n + idx], np.asarray(ref["samples"]["psi"]))
