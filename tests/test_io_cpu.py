"""Molecular-surface and charge files (CPU only): MSMS .vert/.face and PQR
readers of the C ABI (the paper's host reads the molecule and its MSMS
triangulation, Section 2.4, table tb_GPU).  MSMS and PDB data are not
available here, so the files are written by the test from seeded synthetic
surfaces in the formats' layout, read back through the library, and solved
with the CPU oracle: a sphere with a central charge reproduces the Born
energy to the discretization error the in-memory mesh gives."""
import os

import numpy as np
import pytest

import oracle
from closed_forms import born_energy
from paper_1301_5885_amd import gabi
from paper_1301_5885_amd.synth import icosphere, star_surface


def write_msms(base, V, F, normals, header=True):
    with open(base + ".vert", "w") as f:
        if header:
            f.write("# MSMS solvent excluded surface vertices\n")
            f.write("#vertex #sphere density probe_r\n")
        f.write(f"{len(V):7d} {len(V):7d} 1.00 1.50\n")
        for k, (v, n) in enumerate(zip(V, normals)):
            f.write(f"{v[0]:.17g} {v[1]:.17g} {v[2]:.17g} {n[0]:.17g} {n[1]:.17g} "
                    f"{n[2]:.17g} {k + 1} 1 1\n")
    with open(base + ".face", "w") as f:
        if header:
            f.write("# MSMS solvent excluded surface faces\n")
            f.write("#faces  #sphere density probe_r\n")
        f.write(f"{len(F):7d} {len(V):7d} 1.00 1.50\n")
        for t in F:
            f.write(f"{t[0] + 1:6d} {t[1] + 1:6d} {t[2] + 1:6d}  1  1\n")


def write_pqr(path, pos, q, r, chain=True):
    with open(path, "w") as f:
        f.write("REMARK   synthetic charges\n")
        for k, (p, qq, rr) in enumerate(zip(pos, q, r)):
            rec = "ATOM  " if k % 3 else "HETATM"
            ch = " A" if chain else ""
            f.write(f"{rec}{k + 1:5d}  CA  ALA{ch}{k // 2 + 1:4d}    "
                    f"{p[0]:.17g} {p[1]:.17g} {p[2]:.17g} {qq:.17g} {rr:.6f}\n")
        f.write("TER\nEND\n")


def test_msms_round_trip_and_orientation(tmp_path):
    V, F, _ = star_surface(7, 9.0, np.random.default_rng(4))
    nrm = V / np.linalg.norm(V, axis=1, keepdims=True)   # star-shaped: radial is outward
    base = str(tmp_path / "mol")
    Fw = F.copy()
    Fw[::3] = Fw[::3][:, [0, 2, 1]]                      # every third face wound clockwise
    write_msms(base, V, Fw, nrm)
    V2, F2, N2, flipped = gabi.read_msms(base + ".vert", base + ".face", orient=False)
    assert np.array_equal(V2, V) and np.array_equal(N2, nrm) and np.array_equal(F2, Fw)
    assert flipped == 0
    V3, F3, _, flipped = gabi.read_msms(base + ".vert", base + ".face", orient=True)
    assert flipped == len(F[::3])
    # same triangles, every one counter-clockwise seen from outside again
    el_ref = oracle.mesh_elements(V, F)
    el = oracle.mesh_elements(V3, F3)
    for k in ("nx", "ny", "nz", "area", "cx"):
        assert np.allclose(getattr(el, k), getattr(el_ref, k), rtol=0, atol=1e-14)


def test_pqr_records(tmp_path):
    rng = np.random.default_rng(1)
    pos = rng.normal(size=(7, 3))
    q = rng.normal(size=7)
    r = rng.uniform(1, 2, 7)
    for chain in (True, False):
        path = str(tmp_path / f"mol{int(chain)}.pqr")
        write_pqr(path, pos, q, r, chain)
        p2, q2, r2 = gabi.read_pqr(path)
        assert np.array_equal(p2, pos) and np.array_equal(q2, q)
        assert np.allclose(r2, r, atol=1e-6)


def test_bad_files_rejected(tmp_path):
    with pytest.raises(gabi.GabiError):
        gabi.read_pqr(str(tmp_path / "missing.pqr"))
    V, F = icosphere(2, 1.0)
    base = str(tmp_path / "bad")
    F2 = F.copy()
    F2[5, 1] = len(V)                                     # one past the last vertex
    write_msms(base, V, F2, V)
    with pytest.raises(gabi.GabiError) as e:
        gabi.read_msms(base + ".vert", base + ".face")
    assert "EMESH" in str(e.value)
    with open(str(tmp_path / "bad.pqr"), "w") as f:
        f.write("ATOM      1  CA  ALA A   1    1.0 2.0 x.0 0.5 1.8\n")
    with pytest.raises(gabi.GabiError):
        gabi.read_pqr(str(tmp_path / "bad.pqr"))


def test_files_to_born_energy(tmp_path):
    """A sphere of radius 2 with a unit charge at its centre, through files:
    the surface and charge read back give the in-memory problem bit for bit,
    and the oracle's solve reproduces the Born energy at the mesh's O(h)."""
    a = 2.0
    V, F = icosphere(8, a)
    base = str(tmp_path / "born")
    write_msms(base, V, F, V / a)
    write_pqr(str(tmp_path / "born.pqr"), np.zeros((1, 3)), [1.0], [a])
    V2, F2, _, flipped = gabi.read_msms(base + ".vert", base + ".face")
    pos, q, _ = gabi.read_pqr(str(tmp_path / "born.pqr"))
    assert flipped == 0
    el = oracle.mesh_elements(V2, F2)
    _, E, info = oracle.solve(el, pos, q, 1.0, 80.0, 0.1257, tol=1e-10)
    _, E_mem, _ = oracle.solve(oracle.mesh_elements(V, F), np.zeros((1, 3)), [1.0], 1.0, 80.0,
                               0.1257, tol=1e-10)
    assert E == E_mem
    assert abs(E / born_energy(a, 1.0, 1.0, 80.0, 0.1257) - 1) < 0.05
