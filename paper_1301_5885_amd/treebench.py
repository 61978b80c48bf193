"""Time the treecode product on one geodesic sphere (for profiling).

The sphere of frequency nu has N = 20 nu^2 flat triangles at about four
elements per square Angstrom (R = sqrt(N / (16 pi))); the product runs
`reps` times after one warm-up (which builds the tree) and the mean device
time per product (HIP events), the pair count and the error against the
direct FP64 product are printed as one JSON line.

    python paper_1301_5885_amd/treebench.py [--nu 128] [--reps 5]
                                            [--theta 0.7 --degree 5 --leaf 256]
                                            [--precision fp32|fp64]
"""
import argparse
import json
import math
import os
import sys

import numpy as np

if not __package__:  # run as a script (python3 path/to/treebench.py)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--nu", type=int, default=128)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--theta", type=float, default=0.7)
    ap.add_argument("--degree", type=int, default=5)
    ap.add_argument("--leaf", type=int, default=256)
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    a = ap.parse_args(argv)
    import torch

    from paper_1301_5885_amd import gabi
    from paper_1301_5885_amd.synth import icosphere

    n = 20 * a.nu * a.nu
    V, F = icosphere(a.nu, math.sqrt(n / (16 * math.pi)))
    prec = gabi.FP32_PAIR if a.precision == "fp32" else gabi.FP64
    with gabi.Context(0) as ctx:
        ctx.set_surface_mesh(V, F)
        ctx.set_charges(np.zeros((1, 3)), np.ones(1))
        ctx.set_params(1.0, 80.0, 0.1257)
        ctx.set_stream()
        u = torch.tensor(np.random.default_rng(a.nu).normal(size=2 * n), device="cuda")
        y = torch.empty_like(u)
        ref = torch.empty_like(u)
        ctx.matvec_dev(u, ref, gabi.FP64)
        ctx.tree_matvec_dev(u, y, a.theta, a.degree, a.leaf, prec)   # builds the tree
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.reps):
            ctx.tree_matvec_dev(u, y, a.theta, a.degree, a.leaf, prec)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.reps
        info = ctx.tree_info(a.theta, a.degree, a.leaf)
        err = float(torch.linalg.norm(y - ref) / torch.linalg.norm(ref))
    pairs = info["far_pairs"] + info["near_pairs"]
    print(json.dumps({"N": n, "theta": a.theta, "degree": a.degree, "leaf": a.leaf,
                      "precision": a.precision, "reps": a.reps, "ms_per_product": round(ms, 4),
                      "pairs_per_product": pairs,
                      "algorithmic_tflops": round(pairs * 61 / ms / 1e9, 2),
                      "rel_err_vs_direct_fp64": err}), flush=True)


if __name__ == "__main__":
    main()
