"""Autotuner for the decomposition of the boundary-integral product.

The product of one molecule (the double sum over targets i and sources j of
the K1..K4 pair kernels, eqs. (eqdbef1)/(eqdbef2)) is cut into row blocks of
256 * R targets and into source splits: whole 256-source tiles sized so that
about `target_blocks` workgroups run, then `tail_pieces` splits of 64
sources at the end of the source range; a persistent grid drains the
resulting list longest first, so the short tail splits fill the device's
last round.  This module times the whole product (pair kernel plus the
ordered split reduction) on geodesic spheres of one representative size per
N bucket (bucket = floor(log2 N)), for both pair precisions: first every
(R, target_blocks) without a tail, then the three fastest of those with
each tail length (up to every split a 64-source piece), and the symmetric
scheme (whose block pairs come in round-robin rounds; it has no shape
parameter here: its passes follow from the partial-sum budget), and writes
the fastest entry per bucket as JSON.  The
library applies that table when it is loaded (`gabi.TUNING_PATH`).

The decomposition fixes the order of the row sums, so a table change
changes results in the last bits; every result made under one table is
bitwise reproducible.

    python -m paper_1301_5885_amd.tune [--out PATH] [--reps 5]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import gabi
from .synth import icosphere

# One geodesic sphere per N bucket: N = 20 nu^2 (bucket = floor(log2 N)).
BUCKET_NU = {10: 8, 11: 12, 12: 16, 13: 24, 14: 32, 15: 48, 16: 64, 17: 96, 18: 128}
ROWS = (1, 2)
TARGET_BLOCKS = (256, 512, 1024, 2048, 3072, 4096, 6144, 8192, 12288, 16384, 24576, 32768,
                 49152, 65536, 98304, 131072, 196608, 262144)
TAILS = (4, 8, 16, 32, 64, 128)
BANDS = (0,)   # the symmetric scheme's one candidate
PRECISIONS = {"fp64": gabi.FP64, "fp32": gabi.FP32_PAIR}


def log(*a):
    print(*a, flush=True)


def sources_per_split(n, rows_per_thread, target_blocks):
    """Source tiles per split of the decomposition the library derives from
    (N, R, target_blocks) without a tail: candidates with the same (R, result)
    are the same launch and are timed once."""
    row_blocks = -(-n // (256 * rows_per_thread))
    tiles = -(-n // 256)
    want = max(1, -(-target_blocks // row_blocks))
    return max(1, -(-tiles // want))


def time_product(V, F, precision, reps):
    """Median ms of one product (all kernels of gabi_matvec_dev) on torch's
    current stream, after two warm-up products."""
    import torch
    with gabi.Context(0) as ctx:
        ctx.set_surface_mesh(V, F)
        ctx.set_charges(np.zeros((1, 3)), [1.0])
        ctx.set_params(1.0, 80.0, 0.1257)
        n = ctx.n
        gen = torch.Generator(device="cuda").manual_seed(1)
        u = torch.randn(2 * n, dtype=torch.float64, device="cuda", generator=gen)
        y = torch.empty_like(u)
        for _ in range(2):
            ctx.matvec_dev(u, y, precision)
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.matvec_dev(u, y, precision)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))


def tune(buckets, reps, out_path):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the autotuner needs a GPU")
    gabi.load()
    table = {"device": torch.cuda.get_device_name(0), "reps": reps,
             "candidates": {"schemes": ["split", "symmetric"], "rows_per_thread": list(ROWS),
                            "target_blocks": list(TARGET_BLOCKS),
                            "tail_pieces": [0] + list(TAILS), "bands": list(BANDS)},
             "entries": {k: {} for k in PRECISIONS}, "sweep": {k: {} for k in PRECISIONS}}
    t_start = time.time()
    for b in buckets:
        nu = BUCKET_NU[b]
        V, F = icosphere(nu, 2.0 * nu ** 0.5)
        n = len(F)
        assert int(np.floor(np.log2(n))) == b
        for key, prec in PRECISIONS.items():
            default = gabi.tune_get(prec, b)
            rows, seen = [], set()
            for R in ROWS:
                for tb in TARGET_BLOCKS:
                    key_rt = (R, sources_per_split(n, R, tb))
                    if key_rt in seen:
                        continue
                    seen.add(key_rt)
                    gabi.tune_set(prec, b, gabi.SCHEME_SPLIT, R, tb, 0)
                    ms = time_product(V, F, prec, reps)
                    rows.append((ms, gabi.SCHEME_SPLIT, R, tb, 0))
            rows.sort()
            untailed = rows[0]
            # tails up to every source split a 64-source piece: at small N
            # whole 256-source tiles leave most of the device idle
            all_pieces = -(-n // 64)
            tails = sorted({t for t in TAILS if t < all_pieces} | {all_pieces, -(-all_pieces // 2)})
            for _, _, R, tb, _ in rows[:3]:
                for tail in tails:
                    gabi.tune_set(prec, b, gabi.SCHEME_SPLIT, R, tb, tail)
                    ms = time_product(V, F, prec, reps)
                    rows.append((ms, gabi.SCHEME_SPLIT, R, tb, tail))
            sym_rows = []
            for band in BANDS:
                if band and band >= -(-n // 256):
                    continue
                gabi.tune_set(prec, b, gabi.SCHEME_SYMMETRIC, 1, 1, band)
                sym_rows.append((time_product(V, F, prec, reps), gabi.SCHEME_SYMMETRIC, 1, 1, band))
            rows += sym_rows
            sym = min(sym_rows)[0]
            gabi.tune_set(prec, b, *default)
            rows.sort()
            ms, sc, R, tb, tail = rows[0]
            pairs = n * (n - 1)
            table["entries"][key][str(b)] = {"scheme": sc, "rows_per_thread": R,
                                             "target_blocks": tb, "tail_pieces": tail, "n": n,
                                             "ms": round(ms, 5),
                                             "gpairs_per_s": round(pairs / ms / 1e6, 2)}
            table["sweep"][key][str(b)] = [[s_, R, tb, t, round(m, 5)] for m, s_, R, tb, t in rows]
            log(f"bucket {b:2d} N={n:7d} {key}: best scheme={sc} R={R} blocks={tb:6d} "
                f"tail/band={tail:3d} {ms:9.4f} ms ({pairs / ms / 1e6:8.1f} Gpairs/s); split without "
                f"tail {untailed[0]:.4f} ms; best symmetric {sym:.4f} ms; worst {rows[-1][0]:.4f} ms "
                f"[{time.time() - t_start:.0f} s]")
    with open(out_path + ".tmp", "w") as f:
        json.dump(table, f, indent=1)
    os.replace(out_path + ".tmp", out_path)
    log(f"wrote {out_path}")
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=gabi.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--buckets", default=",".join(str(b) for b in BUCKET_NU))
    a = ap.parse_args(argv)
    # tune from the built-in defaults, not from a previous table
    os.environ["GABI_TUNING"] = "none"
    buckets = [int(x) for x in a.buckets.split(",")]
    for b in buckets:
        if b not in BUCKET_NU:
            sys.exit(f"no representative size for bucket {b}")
    tune(buckets, a.reps, a.out)


if __name__ == "__main__":
    main()
