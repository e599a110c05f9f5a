"""Write stored reference values of the FP64 oracle (test infrastructure).

Runs the oracle's IRLS on one seeded synthetic problem and writes a JSON
record with the per-iteration L1 / H_eps history, PCG statistics and
cumulative wall time.  The record is rewritten after every IRLS iteration,
so a partial run is still usable.  Only ``oracle`` and ``synth`` are used.

Usage:
    python -m oracle.make_reference c3 --seed 0 --dtype float32
    python -m oracle.make_reference c2 --seed 0 --dtype float32 --size 2048
    # converged schedule (solves that reach their tolerance): the plain-path
    # parity reference of the 2048^2 field
    python -m oracle.make_reference c2 --seed 0 --dtype float32 --iters 5 \
        --tol 1e-6 --maxit 20000 --tag conv
    # one weight step and exactly 30 PCG iterations from U = 0 (tol 0: no
    # early stop), with U at 10^4 seeded pixels: a record free of the
    # capped schedule's sensitivity
    python -m oracle.make_reference c3 --seed 0 --dtype float32 --iters 1 \
        --tol 0 --maxit 30 --samples 10000 --tag onestep30
    # the paper's running-time shape 4000 x M (Section 4.5): a c2-type field
    # of 4000 x 2000, the capped schedule and the one-step record
    python -m oracle.make_reference c2 --seed 0 --dtype float32 --shape 4000 2000
    python -m oracle.make_reference c2 --seed 0 --dtype float32 --shape 4000 2000 \
        --iters 1 --tol 0 --maxit 30 --samples 10000 --tag onestep30

``--dtype float32`` rounds the inputs (X and the weights) to float32 before
the FP64 solve, which is what the FP32 and mixed GPU paths receive.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import synth  # noqa: E402
from oracle import reduced as R  # noqa: E402

OUT_DIR = os.path.join(HERE, "reference")


SAMPLE_SEED = 12345


def reference_path(gen, seed, size, dtype, tag="", cols=None):
    """size: the side of a square grid, or the row count when cols is given."""
    suffix = f"_{tag}" if tag else ""
    shape = f"{size}" if cols is None or cols == size else f"{size}x{cols}"
    return os.path.join(OUT_DIR, f"{gen}_seed{seed}_{shape}_{dtype}{suffix}.json")


def sample_positions(N, M, k):
    """k seeded pixel positions (row, column), drawn without replacement."""
    rng = np.random.default_rng(SAMPLE_SEED)
    flat = rng.choice(N * M, size=k, replace=False)
    return flat // M, flat % M


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("gen", choices=["c1", "c2", "c3"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--size", type=int, default=None)
    ap.add_argument("--shape", type=int, nargs=2, default=None, metavar=("N", "M"),
                    help="a non-square grid of N rows and M columns")
    ap.add_argument("--dtype", choices=["float32", "float64"], default="float32")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=100)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--tag", default="")
    ap.add_argument("--samples", type=int, default=0,
                    help="store the returned U at this many seeded pixels")
    a = ap.parse_args(argv)
    default = {"c1": 256, "c2": 2048, "c3": 8192}[a.gen]
    n = a.size or default
    m = n
    if a.shape is not None:
        n, m = a.shape
    f = getattr(synth, "field_" + a.gen)(a.seed, n, m)
    X, w = f.X, f.w
    if a.dtype == "float32":
        X = X.astype(np.float32).astype(np.float64)
        w = None if w is None else w.astype(np.float32).astype(np.float64)
    os.makedirs(OUT_DIR, exist_ok=True)
    path = reference_path(a.gen, a.seed, n, a.dtype, a.tag, cols=m)
    rec = dict(gen=a.gen, seed=a.seed, N=n, M=m, input_dtype=a.dtype,
               iters=a.iters, tol=a.tol, maxit=a.maxit, eps=a.eps,
               workers=a.workers, host=platform.node(),
               cpu=platform.processor() or platform.machine(),
               history=[], complete=False)
    t0 = time.perf_counter()

    def cb(h, U):
        h = dict(h)
        h["wall_s"] = time.perf_counter() - t0
        rec["history"].append(h)
        with open(path + ".tmp", "w") as fh:
            json.dump(rec, fh, indent=1)
        os.replace(path + ".tmp", path)
        print(f"k={h['k']} L1={h['L1']:.10g} H={h['H']:.10g} pcg={h['iters']} "
              f"relres={h['relres']:.3e} t={h['wall_s']:.1f}s", flush=True)

    U, hist = R.irls(X, w=w, eps=a.eps, iters=a.iters, tol=a.tol,
                     maxit=a.maxit, workers=a.workers, callback=cb)
    final = dict(hist[-1])
    final["wall_s"] = time.perf_counter() - t0
    rec["history"].append(final)
    rec["L1_final"] = final["L1"]
    rec["H_final"] = final["H"]
    rec["pcg_total"] = int(sum(h.get("iters", 0) for h in hist))
    if a.samples > 0:
        i, j = sample_positions(n, m, a.samples)
        rec["samples"] = dict(seed=SAMPLE_SEED, i=i.tolist(), j=j.tolist(),
                              U=[float(v) for v in U[i, j]])
        rec["U_norm2"] = float(np.sqrt(np.sum(U * U)))
        rec["U_maxabs"] = float(np.max(np.abs(U)))
    rec["complete"] = True
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"final L1={final['L1']:.12g} H={final['H']:.12g} "
          f"wall={final['wall_s']:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    main()
