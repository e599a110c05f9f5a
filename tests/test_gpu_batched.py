"""Batched uneven tiles: one grouped launch per PCG phase over all tiles.

* c4 recipe (small-case generator per tile, seed 1000 + t) satisfies the
  Itoh condition: each tile's U equals plain integration up to a constant
  (checked pointwise; FP32 vectors, BF16 preconditioner, converged solves).
* batched solve == per-tile solves through irlsu_unwrap (objective values;
  the partial-sum partition differs, so not bitwise).
* residue-bearing tiles: final L1 within the mixed bar 1e-3 of the oracle.
"""
import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg
from oracle import reduced as R

pytestmark = pytest.mark.gpu

SHAPES = [(130, 257), (256, 200), (300, 140), (96, 80), (520, 300)]


def params(iters=6, maxit=3000):
    p = pkg.default_params("bf16")
    p.irls_iters, p.pcg_max = iters, maxit
    return p


def test_batched_itoh_tiles_are_integration():
    fields = [synth.field_c4_tile(t, N, M) for t, (N, M) in enumerate(SHAPES)]
    b = pkg.Batch(SHAPES, "bf16")
    Us, st = b.unwrap([torch.from_numpy(f.X.astype(np.float32)).cuda() for f in fields],
                      params=params(3), stats=True)
    torch.cuda.synchronize()
    for f, U, s in zip(fields, Us, st):
        truth = f.phi - f.phi.mean()
        err = np.abs(U.cpu().numpy().astype(np.float64) - truth).max()
        assert err < 2e-3, err
        assert s["history"][0]["iters"] > 0
    b.close()


def test_batched_equals_per_tile_solves():
    fields = [synth.field_c3(20 + t, N, M) for t, (N, M) in enumerate(SHAPES)]
    X = [torch.from_numpy(f.X.astype(np.float32)).cuda() for f in fields]
    W = [torch.from_numpy(f.w.astype(np.float32)).cuda() for f in fields]
    p = params(5)
    b = pkg.Batch(SHAPES, "bf16")
    Ub, sb = b.unwrap(X, W, params=p, stats=True)
    for t, (N, M) in enumerate(SHAPES):
        plan = pkg.Plan(N, M, "bf16")
        U1, s1 = plan.unwrap(X[t], W[t], params=p, stats=True)
        gap = abs(sb[t]["L1_final"] - s1["L1_final"]) / s1["L1_final"]
        assert gap <= 1e-4, (t, gap)
        plan.close()
    b.close()


def test_batched_residue_tiles_vs_oracle():
    shapes = SHAPES[:3]
    fields = [synth.field_c2(30 + t, N, M) for t, (N, M) in enumerate(shapes)]
    X = [f.X.astype(np.float32) for f in fields]
    W = [f.w.astype(np.float32) for f in fields]
    p = params(5)
    b = pkg.Batch(shapes, "bf16")
    Ub, sb = b.unwrap([torch.from_numpy(x).cuda() for x in X],
                      [torch.from_numpy(w).cuda() for w in W], params=p, stats=True)
    for t in range(len(shapes)):
        Uo, h = R.irls(X[t].astype(np.float64), w=W[t].astype(np.float64), iters=5,
                       tol=p.pcg_rtol, maxit=p.pcg_max)
        gap = abs(sb[t]["L1_final"] - h[-1]["L1"]) / h[-1]["L1"]
        print(f"tile {t} {shapes[t]}: L1 gpu {sb[t]['L1_final']:.8g} oracle {h[-1]['L1']:.8g} gap {gap:.2e}")
        assert gap <= 1e-3
    b.close()


def test_batch_rejects_unsupported_precision():
    with pytest.raises(pkg.IrlsuError) as e:
        pkg.Batch([(64, 64)], "f32")
    assert e.value.name == "ERR_UNSUPPORTED"
