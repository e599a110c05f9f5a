"""The launch-shape autotuner: measured choices are applied and cached in a
JSON file keyed by shape, precision, form and architecture (a second call
reads them back); the solves' results do not depend on the launch shapes
beyond the order of the FP64 partial sums (converged FP64 solves agree to
1e-9 in L1; FP32 to the plain path's 1e-5); the batch's tuned band heights
give the untuned batch's results."""
import json

import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,prec", [((512, 512), "f32"), ((1024, 768), "f16"),
                                        ((300, 260), "f64")])
def test_autotune_applies_and_caches(tmp_path, shape, prec):
    cache = tmp_path / "tune.json"
    plan = pkg.Plan(*shape, prec)
    t1 = plan.autotune(cache)
    assert t1["from_cache"] == 0 and t1["stencil_us"] > 0
    assert plan.get_tune()["stencil_rows"] == t1["stencil_rows"]
    doc = json.loads(cache.read_text())
    ent = [e for e in doc["entries"] if e["N"] == shape[0] and e["M"] == shape[1]]
    assert len(ent) == 1 and ent[0]["kind"] == "plan"
    assert ent[0]["arch"].startswith("gfx950")
    assert ent[0]["stencil_rows"] == t1["stencil_rows"]
    plan.set_tune()  # defaults, then read back from the cache
    t2 = plan.autotune(cache)
    assert t2["from_cache"] == 1
    assert (t2["stencil_rows"], t2["update_blocks"], t2["small_tiles"]) == \
        (t1["stencil_rows"], t1["update_blocks"], t1["small_tiles"])
    print(f"{shape} {prec} ({plan.form}): {t1}")
    plan.close()


@pytest.mark.parametrize("prec,form,bar", [("f64", "dense", 1e-9), ("f64", "fast", 1e-9),
                                           ("f32", "folded", 1e-5), ("f16", "dense", 1e-3)])
def test_results_do_not_depend_on_launch_shapes(prec, form, bar):
    N, M = (512, 512) if form == "fast" else (520, 400)
    f = synth.field_c2(2, N, M)
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.from_numpy(f.X).to(device="cuda", dtype=dt)
    w = torch.from_numpy(f.w).to(device="cuda", dtype=dt)
    plan = pkg.Plan(N, M, prec, form=form)
    p = pkg.default_params(prec)
    p.irls_iters, p.pcg_max = 4, 5000
    p.pcg_rtol = 1e-10 if prec == "f64" else 1e-6
    res = []
    for shapes in [(0, 0, 0), (8, 64, 1), (128, 1024, 0), (16, 128, 1)]:
        plan.set_tune(*shapes)
        _, st = plan.unwrap(X, w, params=p, stats=True)
        res.append(st)
    plan.close()
    base = res[0]
    for st in res[1:]:
        for k in range(p.irls_iters + 1):
            a, b = st["history"][k]["L1"], base["history"][k]["L1"]
            assert abs(a - b) <= bar * b, (k, a, b)
    print(f"{prec} {form}: L1 {[r['L1_final'] for r in res]}")


def test_batch_autotune_keeps_results(tmp_path):
    shapes = [(520, 600), (512, 512), (700, 530), (300, 1100)]
    fields = [synth.field_c2(60 + t, n, m) for t, (n, m) in enumerate(shapes)]
    X = [torch.from_numpy(f.X.astype(np.float32)).cuda() for f in fields]
    W = [torch.from_numpy(f.w.astype(np.float32)).cuda() for f in fields]
    p = pkg.default_params("f32")
    p.irls_iters, p.pcg_max, p.pcg_rtol = 3, 4000, 1e-6
    b = pkg.Batch(shapes, "f32")
    _, s0 = b.unwrap(X, W, params=p, stats=True)
    b.autotune(tmp_path / "tune.json")
    _, s1 = b.unwrap(X, W, params=p, stats=True)
    b.close()
    doc = json.loads((tmp_path / "tune.json").read_text())
    assert sum(e["kind"] == "batch_tile" for e in doc["entries"]) == len(shapes)
    for a, c in zip(s0, s1):
        assert abs(a["L1_final"] - c["L1_final"]) <= 1e-5 * a["L1_final"]
