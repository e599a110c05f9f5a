"""PCG iterations replayed from captured HIP graphs give exactly the results
of direct launches (the same kernels with the same arguments in the same
order): U bit for bit, and the same iteration counts and objectives, in
every preconditioner form and precision; and repeated unwraps (each solve
replays the graphs many times, with the host's polls and the weight steps
between replays) stay identical."""
import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg

pytestmark = pytest.mark.gpu

CASES = [((256, 256), "f64", "fast"), ((256, 256), "f16", "fast"), ((512, 256), "f32", "fast"),
         ((300, 260), "f32", "dense"), ((1024, 1100), "bf16", "folded"),
         ((200, 150), "f64", "dense")]


def _unwrap(plan, X, w, graph, prec, true_res_every=32):
    p = pkg.default_params(prec)
    p.irls_iters, p.pcg_max, p.graph = 4, 60, graph
    p.true_res_every = true_res_every
    U, st = plan.unwrap(X, w, params=p, stats=True)
    torch.cuda.synchronize()
    return U.clone(), st


@pytest.mark.parametrize("shape,prec,form", CASES)
def test_graph_replay_matches_direct_launches(shape, prec, form):
    N, M = shape
    f = synth.field_c2(1, N, M)
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.from_numpy(f.X).to(device="cuda", dtype=dt)
    w = torch.from_numpy(f.w).to(device="cuda", dtype=dt)
    plan = pkg.Plan(N, M, prec, form=form)
    U0, s0 = _unwrap(plan, X, w, 0, prec, true_res_every=7)
    U1, s1 = _unwrap(plan, X, w, 1, prec, true_res_every=7)
    U2, s2 = _unwrap(plan, X, w, 1, prec, true_res_every=7)
    plan.close()
    print(f"{shape} {prec} {form}: pcg {s0['pcg_total']} / {s1['pcg_total']} / {s2['pcg_total']}, "
          f"L1 {s0['L1_final']:.12g} / {s1['L1_final']:.12g}")
    assert torch.equal(U0, U1) and torch.equal(U1, U2)
    assert s0["pcg_total"] == s1["pcg_total"] == s2["pcg_total"]
    assert [h["iters"] for h in s0["history"]] == [h["iters"] for h in s1["history"]]
    assert s0["L1_final"] == s1["L1_final"] == s2["L1_final"]


def test_graph_replay_in_the_adjoint_and_the_step_solve():
    """The adjoint's solve and irlsu_pcg go through the same loop."""
    N, M = 256, 256
    f = synth.field_c5(3, N, M)
    X = torch.from_numpy(f.X).to(device="cuda", dtype=torch.float32)
    Cv = torch.from_numpy(f.Cv).to(device="cuda", dtype=torch.float32)
    Ch = torch.from_numpy(f.Ch).to(device="cuda", dtype=torch.float32)
    plan = pkg.Plan(N, M, "f32")
    gU = torch.randn((N, M), device="cuda", generator=torch.Generator(device="cuda").manual_seed(2))
    out = []
    for graph in (0, 1, 1):
        p = pkg.default_params("f32")
        p.irls_iters, p.pcg_max, p.graph = 3, 80, graph
        U = plan.unwrap(X, Cv=Cv, Ch=Ch, params=p)
        pa = pkg.default_params("f32")
        pa.graph = graph
        g = plan.adjoint(gU, params=pa)
        torch.cuda.synchronize()
        out.append([U.clone()] + [t.clone() for t in g if t is not None])
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    for a, b in zip(out[1], out[2]):
        assert torch.equal(a, b)
    plan.close()


def test_batched_graph_replay_matches_direct_launches():
    shapes = [(520, 600), (700, 530), (600, 600), (530, 770)]
    Xs = [torch.from_numpy(synth.field_c4_tile(t, n, m).X).to(device="cuda", dtype=torch.float32)
          for t, (n, m) in enumerate(shapes)]
    batch = pkg.Batch(shapes, "bf16")
    res = []
    for graph in (0, 1, 1):
        p = pkg.default_params("bf16")
        p.irls_iters, p.pcg_max, p.graph, p.true_res_every = 3, 40, graph, 9
        Us, st = batch.unwrap(Xs, params=p, stats=True)
        torch.cuda.synchronize()
        res.append(([u.clone() for u in Us], [s["pcg_total"] for s in st]))
    batch.close()
    for a, b in zip(res[0][0], res[1][0]):
        assert torch.equal(a, b)
    for a, b in zip(res[1][0], res[2][0]):
        assert torch.equal(a, b)
    assert res[0][1] == res[1][1] == res[2][1]
