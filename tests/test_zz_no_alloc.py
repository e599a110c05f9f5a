"""The operator entry point without allocation (irlsu_operator_noalloc: no
workspace, the per-block partial sums in the library's scratch array)
against irlsu_operator on the same inputs: q and p . q identical bit for
bit (the same kernel, the same reduction order), on two calls in a row, the
second with a smaller input than the first (the scratch keeps the larger
call's partials); a plan beyond the scratch's limit is rejected."""
import ctypes

import pytest
import torch

import paper_2401_09961_amd as pkg

pytestmark = pytest.mark.gpu


def _inputs(plan, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    shape = (plan.Np, plan.ld)
    p = torch.zeros(shape, device="cuda", dtype=plan.dtype)
    Ov = torch.zeros_like(p)
    Oh = torch.zeros_like(p)
    N, M = plan.N, plan.M
    p[:N, :M] = torch.randn((N, M), device="cuda", generator=g).to(plan.dtype)
    Ov[:N - 1, :M] = (torch.rand((N - 1, M), device="cuda", generator=g) + 0.05).to(plan.dtype)
    Oh[:N, :M - 1] = (torch.rand((N, M - 1), device="cuda", generator=g) + 0.05).to(plan.dtype)
    return Ov, Oh, p


def _call(lib, plan, Ov, Oh, p, q, pq):
    return lib.irlsu_operator_noalloc(plan.handle, ctypes.c_void_p(Ov.data_ptr()),
                                      ctypes.c_void_p(Oh.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                                      ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(pq.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("prec", ["f32", "f64", "f16"])
def test_noalloc_operator_matches_operator_on_two_calls(prec):
    lib = pkg.load_library()
    cases = []
    for k, (N, M) in enumerate([(1500, 2100), (300, 200)]):  # the second smaller
        plan = pkg.Plan(N, M, prec)
        Ov, Oh, p = _inputs(plan, 10 + k)
        q_ref, pq_ref = plan.operator(Ov, Oh, p)
        q = torch.full_like(p, float("nan"))
        pq = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        cases.append((plan, Ov, Oh, p, q, pq, q_ref, pq_ref))
    torch.cuda.synchronize()
    for plan, Ov, Oh, p, q, pq, _, _ in cases:  # two calls in a row
        assert _call(lib, plan, Ov, Oh, p, q, pq) == 0
    torch.cuda.synchronize()
    for plan, Ov, Oh, p, q, pq, q_ref, pq_ref in cases:
        print(f"{prec} {plan.N}x{plan.M}: p.q {pq.item():.17g} (operator {pq_ref.item():.17g})")
        assert torch.equal(q, q_ref)
        assert pq.item() == pq_ref.item()
        plan.close()


def test_noalloc_operator_rejects_plans_beyond_its_scratch():
    """16384 x 32768 needs 8192 operator blocks, more than the scratch's 4096
    partial sums: ERR_SHAPE, before any launch (the small buffers passed are
    never touched)."""
    lib = pkg.load_library()
    plan = pkg.Plan(16384, 32768, "f32")
    t = torch.zeros(16, device="cuda")
    pq = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert _call(lib, plan, t, t, t, t.clone(), pq) == -2
    plan.close()
    plan = pkg.Plan(16384, 16384, "f32")  # 4096 blocks: the largest accepted square
    Ov = torch.zeros((plan.Np, plan.ld), device="cuda")
    q, pq = plan.operator_noalloc(Ov, Ov, Ov.clone())
    torch.cuda.synchronize()
    assert pq.item() == 0.0 and torch.count_nonzero(q).item() == 0
    plan.close()
