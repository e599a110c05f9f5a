"""The solve on its own (irlsu_pcg, Algorithm 2) against the oracle's PCG,
and the error statuses of the boundary forced from the host: breakdown of
CG on weights that are not positive, a solve stopped at its iteration cap,
and out-of-memory during plan and batch creation (through the library's
allocation-failure hook, so no real allocation fails and nothing on the
GPU misbehaves).

Bars of the PCG parity (x after 12 iterations, no early stop, relative to
max |x|): FP64 1e-11, FP32 1e-5; the final relative residual within 1e-9
(FP64) and 1e-2 (FP32) of the oracle's.  The weights span one decade and
the solve stops at relative residual ~6e-5: there the oracle's own iterate
moves by 1e-14 when its preconditioner output is perturbed by 1e-15
relative and by 6e-10 at 1e-7, so the bars test the arithmetic (the same
in another summation order for FP64; vectors and transforms at 2^-24 for
FP32).  Cases that make no parity test: weights spanning three decades
with 40 iterations, whose iterate is not determined (at 200 x 150 a 1e-15
perturbation moves it by 1e-8, a 1e-7 one by 1.5e-3), and iterating far
past the FP32 floor, where p^T A p and rho are rounding noise.
"""
import ctypes

import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg
from oracle import reduced as R

pytestmark = pytest.mark.gpu

PCG_BAR = {"f64": 1e-11, "f32": 1e-5}
PCG_RELRES = {"f64": 1e-9, "f32": 1e-2}
PCG_ITERS = 12


def _problem(N, M, seed, decades=1.0):
    """Weights spanning `decades` decades and b = D^T Omega G for wrapped G."""
    rng = np.random.default_rng(seed)
    Ov = 10.0 ** rng.uniform(-decades / 2, decades / 2, (N - 1, M))
    Oh = 10.0 ** rng.uniform(-decades / 2, decades / 2, (N, M - 1))
    Gv = R.wrap(rng.normal(0.0, 1.5, (N - 1, M)))
    Gh = R.wrap(rng.normal(0.0, 1.5, (N, M - 1)))
    b = R.div(Ov * Gv, Oh * Gh)
    return Ov, Oh, b


def _internal(plan, A):
    out = torch.zeros((plan.Np, plan.ld), dtype=plan.dtype, device="cuda")
    out[:A.shape[0], :A.shape[1]] = torch.from_numpy(A).to(plan.dtype)
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(256, 256), (200, 150)])
def test_pcg_matches_oracle(prec, shape):
    N, M = shape
    Ov, Oh, b = _problem(N, M, 3)
    plan = pkg.Plan(N, M, prec)
    dt = np.float64 if prec == "f64" else np.float32
    # the GPU receives the weights and b rounded to its element type; the
    # oracle solves with those same values
    Ov, Oh, b = (a.astype(dt).astype(np.float64) for a in (Ov, Oh, b))
    b = b - b.mean()
    p = pkg.default_params(prec)
    p.pcg_max, p.pcg_rtol, p.true_res_every = PCG_ITERS, 0.0, 0
    p.flexible = 0
    x, code, it, rel = plan.pcg(_internal(plan, np.vstack([Ov, np.zeros((1, M))])),
                                _internal(plan, np.hstack([Oh, np.zeros((N, 1))])),
                                _internal(plan, b), params=p)
    xg = x[:N, :M].cpu().numpy()
    form = plan.form
    plan.close()
    xo, info = R.pcg(lambda v: R.apply_A(Ov, Oh, v), R.apply_precond, b, np.zeros((N, M)), 0.0,
                     PCG_ITERS)
    err = np.abs(xg - xo).max() / np.abs(xo).max()
    print(f"pcg {prec} {shape} ({form}): it {it} code {code} relres {rel:.3e} "
          f"(oracle {info['relres']:.3e}), max|dx|/max|x| {err:.2e}")
    assert code == 1 and it == PCG_ITERS  # the cap reached with no early stop: NOT_CONVERGED
    assert err <= PCG_BAR[prec]
    assert abs(rel - info["relres"]) <= PCG_RELRES[prec] * info["relres"]


def test_pcg_converges_to_tolerance():
    """With a tolerance the solve stops at ||r|| <= tol ||b||, like the oracle."""
    N = M = 128
    Ov, Oh, b = _problem(N, M, 4)
    b = b - b.mean()
    plan = pkg.Plan(N, M, "f64")
    p = pkg.default_params("f64")
    p.pcg_max, p.pcg_rtol, p.true_res_every = 500, 1e-10, 0
    x, code, it, rel = plan.pcg(_internal(plan, np.vstack([Ov, np.zeros((1, M))])),
                                _internal(plan, np.hstack([Oh, np.zeros((N, 1))])),
                                _internal(plan, b), params=p)
    plan.close()
    xo, info = R.pcg(lambda v: R.apply_A(Ov, Oh, v), R.apply_precond, b, np.zeros((N, M)),
                     1e-10, 500)
    print(f"pcg tol 1e-10: GPU {it} iterations relres {rel:.2e}; oracle {info['iters']}")
    assert code == 0 and rel <= 1e-10
    # poll granularity: the host reads the flag every poll_every iterations,
    # but the device stops at the first iteration that meets the tolerance
    assert it == info["iters"]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_pcg_breakdown_on_negative_weights(prec):
    """Weights that are not positive make D^T Omega D indefinite: p^T A p
    <= 0 is detected on the device and reported as ERR_BREAKDOWN."""
    N = M = 256
    Ov, Oh, b = _problem(N, M, 5)
    Ov, Oh = -Ov, -Oh
    plan = pkg.Plan(N, M, prec)
    with pytest.raises(pkg.IrlsuError) as e:
        plan.pcg(_internal(plan, np.vstack([Ov, np.zeros((1, M))])),
                 _internal(plan, np.hstack([Oh, np.zeros((N, 1))])), _internal(plan, b))
    plan.close()
    assert e.value.code == -5


def test_unwrap_not_converged_at_cap():
    """A residue field with a two-iteration cap: every solve stops at the
    cap, the call returns NOT_CONVERGED (a warning) with a finite U."""
    f = synth.field_c2(0, 128, 128)
    plan = pkg.Plan(128, 128, "f32")
    p = pkg.default_params("f32")
    p.irls_iters, p.pcg_max = 3, 2
    U, st = plan.unwrap(torch.from_numpy(f.X.astype(np.float32)).cuda(),
                        torch.from_numpy(f.w.astype(np.float32)).cuda(), params=p, stats=True)
    plan.close()
    assert st["code"] == 1
    assert all(h["status"] == 1 and h["iters"] == 2 for h in st["history"][:3])
    assert torch.isfinite(U).all()


def _create(lib, N, M, prec, form):
    h = ctypes.c_void_p()
    code = lib.irlsu_plan_create_ex(ctypes.byref(h), N, M, pkg.PRECISIONS[prec], form, None)
    return code, h


@pytest.mark.parametrize("N,M,prec,form", [(256, 256, "f16", 3), (256, 512, "f32", 3),
                                           (1024, 1024, "bf16", 2), (1000, 600, "f16", 2),
                                           (200, 150, "f64", 1), (200, 300, "f32", 1)])
def test_plan_create_out_of_memory_leaks_nothing(N, M, prec, form):
    """Each allocation of plan creation failed in turn: ERR_OOM, no plan
    returned, and the device's free memory afterwards is what it was."""
    lib = pkg.load_library()
    code, h = _create(lib, N, M, prec, form)  # warm the runtime's own state
    assert code == 0
    lib.irlsu_plan_destroy(h)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failures = 0
    for nth in range(64):
        lib.irlsu_test_fail_alloc(nth)
        code, h = _create(lib, N, M, prec, form)
        if code == 0:
            lib.irlsu_plan_destroy(h)
            break
        assert code == -7, code
        assert not h.value
        failures += 1
    lib.irlsu_test_fail_alloc(-1)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"plan {N}x{M} {prec} form {form}: {failures} allocations failed in turn, "
          f"free memory {free0} -> {free1}")
    assert failures >= 3
    assert free1 == free0


def test_batch_create_out_of_memory_leaks_nothing():
    lib = pkg.load_library()
    shapes = (ctypes.c_int64 * 6)(600, 520, 700, 600, 520, 520)

    def create():
        h = ctypes.c_void_p()
        return lib.irlsu_batch_create(ctypes.byref(h), shapes, 3, pkg.PRECISIONS["bf16"], None), h

    code, h = create()
    assert code == 0
    lib.irlsu_batch_destroy(h)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failures = 0
    for nth in range(64):
        lib.irlsu_test_fail_alloc(nth)
        code, h = create()
        if code == 0:
            lib.irlsu_batch_destroy(h)
            break
        assert code == -7, code
        assert not h.value
        failures += 1
    lib.irlsu_test_fail_alloc(-1)
    torch.cuda.synchronize()
    assert failures >= 5
    assert torch.cuda.mem_get_info()[0] == free0
