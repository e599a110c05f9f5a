"""Parity at the benchmark's full size: the 8192 x 8192 fringe-dense field
(c3, seed 0) in the plan configurations bench.py times (mixed FP16, fast
preconditioner; and FP64).  The oracle cannot run whole solves at this size
in a test, so each step is checked on sampled outputs the oracle computes
one by one, or through properties that hold at any size, and the whole path
against the stored FP64 oracle reference of this field
(oracle/reference/c3_seed0_8192_float32.json, written by
oracle/make_reference.py).

Bars (derived per check, see each test): setup bit-exact; operator
element-wise 8 u sum omega (|p_i| + |p_j|); preconditioner against the
oracle's FP64 transform; IRLS objectives against the reference history.
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg
from oracle import reduced as R

pytestmark = pytest.mark.gpu

N = M = 8192
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REF = os.path.join(ROOT, "oracle", "reference", "c3_seed0_8192_float32.json")
# one weight step from U = 0 and exactly 30 PCG iterations (no early stop),
# with U at 10^4 seeded pixels (oracle/make_reference.py --tag onestep30)
REF30 = os.path.join(ROOT, "oracle", "reference", "c3_seed0_8192_float32_onestep30.json")


@pytest.fixture(scope="module")
def field():
    f = synth.field_c3(0, N, M)
    # the reference was computed on the FP32-rounded inputs
    return f.X.astype(np.float32), f.w.astype(np.float32)


@pytest.fixture(scope="module")
def ref():
    with open(REF) as fh:
        return json.load(fh)


def test_setup_bit_exact_on_sampled_edges(field):
    X, w = field
    plan = pkg.Plan(N, M, "f16")
    assert plan.form == "fast"
    Gv, Gh, Cv, Ch, flags = plan.setup(torch.from_numpy(X).cuda(), torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    i = rng.integers(0, N - 1, 200000)
    j = rng.integers(0, M, 200000)
    X64 = X.astype(np.float64)
    gv_o = R.wrap(X64[i + 1, j] - X64[i, j]).astype(np.float32)
    cv_o = np.minimum(w[i + 1, j], w[i, j])
    gv = Gv[torch.from_numpy(i).cuda(), torch.from_numpy(j).cuda()].cpu().numpy()
    cv = Cv[torch.from_numpy(i).cuda(), torch.from_numpy(j).cuda()].cpu().numpy()
    assert np.array_equal(gv, gv_o)
    assert np.array_equal(cv, cv_o)
    i2 = rng.integers(0, N, 200000)
    j2 = rng.integers(0, M - 1, 200000)
    gh_o = R.wrap(X64[i2, j2 + 1] - X64[i2, j2]).astype(np.float32)
    gh = Gh[torch.from_numpy(i2).cuda(), torch.from_numpy(j2).cuda()].cpu().numpy()
    assert np.array_equal(gh, gh_o)
    plan.close()


def test_operator_on_sampled_pixels():
    """q = D^T Omega D p: each sampled output against its four-term sum in
    FP64 from the same FP32 inputs; bound 8 u sum omega (|p_i| + |p_j|)."""
    plan = pkg.Plan(N, M, "f16")
    g = torch.Generator(device="cuda").manual_seed(5)
    p = torch.randn((N, M), device="cuda", generator=g)
    Ov = torch.rand((N, M), device="cuda", generator=g) + 0.05
    Oh = torch.rand((N, M), device="cuda", generator=g) + 0.05
    Ov[N - 1, :] = 0
    Oh[:, M - 1] = 0
    q, _ = plan.operator(Ov, Oh, p)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    i = rng.integers(0, N, 100000)
    j = rng.integers(0, M, 100000)
    ti, tj = torch.from_numpy(i).cuda(), torch.from_numpy(j).cuda()

    def at(t, a, b):
        a = np.clip(a, 0, N - 1)
        b = np.clip(b, 0, M - 1)
        return t[torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()].double().cpu().numpy()

    pc = at(p, i, j)
    terms, bound = np.zeros_like(pc), np.zeros_like(pc)
    for (di, dj, om) in ((1, 0, at(Ov, i, j)), (0, 1, at(Oh, i, j)),
                         (-1, 0, at(Ov, i - 1, j)), (0, -1, at(Oh, i, j - 1))):
        ok = (i + di >= 0) & (i + di < N) & (j + dj >= 0) & (j + dj < M)
        pn = at(p, i + di, j + dj)
        terms += np.where(ok, om * (pc - pn), 0.0)
        bound += np.where(ok, om * (np.abs(pc) + np.abs(pn)), 0.0)
    qg = q[ti, tj].double().cpu().numpy()
    assert np.all(np.abs(qg - terms) <= 8 * 2.0 ** -24 * bound + 1e-30)
    plan.close()


@pytest.mark.parametrize("prec", ["f16", "f32", "f64"])
def test_preconditioner_against_oracle_full_size(prec):
    """z = L^+ r at 8192^2 against the oracle's FP64 transform (scipy's
    orthonormal DCT), relative error in the 2-norm: FP64 1e-12 (transform
    rounding); FP32 1e-5 (log2 n roundings of 2^-24); FP16 storage 1e-2
    (two stored intermediates, each rounded to 2^-11 relative; the norm of
    z is carried by the low modes, which FP16 holds to that precision).

    Reported beside it, the residual ||L z - (r - mean r)|| / ||r||: FP16
    storage loses the high-frequency part of z after the spectral division
    (values dominated by the low modes, amplified up to 1 / lambda_1 ~ 7e6,
    leave FP16 no digits for content 1e-4 of their size), which L
    amplifies; on white-noise r this residual is O(1) for FP16 (see the
    design notes) while the full-size solve still converges like FP32."""
    plan = pkg.Plan(N, M, prec)
    assert plan.form == "fast"
    g = torch.Generator(device="cuda").manual_seed(6)
    r = torch.randn((N, M), device="cuda", generator=g, dtype=plan.dtype)
    z, _ = plan.precond(r)
    torch.cuda.synchronize()
    rn = r.double().cpu().numpy()
    zn = z.double().cpu().numpy()
    plan.close()
    del r, z
    zo = R.apply_precond(rn, workers=min(16, os.cpu_count() or 1))
    rel = np.linalg.norm(zn - zo) / np.linalg.norm(zo)
    Lz = R.apply_A(np.ones((N - 1, M)), np.ones((N, M - 1)), zn)
    res = np.linalg.norm(Lz - (rn - rn.mean())) / np.linalg.norm(rn)
    print(f"precond {prec} 8192^2: rel err {rel:.3e}, ||L z - (r - mean r)|| / ||r|| = {res:.3e}")
    assert rel <= {"f16": 1e-2, "f32": 1e-5, "f64": 1e-12}[prec]
    if prec == "f64":
        assert res <= 1e-10
    assert abs(zn.mean()) <= 1e-6 * np.abs(zn).max()


def test_fp64_capped_iterates_smoke(field, ref):
    """Smoke check of two capped IRLS iterations at full size in FP64 (fast
    form) against the oracle's stored history.  Before any solve (k = 0:
    setup and weights) the objectives agree to 1e-12.  After a capped solve
    only order-one agreement is asserted (5e-3): at the 100-iteration cap
    the CG iterate is not determined to more digits by FP64 arithmetic (the
    oracle run with 6 and with 8 FFT threads gives L1 at k = 1 that differ
    by 1.6e-3).  The element-wise parity of a solve at this size is
    test_one_weight_step_thirty_iterations, which stops at a fixed iteration
    count well before that sensitivity sets in."""
    X, w = field
    plan = pkg.Plan(N, M, "f64")
    p = pkg.default_params("f64")
    p.irls_iters, p.pcg_max, p.eps, p.pcg_rtol = 2, ref["maxit"], ref["eps"], ref["tol"]
    _, st = plan.unwrap(torch.from_numpy(X.astype(np.float64)).cuda(),
                        torch.from_numpy(w.astype(np.float64)).cuda(), params=p, stats=True)
    plan.close()
    for k in range(3):
        bar = 1e-12 if k == 0 else 5e-3
        a, b = st["history"][k]["L1"], ref["history"][k]["L1"]
        print(f"k={k}: GPU L1 {a:.10g} oracle {b:.10g} rel {abs(a - b) / b:.2e}")
        assert abs(a - b) <= bar * b, k
        a, b = st["history"][k]["H"], ref["history"][k]["H"]
        assert abs(a - b) <= bar * b, k


def test_mixed_fp16_reaches_reference_quality(field, ref):
    """The benchmark's configuration end to end: mixed FP16, fast form,
    100 PCG iterations per IRLS iteration: the L1 target L1_ref (1 + 1e-3)
    is reached, and the L1 at that point is within 1e-3 of L1_ref."""
    X, w = field
    plan = pkg.Plan(N, M, "f16")
    p = pkg.default_params("f16")
    L1_ref = ref["L1_final"]
    p.irls_iters, p.pcg_max, p.eps = 40, ref["maxit"], ref["eps"]
    p.l1_target = L1_ref * (1 + 1e-3)
    _, st = plan.unwrap(torch.from_numpy(X).cuda(), torch.from_numpy(w).cuda(), params=p,
                        stats=True)
    plan.close()
    assert st["target_hit"]
    l1 = st["history"][st["irls_done"]]["L1"]
    print(f"mixed FP16: target at IRLS {st['irls_done']}, L1 {l1:.10g} (ref {L1_ref:.10g})")
    assert abs(l1 - L1_ref) <= 1e-3 * L1_ref


# Bars of the one-step check: relative on L1 and H, and on the sampled U
# relative to max |U|.  FP64: the GPU and the oracle run the same
# arithmetic in different summation orders (the DCT's, the reductions'),
# each rounding at 2^-53; 30 CG iterations amplify such differences by the
# iteration's sensitivity, measured below 1e-11 on this field.  FP32:
# vectors and transforms round at 2^-24.  FP16 storage of the
# preconditioner's intermediates (2^-11) changes the preconditioner itself,
# so its iterate is a different (equally valid) CG trajectory; the bar is
# the mixed path's 1e-3 on the objectives.
ONESTEP_BARS = {"f64": (1e-9, 1e-9), "f32": (1e-5, 1e-4), "f16": (1e-3, 1e-1)}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_one_weight_step_thirty_iterations(field, prec):
    """From U = 0: one weight step (Section 3.1 closed-form weights) and
    exactly 30 PCG iterations (Algorithm 2, no early stop: pcg_rtol = 0),
    then mean removal, against the oracle's record of the same steps in
    FP64: L1 and H of U^1, and U^1 itself at 10^4 seeded pixels."""
    with open(REF30) as fh:
        ref = json.load(fh)
    assert ref["complete"] and ref["maxit"] == 30 and ref["tol"] == 0.0 and ref["iters"] == 1
    X, w = field
    plan = pkg.Plan(N, M, prec)
    assert plan.form == "fast"
    p = pkg.default_params(prec)
    p.irls_iters, p.pcg_max, p.pcg_rtol, p.eps = 1, 30, 0.0, ref["eps"]
    p.true_res_every = 0
    dt = np.float64 if prec == "f64" else np.float32
    U, st = plan.unwrap(torch.from_numpy(X.astype(dt)).cuda(), torch.from_numpy(w.astype(dt)).cuda(),
                        params=p, stats=True)
    torch.cuda.synchronize()
    si = torch.from_numpy(np.asarray(ref["samples"]["i"])).cuda()
    sj = torch.from_numpy(np.asarray(ref["samples"]["j"])).cuda()
    Us = U[si, sj].double().cpu().numpy()
    Umax = float(U.abs().max().item())
    plan.close()
    assert st["pcg_total"] == 30
    Uo = np.asarray(ref["samples"]["U"])
    dL1 = abs(st["L1_final"] - ref["L1_final"]) / ref["L1_final"]
    dH = abs(st["H_final"] - ref["H_final"]) / ref["H_final"]
    dU = float(np.max(np.abs(Us - Uo))) / ref["U_maxabs"]
    print(f"one step, 30 PCG, {prec}: L1 {st['L1_final']:.12g} (oracle {ref['L1_final']:.12g}, "
          f"rel {dL1:.2e}), H rel {dH:.2e}, sampled U max|dU|/max|U| {dU:.2e}, "
          f"max|U| {Umax:.6g} (oracle {ref['U_maxabs']:.6g})")
    bar_obj, bar_u = ONESTEP_BARS[prec]
    assert dL1 <= bar_obj and dH <= bar_obj
    assert dU <= bar_u
    assert abs(Umax - ref["U_maxabs"]) <= bar_u * ref["U_maxabs"]
