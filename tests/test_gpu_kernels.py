"""Kernel-level parity of the HIP path against the FP64 oracle, through the
C ABI (step entry points), on seeded inputs that span several tiles and a
ragged tail.

Tolerances (derived from the arithmetic, per precision of the plan):
* setup: bit-exact -- both sides difference and wrap in FP64 with the same
  rounded operations, the FP32 plan then rounds to nearest.
* weights / operator: element-wise bound 8 u sum_e Omega_e (|p_i| + |p_j|)
  (u the unit roundoff of the vector type; each output sums four terms).
* preconditioner: element-wise, |z_gpu - z| <= 8 sigma_ij with sigma_ij
  from the probabilistic rounding model of each form (tests/precond_bound.py:
  the roundings of each stage propagated through the rest of the map), and
  norm-wise relative error beside it: FP64 1e-11, FP32 2e-5, BF16 3e-2
  (operands rounded to 8 mantissa bits in four chained products).
"""
import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg
import precond_bound as PB
from oracle import reduced as R

pytestmark = pytest.mark.gpu

SHAPES = [(96, 80), (131, 257), (256, 256)]
# sizes whose padded dimensions are multiples of 256 select the 256 x 256 tile
BIG_SHAPES = [(512, 768), (1000, 515)]
UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -24}
PRECOND_RTOL = {"f64": 1e-11, "f32": 2e-5, "bf16": 3e-2}


def npdt(prec):
    return np.float64 if prec == "f64" else np.float32


def internal(plan, A, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    return plan.to_internal(t, dtype=dtype)


def assert_elementwise(zg, r, form, prec):
    """Every element of z within 8 sigma of the oracle's FP64 z (Section 3.3
    eigendecomposition solve, Appendix B zero mode), sigma from the rounding
    model of the plan's form and precision."""
    S = PB.stages(np.asarray(r, np.float64))
    sig = PB.plan_sigma(S, form, prec)
    ok, worst, idx = PB.check(zg, S, sig)
    print(f"  element-wise {form} {prec} {S['z'].shape}: worst |dz|/sigma {worst:.3f} at {idx}, "
          f"8 sigma / max|z| = {PB.KAPPA * sig.max() / np.abs(S['z']).max():.2e}")
    assert ok, (worst, idx)


def edge_v(plan, Ev, dtype=None):
    return internal(plan, Ev, dtype)  # (N-1) x M in the top-left corner


@pytest.fixture(scope="module", params=["f64", "f32", "bf16"])
def prec(request):
    return request.param


@pytest.mark.parametrize("shape", SHAPES)
def test_setup_bit_exact(prec, shape):
    N, M = shape
    f = synth.field_c2(1, N, M)
    dt = npdt(prec)
    X, w = f.X.astype(dt), f.w.astype(dt)
    plan = pkg.Plan(N, M, prec)
    Gv, Gh, Cv, Ch, flags = plan.setup(torch.from_numpy(X).cuda(), torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    Gv_o, Gh_o = R.wrapped_gradients(X.astype(np.float64))
    Cv_o, Ch_o = R.edge_weights(N, M, w=w.astype(np.float64))
    Gv_g, Gh_g = Gv.cpu().numpy(), Gh.cpu().numpy()
    assert np.array_equal(Gv_g[: N - 1, :M], Gv_o.astype(dt))
    assert np.array_equal(Gh_g[:N, : M - 1], Gh_o.astype(dt))
    assert np.array_equal(Cv.cpu().numpy()[: N - 1, :M], Cv_o.astype(dt))
    assert np.array_equal(Ch.cpu().numpy()[:N, : M - 1], Ch_o.astype(dt))
    # padding and missing edges are zero
    for A, r, c in ((Gv_g, N - 1, M), (Gh_g, N, M - 1)):
        Z = A.copy()
        Z[:r, :c] = 0
        assert not Z.any()
    plan.close()


def test_setup_flags_bad_inputs():
    plan = pkg.Plan(40, 33, "f32")
    X = torch.zeros((40, 33), dtype=torch.float32, device="cuda")
    w = torch.ones_like(X)
    X[3, 4] = float("nan")
    *_, flags = plan.setup(X, w)
    assert int(flags.item()) & 1
    X[3, 4] = 0.0
    w[5, 6] = 0.0
    *_, flags = plan.setup(X, w)
    assert int(flags.item()) & 2
    plan.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_weights_step(prec, shape):
    N, M = shape
    f = synth.field_c3(2, N, M)
    dt = npdt(prec)
    plan = pkg.Plan(N, M, prec)
    Gv, Gh, Cv, Ch, _ = plan.setup(torch.from_numpy(f.X.astype(dt)).cuda(),
                                   torch.from_numpy(f.w.astype(dt)).cuda())
    rng = np.random.default_rng(3)
    U = f.phi - f.phi.mean() + rng.normal(0, 0.3, (N, M))
    Ui = internal(plan, U, torch.float64)
    eps = 1e-3
    Ov, Oh, b, obj = plan.weights(eps, Ui, Gv, Gh, Cv, Ch)
    torch.cuda.synchronize()
    Gv_o = Gv.cpu().numpy()[: N - 1, :M].astype(np.float64)
    Gh_o = Gh.cpu().numpy()[:N, : M - 1].astype(np.float64)
    Cv_o = Cv.cpu().numpy()[: N - 1, :M].astype(np.float64)
    Ch_o = Ch.cpu().numpy()[:N, : M - 1].astype(np.float64)
    Ov_o, Oh_o, b_o, L1, H = R.weight_step(U, Gv_o, Gh_o, Cv_o, Ch_o, eps)
    u = UNIT[prec]
    Ov_g = Ov.cpu().numpy()
    Oh_g = Oh.cpu().numpy()
    assert np.all(np.abs(Ov_g[: N - 1, :M] - Ov_o) <= 2 * u * np.abs(Ov_o))
    assert np.all(np.abs(Oh_g[:N, : M - 1] - Oh_o) <= 2 * u * np.abs(Oh_o))
    assert not Ov_g[N - 1:, :].any() and not Oh_g[:, M - 1:].any()
    fv, fh = np.abs(Ov_o * Gv_o), np.abs(Oh_o * Gh_o)
    bound = (np.pad(fv, ((0, 1), (0, 0))) + np.pad(fv, ((1, 0), (0, 0)))
             + np.pad(fh, ((0, 0), (0, 1))) + np.pad(fh, ((0, 0), (1, 0))))
    err = np.abs(b.cpu().numpy()[:N, :M] - b_o)
    assert np.all(err <= 8 * u * bound + 1e-300)
    o = obj.cpu().numpy()
    assert abs(o[0] - L1) <= 1e-12 * L1
    assert abs(o[1] - H) <= 1e-12 * H
    bb = float(np.sum(b.cpu().numpy().astype(np.float64) ** 2))
    assert abs(o[2] - bb) <= 1e-12 * bb
    plan.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_operator_and_dot(prec, shape):
    N, M = shape
    dt = npdt(prec)
    rng = np.random.default_rng(4)
    Ov = rng.uniform(0.0, 50.0, (N - 1, M)).astype(dt)
    Oh = rng.uniform(0.0, 50.0, (N, M - 1)).astype(dt)
    p = rng.standard_normal((N, M)).astype(dt)
    plan = pkg.Plan(N, M, prec)
    q, pq = plan.operator(internal(plan, Ov), internal(plan, Oh), internal(plan, p))
    torch.cuda.synchronize()
    Ovd, Ohd, pd = Ov.astype(np.float64), Oh.astype(np.float64), p.astype(np.float64)
    q_o = R.apply_A(Ovd, Ohd, pd)
    absd_v = np.abs(Ovd) * (np.abs(pd[1:, :]) + np.abs(pd[:-1, :]))
    absd_h = np.abs(Ohd) * (np.abs(pd[:, 1:]) + np.abs(pd[:, :-1]))
    bound = (np.pad(absd_v, ((0, 1), (0, 0))) + np.pad(absd_v, ((1, 0), (0, 0)))
             + np.pad(absd_h, ((0, 0), (0, 1))) + np.pad(absd_h, ((0, 0), (1, 0))))
    qg = q.cpu().numpy()
    assert np.all(np.abs(qg[:N, :M] - q_o) <= 8 * UNIT[prec] * bound)
    assert not qg[N:, :].any() and not qg[:, M:].any()
    ref = float(np.sum(pd * qg[:N, :M].astype(np.float64)))
    assert abs(pq.item() - ref) <= 1e-12 * np.sum(np.abs(pd * q_o)) + 1e-300
    plan.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_precond_matches_dct_oracle(prec, shape):
    N, M = shape
    dt = npdt(prec)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((N, M)).astype(dt)
    plan = pkg.Plan(N, M, prec, form="dense")
    z, rz = plan.precond(internal(plan, r))
    torch.cuda.synchronize()
    z_o = R.apply_precond(r.astype(np.float64))
    zg = z.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(zg[:N, :M] - z_o) / np.linalg.norm(z_o)
    print(f"precond {prec} {shape}: rel err {rel:.3e}")
    assert rel <= PRECOND_RTOL[prec]
    assert_elementwise(zg[:N, :M], r, "dense", prec)
    assert np.abs(zg[N:, :]).max(initial=0) == 0 and np.abs(zg[:, M:]).max(initial=0) == 0
    ref = float(np.sum(r.astype(np.float64) * z_o))
    assert abs(rz.item() - ref) <= 2 * PRECOND_RTOL[prec] * abs(ref)
    plan.close()


@pytest.mark.parametrize("shape", BIG_SHAPES)
@pytest.mark.parametrize("p16", ["bf16", "f16"])
def test_precond_big_tiles(p16, shape):
    N, M = shape
    rng = np.random.default_rng(7)
    r = rng.standard_normal((N, M)).astype(np.float32)
    plan = pkg.Plan(N, M, p16, form="dense")
    z, rz = plan.precond(internal(plan, r))
    torch.cuda.synchronize()
    z_o = R.apply_precond(r.astype(np.float64))
    zg = z.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(zg[:N, :M] - z_o) / np.linalg.norm(z_o)
    print(f"precond {p16} {shape}: rel err {rel:.3e}")
    assert rel <= PRECOND_RTOL["bf16"]
    assert_elementwise(zg[:N, :M], r, "dense", p16)
    assert np.abs(zg[N:, :]).max(initial=0) == 0 and np.abs(zg[:, M:]).max(initial=0) == 0
    plan.close()


# even sides: the folded (even / odd) form; N/2 or M/2 not a multiple of 128
# pads the half-size products
FOLD_SHAPES = [(96, 80), (130, 514), (256, 256), (1000, 512)]


@pytest.mark.parametrize("shape", FOLD_SHAPES)
@pytest.mark.parametrize("fprec", ["f64", "f32", "bf16", "f16"])
def test_precond_folded_matches_dct_oracle(fprec, shape):
    N, M = shape
    dt = npdt(fprec)
    rng = np.random.default_rng(8)
    r = rng.standard_normal((N, M)).astype(dt)
    plan = pkg.Plan(N, M, fprec, form="folded")
    assert plan.folded
    z, rz = plan.precond(internal(plan, r))
    torch.cuda.synchronize()
    z_o = R.apply_precond(r.astype(np.float64))
    zg = z.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(zg[:N, :M] - z_o) / np.linalg.norm(z_o)
    print(f"precond folded {fprec} {shape}: rel err {rel:.3e}")
    assert rel <= PRECOND_RTOL["bf16" if fprec == "f16" else fprec]
    assert_elementwise(zg[:N, :M], r, "folded", fprec)
    assert np.abs(zg[N:, :]).max(initial=0) == 0 and np.abs(zg[:, M:]).max(initial=0) == 0
    ref = float(np.sum(r.astype(np.float64) * z_o))
    assert abs(rz.item() - ref) <= 2 * PRECOND_RTOL["bf16" if fprec == "f16" else fprec] * abs(ref)
    plan.close()


def test_precond_folded_is_pseudo_inverse_property_f64():
    """The folded form solves the same Neumann problem: L z = r - mean(r)."""
    N, M = 384, 200
    rng = np.random.default_rng(6)
    r = rng.standard_normal((N, M))
    plan = pkg.Plan(N, M, "f64", form="folded")
    z, _ = plan.precond(internal(plan, r))
    zg = z.cpu().numpy()[:N, :M]
    Lz = R.apply_A(np.ones((N - 1, M)), np.ones((N, M - 1)), zg)
    assert np.abs(Lz - (r - r.mean())).max() < 1e-10
    assert abs(zg.mean()) < 1e-12
    plan.close()


# powers of two: the fast (cosine-transform) form; one and several rows per
# block, square and both orientations of rectangles
FAST_SHAPES = [(128, 128), (128, 512), (1024, 256), (256, 4096), (2048, 8192), (256, 16384)]
# FP32 / FP64 plans: transform arithmetic and storage in the plan's type, a
# few roundings per transform; mixed plans store the two intermediates in
# BF16 / FP16 (FP32 arithmetic), the bound of the 16-bit products
FAST_RTOL = {"f64": 1e-13, "f32": 2e-6, "bf16": 3e-2, "f16": 3e-2}


@pytest.mark.parametrize("shape", FAST_SHAPES)
@pytest.mark.parametrize("fprec", ["f64", "f32", "bf16", "f16"])
def test_precond_fast_matches_dct_oracle(fprec, shape):
    """The fast form computes in FP32 for FP32 and mixed plans (FP64 for
    FP64); mixed plans keep its two intermediates in their 16-bit type."""
    N, M = shape
    dt = npdt(fprec)
    rng = np.random.default_rng(9)
    r = rng.standard_normal((N, M)).astype(dt)
    plan = pkg.Plan(N, M, fprec, form="fast")
    assert plan.form == "fast"
    z, rz = plan.precond(internal(plan, r))
    torch.cuda.synchronize()
    z_o = R.apply_precond(r.astype(np.float64))
    zg = z.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(zg[:N, :M] - z_o) / np.linalg.norm(z_o)
    print(f"precond fast {fprec} {shape}: rel err {rel:.3e}")
    assert rel <= FAST_RTOL[fprec]
    assert_elementwise(zg[:N, :M], r, "fast", fprec)
    ref = float(np.sum(r.astype(np.float64) * z_o))
    assert abs(rz.item() - ref) <= 2 * FAST_RTOL[fprec] * abs(ref)
    plan.close()


# sides that are not powers of two: the same passes with run-time sizes and
# FFT stages of radix 2^k, 3 and 5 (h = n/2 = 60, 100, 300, 500, 48, 2000,
# 8000); one side a power of two with the other general; one and several
# rows per block and the largest half-length (16000 = 2 x 8000)
GENERAL_SHAPES = [(120, 200), (600, 1000), (4000, 96), (240, 4000), (8192, 1000), (1000, 16000)]


@pytest.mark.parametrize("shape", GENERAL_SHAPES)
@pytest.mark.parametrize("fprec", ["f64", "f32", "bf16", "f16"])
def test_precond_fast_general_sides_match_dct_oracle(fprec, shape):
    """The fast form on sides whose halves factor into 2, 3 and 5 against
    scipy's orthonormal DCT: the same bars and element-wise bound as the
    power-of-two sides."""
    N, M = shape
    dt = npdt(fprec)
    rng = np.random.default_rng(11)
    r = rng.standard_normal((N, M)).astype(dt)
    plan = pkg.Plan(N, M, fprec, form="fast")
    assert plan.form == "fast"
    z, rz = plan.precond(internal(plan, r))
    torch.cuda.synchronize()
    z_o = R.apply_precond(r.astype(np.float64))
    zg = z.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(zg[:N, :M] - z_o) / np.linalg.norm(z_o)
    print(f"precond fast (general sides) {fprec} {shape}: rel err {rel:.3e}")
    assert rel <= FAST_RTOL[fprec]
    assert_elementwise(zg[:N, :M], r, "fast", fprec)
    # the padding of the plan's arrays stays zero
    assert np.all(zg[N:, :] == 0) and np.all(zg[:, M:] == 0)
    ref = float(np.sum(r.astype(np.float64) * z_o))
    assert abs(rz.item() - ref) <= 2 * FAST_RTOL[fprec] * abs(ref)
    plan.close()


# the smallest general sides: one stage (h = 4), one block holding every
# row, radix-3 and radix-5 stages on tiny rows, padding far larger than the
# image
SMALL_GENERAL = [(8, 8), (8, 24), (24, 40), (48, 72), (96, 120), (40, 200)]


@pytest.mark.parametrize("shape", SMALL_GENERAL)
@pytest.mark.parametrize("fprec", ["f64", "f32"])
def test_precond_fast_small_general_sides(fprec, shape):
    N, M = shape
    dt = npdt(fprec)
    rng = np.random.default_rng(13)
    r = rng.standard_normal((N, M)).astype(dt)
    plan = pkg.Plan(N, M, fprec, form="fast")
    assert plan.form == "fast"
    z, _ = plan.precond(internal(plan, r))
    torch.cuda.synchronize()
    z_o = R.apply_precond(r.astype(np.float64))
    zg = z.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(zg[:N, :M] - z_o) / np.linalg.norm(z_o)
    print(f"precond fast (small general sides) {fprec} {shape}: rel err {rel:.3e}")
    assert rel <= FAST_RTOL[fprec]
    assert_elementwise(zg[:N, :M], r, "fast", fprec)
    assert np.all(zg[N:, :] == 0) and np.all(zg[:, M:] == 0)
    plan.close()


def test_precond_fast_general_is_pseudo_inverse_property_f64():
    """L z = r - mean(r) for the general-size fast form (600 x 120)."""
    N, M = 600, 120
    rng = np.random.default_rng(12)
    r = rng.standard_normal((N, M))
    plan = pkg.Plan(N, M, "f64", form="fast")
    z, _ = plan.precond(internal(plan, r))
    zg = z.cpu().numpy()[:N, :M]
    Lz = R.apply_A(np.ones((N - 1, M)), np.ones((N, M - 1)), zg)
    assert np.abs(Lz - (r - r.mean())).max() < 1e-10
    assert abs(zg.mean()) < 1e-12
    plan.close()


def test_precond_fast_is_pseudo_inverse_property_f64():
    """The fast form solves the Neumann problem: L z = r - mean(r)."""
    N, M = 512, 256
    rng = np.random.default_rng(10)
    r = rng.standard_normal((N, M))
    plan = pkg.Plan(N, M, "f64", form="fast")
    z, _ = plan.precond(internal(plan, r))
    zg = z.cpu().numpy()[:N, :M]
    Lz = R.apply_A(np.ones((N - 1, M)), np.ones((N, M - 1)), zg)
    assert np.abs(Lz - (r - r.mean())).max() < 1e-10
    assert abs(zg.mean()) < 1e-12
    plan.close()


def test_precond_is_pseudo_inverse_property_f64():
    """L z = r - mean(r) with L the unweighted Neumann Laplacian (applied by
    the oracle's plain stencil), at a size with several GEMM tiles."""
    N, M = 384, 200
    rng = np.random.default_rng(6)
    r = rng.standard_normal((N, M))
    plan = pkg.Plan(N, M, "f64", form="dense")
    z, _ = plan.precond(internal(plan, r))
    zg = z.cpu().numpy()[:N, :M]
    Lz = R.apply_A(np.ones((N - 1, M)), np.ones((N, M - 1)), zg)
    assert np.abs(Lz - (r - r.mean())).max() < 1e-10
    assert abs(zg.mean()) < 1e-12
    plan.close()
