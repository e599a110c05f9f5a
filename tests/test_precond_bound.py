"""The element-wise error bound of the preconditioner (tests/precond_bound.py)
against pipelines that round where the GPU forms round, computed on the CPU
with numpy / torch dtype casts (FP16, BF16 storage and operands; FP32
transform arithmetic through scipy's single-precision DCT).  The bound must
hold for these faithful pipelines, and must reject a single planted error
that the former 2-norm bars let through.
"""
import math

import numpy as np
import pytest
import scipy.fft
import torch

import precond_bound as PB
from oracle import reduced as R


def _q(A, t):
    if t == "f16":
        return A.astype(np.float16).astype(np.float32)
    if t == "bf16":
        return torch.from_numpy(np.ascontiguousarray(A, np.float32)).to(torch.bfloat16).float().numpy()
    return A.astype(np.float32)


def _lam(N, M):
    L = PB._eig(N)[:, None] + PB._eig(M)[None, :]
    L[0, 0] = np.inf
    return L.astype(np.float32)


def _scale(r, t):
    return 1e-3 * math.sqrt(r.size / float(np.sum(r.astype(np.float64) ** 2))) if t == "f16" else 1.0


def fast_pipeline(r, store):
    """FP32 transforms, intermediates after the row DCT-II and the column
    DCT-III rounded to `store` (FP16 with the 1e-3 rms input scale)."""
    N, M = r.shape
    s = np.float32(_scale(r, store))
    R1 = _q(scipy.fft.dct(r.astype(np.float32) * s, type=2, norm="ortho", axis=1), store)
    Zh = (scipy.fft.dct(R1, type=2, norm="ortho", axis=0) / _lam(N, M)).astype(np.float32)
    Z1 = _q(scipy.fft.idct(Zh, type=2, norm="ortho", axis=0), store)
    return (scipy.fft.idct(Z1, type=2, norm="ortho", axis=1) / s).astype(np.float32)


def dense_pipeline(r, op):
    """Four products with bases and operands rounded to `op`, FP32
    accumulation, every intermediate rounded to `op`."""
    N, M = r.shape
    PN, PM = _q(R.dct_basis(N), op), _q(R.dct_basis(M), op)
    s = np.float32(_scale(r, op))
    T1 = _q(_q(r.astype(np.float32) * s, op) @ PM, op)
    T2 = _q((PN.T @ T1) / _lam(N, M), op)
    T3 = _q(PN @ T2, op)
    return ((T3 @ PM.T) / s).astype(np.float32)


CASES = [("fast", "f16"), ("fast", "bf16"), ("fast", "f32"),
         ("dense", "bf16"), ("dense", "f16"), ("dense", "f32")]


@pytest.mark.parametrize("form,prec", CASES)
def test_bound_holds_for_emulated_rounding(form, prec):
    rng = np.random.default_rng(5)
    r = rng.standard_normal((256, 512)).astype(np.float32)
    S = PB.stages(r)
    zg = fast_pipeline(r, prec) if form == "fast" else dense_pipeline(r, prec)
    sig = PB.plan_sigma(S, form, prec)
    ok, worst, idx = PB.check(zg, S, sig)
    print(f"{form} {prec}: worst |dz| / sigma = {worst:.3f} at {idx}")
    assert ok, worst
    # the bound is not vacuous: it sits well below the size of z
    assert PB.KAPPA * sig.max() <= 0.2 * np.abs(S["z"]).max()


@pytest.mark.parametrize("form,prec", [("fast", "f16"), ("dense", "bf16")])
def test_bound_rejects_one_planted_error(form, prec):
    """One element of an otherwise faithful result moved by 20 sigma: the
    relative 2-norm error stays below the 2-norm bars used before (1e-2 for
    FP16 storage, 3e-2 for BF16 products), the element-wise bound fails."""
    rng = np.random.default_rng(6)
    r = rng.standard_normal((256, 512)).astype(np.float32)
    S = PB.stages(r)
    zg = fast_pipeline(r, prec) if form == "fast" else dense_pipeline(r, prec)
    sig = PB.plan_sigma(S, form, prec)
    zg = zg.astype(np.float64)
    zg[100, 300] += 20.0 * sig[100, 300]
    rel2 = np.linalg.norm(zg - S["z"]) / np.linalg.norm(S["z"])
    assert rel2 <= (1e-2 if prec == "f16" else 3e-2)
    ok, worst, idx = PB.check(zg, S, sig)
    assert not ok and idx == (100, 300)


def test_propagation_of_a_single_spectral_error_is_bounded():
    """A unit error on one spectral coefficient (k, l) before the division
    reaches z as P_N[:, k] P_M[:, l]^T / (lambda_k + mu_l); its largest
    element squared is within the uniform factor (4 / N M) W_kl."""
    N, M = 64, 48
    PN, PM = R.dct_basis(N), R.dct_basis(M)
    lam = PB._eig(N)[:, None] + PB._eig(M)[None, :]
    for (k, l) in ((0, 1), (1, 0), (5, 7), (N - 1, M - 1)):
        dz = np.outer(PN[:, k], PM[:, l]) / lam[k, l]
        assert np.max(dz * dz) <= 4.0 / (N * M) / lam[k, l] ** 2 * (1 + 1e-12)
