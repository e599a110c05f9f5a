"""The paper's scaling shape 4000 x M, M from 2000 to 16000 (the running-time
study of Section 4): sides that are not powers of two run the MFMA forms
with rectangular bases (P_N != P_M), folded when both sides are even.

Bars: the preconditioner against the oracle's FP64 transform (scipy's
orthonormal DCT) at full size, relative 2-norm error -- 16-bit operands
3e-2 (the dense-product bar), FP32 2e-5; the whole path at a tenth of the
size and the same aspect ratio against the oracle, converged solves, L1
within the FP32 / mixed bars of the other unwrap tests.
"""
import os

import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg
from oracle import reduced as R

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,prec", [(2000, "f16"), (16000, "f16"), (6000, "f32")])
def test_preconditioner_4000_by_m(M, prec):
    N = 4000
    plan = pkg.Plan(N, M, prec)
    assert plan.form == "folded"
    g = torch.Generator(device="cuda").manual_seed(8)
    r = torch.zeros((plan.Np, plan.ld), device="cuda", dtype=plan.dtype)
    r[:N, :M] = torch.randn((N, M), device="cuda", generator=g, dtype=plan.dtype)
    z, _ = plan.precond(r)
    torch.cuda.synchronize()
    zn = z[:N, :M].double().cpu().numpy()
    for pad in (z[N:, :], z[:, M:]):
        assert pad.numel() == 0 or float(pad.abs().max()) == 0
    rn = r[:N, :M].double().cpu().numpy()
    plan.close()
    del r, z
    zo = R.apply_precond(rn, workers=min(16, os.cpu_count() or 1))
    rel = np.linalg.norm(zn - zo) / np.linalg.norm(zo)
    print(f"precond {prec} 4000x{M}: rel err {rel:.3e}")
    assert rel <= {"f16": 3e-2, "f32": 2e-5}[prec]


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_unwrap_tenth_scale_400_by_1600(prec):
    """400 x 1600 (the 4000 x 16000 aspect): dense form, c2-type residue
    field, converged solves, L1 against the oracle."""
    f = synth.field_c2(9, 400, 1600)
    dt = np.float32
    X = f.X.astype(dt)
    w = f.w.astype(dt)
    plan = pkg.Plan(400, 1600, prec)
    p = pkg.default_params(prec)
    p.irls_iters, p.pcg_max, p.pcg_rtol = 4, 3000, 1e-6
    _, st = plan.unwrap(torch.from_numpy(X).cuda(), torch.from_numpy(w).cuda(), params=p,
                        stats=True)
    plan.close()
    Uo, hist = R.irls(X.astype(np.float64), w=w.astype(np.float64), iters=4, tol=1e-6,
                      maxit=3000, workers=min(16, os.cpu_count() or 1))
    gap = abs(st["L1_final"] - hist[-1]["L1"]) / hist[-1]["L1"]
    print(f"{prec} 400x1600: GPU L1 {st['L1_final']:.8g} oracle {hist[-1]['L1']:.8g} gap {gap:.2e}")
    assert gap <= {"f32": 1e-5, "f16": 1e-3}[prec]
