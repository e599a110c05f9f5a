"""Config 5 at size: a batch of 16 grids of 1024 x 1024 (the small-case
generator, per-edge weights sigmoid(N(0,1) logits)) through UnwrapFn in
FP32, loss = MSE between the mean-aligned U and the true phase; gradients
with respect to the logits and the wrapped input by torch.autograd through
the hand-written adjoint (one PCG solve per grid on the converged system).

The true phase of the loss is the generator's noise-free phase (its
Gaussians and ramp; the N(0, 0.3^2) noise is what the measurement adds).
The small-case generator meets the Itoh condition at this size (the oracle
reaches L1 ~ 0 after its first solve: U reproduces the noisy phase), so the
loss does not depend on the weights to first order: dL/dC vanishes and
dL/dX carries the gradient.
Checks on grid 0, against the oracle's FP64 adjoint at the GPU's U (the same
frozen-weight map): gX within 2e-3 relative in the 2-norm (the FP32 bar of
the smaller adjoint tests); FP64 central differences of the frozen map on
sampled pixels of X (h = 1e-4, pixels whose differences lie within 1e-2 of
+-pi skipped, so no wrap branch is crossed) within 1e-3 of max |gX|; and
the weight gradient at that vanishing level.  A residue-bearing 512^2
field (where dL/dC does not vanish) checks the weight gradients against
the oracle and against central differences on sampled edges.  Each
perturbed solve of the differences solves the correction from the
unperturbed solution to 1e-12 of its own right-hand side.
"""
import os

import numpy as np
import pytest
import torch

import synth
import paper_2401_09961_amd as pkg
from oracle import reduced as R

pytestmark = pytest.mark.gpu

B, N, M = 16, 1024, 1024
WORKERS = min(16, os.cpu_count() or 1)  # the oracle's FFT threads (the host-CPU share of one GPU)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _params():
    p = pkg.default_params("f32")
    p.irls_iters, p.pcg_max, p.pcg_rtol = 30, 3000, 1e-6
    return p


def test_config5_batch_of_16_through_unwrapfn():
    fields = [synth.field_c5(s, N, M) for s in range(B)]
    X = torch.from_numpy(np.stack([f.X for f in fields]).astype(np.float32)).cuda()
    X.requires_grad_(True)
    zv = torch.from_numpy(np.stack([f.meta["zv"] for f in fields]).astype(np.float32)).cuda()
    zh = torch.from_numpy(np.stack([f.meta["zh"] for f in fields]).astype(np.float32)).cuda()
    zv.requires_grad_(True)
    zh.requires_grad_(True)
    truth = [synth.field_c5_truth(s, N, M) for s in range(B)]
    phi = torch.from_numpy(np.stack([t - t.mean() for t in truth]).astype(np.float32)).cuda()
    plan = pkg.Plan(N, M, "f32")
    p = _params()
    Cv, Ch = torch.sigmoid(zv), torch.sigmoid(zh)
    U = pkg.UnwrapFn.apply(X, Cv, Ch, plan, p)
    Uc = U - U.mean(dim=(1, 2), keepdim=True)
    loss = ((Uc - phi) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    plan.close()
    for g in (X.grad, zv.grad, zh.grad):
        assert g is not None and torch.isfinite(g).all()
    print(f"c5: loss {loss.item():.6e}, |gX| {X.grad.norm().item():.3e}, "
          f"|g_zv| {zv.grad.norm().item():.3e}, |g_zh| {zh.grad.norm().item():.3e}")

    Ug = U[0].detach().double().cpu().numpy()
    X0 = fields[0].X.astype(np.float32).astype(np.float64)
    Cv0 = Cv[0].detach().double().cpu().numpy()
    Ch0 = Ch[0].detach().double().cpu().numpy()
    ph0 = phi[0].double().cpu().numpy()
    gU = 2.0 * (Ug - Ug.mean() - ph0) / (B * N * M)
    Gv, Gh = R.wrapped_gradients(X0)
    ref = R.adjoint(Ug, Gv, Gh, Cv0, Ch0, p.eps, gU, tol=1e-12, maxit=20000, workers=WORKERS)
    gXg = X.grad[0].double().cpu().numpy()
    e = rel(gXg, ref["gX"])
    scale = float(np.abs(gXg).max())
    gCv = zv.grad[0].double().cpu().numpy() / (Cv0 * (1.0 - Cv0))
    print(f"c5 grid 0: gX rel err vs oracle {e:.2e}; max|gX| {scale:.3e}, "
          f"max|gCv| {np.abs(gCv).max():.3e} (oracle {np.abs(ref['gCv']).max():.3e})")
    assert e <= 2e-3
    # the weights' gradient is at the vanishing level of the Itoh case
    assert np.abs(gCv).max() <= 1e-3 * scale

    # central differences of the frozen map in X on sampled pixels
    wv, wh = ref["wv"], ref["wh"]
    base = R.frozen_solve(Cv0, Ch0, Gv, Gh, wv, wh, tol=1e-12, maxit=20000, workers=WORKERS)
    loss_of = lambda Uc: float(np.mean((Uc - Uc.mean() - ph0) ** 2)) / B  # noqa: E731
    rng = np.random.default_rng(9)
    h, done = 1e-4, 0
    while done < 3:
        i, j = int(rng.integers(1, N - 1)), int(rng.integers(1, M - 1))
        d = [X0[i + 1, j] - X0[i, j], X0[i, j] - X0[i - 1, j], X0[i, j + 1] - X0[i, j],
             X0[i, j] - X0[i, j - 1]]
        if min(abs(abs(R.wrap(np.array(d))) - np.pi)) < 1e-2:
            continue
        vals = []
        for sgn in (1.0, -1.0):
            Xp = X0.copy()
            Xp[i, j] += sgn * h
            Gvp, Ghp = R.wrapped_gradients(Xp)
            vals.append(loss_of(R.frozen_solve(Cv0, Ch0, Gvp, Ghp, wv, wh, tol=1e-12,
                                               maxit=20000, x0=base, workers=WORKERS)))
        fd = (vals[0] - vals[1]) / (2 * h)
        print(f"pixel ({i},{j}): FD {fd:.6e} GPU {gXg[i, j]:.6e} oracle {ref['gX'][i, j]:.6e}")
        assert abs(fd - gXg[i, j]) <= 1e-3 * scale
        done += 1


def test_config5_weights_residue_field_weight_gradients():
    """A 512^2 field with residues and the config-5 weights: the weight
    gradients against the oracle's adjoint and central differences."""
    N = M = 512
    rng = np.random.default_rng(11)
    phi = synth.gaussian_sum_field(rng, N, M, amp=3.0, noise=1.2)
    X0 = synth.observe(phi).astype(np.float32)
    w5 = synth.field_c5(21, N, M)
    Cv0, Ch0 = w5.Cv.astype(np.float32), w5.Ch.astype(np.float32)
    plan = pkg.Plan(N, M, "f32")
    p = _params()
    U = plan.unwrap(torch.from_numpy(X0).cuda(), Cv=torch.from_numpy(Cv0).cuda(),
                    Ch=torch.from_numpy(Ch0).cuda(), params=p)
    a = np.random.default_rng(12).standard_normal((N, M)).astype(np.float32)
    gCv, gCh, gX = plan.adjoint(torch.from_numpy(a).cuda(), params=p)
    torch.cuda.synchronize()
    plan.close()
    Ug = U.double().cpu().numpy()
    X64, Cv64, Ch64 = (v.astype(np.float64) for v in (X0, Cv0, Ch0))
    Gv, Gh = R.wrapped_gradients(X64)
    ref = R.adjoint(Ug, Gv, Gh, Cv64, Ch64, p.eps, a.astype(np.float64), tol=1e-12, maxit=20000,
                    workers=WORKERS)
    gv, gh, gx = (t.double().cpu().numpy() for t in (gCv, gCh, gX))
    e = [rel(gv, ref["gCv"]), rel(gh, ref["gCh"]), rel(gx, ref["gX"])]
    print(f"residue 512^2: rel err gCv {e[0]:.2e} gCh {e[1]:.2e} gX {e[2]:.2e}")
    assert max(e) <= 2e-3
    wv, wh = ref["wv"], ref["wh"]
    base = R.frozen_solve(Cv64, Ch64, Gv, Gh, wv, wh, tol=1e-12, maxit=20000, workers=WORKERS)
    a64 = a.astype(np.float64)
    loss_of = lambda Uc: float(np.sum(a64 * Uc))  # noqa: E731
    scale = float(np.abs(gv).max())
    h = 1e-3
    rs = np.random.default_rng(13)
    for _ in range(3):
        i, j = int(rs.integers(0, N - 1)), int(rs.integers(0, M))
        vals = []
        for sgn in (1.0, -1.0):
            Cp = Cv64.copy()
            Cp[i, j] += sgn * h
            vals.append(loss_of(R.frozen_solve(Cp, Ch64, Gv, Gh, wv, wh, tol=1e-12, maxit=20000,
                                               x0=base, workers=WORKERS)))
        fd = (vals[0] - vals[1]) / (2 * h)
        print(f"edge ({i},{j}): FD {fd:.6e} GPU {gv[i, j]:.6e} oracle {ref['gCv'][i, j]:.6e}")
        assert abs(fd - gv[i, j]) <= 1e-3 * scale
