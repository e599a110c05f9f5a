"""FP64 oracle of the paper's augmented form in (U, V^v, V^h).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Follows the paper (arXiv 2401.09961) step by step:

* Objective F_delta of (eq:F_delta): sum sqrt(C^2 V^2 + delta^2) plus the
  quadratic penalty ||S U - G^v - V^v||^2 / (2 tau) + ||U T - G^h - V^h||^2 / (2 tau).
* Algorithm 1: U^0 = 0, V^0 = S U^0 - G^v (and likewise for h); each
  iteration takes the closed-form weights (eq:weight-matrices-closed-form)
  W = sqrt(C^2 V^2 + delta^2), solves the linear system of Proposition 1
  with CG, then removes the mean of U.
* The linear map is the symmetric matrix of (eq:matrix-soft-constraints)
  (1/tau on the whole first block row); Algorithm 1 prints the first row
  without 1/tau, which is the same equation but not a symmetric operator.
* Block-diagonal preconditioner (eq:preconditioner-definition): tau L^+ on
  the U block (L the Neumann Laplacian, pseudo-inverse of Appendix B) and
  the diagonal (D + I / tau)^-1 on the slack blocks.

Cross-checks (tests): the Schur reduction of the slack rows gives the
weighted 5-point system with per-edge K = tau C^2 / (W + tau C^2); with
C = 1 and tau = eps the minimum of F over V equals the reduced Huber
objective, so both oracles reach the same optimum value.
"""
from __future__ import annotations

import math

import numpy as np

from . import reduced as R


def f_delta(U, Vv, Vh, Gv, Gh, Cv, Ch, tau, delta):
    """F_delta(U, V^v, V^h) of (eq:F_delta); delta = 0 gives F."""
    ev = R.diff_v(U) - Gv - Vv
    eh = R.diff_h(U) - Gh - Vh
    return float(np.sum(np.sqrt(Cv * Cv * Vv * Vv + delta * delta))
                 + np.sum(np.sqrt(Ch * Ch * Vh * Vh + delta * delta))
                 + (np.sum(ev * ev) + np.sum(eh * eh)) / (2.0 * tau))


def h_delta(U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch, tau, delta):
    """The function minimised in (prob:alt1), evaluated at given weights W:
    1/2 sum ((C^2 V^2 + delta^2) / W + W) plus the quadratic penalty."""
    ev = R.diff_v(U) - Gv - Vv
    eh = R.diff_h(U) - Gh - Vh
    return float(0.5 * np.sum((Cv * Cv * Vv * Vv + delta * delta) / Wv + Wv)
                 + 0.5 * np.sum((Ch * Ch * Vh * Vh + delta * delta) / Wh + Wh)
                 + (np.sum(ev * ev) + np.sum(eh * eh)) / (2.0 * tau))


def closed_form_weights(Vv, Vh, Cv, Ch, delta):
    """W = sqrt(C^2 V^2 + delta^2) (eq:weight-matrices-closed-form)."""
    return (np.sqrt(Cv * Cv * Vv * Vv + delta * delta),
            np.sqrt(Ch * Ch * Vh * Vh + delta * delta))


class Augmented:
    """Matrix-free linear map, right-hand side and preconditioner of
    Proposition 1 / (eq:matrix-soft-constraints) for fixed weights W."""

    def __init__(self, Gv, Gh, Cv, Ch, Wv, Wh, tau):
        self.Gv, self.Gh, self.tau = Gv, Gh, tau
        self.Dv = Cv * Cv / Wv
        self.Dh = Ch * Ch / Wh
        self.N, self.M = Gv.shape[0] + 1, Gh.shape[1] + 1

    def split(self, x):
        N, M = self.N, self.M
        a = N * M
        b = a + (N - 1) * M
        return (x[:a].reshape(N, M), x[a:b].reshape(N - 1, M),
                x[b:].reshape(N, M - 1))

    @staticmethod
    def join(u, vv, vh):
        return np.concatenate([u.ravel(), vv.ravel(), vh.ravel()])

    def A(self, x):
        u, vv, vh = self.split(x)
        t = self.tau
        top = R.div(R.diff_v(u) - vv, R.diff_h(u) - vh) / t
        mid = -R.diff_v(u) / t + (self.Dv + 1.0 / t) * vv
        bot = -R.diff_h(u) / t + (self.Dh + 1.0 / t) * vh
        return self.join(top, mid, bot)

    def rhs(self):
        t = self.tau
        return self.join(R.div(self.Gv, self.Gh) / t, -self.Gv / t, -self.Gh / t)

    def precond(self, r):
        ra, rb, rc = self.split(r)
        t = self.tau
        return self.join(t * R.apply_precond(ra), rb / (self.Dv + 1.0 / t),
                         rc / (self.Dh + 1.0 / t))


def candidate_step(U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch, tau, delta):
    """The gradient step of Theorem 3 (eq:candidate-gd-step) from (U, V) at
    the weights W: each block moves by -1/L times the partial gradient of the
    (prob:alt1) objective at fixed W, with L of Theorem 3.

    grad_U = (S^T (S U - G^v - V^v) + (U T - G^h - V^h) T^T) / tau
    grad_V = C^2 V / W + (V - (D U - G)) / tau   (each slack block)
    """
    L = lipschitz_L(Cv, Ch, tau, delta)
    ev = R.diff_v(U) - Gv - Vv
    eh = R.diff_h(U) - Gh - Vh
    gU = R.div(ev, eh) / tau
    gVv = Cv * Cv * Vv / Wv - ev / tau
    gVh = Ch * Ch * Vh / Wh - eh / tau
    return U - gU / L, Vv - gVv / L, Vh - gVh / L


def irls(X=None, *, G=None, w=None, Cv=None, Ch=None, tau=1e-2, delta=1e-6,
         iters=20, tol=1e-8, maxit=100, max_cg=None, guard=0):
    """Algorithm 1 verbatim; returns (U, Vv, Vh, history).

    ``max_cg`` (callable k -> int) overrides ``maxit`` per IRLS iteration,
    which is how the Section 4.3 schedule drives it.

    ``guard`` -- the sufficient-decrease condition of Theorem 3
    (eq:sufficient-decrease): 0 does not check it; 1 checks it after each CG
    solve (the paper reports it always held) and takes the candidate step
    when it fails; 2 takes only the candidate steps, no CG (the variant of
    the remark after Theorem 3).  history[k]['guard'] is 0 (not checked),
    1 (held) or 2 (candidate taken).
    """
    if G is None:
        Gv, Gh = R.wrapped_gradients(X)
    else:
        Gv, Gh = (np.asarray(g, np.float64) for g in G)
    N, M = Gv.shape[0] + 1, Gh.shape[1] + 1
    Cv, Ch = R.edge_weights(N, M, w, Cv, Ch)
    U = np.zeros((N, M))
    Vv, Vh = R.diff_v(U) - Gv, R.diff_h(U) - Gh
    hist = []
    for k in range(iters):
        Wv, Wh = closed_form_weights(Vv, Vh, Cv, Ch, delta)
        sysk = Augmented(Gv, Gh, Cv, Ch, Wv, Wh, tau)
        cand = None
        if guard:
            cand = candidate_step(U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch, tau, delta)
        if guard == 2:
            U, Vv, Vh = cand
            info, g = dict(iters=0), 2
        else:
            x0 = sysk.join(U, Vv, Vh)
            m = maxit if max_cg is None else max_cg(k)
            x, info = R.pcg(sysk.A, sysk.precond, sysk.rhs(), x0, tol, m)
            U, Vv, Vh = sysk.split(x)
            g = 0
            if guard == 1:
                h_new = h_delta(U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch, tau, delta)
                h_cand = h_delta(*cand, Wv, Wh, Gv, Gh, Cv, Ch, tau, delta)
                g = 1 if h_new <= h_cand else 2
                if g == 2:
                    U, Vv, Vh = cand
        U = U - U.mean()
        hist.append(dict(k=k, F_delta=f_delta(U, Vv, Vh, Gv, Gh, Cv, Ch, tau, delta),
                         L1=R.l1_objective(U, Gv, Gh, Cv, Ch), guard=g, **info))
    return U, Vv, Vh, hist


def schur_solve(Gv, Gh, Cv, Ch, Wv, Wh, tau, tol=1e-13, maxit=5000):
    """Eliminate the slack rows of Proposition 1: V = (DU - G) / (1 + tau C^2 / W)
    leaves D^T K D U = D^T K G with K = tau C^2 / (W + tau C^2).
    Returns (U, Vv, Vh) with U mean-zero."""
    Kv = tau * Cv * Cv / (Wv + tau * Cv * Cv)
    Kh = tau * Ch * Ch / (Wh + tau * Ch * Ch)
    b = R.div(Kv * Gv, Kh * Gh)
    U, _ = R.pcg(lambda p: R.apply_A(Kv, Kh, p), R.apply_precond, b,
                 np.zeros_like(b), tol, maxit)
    U = U - U.mean()
    Vv = (R.diff_v(U) - Gv) / (1.0 + tau * Cv * Cv / Wv)
    Vh = (R.diff_h(U) - Gh) / (1.0 + tau * Ch * Ch / Wh)
    return U, Vv, Vh


def smoothing_gap_bound(N, M, delta):
    """Theorem 2: F <= F_delta <= F + delta ((N-1) M + N (M-1))."""
    return delta * ((N - 1) * M + N * (M - 1))


def lipschitz_L(Cv, Ch, tau, delta):
    """L = 12 / tau + C_max^2 / delta of Theorem 3."""
    cmax = max(float(np.max(Cv)), float(np.max(Ch)))
    return 12.0 / tau + cmax * cmax / delta


__all__ = ["f_delta", "closed_form_weights", "Augmented", "irls", "candidate_step",
           "schur_solve", "smoothing_gap_bound", "lipschitz_L", "h_delta"]
