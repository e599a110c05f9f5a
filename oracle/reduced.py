"""FP64 oracle of the reduced (slack-eliminated) IRLS + PCG method.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

What is computed (paper arXiv 2401.09961):

* Wrapped gradients G^v, G^h of the observed phase X (Section 2, the
  definitions before problem (prob:main)); the residue function W maps a
  difference to [-pi, pi).
* Edge weights C^v, C^h (Section 2 and the ``unwrap`` interface of Section
  4.4): given per edge, else the smaller of the two endpoint pixel weights,
  else 1.
* The weighted L1 objective of problem (prob:main-matrix-form) and its
  Huber smoothing H_eps = sum C h_eps(DU - G).  Eliminating the slacks of
  problem (prob:soft-constraints) gives exactly this Huber form (Moreau
  envelope of |.|), so H_eps is the objective IRLS decreases.
* IRLS (structure of Algorithm 1): U^0 = 0; per iteration the weights
  Omega = C / max(|DU - G|, eps), a preconditioned CG solve of
  D^T Omega D U = D^T Omega G warm-started at the current U, then the mean
  is removed (last step of Algorithm 1).
* PCG as in Algorithm 2, matrix-free; stop when ||r|| <= tol ||b||.
* Preconditioner: the U block of (eq:preconditioner-definition), the
  unweighted Neumann Laplacian I (x) S^T S + T T^T (x) I, solved through its
  eigendecomposition (eq:eigendecompositions) -- the eigenvectors are the
  orthonormal DCT-II basis and the eigenvalues 2 - 2 cos(pi k / n) -- with
  mode (0, 0) set to zero (the pseudo-inverse choice of Appendix B).  The
  tau factor is dropped: CG iterates do not change when the preconditioner
  is scaled by a positive constant.
* The Section 4.3 surrogate and the rounded (2 pi-congruent) output.
* Adjoints: of the frozen-weight least-squares map (``adjoint``), and the
  full implicit derivative of the Huber minimiser (``huber_minimiser``, an
  exact active-set solve of the stationarity condition, and
  ``adjoint_implicit``).

Pins (tests/test_oracle_pins.py): closed-form eigenpairs, dense matrix
definitions of S, T and D^T Omega D, pseudo-inverse identities, one-step
convergence for unit weights, dense least squares, the Itoh integration
case, monotone decrease of H_eps, linear-programming brute force on small
grids, the 2 x 2 single-loop closed form, the paper-form cross-oracle,
finite differences of both adjoints (of the frozen map; of the exact
minimiser in C and X), the Itoh closed form of the implicit adjoint.
Parity unpinned: pointwise U when the L1 / Huber minimiser is not unique.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------
# Problem data (Section 2)
# ----------------------------------------------------------------------------
def wrap(x):
    """Residue of x modulo 2 pi in [-pi, pi): x - 2 pi floor((x + pi) / 2 pi)."""
    x = np.asarray(x, dtype=np.float64)
    return x - TWO_PI * np.floor((x + math.pi) / TWO_PI)


def wrapped_gradients(X):
    """G^v_{ij} = W(X_{i+1,j} - X_{ij}), G^h_{ij} = W(X_{i,j+1} - X_{ij})."""
    X = np.asarray(X, dtype=np.float64)
    return wrap(X[1:, :] - X[:-1, :]), wrap(X[:, 1:] - X[:, :-1])


def edge_weights(N, M, w=None, Cv=None, Ch=None):
    """Per-edge weights: explicit (Cv, Ch) win; else min of the endpoint
    pixel weights; else unit weights."""
    if Cv is not None or Ch is not None:
        if Cv is None or Ch is None:
            raise ValueError("Cv and Ch must be given together")
        return np.asarray(Cv, np.float64), np.asarray(Ch, np.float64)
    if w is not None:
        w = np.asarray(w, dtype=np.float64)
        return np.minimum(w[1:, :], w[:-1, :]), np.minimum(w[:, 1:], w[:, :-1])
    return np.ones((N - 1, M)), np.ones((N, M - 1))


# ----------------------------------------------------------------------------
# Difference operators (matrices S and T of Section 2, Appendix A)
# ----------------------------------------------------------------------------
def diff_v(U):
    """S U: vertical forward differences, (N-1) x M."""
    return U[1:, :] - U[:-1, :]


def diff_h(U):
    """U T: horizontal forward differences, N x (M-1)."""
    return U[:, 1:] - U[:, :-1]


def div(Fv, Fh):
    """D^T F = S^T F^v + F^h T^T (adjoint of the two difference maps)."""
    N = Fv.shape[0] + 1
    M = Fh.shape[1] + 1
    q = np.zeros((N, M), dtype=np.float64)
    q[:-1, :] -= Fv
    q[1:, :] += Fv
    q[:, :-1] -= Fh
    q[:, 1:] += Fh
    return q


def apply_A(Ov, Oh, P):
    """Weighted 5-point operator D^T Omega D applied to an N x M image."""
    return div(Ov * diff_v(P), Oh * diff_h(P))


def sparse_D(N, M):
    """Explicit sparse D = [I_M kron S ; T^T kron I_N] acting on the
    column-major vec of the paper's notation section."""
    import scipy.sparse as sp
    S = sp.diags([-np.ones(N - 1), np.ones(N - 1)], [0, 1], shape=(N - 1, N))
    T = sp.diags([-np.ones(M - 1), np.ones(M - 1)], [0, -1], shape=(M, M - 1))
    return sp.vstack([sp.kron(sp.identity(M), S), sp.kron(T.T, sp.identity(N))]).tocsr()


def vec(A):
    """Column-major vectorisation (the paper's vec)."""
    return np.asarray(A).flatten(order="F")


# ----------------------------------------------------------------------------
# Objectives (problem (prob:main-matrix-form) and its Huber smoothing)
# ----------------------------------------------------------------------------
def residuals(U, Gv, Gh):
    return diff_v(U) - Gv, diff_h(U) - Gh


def l1_objective(U, Gv, Gh, Cv, Ch):
    rv, rh = residuals(U, Gv, Gh)
    return float(np.sum(Cv * np.abs(rv)) + np.sum(Ch * np.abs(rh)))


def huber(r, eps):
    a = np.abs(r)
    return np.where(a <= eps, 0.5 * r * r / eps, a - 0.5 * eps)


def huber_objective(U, Gv, Gh, Cv, Ch, eps):
    rv, rh = residuals(U, Gv, Gh)
    return float(np.sum(Cv * huber(rv, eps)) + np.sum(Ch * huber(rh, eps)))


# ----------------------------------------------------------------------------
# IRLS weight step: closed-form weights, right-hand side, objectives
# ----------------------------------------------------------------------------
def weight_step(U, Gv, Gh, Cv, Ch, eps):
    """Omega = C / max(|DU - G|, eps); b = D^T Omega G; L1 and H_eps at U."""
    rv, rh = residuals(U, Gv, Gh)
    Ov = Cv / np.maximum(np.abs(rv), eps)
    Oh = Ch / np.maximum(np.abs(rh), eps)
    b = div(Ov * Gv, Oh * Gh)
    L1 = float(np.sum(Cv * np.abs(rv)) + np.sum(Ch * np.abs(rh)))
    H = float(np.sum(Cv * huber(rv, eps)) + np.sum(Ch * huber(rh, eps)))
    return Ov, Oh, b, L1, H


def surrogate(U, Gv, Gh, Cv, Ch, Ov, Oh):
    """The quadratic IRLS model at fixed edge weights Omega = C omega, the
    reduced analogue of the function H(U, W) minimised by the alternating
    scheme (Section 3.1): sum Omega r^2 / 2 + C^2 / (2 Omega), r = DU - G.
    Minimised over omega <= 1/eps at omega = 1/max(|r|, eps), where it equals
    sum C (h_eps(r) + eps/2)."""
    rv, rh = residuals(U, Gv, Gh)
    return float(np.sum(Ov * rv * rv / 2.0 + Cv * Cv / (2.0 * Ov))
                 + np.sum(Oh * rh * rh / 2.0 + Ch * Ch / (2.0 * Oh)))


# ----------------------------------------------------------------------------
# Preconditioner: eigendecomposition of the Neumann Laplacian (Section 3.3)
# ----------------------------------------------------------------------------
def laplacian_eigenvalues(n):
    """Eigenvalues of S^T S (n x n): 2 - 2 cos(pi k / n), k = 0..n-1
    (Appendix A), evaluated as 4 sin^2(pi k / 2n) -- the same numbers by the
    half-angle identity, without the cancellation of 2 - 2 cos near k = 0
    (which would cost a relative error of about u / lambda_1 in the lowest
    modes of the preconditioner)."""
    k = np.arange(n, dtype=np.float64)
    return 4.0 * np.sin(math.pi * k / (2.0 * n)) ** 2


def dct_basis(n):
    """Orthonormal eigenvectors of S^T S: P[i, k] = c_k cos(pi k (2i+1) / 2n)."""
    i = np.arange(n, dtype=np.float64)[:, None]
    k = np.arange(n, dtype=np.float64)[None, :]
    P = np.cos(math.pi * k * (2.0 * i + 1.0) / (2.0 * n)) * math.sqrt(2.0 / n)
    P[:, 0] = math.sqrt(1.0 / n)
    return P


def _spectral_divide(Rh):
    N, M = Rh.shape
    lam = laplacian_eigenvalues(N)[:, None] + laplacian_eigenvalues(M)[None, :]
    lam[0, 0] = np.inf  # pseudo-inverse: the constant mode maps to zero
    return Rh / lam


def apply_precond(R, workers=None):
    """z = L^+ r for the unweighted Neumann Laplacian L, via the orthonormal
    DCT-II (forward) and DCT-III (inverse) on both axes."""
    Rh = scipy.fft.dctn(np.asarray(R, np.float64), type=2, norm="ortho",
                        workers=workers)
    return scipy.fft.idctn(_spectral_divide(Rh), type=2, norm="ortho",
                           workers=workers)


def apply_precond_explicit(R):
    """Same map with the dense eigenbasis products P_N^T R P_M and
    P_N Z' P_M^T written out (small grids only)."""
    N, M = R.shape
    PN, PM = dct_basis(N), dct_basis(M)
    return PN @ _spectral_divide(PN.T @ R @ PM) @ PM.T


# ----------------------------------------------------------------------------
# Preconditioned conjugate gradient (Algorithm 2)
# ----------------------------------------------------------------------------
class Breakdown(RuntimeError):
    pass


def pcg(A, Minv, b, x0, tol, maxit):
    """Algorithm 2 with a matrix-free A and preconditioner solve Minv.

    Stops when ||r|| <= tol ||b|| (checked on the recursively updated
    residual, before the preconditioner) or after maxit iterations.
    Returns x and a dict with iterations, recursive and true relative
    residuals.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A(x)
    bnorm = math.sqrt(float(np.vdot(b, b)))
    it = 0
    if math.sqrt(float(np.vdot(r, r))) > tol * bnorm:
        z = Minv(r)
        p = z.copy()
        rho = float(np.vdot(r, z))
        while it < maxit:
            q = A(p)
            pq = float(np.vdot(p, q))
            if not pq > 0.0:
                raise Breakdown("p^T A p <= 0")
            alpha = rho / pq
            x += alpha * p
            r -= alpha * q
            it += 1
            if math.sqrt(float(np.vdot(r, r))) <= tol * bnorm:
                break
            z = Minv(r)
            rho_new = float(np.vdot(r, z))
            beta = rho_new / rho
            rho = rho_new
            p = z + beta * p
    rt = b - A(x)
    denom = bnorm if bnorm > 0 else 1.0
    return x, dict(iters=it,
                   relres=math.sqrt(float(np.vdot(r, r))) / denom,
                   true_relres=math.sqrt(float(np.vdot(rt, rt))) / denom)


# ----------------------------------------------------------------------------
# IRLS outer loop (Algorithm 1 structure, reduced form)
# ----------------------------------------------------------------------------
def irls(X=None, *, G=None, w=None, Cv=None, Ch=None, eps=1e-3, iters=20,
         tol=1e-8, maxit=100, U0=None, precond="dct", workers=None,
         callback=None, schedule=None):
    """Unwrap X (or given gradients G = (Gv, Gh)); return (U, history).

    history[k] holds L1 and H_eps at U^k (before solve k) and the solve
    statistics; history[iters] holds L1 and H_eps of the returned U.

    ``schedule`` (an ``oracle.schedule.CgSchedule``) replaces the fixed
    ``maxit`` by the Section 4.3 rules: before solve k >= 1 the relative
    improvement Delta of the surrogate at U^k between the previous and the
    new weights picks the solve's iteration cap, or stops the loop (the
    returned history then ends with that U's entry, marked stopped=True).
    """
    if G is None:
        Gv, Gh = wrapped_gradients(X)
    else:
        Gv, Gh = (np.asarray(g, np.float64) for g in G)
    N, M = Gv.shape[0] + 1, Gh.shape[1] + 1
    Cv, Ch = edge_weights(N, M, w, Cv, Ch)
    if precond == "dct":
        Minv = lambda r: apply_precond(r, workers=workers)  # noqa: E731
    elif precond == "explicit":
        Minv = apply_precond_explicit
    elif precond == "none":
        Minv = lambda r: r.copy()  # noqa: E731
    else:
        raise ValueError(precond)
    U = np.zeros((N, M)) if U0 is None else np.array(U0, np.float64, copy=True)
    hist = []
    prev = None
    for k in range(iters):
        Ov, Oh, b, L1, H = weight_step(U, Gv, Gh, Cv, Ch, eps)
        m, extra = maxit, {}
        if schedule is not None:
            m = schedule.current()
            if prev is not None:
                s_old = surrogate(U, Gv, Gh, Cv, Ch, *prev)
                s_new = surrogate(U, Gv, Gh, Cv, Ch, Ov, Oh)
                delta = (s_old - s_new) / s_old
                m = schedule.update(delta)
                extra = dict(delta=delta)
                if m is None:
                    hist.append(dict(k=k, L1=L1, H=H, stopped=True, **extra))
                    return U, hist
            extra["cap"] = m
        U, info = pcg(lambda p: apply_A(Ov, Oh, p), Minv, b, U, tol, m)
        U = U - U.mean()
        prev = (Ov, Oh)
        rec = dict(k=k, L1=L1, H=H, **info, **extra)
        hist.append(rec)
        if callback is not None:
            callback(rec, U)
    hist.append(dict(k=iters, L1=l1_objective(U, Gv, Gh, Cv, Ch),
                     H=huber_objective(U, Gv, Gh, Cv, Ch, eps)))
    return U, hist


# ----------------------------------------------------------------------------
# Full implicit derivative of the Huber minimiser (the map whose minimiser the
# IRLS fixed point is): with r = DU* - G, the quadratic zone Q = {|r| < eps}
# and Hessian weights kappa = C / eps on Q (0 off Q), the stationarity
# condition D^T (C h_eps'(r)) = 0 differentiates to
#   dL/dG = kappa (D lambda),  dL/dC = -h_eps'(r) (D lambda),
#   dL/dX = D^T dL/dG,         D^T diag(kappa) D lambda = gU (projected).
# ----------------------------------------------------------------------------
def incidence(N, M):
    """Sparse D (rows: the vertical edges then the horizontal ones, each in
    row-major order of their (N-1) x M and N x (M-1) arrays) acting on the
    row-major ravel of U: (D u)_e = u[end] - u[start]."""
    import scipy.sparse as sp
    idx = np.arange(N * M).reshape(N, M)
    a = np.concatenate([idx[:-1, :].ravel(), idx[:, :-1].ravel()])
    b = np.concatenate([idx[1:, :].ravel(), idx[:, 1:].ravel()])
    ne = a.size
    rows = np.concatenate([np.arange(ne), np.arange(ne)])
    cols = np.concatenate([b, a])
    vals = np.concatenate([np.ones(ne), -np.ones(ne)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(ne, N * M))


def _components(N, M, q):
    """Connected components of the pixel graph whose edges are those with q."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    idx = np.arange(N * M).reshape(N, M)
    a = np.concatenate([idx[:-1, :].ravel(), idx[:, :-1].ravel()])[q]
    b = np.concatenate([idx[1:, :].ravel(), idx[:, 1:].ravel()])[q]
    G = sp.csr_matrix((np.ones(a.size), (a, b)), shape=(N * M, N * M))
    return connected_components(G, directed=False)


def _solve_mean_zero(H, rhs, keep):
    """Solve H x = rhs on the pixels `keep` with sum(x[keep]) = 0 and
    x = 0 elsewhere (sparse direct, bordered by the constraint)."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import spsolve
    k = np.flatnonzero(keep)
    Hk = H[k][:, k]
    one = sp.csr_matrix(np.ones((k.size, 1)))
    A = sp.bmat([[Hk, one], [one.T, None]]).tocsc()
    sol = spsolve(A, np.concatenate([rhs[k], [0.0]]))
    x = np.zeros(H.shape[0])
    x[k] = sol[:-1]
    return x


def huber_minimiser(Gv, Gh, Cv, Ch, eps, U0, max_rounds=100):
    """The exact mean-zero minimiser of sum C h_eps(DU - G), from a start U0
    near it: with the quadratic zone Q of the current iterate fixed, the
    stationarity condition is linear,
        D^T diag(kappa) D U = D^T (kappa G - C s),
        kappa = C / eps on Q (0 off it),  s = sign(r) off Q (0 on it),
    and is solved directly; repeated until Q and the signs settle.  Raises
    when they do not, or when the Q-graph does not connect every pixel (the
    minimiser is then not unique).  Returns (U, qv, qh)."""
    N, M = U0.shape
    D = incidence(N, M)
    g = np.concatenate([Gv.ravel(), Gh.ravel()])
    c = np.concatenate([Cv.ravel(), Ch.ravel()])
    u = (U0 - U0.mean()).ravel()
    r = D @ u - g
    q, s = np.abs(r) < eps, np.sign(r)
    for _ in range(max_rounds):
        if _components(N, M, q)[0] != 1:
            raise ValueError("quadratic-zone graph does not connect every pixel")
        kap = np.where(q, c / eps, 0.0)
        sl = np.where(q, 0.0, s)
        H = (D.T @ (D.multiply(kap[:, None]))).tocsr()
        u = _solve_mean_zero(H, D.T @ (kap * g - c * sl), np.ones(N * M, bool))
        r = D @ u - g
        q2, s2 = np.abs(r) < eps, np.sign(r)
        if np.array_equal(q2, q) and np.array_equal(np.where(q, 0.0, s2), sl):
            ne = (N - 1) * M
            return u.reshape(N, M), q[:ne].reshape(N - 1, M), q[ne:].reshape(N, M - 1)
        q, s = q2, s2
    raise ValueError("quadratic zone did not settle")


def huber_stationarity(U, Gv, Gh, Cv, Ch, eps):
    """max |D^T (C h_eps'(DU - G))|: zero at the Huber minimiser."""
    rv, rh = residuals(U, Gv, Gh)
    dv = np.where(np.abs(rv) <= eps, rv / eps, np.sign(rv))
    dh = np.where(np.abs(rh) <= eps, rh / eps, np.sign(rh))
    return float(np.abs(div(Cv * dv, Ch * dh)).max())


def adjoint_implicit(U, Gv, Gh, Cv, Ch, eps, gU):
    """Gradients of a loss with dL/dU = gU through the Huber minimiser U* =
    U (full implicit derivative, no frozen weights).

    Pixels with no quadratic-zone edge ("isolated": the minimiser is not
    unique there) are left out: gU is taken as zero on them and lambda = 0
    there; the remaining pixels must form one Q-component (else ValueError).
    lambda solves D^T diag(kappa) D lambda = gU - mean(gU) over them."""
    N, M = U.shape
    rv, rh = residuals(U, Gv, Gh)
    qv, qh = np.abs(rv) < eps, np.abs(rh) < eps
    kv, kh = np.where(qv, Cv / eps, 0.0), np.where(qh, Ch / eps, 0.0)
    deg = np.zeros((N, M), int)
    deg[:-1, :] += qv
    deg[1:, :] += qv
    deg[:, :-1] += qh
    deg[:, 1:] += qh
    iso = deg == 0
    ncomp, lab = _components(N, M, np.concatenate([qv.ravel(), qh.ravel()]))
    if ncomp - int(iso.sum()) != 1:
        raise ValueError("quadratic zone splits the image")
    g = np.where(iso, 0.0, np.asarray(gU, np.float64))
    g[~iso] -= g[~iso].mean()
    D = incidence(N, M)
    kap = np.concatenate([kv.ravel(), kh.ravel()])
    H = (D.T @ (D.multiply(kap[:, None]))).tocsr()
    lam = _solve_mean_zero(H, g.ravel(), ~iso.ravel()).reshape(N, M)
    dv, dh = diff_v(lam), diff_h(lam)
    hv = np.where(qv, rv / eps, np.sign(rv))
    hh = np.where(qh, rh / eps, np.sign(rh))
    gGv, gGh = kv * dv, kh * dh
    return dict(lam=lam, gCv=-hv * dv, gCh=-hh * dh, gGv=gGv, gGh=gGh,
                gX=div(gGv, gGh), isolated=iso, kv=kv, kh=kh)


# ----------------------------------------------------------------------------
# Rounded output (Section 4, "rounded IRLS"): the unwrapped U made
# 2 pi-congruent to the input.  U is defined up to a constant; the constant c
# aligning U with X modulo 2 pi is the circular mean of X - U.
# ----------------------------------------------------------------------------
def congruent_shift(U, X):
    """c = arg sum exp(i (X - U))."""
    d = np.asarray(X, np.float64) - np.asarray(U, np.float64)
    return math.atan2(float(np.sum(np.sin(d))), float(np.sum(np.cos(d))))


def rounded(U, X):
    """X + 2 pi k with k = round((U + c - X) / 2 pi) (ties to even), and k."""
    X = np.asarray(X, np.float64)
    c = congruent_shift(U, X)
    k = np.rint((np.asarray(U, np.float64) + c - X) / TWO_PI)
    return X + TWO_PI * k, k


# ----------------------------------------------------------------------------
# Adjoint of the converged (frozen-weight) least-squares map
# ----------------------------------------------------------------------------
def frozen_weights(U, Gv, Gh, eps):
    """omega_bar = 1 / max(|DU - G|, eps) at a converged U."""
    rv, rh = residuals(U, Gv, Gh)
    return 1.0 / np.maximum(np.abs(rv), eps), 1.0 / np.maximum(np.abs(rh), eps)


def frozen_solve(Cv, Ch, Gv, Gh, wv, wh, tol=1e-14, maxit=5000, x0=None, workers=None):
    """U = argmin over mean-zero U of sum C omega_bar (DU - G)^2.

    With x0 given, the correction from x0 is solved instead, to tol relative
    to its own right-hand side (the residual at x0): a small change of the
    weights then still gets a solve converged relative to that change."""
    Ov, Oh = Cv * wv, Ch * wh
    b = div(Ov * Gv, Oh * Gh)
    N, M = b.shape
    A = lambda p: apply_A(Ov, Oh, p)  # noqa: E731
    Minv = lambda r: apply_precond(r, workers=workers)  # noqa: E731
    if x0 is None:
        U, _ = pcg(A, Minv, b, np.zeros((N, M)), tol, maxit)
    else:
        res = b - A(x0)
        dU, _ = pcg(A, Minv, res - res.mean(), np.zeros((N, M)), tol, maxit)
        U = x0 + dU
    return U - U.mean()


def adjoint(U, Gv, Gh, Cv, Ch, eps, gU, tol=1e-14, maxit=5000, weights=None, workers=None):
    """Gradients of a loss with dL/dU = gU through the frozen map.

    U must solve the frozen system for the weights omega_bar, which are
    ``weights`` = (wv, wh) if given, else 1 / max(|DU - G|, eps) at U (the
    fixed point of converged IRLS).  lambda solves D^T Omega D lambda = gU - mean(gU); then per edge
    g_Omega = -(D lambda) r, g_C = omega_bar g_Omega,
    g_G = Omega (D lambda), and g_X = D^T g_G (the residue map W has
    derivative 1 away from its jumps).
    """
    rv, rh = residuals(U, Gv, Gh)
    wv, wh = frozen_weights(U, Gv, Gh, eps) if weights is None else weights
    Ov, Oh = Cv * wv, Ch * wh
    g = np.asarray(gU, np.float64)
    g = g - g.mean()
    lam, _ = pcg(lambda p: apply_A(Ov, Oh, p), lambda r: apply_precond(r, workers=workers), g,
                 np.zeros_like(g), tol, maxit)
    lam -= lam.mean()
    dv, dh = diff_v(lam), diff_h(lam)
    gOv, gOh = -dv * rv, -dh * rh
    gCv, gCh = wv * gOv, wh * gOh
    gGv, gGh = Ov * dv, Oh * dh
    gX = div(gGv, gGh)
    return dict(lam=lam, gCv=gCv, gCh=gCh, gGv=gGv, gGh=gGh, gX=gX,
                wv=wv, wh=wh)
