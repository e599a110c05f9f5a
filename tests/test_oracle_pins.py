"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: matrices are
rebuilt from the paper's element-wise definitions, solutions come from
dense linear algebra or linear programming, and special cases use closed
forms.  Paper: arXiv 2401.09961.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import synth
from oracle import paper_form as PF
from oracle import reduced as R
from oracle import schedule as SCH

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PI = math.pi


# ---------------------------------------------------------------------------
# Independent builders from the paper's definitions (Section 2, Appendix A)
# ---------------------------------------------------------------------------
def S_mat(N):
    """S in R^{(N-1) x N}: S_ij = 1 if j = i+1, -1 if j = i, else 0."""
    S = np.zeros((N - 1, N))
    for i in range(N - 1):
        for j in range(N):
            if j == i + 1:
                S[i, j] = 1.0
            elif j == i:
                S[i, j] = -1.0
    return S


def T_mat(M):
    """T in R^{M x (M-1)}: T_ij = 1 if i = j+1, -1 if i = j, else 0."""
    T = np.zeros((M, M - 1))
    for i in range(M):
        for j in range(M - 1):
            if i == j + 1:
                T[i, j] = 1.0
            elif i == j:
                T[i, j] = -1.0
    return T


def D_dense(N, M):
    """D = [I_M kron S ; T^T kron I_N] on the column-major vec (notation
    section property vec(XYZ) = (Z^T kron X) vec(Y))."""
    return np.vstack([np.kron(np.eye(M), S_mat(N)), np.kron(T_mat(M).T, np.eye(N))])


def vecF(A):
    return np.asarray(A).flatten(order="F")


def laplacian_dense(N, M):
    return (np.kron(np.eye(M), S_mat(N).T @ S_mat(N))
            + np.kron(T_mat(M) @ T_mat(M).T, np.eye(N)))


def lp_l1_star(Gv, Gh, Cv, Ch):
    """Brute-force L1* of problem (prob:main) as a linear program
    (the constraint matrix is totally unimodular, Section 2)."""
    N, M = Gv.shape[0] + 1, Gh.shape[1] + 1
    D = sp.csr_matrix(D_dense(N, M))
    g = np.concatenate([vecF(Gv), vecF(Gh)])
    c = np.concatenate([vecF(Cv), vecF(Ch)])
    E, n = D.shape
    A = sp.hstack([D, -sp.identity(E), sp.identity(E)])
    cost = np.concatenate([np.zeros(n), c, c])
    bounds = [(None, None)] * n + [(0, None)] * (2 * E)
    res = linprog(cost, A_eq=A, b_eq=g, bounds=bounds, method="highs")
    assert res.status == 0
    return float(res.fun)


def residue_count(X):
    Gv, Gh = R.wrapped_gradients(X)
    s = Gh[:-1, :] + Gv[:, 1:] - Gh[1:, :] - Gv[:, :-1]
    return int(np.sum(np.abs(s) > 1.0))


# ---------------------------------------------------------------------------
# Problem data
# ---------------------------------------------------------------------------
def test_eigenvalues_equal_printed_form_in_extended_precision():
    """Appendix A's eigenvalues 2 - 2 cos(pi k / n), evaluated at 50 digits
    (no cancellation left at that precision), equal the oracle's FP64 values
    to a few ulps for every k, the lowest modes included."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    for n in (2, 3, 64, 1000, 8192):
        lam = R.laplacian_eigenvalues(n)
        assert lam[0] == 0.0
        ks = sorted(set([1, 2, 3, n // 2, n - 1] + list(range(1, min(n, 40)))))
        for k in ks:
            if k < 1 or k >= n:
                continue
            exact = 2 - 2 * mpmath.cos(mpmath.pi * k / n)
            rel = abs(float((mpmath.mpf(float(lam[k])) - exact) / exact))
            assert rel < 5e-16 * 8, (n, k, rel)


def test_wrap_is_symmetric_residue():
    x = np.array([0.0, PI, -PI, 1.5 * PI, -1.5 * PI, 7.0, -7.0, 2 * PI, 1e-17, 100.0])
    w = R.wrap(x)
    assert np.all(w >= -PI) and np.all(w < PI)
    k = (x - w) / (2 * PI)
    assert np.allclose(k, np.round(k), atol=1e-12)
    assert R.wrap(PI) == -PI
    assert R.wrap(-PI) == -PI
    assert abs(R.wrap(1.5 * PI) + 0.5 * PI) < 1e-15


def test_wrapped_gradients_match_definition():
    rng = np.random.default_rng(1)
    X = rng.uniform(-PI, PI, (5, 4))
    Gv, Gh = R.wrapped_gradients(X)
    for i in range(4):
        for j in range(4):
            d = X[i + 1, j] - X[i, j]
            assert abs(Gv[i, j] - (((d + PI) % (2 * PI)) - PI)) < 1e-14
    for i in range(5):
        for j in range(3):
            d = X[i, j + 1] - X[i, j]
            assert abs(Gh[i, j] - (((d + PI) % (2 * PI)) - PI)) < 1e-14


def test_edge_weight_rules():
    rng = np.random.default_rng(2)
    w = rng.uniform(0.1, 1.0, (4, 5))
    Cv, Ch = R.edge_weights(4, 5, w=w)
    assert Cv[1, 2] == min(w[1, 2], w[2, 2]) and Ch[3, 1] == min(w[3, 1], w[3, 2])
    Cv1, Ch1 = R.edge_weights(4, 5)
    assert np.all(Cv1 == 1) and Cv1.shape == (3, 5) and Ch1.shape == (4, 4)
    Cv2, Ch2 = R.edge_weights(4, 5, w=w, Cv=Cv * 2, Ch=Ch * 2)
    assert np.allclose(Cv2, 2 * Cv)


# ---------------------------------------------------------------------------
# P1 eigenpairs of S^T S and T T^T (eq:eigendecompositions)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 5, 8, 17, 64])
def test_P1_dct_basis_is_eigenbasis(n):
    S, T = S_mat(n), T_mat(n)
    P, lam = R.dct_basis(n), R.laplacian_eigenvalues(n)
    assert np.allclose((S.T @ S) @ P, P * lam[None, :], atol=1e-12)
    assert np.allclose((T @ T.T) @ P, P * lam[None, :], atol=1e-12)
    assert np.allclose(P.T @ P, np.eye(n), atol=1e-12)
    assert np.allclose(np.sort(np.linalg.eigvalsh(S.T @ S)), np.sort(lam), atol=1e-12)
    assert lam[0] == 0.0 and np.all(lam[1:] > 0)


# ---------------------------------------------------------------------------
# P2 the DCT route equals the dense eigenbasis products
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(9, 14), (16, 16), (2, 7), (33, 5)])
def test_P2_dct_route_equals_dense_products(shape):
    import scipy.fft
    rng = np.random.default_rng(3)
    Rm = rng.standard_normal(shape)
    PN, PM = R.dct_basis(shape[0]), R.dct_basis(shape[1])
    assert np.allclose(scipy.fft.dctn(Rm, type=2, norm="ortho"), PN.T @ Rm @ PM, atol=1e-13)
    assert np.allclose(R.apply_precond(Rm), R.apply_precond_explicit(Rm), atol=1e-12)


# ---------------------------------------------------------------------------
# P3 the operator equals the dense D^T diag(omega) D
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(6, 5), (2, 2), (3, 7)])
def test_P3_operator_equals_dense(shape):
    N, M = shape
    rng = np.random.default_rng(4)
    Ov = rng.uniform(0.1, 3.0, (N - 1, M))
    Oh = rng.uniform(0.1, 3.0, (N, M - 1))
    P = rng.standard_normal((N, M))
    D = D_dense(N, M)
    A = D.T @ np.diag(np.concatenate([vecF(Ov), vecF(Oh)])) @ D
    assert np.allclose(vecF(R.apply_A(Ov, Oh, P)), A @ vecF(P), atol=1e-12)
    assert np.allclose(A, A.T)
    assert np.allclose(A @ np.ones(N * M), 0.0, atol=1e-12)
    assert np.allclose(R.sparse_D(N, M).toarray(), D)
    # D^T F for edge fields: div is the adjoint of the difference maps
    Fv, Fh = rng.standard_normal((N - 1, M)), rng.standard_normal((N, M - 1))
    assert np.allclose(vecF(R.div(Fv, Fh)), D.T @ np.concatenate([vecF(Fv), vecF(Fh)]))


# ---------------------------------------------------------------------------
# P4 preconditioner is the pseudo-inverse of the Neumann Laplacian
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(7, 6), (4, 9), (2, 2)])
def test_P4_precond_is_pseudo_inverse(shape):
    N, M = shape
    rng = np.random.default_rng(5)
    r = rng.standard_normal((N, M))
    z = R.apply_precond(r)
    L = laplacian_dense(N, M)
    assert np.allclose(L @ vecF(z), vecF(r - r.mean()), atol=1e-11)
    assert np.allclose(np.linalg.pinv(L) @ vecF(r), vecF(z), atol=1e-11)
    assert abs(z.mean()) < 1e-13


# ---------------------------------------------------------------------------
# P5 PCG special cases
# ---------------------------------------------------------------------------
def test_P5_unit_weights_converge_in_one_iteration():
    rng = np.random.default_rng(6)
    N, M = 20, 13
    Gv, Gh = rng.uniform(-PI, PI, (N - 1, M)), rng.uniform(-PI, PI, (N, M - 1))
    Ov, Oh = np.ones((N - 1, M)), np.ones((N, M - 1))
    b = R.div(Gv, Gh)
    x, info = R.pcg(lambda p: R.apply_A(Ov, Oh, p), R.apply_precond, b,
                    np.zeros((N, M)), 1e-12, 50)
    assert info["iters"] == 1 and info["true_relres"] < 1e-12


def test_P5_weighted_solve_equals_dense_lstsq():
    rng = np.random.default_rng(7)
    N, M = 12, 9
    Ov = rng.uniform(0.05, 20.0, (N - 1, M))
    Oh = rng.uniform(0.05, 20.0, (N, M - 1))
    Gv, Gh = rng.uniform(-PI, PI, (N - 1, M)), rng.uniform(-PI, PI, (N, M - 1))
    b = R.div(Ov * Gv, Oh * Gh)
    x, info = R.pcg(lambda p: R.apply_A(Ov, Oh, p), R.apply_precond, b,
                    np.zeros((N, M)), 1e-13, 500)
    D = D_dense(N, M)
    sw = np.sqrt(np.concatenate([vecF(Ov), vecF(Oh)]))
    xs = np.linalg.lstsq(sw[:, None] * D, sw * np.concatenate([vecF(Gv), vecF(Gh)]), rcond=None)[0]
    xs = xs - xs.mean()
    assert np.allclose(vecF(x - x.mean()), xs, atol=1e-9)


def test_P5_energy_error_non_increasing():
    rng = np.random.default_rng(8)
    N, M = 10, 11
    Ov = rng.uniform(0.01, 10.0, (N - 1, M))
    Oh = rng.uniform(0.01, 10.0, (N, M - 1))
    b = R.div(Ov * rng.standard_normal((N - 1, M)), Oh * rng.standard_normal((N, M - 1)))
    A = lambda p: R.apply_A(Ov, Oh, p)  # noqa: E731
    xs, _ = R.pcg(A, R.apply_precond, b, np.zeros((N, M)), 1e-14, 1000)
    errs = []
    for k in range(1, 15):
        xk, _ = R.pcg(A, R.apply_precond, b, np.zeros((N, M)), 0.0, k)
        e = xk - xs
        errs.append(float(np.vdot(e, A(e))))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) + 1e-24 for i in range(len(errs) - 1))


# ---------------------------------------------------------------------------
# P6 unweighted L2 unwrapping in one preconditioned step
# ---------------------------------------------------------------------------
def test_P6_unweighted_l2_is_one_laplacian_solve():
    f = synth.field_c3(4, 16, 12)
    Gv, Gh = R.wrapped_gradients(f.X)
    N, M = f.X.shape
    b = R.div(Gv, Gh)
    x, info = R.pcg(lambda p: R.apply_A(np.ones_like(Gv), np.ones_like(Gh), p),
                    R.apply_precond, b, np.zeros((N, M)), 1e-12, 10)
    D = D_dense(N, M)
    xs = np.linalg.lstsq(D, np.concatenate([vecF(Gv), vecF(Gh)]), rcond=None)[0]
    assert info["iters"] == 1
    assert np.allclose(vecF(x), xs - xs.mean(), atol=1e-11)


# ---------------------------------------------------------------------------
# P7 Itoh condition: the L1 solution is plain integration (Section 1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,shape", [(0, (24, 20)), (1, (40, 33)), (2, (7, 9))])
def test_P7_itoh_case_recovers_integration(seed, shape):
    f = synth.smooth_field(seed, *shape)
    assert max(np.abs(np.diff(f.phi, axis=0)).max(), np.abs(np.diff(f.phi, axis=1)).max()) < PI
    U, hist = R.irls(f.X, iters=2, tol=1e-13, maxit=500)
    assert np.abs(U - (f.phi - f.phi.mean())).max() < 1e-9
    assert hist[-1]["L1"] < 1e-8


def test_P7_small_case_generator_satisfies_itoh():
    f = synth.field_c1(0, 128, 128)
    assert residue_count(f.X) == 0
    U, hist = R.irls(f.X, iters=2, tol=1e-12, maxit=200)
    assert np.abs(U - (f.phi - f.phi.mean())).max() < 1e-8


# ---------------------------------------------------------------------------
# P8 monotone decrease of the smoothed objective (majorise-minimise)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gen,seed", [("c2", 0), ("c3", 1), ("c2", 5)])
def test_P8_huber_objective_monotone(gen, seed):
    f = getattr(synth, "field_" + gen)(seed, 48, 40)
    U, hist = R.irls(f.X, w=f.w, iters=15, tol=1e-8, maxit=60)
    H = [h["H"] for h in hist]
    assert all(H[k + 1] <= H[k] * (1 + 1e-12) for k in range(len(H) - 1))
    assert H[-1] < 0.9 * H[0]


# ---------------------------------------------------------------------------
# P9 bracket with the LP optimum, P10 single-loop closed form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_P9_lp_bracket(seed):
    n = 3 + seed % 4  # 3..6
    f = synth.field_c3(seed, n, n + (seed % 2))
    N, M = f.X.shape
    Gv, Gh = R.wrapped_gradients(f.X)
    Cv, Ch = R.edge_weights(N, M, w=f.w)
    L1s = lp_l1_star(Gv, Gh, Cv, Ch)
    eps = 1e-3
    U, hist = R.irls(f.X, w=f.w, iters=300, tol=1e-13, maxit=400, eps=eps)
    H, L1 = hist[-1]["H"], hist[-1]["L1"]
    slack = eps / 2 * (Cv.sum() + Ch.sum())
    assert H <= L1s + 1e-9 * max(1.0, L1s)
    assert L1s <= L1 + 1e-9
    assert L1 <= H + slack + 1e-12


def test_P10_single_loop_closed_form():
    g = json.load(open(os.path.join(GOLDEN, "loop2x2.json")))
    X = np.array(g["X"])
    Gv, Gh = R.wrapped_gradients(X)
    loop = Gh[0, 0] + Gv[0, 1] - Gh[1, 0] - Gv[0, 0]
    assert abs(loop - 2 * PI * g["loop_sum_over_2pi"]) < 1e-12
    Cv, Ch = np.array(g["Cv"]), np.array(g["Ch"])
    assert abs(lp_l1_star(Gv, Gh, Cv, Ch) - g["L1_star_given_weights"]) < 1e-9
    one_v, one_h = np.ones_like(Cv), np.ones_like(Ch)
    assert abs(lp_l1_star(Gv, Gh, one_v, one_h) - g["L1_star_unit_weights"]) < 1e-9
    eps = 1e-4
    U, hist = R.irls(X, Cv=Cv, Ch=Ch, iters=200, tol=1e-14, maxit=100, eps=eps)
    L1 = hist[-1]["L1"]
    assert g["L1_star_given_weights"] - 1e-9 <= L1 <= g["L1_star_given_weights"] + eps * 4


# ---------------------------------------------------------------------------
# P11 cross-oracle: Algorithm 1 verbatim reaches the reduced optimum
# ---------------------------------------------------------------------------
def test_P11_paper_form_reaches_reduced_optimum():
    f = synth.field_c3(1, 12, 12)
    assert residue_count(f.X) > 0
    Gv, Gh = R.wrapped_gradients(f.X)
    Cv, Ch = R.edge_weights(12, 12)
    eps = 1e-2
    U1, h1 = R.irls(f.X, iters=300, tol=1e-13, maxit=500, eps=eps)
    U2, Vv, Vh, h2 = PF.irls(f.X, tau=eps, delta=1e-9, iters=300, tol=1e-13, maxit=2000)
    F2 = PF.f_delta(U2, Vv, Vh, Gv, Gh, Cv, Ch, eps, 0.0)
    assert abs(h1[-1]["H"] - F2) < 1e-6 * h1[-1]["H"]
    assert abs(R.huber_objective(U2, Gv, Gh, Cv, Ch, eps) - h1[-1]["H"]) < 1e-7 * h1[-1]["H"]
    # F over V at fixed U is minimised by the soft threshold (Moreau envelope)
    rv, rh = R.residuals(U2, Gv, Gh)
    Vv_st = np.sign(rv) * np.maximum(np.abs(rv) - eps, 0)
    Vh_st = np.sign(rh) * np.maximum(np.abs(rh) - eps, 0)
    F_env = PF.f_delta(U2, Vv_st, Vh_st, Gv, Gh, Cv, Ch, eps, 0.0)
    assert abs(F_env - R.huber_objective(U2, Gv, Gh, Cv, Ch, eps)) < 1e-10 * F_env


# ---------------------------------------------------------------------------
# P12 rewrapping U gives back X (Itoh case)
# ---------------------------------------------------------------------------
def test_P12_rewrap_gives_back_input():
    f = synth.smooth_field(5, 30, 26)
    U, _ = R.irls(f.X, iters=2, tol=1e-13, maxit=500)
    c = np.angle(np.sum(np.exp(1j * (f.X - U))))
    back = np.angle(np.exp(1j * (U + c - f.X)))
    assert np.abs(back).max() < 1e-9


# ---------------------------------------------------------------------------
# P13 Schur reduction of Proposition 1
# ---------------------------------------------------------------------------
def test_P13_schur_reduction_equals_augmented_solve():
    rng = np.random.default_rng(9)
    N, M, tau, delta = 5, 6, 1e-2, 1e-6
    f = synth.field_c3(3, N, M)
    Gv, Gh = R.wrapped_gradients(f.X)
    Cv, Ch = rng.uniform(0.2, 1.5, (N - 1, M)), rng.uniform(0.2, 1.5, (N, M - 1))
    Wv, Wh = rng.uniform(delta, 2.0, (N - 1, M)), rng.uniform(delta, 2.0, (N, M - 1))
    sysk = PF.Augmented(Gv, Gh, Cv, Ch, Wv, Wh, tau)
    n = sysk.rhs().size
    A = np.column_stack([sysk.A(e) for e in np.eye(n)])
    assert np.allclose(A, A.T, atol=1e-9 * np.abs(A).max())
    x = np.linalg.lstsq(A, sysk.rhs(), rcond=None)[0]
    u, vv, vh = sysk.split(x)
    U, Vv, Vh = PF.schur_solve(Gv, Gh, Cv, Ch, Wv, Wh, tau)
    assert np.allclose(u - u.mean(), U, atol=1e-9)
    assert np.allclose(vv, Vv, atol=1e-9) and np.allclose(vh, Vh, atol=1e-9)
    # the augmented PCG of Algorithm 2 with the block preconditioner agrees
    xp, info = R.pcg(sysk.A, sysk.precond, sysk.rhs(), np.zeros(n), 1e-13, 2000)
    up, _, _ = sysk.split(xp)
    assert np.allclose(up - up.mean(), U, atol=1e-8)


# ---------------------------------------------------------------------------
# Theorem 2 bound and the paper-form objective
# ---------------------------------------------------------------------------
def test_theorem2_smoothing_bound():
    rng = np.random.default_rng(10)
    N, M, tau = 7, 5, 1e-2
    U = rng.standard_normal((N, M))
    Gv, Gh = rng.uniform(-PI, PI, (N - 1, M)), rng.uniform(-PI, PI, (N, M - 1))
    Vv, Vh = rng.standard_normal((N - 1, M)), rng.standard_normal((N, M - 1))
    Cv, Ch = rng.uniform(0.1, 2, (N - 1, M)), rng.uniform(0.1, 2, (N, M - 1))
    for delta in (1e-6, 1e-2, 0.5):
        F = PF.f_delta(U, Vv, Vh, Gv, Gh, Cv, Ch, tau, 0.0)
        Fd = PF.f_delta(U, Vv, Vh, Gv, Gh, Cv, Ch, tau, delta)
        assert F <= Fd <= F + PF.smoothing_gap_bound(N, M, delta) + 1e-12
    # closed-form weights minimise the surrogate of (prob:alt1) over W
    Wv, Wh = PF.closed_form_weights(Vv, Vh, Cv, Ch, 0.1)
    h0 = PF.h_delta(U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch, tau, 0.1)
    assert abs(h0 - PF.f_delta(U, Vv, Vh, Gv, Gh, Cv, Ch, tau, 0.1)) < 1e-10 * h0
    assert h0 <= PF.h_delta(U, Vv, Vh, Wv * 1.1, Wh * 0.9, Gv, Gh, Cv, Ch, tau, 0.1)


def test_theorem2_gap_is_attained_at_zero_slack():
    """Both sides of Theorem 2 are tight: at V = 0 every smoothed term is
    sqrt(0 + delta^2) = delta, so F_delta - F equals delta times the number
    of edges (counted here as the rows of the dense D of Section 2), and for
    slacks far larger than delta / C the gap vanishes.  An over- or
    under-count of the edges in the oracle's bound fails the first check."""
    rng = np.random.default_rng(11)
    tau = 1e-2
    for (N, M) in ((7, 5), (4, 9), (2, 2)):
        n_edges = D_dense(N, M).shape[0]
        assert n_edges == (N - 1) * M + N * (M - 1)
        U = rng.standard_normal((N, M))
        Gv, Gh = rng.uniform(-PI, PI, (N - 1, M)), rng.uniform(-PI, PI, (N, M - 1))
        Cv, Ch = rng.uniform(0.1, 2, (N - 1, M)), rng.uniform(0.1, 2, (N, M - 1))
        Z0v, Z0h = np.zeros((N - 1, M)), np.zeros((N, M - 1))
        for delta in (1e-6, 1e-2, 0.5):
            F = PF.f_delta(U, Z0v, Z0h, Gv, Gh, Cv, Ch, tau, 0.0)
            Fd = PF.f_delta(U, Z0v, Z0h, Gv, Gh, Cv, Ch, tau, delta)
            assert abs((Fd - F) - delta * n_edges) <= 1e-12 * max(Fd, 1.0)
            assert PF.smoothing_gap_bound(N, M, delta) == pytest.approx(delta * n_edges, rel=1e-15)
        big = 1e6
        Vv, Vh = np.full((N - 1, M), big), np.full((N, M - 1), -big)
        delta = 1e-3
        gap = (PF.f_delta(U, Vv, Vh, Gv, Gh, Cv, Ch, tau, delta)
               - PF.f_delta(U, Vv, Vh, Gv, Gh, Cv, Ch, tau, 0.0))
        # sqrt(C^2 V^2 + d^2) - C|V| = d^2 / (2 C |V|) + O(d^4): far below d
        assert 0.0 <= gap <= delta * n_edges * 1e-6


def test_theorem3_L_equals_the_printed_value():
    """L = 12 / tau + C_max^2 / delta at the paper's tau and delta
    (Section 4.4) and unit weights, against the stored constant 1 001 200;
    C_max enters squared and only through the largest weight."""
    with open(os.path.join(GOLDEN, "paper_parameters.json")) as fh:
        g = json.load(fh)
    tau, delta = g["tau"], g["delta"]
    ones_v, ones_h = np.ones((5, 6)), np.ones((6, 5))
    assert PF.lipschitz_L(ones_v, ones_h, tau, delta) == pytest.approx(
        g["theorem3_L_unit_weights"], rel=1e-15)
    Cv = np.full((5, 6), 0.5)
    Cv[2, 3] = 2.0
    assert PF.lipschitz_L(Cv, ones_h, tau, delta) == pytest.approx(1200.0 + 4e6, rel=1e-15)
    assert PF.lipschitz_L(0.5 * ones_v, 0.5 * ones_h, tau, delta) == pytest.approx(
        1200.0 + 0.25e6, rel=1e-15)


def test_paper_form_alg1_monotone_f_delta():
    f = synth.field_c2(2, 16, 14)
    U, Vv, Vh, hist = PF.irls(f.X, w=f.w, tau=1e-2, delta=1e-6, iters=10, tol=1e-12, maxit=400)
    Fd = [h["F_delta"] for h in hist]
    assert all(Fd[k + 1] <= Fd[k] * (1 + 1e-10) for k in range(len(Fd) - 1))


# ---------------------------------------------------------------------------
# Theorem 3: the candidate gradient step and the sufficient-decrease guard
# ---------------------------------------------------------------------------
def _thm3_problem(seed, N=6, M=5, delta=0.05):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((N, M))
    Gv, Gh = rng.uniform(-PI, PI, (N - 1, M)), rng.uniform(-PI, PI, (N, M - 1))
    Vv, Vh = rng.standard_normal((N - 1, M)), rng.standard_normal((N, M - 1))
    Cv, Ch = rng.uniform(0.1, 2, (N - 1, M)), rng.uniform(0.1, 2, (N, M - 1))
    # weights of the previous iterate (not those of V: the step is taken at W^k)
    Wv, Wh = PF.closed_form_weights(rng.standard_normal((N - 1, M)),
                                    rng.standard_normal((N, M - 1)), Cv, Ch, delta)
    return U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch


def _pack(U, Vv, Vh):
    return np.concatenate([U.ravel(), Vv.ravel(), Vh.ravel()])


def _unpack(x, N, M):
    a, b = N * M, N * M + (N - 1) * M
    return x[:a].reshape(N, M), x[a:b].reshape(N - 1, M), x[b:].reshape(N, M - 1)


def test_thm3_candidate_direction_is_the_gradient_by_finite_differences():
    """(x - x~) L must equal the gradient of the (prob:alt1) objective at
    fixed W, here by central differences of h_delta itself."""
    tau, delta = 0.3, 0.05
    U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch = _thm3_problem(1, delta=delta)
    N, M = U.shape
    L = PF.lipschitz_L(Cv, Ch, tau, delta)
    x = _pack(U, Vv, Vh)
    step = (x - _pack(*PF.candidate_step(U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch, tau, delta))) * L
    h = lambda y: PF.h_delta(*_unpack(y, N, M), Wv, Wh, Gv, Gh, Cv, Ch, tau, delta)
    eps = 1e-6
    fd = np.array([(h(x + eps * e) - h(x - eps * e)) / (2 * eps) for e in np.eye(x.size)])
    assert np.abs(fd - step).max() <= 1e-6 * np.abs(fd).max()


def test_thm3_L_bounds_the_hessian_and_gives_the_descent_lemma():
    """L = 12/tau + C_max^2/delta bounds the largest Hessian eigenvalue of
    the objective at fixed W >= delta (dense eigvalsh), so the step decreases
    it by at least ||grad||^2 / (2L) (descent lemma)."""
    tau, delta = 0.2, 0.05
    for seed in range(5):
        U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch = _thm3_problem(seed, delta=delta)
        N, M = U.shape
        L = PF.lipschitz_L(Cv, Ch, tau, delta)
        x = _pack(U, Vv, Vh)
        h = lambda y: PF.h_delta(*_unpack(y, N, M), Wv, Wh, Gv, Gh, Cv, Ch, tau, delta)
        n = x.size
        # the objective is quadratic in x at fixed W: Hessian by second differences
        H = np.zeros((n, n))
        E = np.eye(n)
        h0 = h(np.zeros(n))
        for i in range(n):
            for j in range(i, n):
                H[i, j] = H[j, i] = h(E[i] + E[j]) - h(E[i]) - h(E[j]) + h0
        lam = np.linalg.eigvalsh(H)
        assert lam[0] > -1e-9 and lam[-1] <= L
        xc = _pack(*PF.candidate_step(U, Vv, Vh, Wv, Wh, Gv, Gh, Cv, Ch, tau, delta))
        g = (x - xc) * L
        assert h(xc) <= h(x) - g @ g / (2 * L) + 1e-12 * abs(h(x))


def test_thm3_condition_holds_after_cg_and_candidate_only_is_monotone():
    """The paper reports the condition always held after CG: so it does in
    the guarded oracle run, which then equals the unguarded one.  The
    candidate-only variant decreases F_delta at every iteration (alternating
    minimisation over W never increases it) but far more slowly."""
    f = synth.field_c2(2, 16, 14)
    kw = dict(w=f.w, tau=1e-2, delta=1e-6, iters=6, tol=1e-12, maxit=400)
    U1, _, _, h1 = PF.irls(f.X, guard=1, **kw)
    U0, _, _, h0 = PF.irls(f.X, guard=0, **kw)
    assert all(h["guard"] == 1 for h in h1)
    assert np.array_equal(U1, U0)
    U2, _, _, h2 = PF.irls(f.X, guard=2, **kw)
    F2 = [h["F_delta"] for h in h2]
    assert all(h["guard"] == 2 for h in h2)
    assert all(F2[k + 1] <= F2[k] for k in range(len(F2) - 1))
    assert F2[-1] > h1[-1]["F_delta"] * 1.01


def test_thm3_guard_takes_the_candidate_when_cg_does_worse():
    """Planted on the CPU: a 'solver' that returns a worse point than the
    start must be replaced by the candidate step."""
    f = synth.field_c2(3, 12, 10)
    real = R.pcg
    try:
        R.pcg = lambda A, P, b, x0, tol, m: (x0 + 0.5, dict(iters=1))
        U, _, _, h = PF.irls(f.X, w=f.w, tau=1e-2, delta=1e-6, iters=2, guard=1)
    finally:
        R.pcg = real
    U2, _, _, h2 = PF.irls(f.X, w=f.w, tau=1e-2, delta=1e-6, iters=2, guard=2)
    assert [x["guard"] for x in h] == [2, 2]
    assert np.allclose(U, U2, rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# Section 4.3 schedule rules
# ---------------------------------------------------------------------------
def test_schedule_rules_with_paper_parameters():
    p = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    s = SCH.CgSchedule(p["m_cg_0"], p["eps_tol"], p["alpha"])
    assert s.current() == 5
    assert s.update(0.1) == 5          # rule 1: enough improvement
    assert s.update(1e-4) == 9         # rule 3: ceil(1.7 * 5)
    assert s.update(1e-4) is None      # rule 2: raised last time -> stop
    s2 = SCH.CgSchedule(5, 1e-3, 1.7)
    assert s2.update(1e-3) == 9        # Delta == eps_tol counts as not significant


def test_surrogate_majorises_huber_and_touches_at_own_weights():
    """The reduced IRLS model: at its own weights it equals H_eps + eps/2
    sum C (closed form of the minimum over omega <= 1/eps), at any other
    positive weights it is larger (so Delta >= 0)."""
    rng = np.random.default_rng(21)
    N, M, eps = 9, 7, 1e-2
    Gv, Gh = rng.uniform(-3, 3, (N - 1, M)), rng.uniform(-3, 3, (N, M - 1))
    Cv, Ch = rng.uniform(0.2, 2, (N - 1, M)), rng.uniform(0.2, 2, (N, M - 1))
    U = rng.normal(size=(N, M))
    U[0, :3] = U[1, :3] + Gv[0, :3] + 1e-3          # a few edges inside the Huber corner
    rv, rh = R.residuals(U, Gv, Gh)
    Ov, Oh = Cv / np.maximum(np.abs(rv), eps), Ch / np.maximum(np.abs(rh), eps)
    s_own = R.surrogate(U, Gv, Gh, Cv, Ch, Ov, Oh)
    closed = R.huber_objective(U, Gv, Gh, Cv, Ch, eps) + eps / 2 * (Cv.sum() + Ch.sum())
    assert abs(s_own - closed) <= 1e-12 * closed
    for _ in range(20):
        Pv, Ph = Ov * rng.uniform(0.2, 5, Ov.shape), Oh * rng.uniform(0.2, 5, Oh.shape)
        Pv, Ph = np.minimum(Pv, Cv / eps), np.minimum(Ph, Ch / eps)
        assert R.surrogate(U, Gv, Gh, Cv, Ch, Pv, Ph) >= s_own * (1 - 1e-14)


def test_scheduled_irls_follows_section_4_3_rules():
    """The schedule-driven oracle: caps follow the rules from the recorded
    Delta values, every Delta >= 0, the stop comes only after a raise, and
    the solves use the cap (never more iterations)."""
    f = synth.field_c3(2, 48, 40)
    sch = SCH.CgSchedule(5, 1e-3, 1.7)
    U, hist = R.irls(f.X, w=f.w, iters=60, tol=1e-12, maxit=100, schedule=sch)
    caps = [h["cap"] for h in hist if "cap" in h]
    assert caps[0] == 5
    deltas = [h["delta"] for h in hist if "delta" in h]
    assert all(d >= -1e-14 for d in deltas)
    replay = SCH.CgSchedule(5, 1e-3, 1.7)
    expect = [5]
    for d in deltas:
        m = replay.update(d)
        if m is None:
            break
        expect.append(m)
    assert caps == expect[:len(caps)]
    assert all(h["iters"] <= h["cap"] for h in hist if "cap" in h and "iters" in h)
    if hist[-1].get("stopped"):
        assert caps[-1] != caps[-2] if len(caps) >= 2 else True
        assert hist[-1]["delta"] <= 1e-3


# ---------------------------------------------------------------------------
# Rounded (2 pi-congruent) output
# ---------------------------------------------------------------------------
def test_rounded_output_is_congruent_and_recovers_itoh_phase():
    """Itoh case: the IRLS U is phi - mean(phi); rounding it gives back phi
    up to one multiple of 2 pi, and the output minus X is an exact integer
    multiple of 2 pi pixel by pixel."""
    f = synth.smooth_field(3, 40, 36)
    U, _ = R.irls(f.X, iters=3, tol=1e-12, maxit=500)
    Ur, k = R.rounded(U, f.X)
    assert np.array_equal(Ur, f.X + R.TWO_PI * k)
    m = (Ur - f.phi) / R.TWO_PI
    assert np.abs(m - np.round(m[0, 0])).max() < 1e-9


def test_rounded_output_is_invariant_to_the_constant_of_u():
    """U is defined up to a constant: rounding U + t gives the same output
    (the aligning constant absorbs t), for t off the rounding boundaries."""
    rng = np.random.default_rng(31)
    X = rng.uniform(-np.pi, np.pi, (30, 20))
    U = X + R.TWO_PI * rng.integers(-3, 4, X.shape) + rng.normal(0, 0.3, X.shape)
    Ur, k = R.rounded(U, X)
    for t in (0.7, -2.1, 10.0):
        Ur2, k2 = R.rounded(U + t, X)
        d = (Ur2 - Ur) / R.TWO_PI
        assert np.abs(d - np.round(d)).max() < 1e-12 and np.ptp(np.round(d)) == 0


def test_rounded_output_of_a_congruent_u_keeps_its_integers():
    """A U that already differs from X by 2 pi k (plus a constant) is
    returned as X + 2 pi k (up to one common multiple of 2 pi)."""
    rng = np.random.default_rng(32)
    X = rng.uniform(-np.pi, np.pi, (17, 23))
    K = rng.integers(-5, 6, X.shape)
    Ur, k = R.rounded(X + R.TWO_PI * K - 1.234, X)
    s = k - K
    assert np.ptp(s) == 0


# ---------------------------------------------------------------------------
# Adjoint of the frozen-weight map against FP64 central differences
# ---------------------------------------------------------------------------
def dense_frozen_solve(Cv, Ch, Gv, Gh, wv, wh):
    """Mean-zero minimiser of sum C omega (DU - G)^2: the normal equations
    bordered with the mean constraint, solved by dense LU."""
    N, M = Gv.shape[0] + 1, Gh.shape[1] + 1
    D = D_dense(N, M)
    om = np.concatenate([vecF(Cv * wv), vecF(Ch * wh)])
    A = D.T @ (om[:, None] * D)
    b = D.T @ (om * np.concatenate([vecF(Gv), vecF(Gh)]))
    n = N * M
    K = np.zeros((n + 1, n + 1))
    K[:n, :n], K[:n, n], K[n, :n] = A, 1.0, 1.0
    x = np.linalg.solve(K, np.concatenate([b, [0.0]]))[:n]
    return x.reshape((N, M), order="F")


# ---------------------------------------------------------------------------
# Full implicit derivative of the Huber minimiser
# ---------------------------------------------------------------------------
def _huber_case(seed, N=20, M=18, eps=1e-2):
    """A residue field whose quadratic-zone graph connects every pixel (seeds
    3 and 5 at this size), its weights and its exact Huber minimiser."""
    rng = np.random.default_rng(seed)
    X = synth.observe(synth.gaussian_sum_field(rng, N, M, amp=3.0, noise=1.2))
    Gv, Gh = R.wrapped_gradients(X)
    rng2 = np.random.default_rng(100 + seed)
    Cv, Ch = rng2.uniform(0.5, 1.5, (N - 1, M)), rng2.uniform(0.5, 1.5, (N, M - 1))
    U0, _ = R.irls(G=(Gv, Gh), Cv=Cv, Ch=Ch, eps=eps, iters=200, tol=1e-13, maxit=2000)
    U, qv, qh = R.huber_minimiser(Gv, Gh, Cv, Ch, eps, U0)
    return X, Gv, Gh, Cv, Ch, eps, U, qv, qh


def test_huber_minimiser_is_stationary_and_irls_converges_to_it():
    X, Gv, Gh, Cv, Ch, eps, U, qv, qh = _huber_case(3)
    assert R.huber_stationarity(U, Gv, Gh, Cv, Ch, eps) < 1e-10
    assert 0.5 < qv.mean() < 1.0 and 0.5 < qh.mean() < 1.0    # both zones occur
    U0, _ = R.irls(G=(Gv, Gh), Cv=Cv, Ch=Ch, eps=eps, iters=200, tol=1e-13, maxit=2000)
    assert np.abs(U0 - U).max() < 1e-8


@pytest.mark.parametrize("seed", [3, 5])
def test_implicit_adjoint_matches_finite_differences_of_the_minimiser(seed):
    """dL/dC and dL/dX of L = gU . U*(C, X) by central differences of the
    exact minimiser (re-solved for each perturbed problem, same quadratic
    zone) against the implicit adjoint."""
    X, Gv, Gh, Cv, Ch, eps, U, qv, qh = _huber_case(seed)
    N, M = X.shape
    rng = np.random.default_rng(7 + seed)
    gU = rng.standard_normal((N, M))
    adj = R.adjoint_implicit(U, Gv, Gh, Cv, Ch, eps, gU)
    assert not adj["isolated"].any()
    h = 1e-6
    scale = max(np.abs(adj["gCv"]).max(), np.abs(adj["gCh"]).max())
    for _ in range(10):
        vert = rng.random() < 0.5
        shp = (N - 1, M) if vert else (N, M - 1)
        e = (rng.integers(shp[0]), rng.integers(shp[1]))
        L = []
        for sgn in (1, -1):
            Cv2, Ch2 = Cv.copy(), Ch.copy()
            (Cv2 if vert else Ch2)[e] += sgn * h
            U2, qv2, qh2 = R.huber_minimiser(Gv, Gh, Cv2, Ch2, eps, U)
            assert np.array_equal(qv2, qv) and np.array_equal(qh2, qh)
            L.append(float(np.sum(gU * U2)))
        fd = (L[0] - L[1]) / (2 * h)
        got = (adj["gCv"] if vert else adj["gCh"])[e]
        assert abs(fd - got) <= 1e-6 * scale, (vert, e, fd, got)
    scale = np.abs(adj["gX"]).max()
    checked = 0
    while checked < 8:
        i, j = rng.integers(N), rng.integers(M)
        d = np.concatenate([np.diff(X, axis=0)[max(i - 1, 0):i + 1, j],
                            np.diff(X, axis=1)[i, max(j - 1, 0):j + 1]])
        if np.any(np.abs(np.abs(d) - np.pi) < 1e-3):
            continue
        L = []
        for sgn in (1, -1):
            X2 = X.copy()
            X2[i, j] += sgn * h
            Gv2, Gh2 = R.wrapped_gradients(X2)
            U2, _, _ = R.huber_minimiser(Gv2, Gh2, Cv, Ch, eps, U)
            L.append(float(np.sum(gU * U2)))
        fd = (L[0] - L[1]) / (2 * h)
        assert abs(fd - adj["gX"][i, j]) <= 1e-6 * scale, (i, j, fd, adj["gX"][i, j])
        checked += 1


def test_implicit_adjoint_itoh_case_is_the_mean_removal():
    """No residues: every edge is quadratic and U* integrates G, so
    dL/dX = gU - mean(gU) whatever C, and dL/dC = 0 (h'(0) = 0)."""
    f = synth.smooth_field(2, 24, 20)
    Gv, Gh = R.wrapped_gradients(f.X)
    rng = np.random.default_rng(4)
    Cv, Ch = rng.uniform(0.5, 1.5, Gv.shape), rng.uniform(0.5, 1.5, Gh.shape)
    U0, _ = R.irls(G=(Gv, Gh), Cv=Cv, Ch=Ch, eps=1e-3, iters=3, tol=1e-13, maxit=2000)
    U, qv, qh = R.huber_minimiser(Gv, Gh, Cv, Ch, 1e-3, U0)
    assert qv.all() and qh.all()
    gU = rng.standard_normal(U.shape)
    adj = R.adjoint_implicit(U, Gv, Gh, Cv, Ch, 1e-3, gU)
    assert np.abs(adj["gX"] - (gU - gU.mean())).max() < 1e-9
    assert max(np.abs(adj["gCv"]).max(), np.abs(adj["gCh"]).max()) < 1e-9


def test_implicit_adjoint_leaves_out_isolated_pixels():
    """A pixel whose four edges all lie outside the quadratic zone (its
    minimiser value is not unique) gets lambda = 0 and no share of gU; the
    gradients are then those of the problem with gU zero there."""
    X, Gv, Gh, Cv, Ch, eps, U, qv, qh = _huber_case(3)
    N, M = X.shape
    U2 = U.copy()
    U2[10, 9] += 0.5                      # its four residuals leave the zone
    adj = R.adjoint_implicit(U2, Gv, Gh, Cv, Ch, eps, np.ones((N, M)) + np.arange(N * M).reshape(N, M))
    assert adj["isolated"][10, 9] and adj["isolated"].sum() == 1
    assert adj["lam"][10, 9] == 0.0
    assert abs(adj["lam"][~adj["isolated"]].sum()) < 1e-9


def test_adjoint_matches_finite_differences():
    # residue-bearing moderate-amplitude phase with the sigmoid edge weights
    # of the differentiation case, so that r = DU - G is not identically zero
    rng = np.random.default_rng(12)
    phi = synth.gaussian_sum_field(rng, 9, 8, amp=3.0, noise=1.2)
    X = synth.observe(phi)
    assert residue_count(X) > 0
    w5 = synth.field_c5(0, 9, 8)
    Cv, Ch = w5.Cv, w5.Ch
    N, M = X.shape
    Gv, Gh = R.wrapped_gradients(X)
    eps = 1e-3
    U, _ = R.irls(X, Cv=Cv, Ch=Ch, iters=8, tol=1e-12, maxit=300, eps=eps)
    wv, wh = R.frozen_weights(U, Gv, Gh, eps)
    U0 = dense_frozen_solve(Cv, Ch, Gv, Gh, wv, wh)
    # a linear loss L(U) = <a, U>: the adjoint is linear in dL/dU = a, and
    # finite differences of U avoid cancellation in the loss value
    a = rng.standard_normal((N, M))
    adj = R.adjoint(U0, Gv, Gh, Cv, Ch, eps, a, weights=(wv, wh))
    # h = 1e-3: central-difference truncation ~1e-6 relative; smaller steps
    # drown in the dense solve's rounding (condition number ~1e4)
    h = 1e-3
    loss = lambda Uc: float(np.sum(a * Uc))  # noqa: E731
    for e in range(8):
        i, j = rng.integers(0, N - 1), rng.integers(0, M)
        Cp, Cm = Cv.copy(), Cv.copy()
        Cp[i, j] += h
        Cm[i, j] -= h
        fd = (loss(dense_frozen_solve(Cp, Ch, Gv, Gh, wv, wh))
              - loss(dense_frozen_solve(Cm, Ch, Gv, Gh, wv, wh))) / (2 * h)
        assert abs(fd - adj["gCv"][i, j]) <= 1e-5 * abs(fd) + 1e-11
    def safe(i, j):
        # +-h must not move any incident difference across the jump at +-pi
        d = []
        if i > 0:
            d.append(X[i, j] - X[i - 1, j])
        if i < N - 1:
            d.append(X[i + 1, j] - X[i, j])
        if j > 0:
            d.append(X[i, j] - X[i, j - 1])
        if j < M - 1:
            d.append(X[i, j + 1] - X[i, j])
        return np.min(np.abs(np.abs(d) - PI)) > 10 * h

    done = 0
    while done < 8:
        i, j = rng.integers(0, N), rng.integers(0, M)
        if not safe(i, j):
            continue
        done += 1
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        Gp, Gm = R.wrapped_gradients(Xp), R.wrapped_gradients(Xm)
        fd = (loss(dense_frozen_solve(Cv, Ch, *Gp, wv, wh))
              - loss(dense_frozen_solve(Cv, Ch, *Gm, wv, wh))) / (2 * h)
        assert abs(fd - adj["gX"][i, j]) <= 1e-5 * abs(fd) + 1e-11
    i, j = 2, 3
    Hp, Hm = Ch.copy(), Ch.copy()
    Hp[i, j] += h
    Hm[i, j] -= h
    fd = (loss(dense_frozen_solve(Cv, Hp, Gv, Gh, wv, wh))
          - loss(dense_frozen_solve(Cv, Hm, Gv, Gh, wv, wh))) / (2 * h)
    assert abs(fd - adj["gCh"][i, j]) <= 1e-5 * abs(fd) + 1e-11


def test_irls_returns_mean_zero_from_any_start():
    f = synth.field_c2(1, 20, 18)
    U, _ = R.irls(f.X, w=f.w, iters=2, tol=1e-10, maxit=50, U0=np.full((20, 18), 5.0))
    assert abs(U.mean()) < 1e-12


def test_frozen_solve_correction_from_a_start_point():
    """frozen_solve with x0 solves the correction from x0 (to tol of its own
    right-hand side): for any start point it gives the cold solve's mean-zero
    minimiser, and for a perturbed weight started at the unperturbed
    solution it gives the dense bordered solve of the perturbed problem."""
    N, M = 20, 17
    rng = np.random.default_rng(41)
    X = R.wrap(rng.normal(0, 2.0, (N, M)))
    Gv, Gh = R.wrapped_gradients(X)
    Cv = rng.uniform(0.2, 1.0, (N - 1, M))
    Ch = rng.uniform(0.2, 1.0, (N, M - 1))
    wv = 1.0 / np.maximum(np.abs(rng.normal(0, 1, (N - 1, M))), 1e-3)
    wh = 1.0 / np.maximum(np.abs(rng.normal(0, 1, (N, M - 1))), 1e-3)
    cold = R.frozen_solve(Cv, Ch, Gv, Gh, wv, wh, tol=1e-14, maxit=5000)
    assert np.abs(cold - dense_frozen_solve(Cv, Ch, Gv, Gh, wv, wh)).max() < 1e-9
    warm = R.frozen_solve(Cv, Ch, Gv, Gh, wv, wh, tol=1e-14, maxit=5000,
                          x0=rng.normal(0, 5.0, (N, M)))
    assert np.abs(warm - cold).max() < 1e-9
    Cp = Cv.copy()
    Cp[3, 4] += 1e-3
    pert = R.frozen_solve(Cp, Ch, Gv, Gh, wv, wh, tol=1e-14, maxit=5000, x0=cold)
    dense = dense_frozen_solve(Cp, Ch, Gv, Gh, wv, wh)
    # the change itself (not only the solution) is resolved
    assert np.abs((pert - cold) - (dense - cold)).max() <= 1e-6 * np.abs(dense - cold).max()
