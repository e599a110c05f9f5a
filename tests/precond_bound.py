"""Element-wise error bound for the preconditioner z = L^+ r (test helper).

The map (Section 3.3, eq:eigendecompositions; Appendix B for the zero mode):

    R1 = r P_M            (DCT-II along rows)
    Rh = P_N^T R1         (DCT-II along columns)
    Zh = Rh ./ (lambda_k + mu_l),  Zh[0, 0] = 0
    Z1 = P_N Zh           (DCT-III along columns)
    z  = Z1 P_M^T         (DCT-III along rows)

Every implementation computes these five stages in some order, rounding at
each one: the arithmetic of a transform, the storage of an intermediate in
a narrower type, the rounding of a basis to the operand type.  The bound
here follows the probabilistic model of rounding errors (Higham and Mary,
"A new approach to probabilistic rounding error analysis", SIAM J. Sci.
Comput. 2019): each rounding is an independent error of mean zero and
magnitude at most u |x|, hence variance at most u^2 x^2 / 3.  The variance
each error source puts on z_ij is propagated exactly through the remaining
linear map and then bounded uniformly with |P[i, k]|^2 <= 2 / n:

* an error field e in the Rh domain (before the division) reaches z_ij as
  sum_kl P_ik P_jl e_kl / (lambda_k + mu_l): variance at most
  (4 / NM) sum_kl var(e_kl) W_kl, W = 1 / (lambda + mu)^2 (W_00 = 0);
* an error field in the R1 domain (rows spatial) first maps to the
  spectral domain by an orthonormal transform of its columns:
  var(e_hat_kl) <= (2 / N) sum_i var(e_il), then as above;
* an error in the r domain maps by both transforms:
  var(e_hat_kl) <= (4 / NM) sum var(e), then as above;
* an error in Zh (after the division): variance at most (4 / NM) sum var;
* an error in Z1 (rows spatial, after the column inverse) reaches z_ij
  through row i's DCT-III: at most (2 / M) sum_l var(e_il);
* an error in z itself stays where it is.

A transform of length n computed by a fast algorithm in unit roundoff u
has a normwise error of at most about c u log2(n) relative to its input
(Cooley-Tukey with accurately rounded twiddles, c about 6.7; Higham,
"Accuracy and Stability of Numerical Algorithms", 2nd ed., Section 24.1);
the model spreads that error evenly over the outputs of the line.  A
product with a basis rounded to u contributes, per output,
(u^2 / 3) sum_i P_ik^2 x_i^2 <= (2 u^2 / 3) mean(x^2) of its input line;
its accumulation in unit roundoff u_acc at most (u_acc^2 / 6) ||x||^2
(recursive summation of terms of random sign).

The bound returned is kappa * sigma_ij with sigma_ij^2 the sum of all
contributions; kappa = 8 leaves a Gaussian tail of 1e-15 per element.
16-bit storage with an input scale s (the FP16 plans scale r to an rms of
1e-3 before the first transform) rounds with an absolute floor of
2^-14 / s (the smallest normal FP16 number, in unscaled units).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

# unit roundoff (round to nearest) of each storage / arithmetic type
UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
FFT_C = 6.7
KAPPA = 8.0


def _eig(n):
    k = np.arange(n, dtype=np.float64)
    return 4.0 * np.sin(math.pi * k / (2.0 * n)) ** 2


def stages(r, workers=None):
    """FP64 intermediates R1, Rh, Zh, Z1, z of the map (scipy's orthonormal
    DCT, the oracle's route)."""
    r = np.asarray(r, np.float64)
    R1 = scipy.fft.dct(r, type=2, norm="ortho", axis=1, workers=workers)
    Rh = scipy.fft.dct(R1, type=2, norm="ortho", axis=0, workers=workers)
    lam = _eig(r.shape[0])[:, None] + _eig(r.shape[1])[None, :]
    lam[0, 0] = np.inf
    Zh = Rh / lam
    Z1 = scipy.fft.idct(Zh, type=2, norm="ortho", axis=0, workers=workers)
    z = scipy.fft.idct(Z1, type=2, norm="ortho", axis=1, workers=workers)
    W = 1.0 / lam ** 2
    return dict(r=r, R1=R1, Rh=Rh, Zh=Zh, Z1=Z1, z=z, W=W)


class _Acc:
    """Accumulates variance contributions per domain and propagates them."""

    def __init__(self, S):
        self.S = S
        self.N, self.M = S["z"].shape
        self.pre_spec = np.zeros((self.N, self.M))   # spectral-domain variance before division
        self.post_const = 0.0                        # uniform variance on z
        self.row = np.zeros(self.N)                  # per-row variance on z
        self.elem = np.zeros((self.N, self.M))       # per-element variance on z

    # contributions, each given as a variance array broadcastable to N x M
    def add_r(self, var):
        var = np.broadcast_to(var, (self.N, self.M))
        self.pre_spec += 4.0 / (self.N * self.M) * float(np.sum(var))

    def add_R1(self, var):
        var = np.broadcast_to(var, (self.N, self.M))
        self.pre_spec += (2.0 / self.N) * np.sum(var, axis=0)[None, :]

    def add_Rh(self, var):
        self.pre_spec += np.broadcast_to(var, (self.N, self.M))

    def add_Zh(self, var):
        var = np.broadcast_to(var, (self.N, self.M))
        self.post_const += 4.0 / (self.N * self.M) * float(np.sum(var))

    def add_Z1(self, var):
        var = np.broadcast_to(var, (self.N, self.M))
        self.row += (2.0 / self.M) * np.sum(var, axis=1)

    def add_z(self, var):
        self.elem += np.broadcast_to(var, (self.N, self.M))

    def sigma(self):
        pre = 4.0 / (self.N * self.M) * float(np.sum(self.pre_spec * self.S["W"]))
        return np.sqrt(pre + self.post_const + self.row[:, None] + self.elem)


def _ms_rows(A):
    return np.mean(A * A, axis=1, keepdims=True)


def _ms_cols(A):
    return np.mean(A * A, axis=0, keepdims=True)


def _store_var(A, u, floor):
    a = np.maximum(np.abs(A), floor)
    return u * u * a * a / 3.0


def fp16_floor(r):
    """Smallest normal FP16 value in unscaled units, for the input scale
    s = 1e-3 sqrt(N M / ||r||^2) of the FP16 plans."""
    r = np.asarray(r, np.float64)
    s = 1e-3 * math.sqrt(r.size / float(np.sum(r * r)))
    return 2.0 ** -14 / s


def sigma_fast(S, arith, store, vec, floor=0.0):
    """Fast form: FFT-based DCT-II / DCT-III of each line in unit roundoff
    `arith`, the intermediates after the row DCT-II and after the column
    DCT-III stored in `store`, z stored in `vec`."""
    A = _Acc(S)
    N, M = A.N, A.M
    ua, us, uv = UNIT[arith], UNIT[store], UNIT[vec]
    cM, cN = FFT_C * ua * math.log2(M), FFT_C * ua * math.log2(N)
    A.add_R1(cM * cM * _ms_rows(S["r"]) + _store_var(S["R1"], us, floor))
    A.add_Rh(cN * cN * _ms_cols(S["R1"]))
    A.add_Zh(ua * ua * S["Zh"] ** 2 / 3.0)
    A.add_Z1(cN * cN * _ms_cols(S["Zh"]) + _store_var(S["Z1"], us, floor))
    A.add_z(cM * cM * _ms_rows(S["Z1"]) + uv * uv * S["z"] ** 2 / 3.0)
    return A.sigma()


def sigma_products(S, op, acc, vec, floor=0.0, folded=False):
    """Dense (or folded) form: four products with the cosine bases rounded
    to `op`, accumulated in `acc`; r and every intermediate rounded to `op`,
    z stored in `vec`.  The folded form splits each product into sum /
    difference halves: every operand rounding then sees the sum of two
    values and the half-size basis products twice the dense terms, so its
    operand-rounding variances are taken four times those of the dense
    form."""
    A = _Acc(S)
    N, M = A.N, A.M
    uo, ua, uv = UNIT[op], UNIT[acc], UNIT[vec]
    f = 4.0 if folded else 1.0
    same = op == vec
    # input rounding of r to the operand type (none when they coincide)
    if not same:
        A.add_r(f * _store_var(S["r"], uo, floor))
    # G1: rows
    A.add_R1(f * (2.0 * uo * uo / 3.0) * _ms_rows(S["r"]) + (ua * ua / 6.0) * M * _ms_rows(S["r"])
             + f * _store_var(S["R1"], uo, floor))
    # G2: columns, then the division; the result is stored in the operand type
    A.add_Rh(f * (2.0 * uo * uo / 3.0) * _ms_cols(S["R1"]) + (ua * ua / 6.0) * N * _ms_cols(S["R1"]))
    A.add_Zh(f * _store_var(S["Zh"], uo, floor) + ua * ua * S["Zh"] ** 2 / 3.0)
    # G3: columns inverse
    A.add_Z1(f * (2.0 * uo * uo / 3.0) * _ms_cols(S["Zh"]) + (ua * ua / 6.0) * N * _ms_cols(S["Zh"])
             + f * _store_var(S["Z1"], uo, floor))
    # G4: rows inverse, z in the vector type
    A.add_z(f * (2.0 * uo * uo / 3.0) * _ms_rows(S["Z1"]) + (ua * ua / 6.0) * M * _ms_rows(S["Z1"])
            + f * uv * uv * S["z"] ** 2 / 3.0)
    return A.sigma()


def plan_sigma(S, form, prec, r=None):
    """sigma of z for a plan of precision prec ('f64', 'f32', 'bf16',
    'f16') and preconditioner form ('fast', 'dense', 'folded')."""
    vec = "f64" if prec == "f64" else "f32"
    floor = fp16_floor(S["r"] if r is None else r) if prec == "f16" else 0.0
    if form == "fast":
        arith = "f64" if prec == "f64" else "f32"
        return sigma_fast(S, arith, prec, vec, floor)
    acc = "f64" if prec == "f64" else "f32"
    return sigma_products(S, prec, acc, vec, floor, folded=(form == "folded"))


def check(zg, S, sigma, kappa=KAPPA):
    """Return (ok, worst ratio |z_gpu - z| / sigma, its index)."""
    err = np.abs(np.asarray(zg, np.float64) - S["z"])
    ratio = err / sigma
    idx = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    worst = float(ratio[idx])
    return worst <= kappa, worst, idx
