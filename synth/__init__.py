"""Seeded synthetic InSAR-shaped phase fields (inputs only).

This module draws a true phase field, turns it into the observed wrapped
phase of an interferogram sample (the argument of exp(i*phi)), and draws
per-pixel coherence weights or per-edge weights.  It contains none of the
unwrapping method's arithmetic; it is the one module shared by the oracle,
the tests and the benchmark, so both sides of every parity check see the
same bits.

Draw order inside every generator is fixed (numpy PCG64 via
``numpy.random.default_rng``):

1. Gaussian centres (row, then column), 2. amplitudes, 3. widths,
4. ramp direction, 5. additive noise, 6. extras (step line, band line,
band phases, salt mask and phases, weights, edge logits) in that order.

The paper's own workloads (Sentinel-1 crops of 2048 x 2048 and burst
stitches of about 4000 x 20000, Section 4.1) are not available; these
fields stand in for them with topography-like Gaussian bumps, an orbital
ramp, phase noise, discontinuities and decorrelated areas.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Field", "gaussian_sum_field", "observe", "field_c1", "field_c2",
    "field_c3", "tile_shapes_c4", "field_c4_tile", "field_c5", "smooth_field",
]


@dataclasses.dataclass
class Field:
    """One synthetic problem instance.

    phi: true (unwrapped) phase, float64 N x M.
    X:   observed wrapped phase in (-pi, pi], float64 N x M.
    w:   optional per-pixel weights (> 0), float64 N x M.
    Cv, Ch: optional per-edge weights, float64 (N-1) x M and N x (M-1).
    meta: generator name, seed and parameters.
    """
    phi: np.ndarray
    X: np.ndarray
    w: Optional[np.ndarray] = None
    Cv: Optional[np.ndarray] = None
    Ch: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)


def observe(phi: np.ndarray) -> np.ndarray:
    """Observed interferogram phase: arg(exp(i*phi)) in (-pi, pi]."""
    return np.arctan2(np.sin(phi), np.cos(phi))


def gaussian_sum_field(rng, N, M, n_gauss=8, amp=20.0, sigma=(15.0, 60.0),
                       ramp=0.05, noise=0.3):
    """Sum of isotropic 2-D Gaussians + linear ramp + i.i.d. Gaussian noise.

    Draws, in order: centres (rows, columns), amplitudes U(-amp, amp),
    widths U(sigma), ramp direction U[0, 2pi), noise N(0, noise^2).
    """
    ci = rng.uniform(0.0, N, n_gauss)
    cj = rng.uniform(0.0, M, n_gauss)
    a = rng.uniform(-amp, amp, n_gauss)
    s = rng.uniform(sigma[0], sigma[1], n_gauss)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    ii = np.arange(N, dtype=np.float64)
    jj = np.arange(M, dtype=np.float64)
    phi = np.zeros((N, M), dtype=np.float64)
    for g in range(n_gauss):
        gi = np.exp(-0.5 * ((ii - ci[g]) / s[g]) ** 2)
        gj = np.exp(-0.5 * ((jj - cj[g]) / s[g]) ** 2)
        phi += a[g] * np.outer(gi, gj)
    phi += ramp * (np.cos(theta) * ii[:, None] + np.sin(theta) * jj[None, :])
    if noise > 0:
        phi += rng.normal(0.0, noise, (N, M))
    return phi


def _line_side(N, M, pi_, pj, psi):
    ii = np.arange(N, dtype=np.float64)[:, None]
    jj = np.arange(M, dtype=np.float64)[None, :]
    return (ii - pi_) * np.sin(psi) - (jj - pj) * np.cos(psi)


def field_c1(seed: int, N: int = 256, M: int = 256) -> Field:
    """Small plain case: 8 Gaussians (+-20 rad, widths 15-60 px), ramp
    0.05 rad/px, N(0, 0.3^2) noise, unit weights."""
    rng = np.random.default_rng(seed)
    phi = gaussian_sum_field(rng, N, M, amp=20.0, noise=0.3)
    return Field(phi=phi, X=observe(phi),
                 meta=dict(gen="c1", seed=seed, N=N, M=M))


def field_c2(seed: int, N: int = 2048, M: int = 2048, band: int = 64) -> Field:
    """Plain FP32 case: Gaussians (+-80 rad), N(0, 0.5^2) noise, a 3*pi
    step on one side of a seeded line, a decorrelated band of uniform
    random phase, per-pixel Beta(2,2) coherence (0.05 inside the band)."""
    rng = np.random.default_rng(seed)
    phi = gaussian_sum_field(rng, N, M, amp=80.0, noise=0.5)
    # step line through a uniform point, angle U[0, pi)
    sp = (rng.uniform(0.0, N), rng.uniform(0.0, M), rng.uniform(0.0, np.pi))
    phi += 3.0 * np.pi * (_line_side(N, M, *sp) > 0)
    # decorrelated band centred on a second seeded line
    bp = (rng.uniform(0.0, N), rng.uniform(0.0, M), rng.uniform(0.0, np.pi))
    in_band = np.abs(_line_side(N, M, *bp)) < 0.5 * band
    n_band = int(in_band.sum())
    phi[in_band] = rng.uniform(-np.pi, np.pi, n_band)
    w = rng.beta(2.0, 2.0, (N, M))
    w[in_band] = 0.05
    return Field(phi=phi, X=observe(phi), w=w,
                 meta=dict(gen="c2", seed=seed, N=N, M=M, band=band))


def field_c3(seed: int, N: int = 8192, M: int = 8192, salt: float = 0.02) -> Field:
    """Burst-sized fringe-dense case: Gaussians (+-400 rad), N(0, 0.7^2)
    noise, 2% salt pixels of uniform phase, Beta(2,2) weights."""
    rng = np.random.default_rng(seed)
    phi = gaussian_sum_field(rng, N, M, amp=400.0, noise=0.7)
    mask = rng.random((N, M)) < salt
    phi[mask] = rng.uniform(-np.pi, np.pi, int(mask.sum()))
    w = rng.beta(2.0, 2.0, (N, M))
    return Field(phi=phi, X=observe(phi), w=w,
                 meta=dict(gen="c3", seed=seed, N=N, M=M, salt=salt))


def tile_shapes_c4(master_seed: int = 0, ntiles: int = 64, lo: int = 512,
                   hi: int = 3072) -> np.ndarray:
    """Uneven tile shapes: (ntiles, 2) int64, sides iid uniform in [lo, hi]."""
    rng = np.random.default_rng(master_seed)
    return rng.integers(lo, hi + 1, size=(ntiles, 2)).astype(np.int64)


def field_c4_tile(t: int, N: int, M: int) -> Field:
    """Tile t of the batched case: the small-case generator with seed 1000+t."""
    f = field_c1(1000 + t, N, M)
    f.meta.update(gen="c4", tile=t)
    return f


def field_c5_truth(seed: int, N: int = 1024, M: int = 1024) -> np.ndarray:
    """The noise-free phase of field_c5(seed): the same Gaussians and ramp
    (the noise is the last draw of the phase, so the same stream without it
    gives the signal the noise was added to)."""
    rng = np.random.default_rng(seed)
    return gaussian_sum_field(rng, N, M, amp=20.0, noise=0.0)


def field_c5(seed: int, N: int = 1024, M: int = 1024) -> Field:
    """Differentiation case: small-case generator plus per-edge weights
    sigmoid(z), z ~ N(0, 1), drawn after the phase."""
    f = field_c1(seed, N, M)
    rng = np.random.default_rng(seed)
    # advance past the phase draws so the logits are a fresh stream
    gaussian_sum_field(rng, N, M, amp=20.0, noise=0.3)
    zv = rng.normal(0.0, 1.0, (N - 1, M))
    zh = rng.normal(0.0, 1.0, (N, M - 1))
    f.Cv = 1.0 / (1.0 + np.exp(-zv))
    f.Ch = 1.0 / (1.0 + np.exp(-zh))
    f.meta.update(gen="c5", zv=zv, zh=zh)
    return f


def smooth_field(seed: int, N: int, M: int, amp: float = 2.0) -> Field:
    """Noise-free smooth field whose neighbour differences stay well below
    pi (the Itoh condition holds), for the integration special case."""
    rng = np.random.default_rng(seed)
    phi = gaussian_sum_field(rng, N, M, n_gauss=4, amp=amp,
                             sigma=(max(3.0, N / 6), max(4.0, N / 3)),
                             ramp=0.3, noise=0.0)
    return Field(phi=phi, X=observe(phi),
                 meta=dict(gen="smooth", seed=seed, N=N, M=M))
