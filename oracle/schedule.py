"""Adaptive CG-iteration schedule and IRLS stop rule of Section 4.3.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

m_CG(0) is given.  For k >= 1 the relative improvement
Delta_{k-1,k} = (H(U^k, W^{k-1}) - H(U^k, W^k)) / H(U^k, W^{k-1}) of the
surrogate H (the function minimised in (prob:alt1)) is compared with
eps_tol:

1. Delta > eps_tol: keep m_CG(k) = m_CG(k-1);
2. Delta <= eps_tol and m_CG(k-1) != m_CG(k-2): stop and return U^k;
3. Delta <= eps_tol and m_CG(k-1) == m_CG(k-2): m_CG(k) = alpha m_CG(k-1).

Readings where the paper is silent: at k = 1 the missing m_CG(-1) is taken
equal to m_CG(0) (so rule 3 can fire); alpha m is rounded up to an integer.
The paper's settings are m_CG(0) = 5, eps_tol = 1e-3, alpha = 1.7.
"""
from __future__ import annotations

import math


class CgSchedule:
    def __init__(self, m0=5, eps_tol=1e-3, alpha=1.7):
        self.eps_tol, self.alpha = eps_tol, alpha
        self.m = [int(m0)]

    def current(self):
        return self.m[-1]

    def update(self, delta):
        """Feed Delta_{k-1,k}; returns the new m_CG(k), or None to stop."""
        prev = self.m[-1]
        prev2 = self.m[-2] if len(self.m) >= 2 else self.m[-1]
        if delta > self.eps_tol:
            self.m.append(prev)
        elif prev != prev2:
            return None
        else:
            self.m.append(int(math.ceil(self.alpha * prev)))
        return self.m[-1]


def relative_improvement(h_old_weights, h_new_weights):
    return (h_old_weights - h_new_weights) / h_old_weights
