"""Closed-form reference values used as pins (not the method itself).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  FP64.

bethe_e0(L): ground energy of the periodic spin-1/2 Heisenberg chain (J = 1,
Delta = 1) in the sector n = L/2 from the logarithmic Bethe equations
    2 L arctan(2 l_j) = 2 pi I_j + 2 sum_k arctan(l_j - l_k),  I_j = j - (M - 1)/2,
    E0 = L/4 - sum_j 2 / (1 + 4 l_j^2),
M = L/2 rapidities, solved by Newton-type iteration from the free-magnon guess.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize


def bethe_e0(L: int) -> float:
    if L % 2:
        raise ValueError("L must be even")
    M = L // 2
    I = np.arange(M) - (M - 1) / 2.0

    def eqs(lam):
        d = lam[:, None] - lam[None, :]
        return 2 * L * np.arctan(2 * lam) - 2 * np.pi * I - 2 * np.arctan(d).sum(axis=1)

    lam = scipy.optimize.fsolve(eqs, 0.5 * np.tan(np.pi * I / L), xtol=1e-13)
    if np.max(np.abs(eqs(lam))) > 1e-10:
        raise RuntimeError("Bethe equations did not converge")
    return float(L / 4 - np.sum(2 / (1 + 4 * lam ** 2)))
