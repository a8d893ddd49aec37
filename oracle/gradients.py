"""Oracle: derivatives of y = H(theta) x and of the ground energy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  FP64.

H is linear in the couplings, H = sum_b (Jxy_b A_b + Jz_b Z_b) + sum_i h_i Sz_i with
A_b = (S+_i S-_j + S-_i S+_j)/2 and Z_b = Sz_i Sz_j, and real symmetric.  For a
scalar loss with upstream gradient g = dLoss/dy:

    dLoss/dx      = H^T g = H g
    dLoss/dJxy_b  = g . (A_b x)
    dLoss/dJz_b   = g . (Z_b x)
    dLoss/dh_i    = g . (Sz_i x)

Hellmann-Feynman: for a normalised, non-degenerate ground vector psi0,
dE0/dJxy_b = psi0 . A_b psi0 and dE0/dJz_b = psi0 . Z_b psi0.
With Jxy = J and Jz = J Delta:  d/dJ = d/dJxy + Delta d/dJz,  d/dDelta = J d/dJz.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import apply_h


def adjoint(bs, bonds, jxy, jz, x, g, h=None):
    grad_x = apply_h(bs, bonds, jxy, jz, g, h)
    nb = len(bonds)
    gj = np.zeros(nb)
    gz = np.zeros(nb)
    for b in range(nb):
        gj[b] = float(np.sum(g * apply_h(bs, [bonds[b]], [1.0], [0.0], x)))
        gz[b] = float(np.sum(g * apply_h(bs, [bonds[b]], [0.0], [1.0], x)))
    gh = None
    if h is not None:
        gh = np.zeros(bs.L)
        for i in range(bs.L):
            e = np.zeros(bs.L)
            e[i] = 1.0
            gh[i] = float(np.sum(g * apply_h(bs, [], [], [], x, e)))
    return grad_x, gj, gz, gh


def chain_rule_j_delta(J, Delta, g_jxy, g_jz):
    """Map gradients w.r.t. (Jxy, Jz) to (J, Delta) for Jxy = J, Jz = J*Delta."""
    J = np.asarray(J)
    Delta = np.asarray(Delta)
    return g_jxy + Delta * g_jz, J * g_jz


def hellmann_feynman(bs, bonds, psi0):
    psi0 = psi0 / np.linalg.norm(psi0)
    _, gj, gz, _ = adjoint(bs, bonds, np.zeros(len(bonds)), np.zeros(len(bonds)), psi0, psi0)
    return gj, gz
