"""Oracle: XXZ matrix elements and the matrix-free product y = H x by definition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  FP64 throughout.

Hamiltonian (eq. H_30 and the App. D example, with per-bond couplings):

    H = sum_b [ Jxy_b/2 (S+_i S-_j + S-_i S+_j) + Jz_b Sz_i Sz_j ] + sum_i h_i Sz_i

on a bond list b = (i, j).  Spin S = (Q-1)/2; a site with digit d has
m = d - S, Sz = m, and the ladder factors
    S+ |m> = sqrt(S(S+1) - m(m+1)) |m+1>,   S- |m> = sqrt(S(S+1) - m(m-1)) |m-1>.
A model given by (J_b, Delta_b) has Jxy_b = J_b and Jz_b = J_b * Delta_b.

H is real symmetric, so row s of H x is  sum_{s'} <s'|H|s> x_{s'}: apply H to the
basis state of the row and gather x at the rank of every state it reaches.
"""
from __future__ import annotations

import math

import numpy as np

from .sector import BruteSector, nbits_for, unpack


def spin(Q: int) -> float:
    return (Q - 1) / 2.0


def ladder_up(Q: int, d: int) -> float:
    S, m = spin(Q), d - spin(Q)
    return math.sqrt(max(0.0, S * (S + 1) - m * (m + 1)))


def ladder_down(Q: int, d: int) -> float:
    S, m = spin(Q), d - spin(Q)
    return math.sqrt(max(0.0, S * (S + 1) - m * (m - 1)))


def apply_to_state(state: int, Q: int, L: int, bonds, jxy, jz, h=None):
    """H |s> for one basis state: (diagonal element, list of (s', amplitude))."""
    d = unpack(state, Q, L)
    S = spin(Q)
    nb = nbits_for(Q)
    diag = 0.0
    out = []
    for b, (i, j) in enumerate(bonds):
        diag += jz[b] * (d[i] - S) * (d[j] - S)
        for (a, c) in ((i, j), (j, i)):          # S+_a S-_c
            if d[a] < Q - 1 and d[c] > 0:
                amp = 0.5 * jxy[b] * ladder_up(Q, d[a]) * ladder_down(Q, d[c])
                sp = state + (1 << (nb * (L - 1 - a))) - (1 << (nb * (L - 1 - c)))
                out.append((sp, amp))
    if h is not None:
        for i in range(L):
            diag += h[i] * (d[i] - S)
    return diag, out


def apply_h(bs: BruteSector, bonds, jxy, jz, x, h=None):
    """y = H x on the sector of ``bs`` (rows in its canonical order), FP64.

    x has shape [D] or [D, k].  Vectorised over rows, one bond and one hop
    direction at a time; ranks come from the brute-force sorted order.
    """
    Q, L = bs.Q, bs.L
    nb = nbits_for(Q)
    S = spin(Q)
    x = np.asarray(x, dtype=np.float64)
    st = bs.states
    dmask = np.uint64((1 << nb) - 1)
    dig = [((st >> np.uint64(nb * (L - 1 - i))) & dmask).astype(np.int64) for i in range(L)]
    up = np.array([ladder_up(Q, q) for q in range(Q)])
    dn = np.array([ladder_down(Q, q) for q in range(Q)])
    diag = np.zeros(bs.dim)
    y = np.zeros_like(x)
    for b, (i, j) in enumerate(bonds):
        diag += jz[b] * (dig[i] - S) * (dig[j] - S)
        for (a, c) in ((i, j), (j, i)):
            rows = np.nonzero((dig[a] < Q - 1) & (dig[c] > 0))[0]
            if len(rows) == 0:
                continue
            sp = st[rows] + np.uint64(1 << (nb * (L - 1 - a))) - np.uint64(1 << (nb * (L - 1 - c)))
            cols = bs.rank(sp)
            assert np.all(cols >= 0)
            amp = 0.5 * jxy[b] * up[dig[a][rows]] * dn[dig[c][rows]]
            if x.ndim == 1:
                np.add.at(y, rows, amp * x[cols])
            else:
                np.add.at(y, rows, amp[:, None] * x[cols])
    if h is not None:
        for i in range(L):
            diag += h[i] * (dig[i] - S)
    if x.ndim == 1:
        y += diag * x
    else:
        y += diag[:, None] * x
    return y


def sector_matrix(bs: BruteSector, bonds, jxy, jz, h=None) -> np.ndarray:
    """Dense sector matrix, column c = H e_c, rows and columns in canonical order."""
    return apply_h(bs, bonds, jxy, jz, np.eye(bs.dim), h)


def full_matrix(Q: int, L: int, bonds, jxy, jz, h=None) -> np.ndarray:
    """Dense Q^L x Q^L matrix built column by column from digit strings, no sector index.

    Basis states are numbered by their base-Q value with site 0 most significant.
    """
    dim = Q ** L
    S = spin(Q)
    H = np.zeros((dim, dim))
    powers = [Q ** (L - 1 - i) for i in range(L)]
    for col in range(dim):
        d = [(col // powers[i]) % Q for i in range(L)]
        diag = 0.0
        for b, (i, j) in enumerate(bonds):
            diag += jz[b] * (d[i] - S) * (d[j] - S)
            for (a, c) in ((i, j), (j, i)):
                if d[a] < Q - 1 and d[c] > 0:
                    row = col + powers[a] - powers[c]
                    H[row, col] += 0.5 * jxy[b] * ladder_up(Q, d[a]) * ladder_down(Q, d[c])
        if h is not None:
            for i in range(L):
                diag += h[i] * (d[i] - S)
        H[col, col] += diag
    return H


def full_basis_digit_sums(Q: int, L: int) -> np.ndarray:
    """Digit sum of every full-space basis state, in the numbering of full_matrix."""
    vals = np.arange(Q ** L)
    s = np.zeros(Q ** L, dtype=np.int64)
    for _ in range(L):
        s += vals % Q
        vals //= Q
    return s
