"""Oracle: generic number-conserving local operators, y = O x by definition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  FP64 (or complex128) throughout.

The operator class of Sec. 4.1 builds a Hamiltonian from strings of local
operators (S+, S-, Sz and user-defined local matrices) on lists of sites;
App. C stores the sum of the terms that live inside one cluster of sites as one
sparse matrix.  Here an operator is a list of terms (coef, sites, M): M is a
Q^m x Q^m matrix acting on the digits of the m listed sites, <b|M|a>, with the
local index of a digit string (d_0, ..., d_{m-1}) over those sites being
sum_j d_j Q^(m-1-j) (the first listed site most significant).  The operator is

    O = sum_t coef_t M_t      (each M_t with the identity on every other site).

A term conserves the particle number when every nonzero <b|M|a> joins digit
strings of equal sums; only such terms map a U(1) sector into itself.

Matrices may be complex (the operator's scalar type of Sec. 4.1 is real or complex);
the product is then complex.  ``spin_matrices`` also gives Sx = (S+ + S-)/2 and
Sy = (S+ - S-)/(2i).

The oracle applies the terms one by one in the push form (every basis state of
the sector sends coef <b|M|a> x_s to the state with the term's digits replaced);
it merges nothing.  ``full_space_matrix`` builds the same operator on the whole
Q^L space from tensor reshapes alone (no state arithmetic), as an independent pin.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import ladder_down, ladder_up, spin
from .sector import BruteSector, nbits_for


def spin_matrices(Q: int) -> dict:
    """Single-site matrices on digits 0..Q-1 (m = d - S): Id, Sz, S+ (raises d by one),
    S- (lowers it), with the ladder factors of the XXZ oracle, and Sx, Sy (complex)."""
    S = spin(Q)
    sz = np.diag([d - S for d in range(Q)])
    sp = np.zeros((Q, Q))
    sm = np.zeros((Q, Q))
    for d in range(Q - 1):
        sp[d + 1, d] = ladder_up(Q, d)
    for d in range(1, Q):
        sm[d - 1, d] = ladder_down(Q, d)
    return {"Id": np.eye(Q), "Sz": sz, "S+": sp, "S-": sm, "Sx": (sp + sm) / 2, "Sy": (sp - sm) / 2j}


def string(coef: float, sites, names, Q: int):
    """The term coef * (op_0 on sites[0]) (op_1 on sites[1]) ...: the Kronecker product of
    the named single-site matrices, first site most significant."""
    mats = spin_matrices(Q)
    M = np.ones((1, 1))
    for nm in names:
        M = np.kron(M, mats[nm])
    return (float(coef), tuple(int(s) for s in sites), M)


def conserves(Q: int, m: int, M) -> bool:
    """True when every nonzero <b|M|a> joins local digit strings of equal digit sums."""
    def dsum(a):
        s = 0
        for _ in range(m):
            s += a % Q
            a //= Q
        return s
    rows, cols = np.nonzero(np.asarray(M))
    return all(dsum(int(b)) == dsum(int(a)) for b, a in zip(rows, cols))


def apply_operator(bs: BruteSector, terms, x):
    """y = O x on the sector of ``bs`` (rows in its canonical order), x of shape [D];
    FP64, or complex128 when x or a matrix is complex."""
    Q, L = bs.Q, bs.L
    nb = nbits_for(Q)
    dmask = np.uint64((1 << nb) - 1)
    x = np.asarray(x)
    x = x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)
    cplx = np.iscomplexobj(x) or any(np.iscomplexobj(M) for _, _, M in terms)
    st = bs.states
    y = np.zeros(bs.dim, dtype=np.complex128 if cplx else np.float64)
    for coef, sites, M in terms:
        m = len(sites)
        M = np.asarray(M)
        M = M.astype(np.complex128 if np.iscomplexobj(M) else np.float64)
        if M.shape != (Q ** m, Q ** m):
            raise ValueError("term matrix shape")
        if not conserves(Q, m, M):
            raise ValueError("term does not conserve the particle number")
        shifts = [np.uint64(nb * (L - 1 - s)) for s in sites]
        a = np.zeros(bs.dim, dtype=np.int64)
        for sh in shifts:
            a = a * Q + ((st >> sh) & dmask).astype(np.int64)
        keep = st.copy()
        for sh in shifts:
            keep &= ~(dmask << sh)
        for bl, al in zip(*np.nonzero(M)):
            rows = np.nonzero(a == al)[0]
            if rows.size == 0:
                continue
            new = keep[rows].copy()
            v = int(bl)
            for j in range(m - 1, -1, -1):  # the last listed site is the least significant digit
                new |= np.uint64(v % Q) << shifts[j]
                v //= Q
            y[bs.rank(new)] += coef * M[bl, al] * x[rows]
    return y


def full_space_matrix(Q: int, L: int, terms):
    """O on the whole Q^L space (basis index sum_i d_i Q^(L-1-i)), by contracting each
    term's matrix into the tensor legs of its sites."""
    dim = Q ** L
    cplx = any(np.iscomplexobj(M) for _, _, M in terms)
    out = np.zeros((dim, dim), dtype=np.complex128 if cplx else np.float64)
    for coef, sites, M in terms:
        m = len(sites)
        T = np.asarray(M).reshape([Q] * (2 * m))  # out legs, then in legs
        eye = np.eye(dim).reshape([Q] * L + [dim])
        # apply the term to every basis column: contract its in legs with the sites' legs
        res = np.tensordot(T, eye, axes=(list(range(m, 2 * m)), list(sites)))
        # res legs: the term's out legs, the remaining site legs in order, the column
        rest = [i for i in range(L) if i not in sites]
        order = [0] * L
        for j, s in enumerate(sites):
            order[s] = j
        for r, s in enumerate(rest):
            order[s] = m + r
        res = np.transpose(res, order + [L]).reshape(dim, dim)
        out += coef * res
    return out


def sector_matrix(bs: BruteSector, terms):
    """O restricted to the sector, from the full-space matrix (rows and columns of the
    sector's basis states)."""
    Q, L = bs.Q, bs.L
    nb = nbits_for(Q)
    dmask = np.uint64((1 << nb) - 1)
    idx = np.zeros(bs.dim, dtype=np.int64)
    for i in range(L):
        idx = idx * Q + ((bs.states >> np.uint64(nb * (L - 1 - i))) & dmask).astype(np.int64)
    F = full_space_matrix(Q, L, terms)
    return F[np.ix_(idx, idx)]


def lindbladian_dense(bs: BruteSector, h_terms, jumps, rho):
    """L[rho] = -i [H, rho] + sum_k g_k (A_k rho A_k^+ - 1/2 {A_k^+ A_k, rho}) (the
    Lindblad form the paper's operator class targets, Sec. 4.1), with H and every jump
    operator A_k = coef_k M_k given as terms on the sector of ``bs`` (A_k must conserve
    the particle number so that the (n, n) block of rho maps to itself).  Dense
    matrices in the sector basis; ``jumps`` is a list of (g_k, term)."""
    H = sector_matrix(bs, h_terms)
    rho = np.asarray(rho, dtype=np.complex128)
    out = -1j * (H @ rho - rho @ H)
    for g, term in jumps:
        A = sector_matrix(bs, [term])
        AdA = A.conj().T @ A
        out += g * (A @ rho @ A.conj().T - 0.5 * (AdA @ rho + rho @ AdA))
    return out
