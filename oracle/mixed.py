"""Oracle: sectors and local operators on sites of different local dimensions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain Python integers, numpy,
FP64 / complex128.

Sec. 5 remarks that the method extends to a local dimension q_i per site (mixed
spins, Bose-Fermi mixtures) at the cost of more bookkeeping, without writing it
out.  The definitions here are the single-Q ones with every Q made per site:

  * the sector holds the digit strings d with 0 <= d_i < q_i and sum_i d_i = n;
    its dimension is the coefficient of x^n in prod_i (1 + x + ... + x^(q_i - 1))
    (App. A's generating function, one factor per site);
  * a state is packed as for one Q with nb = ceil(log2 max_i q_i) bits per site,
    site 0 in the most significant field;
  * the canonical order is that of Sec. 3.1-3.2: P_0 varies slowest, inside each
    subsystem states go by local digit sum, then by word;
  * a local term's matrix has one row and one column per digit string on its
    listed sites, its local index the mixed-radix number of the digits with the
    first listed site most significant.

The sector is found by enumerating every digit string and sorting (no index
arithmetic); the operator is applied term by term in the push form, and also
built on the whole space from tensor contractions as an independent check.
"""
from __future__ import annotations

import itertools

import numpy as np

from .sector import canonical_keys, default_split, nbits_for, pack_array


def dim_poly(dims, n: int) -> int:
    """Coefficient of x^n in prod_i (1 + x + ... + x^(q_i - 1)), by exact polynomial
    multiplication with Python integers."""
    poly = [1]
    for q in dims:
        new = [0] * (len(poly) + q - 1)
        for a, c in enumerate(poly):
            for d in range(q):
                new[a + d] += c
        poly = new
    return poly[n] if 0 <= n < len(poly) else 0


def sector_digits(dims, n: int) -> np.ndarray:
    """Every digit string with d_i < dims[i] and digit sum n, shape [D, L] (any order)."""
    total = int(np.prod([int(q) for q in dims]))
    if total > 20_000_000:
        raise ValueError("sector too large for brute force")
    rows = [d for d in itertools.product(*[range(int(q)) for q in dims]) if sum(d) == n]
    return np.array(rows, dtype=np.int8).reshape(len(rows), len(dims))


class MixedSector:
    """Canonical order of a sector with per-site local dimensions, by a plain sort.

    rank(s) is the position of s in the sorted list (-1 if s is not in the sector),
    unrank(i) its i-th entry."""

    def __init__(self, dims, n: int, split=None):
        self.dims = [int(q) for q in dims]
        self.L, self.n = len(self.dims), n
        self.Q = max(self.dims)  # sets the packing width
        self.split = list(split) if split is not None else default_split(self.Q, self.L)
        if sum(self.split) != self.L:
            raise ValueError("split does not sum to L")
        st = pack_array(sector_digits(self.dims, n), self.Q)
        keys = canonical_keys(st, self.Q, self.split)
        order = np.lexsort(keys.T[::-1])
        self.states = st[order]
        self.dim = len(self.states)
        self._pos = {int(s): i for i, s in enumerate(self.states)}

    def rank(self, states) -> np.ndarray:
        return np.array([self._pos.get(int(s), -1) for s in np.asarray(states, dtype=np.uint64)], dtype=np.int64)

    def unrank(self, idx) -> np.ndarray:
        return self.states[np.asarray(idx, dtype=np.int64)]


def _digits_of(a: int, radices):
    """Mixed-radix digits of a, first position most significant."""
    out = []
    for q in reversed(radices):
        out.append(a % q)
        a //= q
    return out[::-1]


def conserves(radices, M) -> bool:
    """True when every nonzero <b|M|a> joins digit strings of equal digit sums."""
    rows, cols = np.nonzero(np.asarray(M))
    return all(sum(_digits_of(int(b), radices)) == sum(_digits_of(int(a), radices)) for b, a in zip(rows, cols))


def apply_operator(ms: MixedSector, terms, x):
    """y = O x on the sector of ``ms`` (rows in its canonical order): each term
    (coef, sites, M) sends coef <b|M|a> x_s from every state s whose digits on the
    sites are a to the state with them replaced by b (push form).  FP64, or
    complex128 when x or a matrix is complex."""
    nb = nbits_for(ms.Q)
    L = ms.L
    x = np.asarray(x)
    cplx = np.iscomplexobj(x) or any(np.iscomplexobj(M) for _, _, M in terms)
    y = np.zeros(ms.dim, dtype=np.complex128 if cplx else np.float64)
    digits = [[(int(s) >> (nb * (L - 1 - i))) & ((1 << nb) - 1) for i in range(L)] for s in ms.states]
    for coef, sites, M in terms:
        radices = [ms.dims[v] for v in sites]
        n = int(np.prod(radices))
        M = np.asarray(M)
        if M.shape != (n, n):
            raise ValueError("term matrix shape")
        if not conserves(radices, M):
            raise ValueError("term does not conserve the particle number")
        for r, d in enumerate(digits):
            a = 0
            for v, q in zip(sites, radices):
                a = a * q + d[v]
            for b in np.nonzero(M[:, a])[0]:
                new = list(d)
                for v, db in zip(sites, _digits_of(int(b), radices)):
                    new[v] = db
                s2 = 0
                for i in range(L):
                    s2 |= new[i] << (nb * (L - 1 - i))
                y[ms._pos[s2]] += coef * M[b, a] * x[r]
    return y


def full_space_matrix(dims, terms):
    """O on the whole space of prod_i dims[i] states (basis index: the mixed-radix
    number of all L digits, site 0 most significant), by contracting each term's
    matrix into the tensor legs of its sites."""
    dims = [int(q) for q in dims]
    L = len(dims)
    dim = int(np.prod(dims))
    cplx = any(np.iscomplexobj(M) for _, _, M in terms)
    out = np.zeros((dim, dim), dtype=np.complex128 if cplx else np.float64)
    for coef, sites, M in terms:
        m = len(sites)
        legs = [dims[v] for v in sites]
        T = np.asarray(M).reshape(legs + legs)  # out legs, then in legs
        eye = np.eye(dim).reshape(dims + [dim])
        res = np.tensordot(T, eye, axes=(list(range(m, 2 * m)), list(sites)))
        rest = [i for i in range(L) if i not in sites]
        order = [0] * L
        for j, v in enumerate(sites):
            order[v] = j
        for r, v in enumerate(rest):
            order[v] = m + r
        out += coef * np.transpose(res, order + [L]).reshape(dim, dim)
    return out


def sector_matrix(ms: MixedSector, terms):
    """O restricted to the sector: the full-space matrix at the sector's states."""
    nb = nbits_for(ms.Q)
    L = ms.L
    idx = np.zeros(ms.dim, dtype=np.int64)
    for i in range(L):
        d = ((ms.states >> np.uint64(nb * (L - 1 - i))) & np.uint64((1 << nb) - 1)).astype(np.int64)
        idx = idx * ms.dims[i] + d
    F = full_space_matrix(ms.dims, terms)
    return F[np.ix_(idx, idx)]
