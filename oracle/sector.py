"""Oracle: sector dimension, canonical order, rank / unrank / increment.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain Python integers and
numpy; no blocking, no fused tables.

Notation follows the paper (arXiv:2407.14591): Q states per site, L sites, n
particles (digit sum), N subsystems P_0..P_{N-1} of lengths L_k, local particle
numbers n_k, lambda_k = particles in P_0..P_{k-1}, Gamma_k = length of the
complement to the right of P_k.

State encoding (the library's format, also used here): one unsigned 64-bit
word, ceil(log2 Q) bits per site, site 0 in the most significant field, plain
binary digits (Sec. 4.2, the |3;2;1;0> -> 228 example).

Readings of the paper taken here (each also listed in the design notes):
  * Gamma_i is the length to the right of P_i, i.e. L - sum_{l<=i} L_l: the
    general-recipe text writes the sum up to i-1 while the stride formula and the
    worked example (offset_B = 10) need the complement after P_i.
  * D_Q(0, m) = [m == 0]; D_Q(l, m) = 0 for m < 0 or m > (Q-1) l.
  * The order inside a local particle-number sector is lexicographic in the
    sites (first site most significant), which is what the on-the-fly rank
    assigns when the paper builds its tables (Sec. 4.2, table lookup).
  * Unrank searches n_k only over the feasible range [n_low, n_high].
  * Increment does not wrap: past the last state it returns None.
"""
from __future__ import annotations

import functools
import itertools
import math

import numpy as np


# ----------------------------------------------------------------------------
# Encoding helpers (independent of the GPU library's own)
# ----------------------------------------------------------------------------

def nbits_for(Q: int) -> int:
    """Bits per site, ceil(log2 Q) (Sec. 4.2)."""
    if Q < 2:
        raise ValueError("Q must be >= 2")
    return (Q - 1).bit_length()


def pack(digits, Q: int) -> int:
    nb = nbits_for(Q)
    v = 0
    for d in digits:
        v = (v << nb) | int(d)
    return v


def unpack(state: int, Q: int, L: int):
    nb = nbits_for(Q)
    m = (1 << nb) - 1
    return [(int(state) >> (nb * (L - 1 - i))) & m for i in range(L)]


def default_split(Q: int, L: int):
    """Most-equal split into ceil(L / floor(9 / Nbits)) parts, shorter parts first.

    The paper recommends the most-equal partition (Sec. 4.3) but its default
    length (16 sites) is not the split the workloads here use; parts of at most
    9 sites reproduce the 8/8, 8/8/8/8 and 8/8/9/9 splits of the workloads.
    """
    per = max(1, 9 // nbits_for(Q))
    N = max(1, -(-L // per))
    base, extra = divmod(L, N)
    return [base] * (N - extra) + [base + 1] * extra


# ----------------------------------------------------------------------------
# Dimension (Sec. 2.1 eq. dim; App. A)
# ----------------------------------------------------------------------------

def dim_poly(Q: int, L: int, n: int) -> int:
    """Coefficient of x^n in (1 + x + ... + x^{Q-1})^L, by repeated convolution.

    This is the plain definition of the sector dimension (App. A): every word
    with digit sum n contributes one to that coefficient.
    """
    poly = [1]
    for _ in range(L):
        new = [0] * (len(poly) + Q - 1)
        for e, c in enumerate(poly):
            if c:
                for d in range(Q):
                    new[e + d] += c
        poly = new
    return poly[n] if 0 <= n < len(poly) else 0


def dim_closed(Q: int, L: int, n: int) -> int:
    """Closed form, eq. dim: sum_k (-1)^k C(L,k) C(L-1+n-Qk, L-1)."""
    if n < 0 or n > (Q - 1) * L:
        return 0
    if L == 0:
        return 1 if n == 0 else 0
    return sum((-1) ** k * math.comb(L, k) * math.comb(L - 1 + n - Q * k, L - 1)
               for k in range(n // Q + 1))


@functools.lru_cache(maxsize=None)
def D(Q: int, l: int, m: int) -> int:
    """Sector dimension with the range guard (0 outside 0 <= m <= (Q-1) l)."""
    if l < 0 or m < 0 or m > (Q - 1) * l:
        return 0
    return dim_poly(Q, l, m)


# ----------------------------------------------------------------------------
# Brute force: all words of the sector and the canonical order by sorting
# ----------------------------------------------------------------------------

def sector_digits(Q: int, L: int, n: int) -> np.ndarray:
    """All digit strings of length L with digit sum n, shape [D, L] (any order)."""
    total = Q ** L
    if total > 200_000_000:
        raise ValueError("sector too large for brute force")
    vals = np.arange(total, dtype=np.int64)
    digits = np.empty((total, L), dtype=np.int8)
    for i in range(L - 1, -1, -1):
        digits[:, i] = vals % Q
        vals //= Q
    keep = digits.sum(axis=1, dtype=np.int64) == n
    return digits[keep]


def pack_array(digits: np.ndarray, Q: int) -> np.ndarray:
    nb = nbits_for(Q)
    L = digits.shape[1]
    out = np.zeros(digits.shape[0], dtype=np.uint64)
    for i in range(L):
        out |= digits[:, i].astype(np.uint64) << np.uint64(nb * (L - 1 - i))
    return out


def _subsystem_fields(Q, split):
    """(shift, mask) of each subsystem word inside the packed state, P_0 first."""
    nb = nbits_for(Q)
    L = sum(split)
    fields = []
    start = 0
    for Lk in split:
        shift = nb * (L - start - Lk)
        fields.append((shift, (1 << (nb * Lk)) - 1))
        start += Lk
    return fields


def _digit_sum_words(words: np.ndarray, Q: int, length: int) -> np.ndarray:
    nb = nbits_for(Q)
    m = np.uint64((1 << nb) - 1)
    s = np.zeros(words.shape, dtype=np.int64)
    for i in range(length):
        s += ((words >> np.uint64(nb * i)) & m).astype(np.int64)
    return s


def canonical_keys(states: np.ndarray, Q: int, split) -> np.ndarray:
    """Sort keys (n_0, w_0, n_1, w_1, ...) for packed states, as [len(states), 2N].

    The canonical order (Sec. 3.1-3.2): P_0 varies slowest and P_{N-1} fastest;
    inside each subsystem, states are grouped by local particle number (lower
    first) and then ordered lexicographically (numeric order of the word).
    """
    cols = []
    for (shift, mask), Lk in zip(_subsystem_fields(Q, split), split):
        w = (states >> np.uint64(shift)) & np.uint64(mask)
        cols.append(_digit_sum_words(w, Q, Lk))
        cols.append(w.astype(np.int64))
    return np.stack(cols, axis=1)


class BruteSector:
    """Canonical order of one sector by a plain sort of all its words.

    rank(s) is the position of s in this sorted list, unrank(i) its i-th entry.
    """

    def __init__(self, Q: int, L: int, n: int, split=None):
        self.Q, self.L, self.n = Q, L, n
        self.split = list(split) if split is not None else default_split(Q, L)
        if sum(self.split) != L:
            raise ValueError("split does not sum to L")
        st = pack_array(sector_digits(Q, L, n), Q)
        keys = canonical_keys(st, Q, self.split)
        order = np.lexsort(keys.T[::-1])
        self.states = st[order]
        self.dim = len(self.states)
        # composite key for lookup: fields concatenated, checked to fit 63 bits
        self._widths = []
        for Lk in self.split:
            self._widths.append(((Q - 1) * Lk).bit_length())
            self._widths.append(nbits_for(Q) * Lk)
        if sum(self._widths) > 63:
            raise ValueError("composite key too wide for this oracle helper")
        self._sorted_keys = self._composite(self.states)
        assert np.all(np.diff(self._sorted_keys.astype(np.int64)) > 0)

    def _composite(self, states: np.ndarray) -> np.ndarray:
        keys = canonical_keys(states, self.Q, self.split)
        out = np.zeros(len(states), dtype=np.uint64)
        for c, w in enumerate(self._widths):
            out = (out << np.uint64(w)) | keys[:, c].astype(np.uint64)
        return out

    def rank(self, states) -> np.ndarray:
        """Positions of packed states; -1 for words that are not in the sector."""
        states = np.asarray(states, dtype=np.uint64)
        key = self._composite(states)
        pos = np.searchsorted(self._sorted_keys, key)
        pos_c = np.minimum(pos, self.dim - 1)
        ok = (pos < self.dim) & (self.states[pos_c] == states)
        return np.where(ok, pos_c.astype(np.int64), -1)

    def unrank(self, idx) -> np.ndarray:
        return self.states[np.asarray(idx, dtype=np.int64)]


# ----------------------------------------------------------------------------
# Lexicographic rank within a digit-sum sector (eq. N=L; Alg. on-the-fly)
# ----------------------------------------------------------------------------

def lex_rank(digits, Q: int) -> int:
    """Position of a word among all words of its length and digit sum, in lex order.

    eq. N=L: every site contributes the number of completions that put a
    smaller digit at that site, sum_{k < q_i} D_Q(Gamma_i, n - lambda_i - k)
    with Gamma_i = L-1-i sites to the right; the range guard of D removes the
    infeasible terms (the n_low bound).
    """
    L = len(digits)
    n = sum(digits)
    idx, lam = 0, 0
    for i, q in enumerate(digits):
        gam = L - 1 - i
        for k in range(q):
            idx += D(Q, gam, n - lam - k)
        lam += q
    return idx


def lex_unrank(i: int, Q: int, L: int, m: int):
    """The i-th word (lex order) among words of length L with digit sum m."""
    if not 0 <= i < D(Q, L, m):
        raise ValueError("local index out of range")
    digits = []
    rem = m
    for pos in range(L):
        gam = L - 1 - pos
        for q in range(Q):
            cnt = D(Q, gam, rem - q)
            if i < cnt:
                digits.append(q)
                rem -= q
                break
            i -= cnt
    return digits


def cover_rank(S, x) -> int:
    """Cover's enumerative index of word x in the set S of words (eq. cover).

    index = sum_k sum_{l < x_k} n_S(x_0..x_{k-1}, l), with n_S(prefix) the
    number of words of S that start with prefix.
    """
    S = [tuple(s) for s in S]

    def n_S(prefix):
        return sum(1 for s in S if s[:len(prefix)] == tuple(prefix))

    return sum(n_S(tuple(x[:k]) + (l,)) for k in range(len(x)) for l in range(x[k]))


# ----------------------------------------------------------------------------
# Closed form: offsets, strides, rank, unrank, increment (Sec. 3.2, App. B)
# ----------------------------------------------------------------------------

class Sector:
    """The divide-and-conquer index with Python integers, eq. index / ck / offset / stride."""

    def __init__(self, Q: int, L: int, n: int, split=None):
        if not 0 <= n <= (Q - 1) * L:
            raise ValueError("n out of range")
        self.Q, self.L, self.n = Q, L, n
        self.split = list(split) if split is not None else default_split(Q, L)
        if sum(self.split) != L or any(s <= 0 for s in self.split):
            raise ValueError("bad split")
        self.N = len(self.split)
        self.nb = nbits_for(Q)
        self.fields = _subsystem_fields(Q, self.split)
        self.start = [sum(self.split[:k]) for k in range(self.N)]
        # Gamma_k: sites to the right of P_k (reading: the complement after P_k)
        self.gamma = [L - sum(self.split[:k + 1]) for k in range(self.N)]
        self.dim = D(Q, L, n)

    def n_low(self, k: int, lam: int) -> int:
        return max(0, self.n - lam - (self.Q - 1) * self.gamma[k])

    def n_high(self, k: int, lam: int) -> int:
        return min((self.Q - 1) * self.split[k], self.n - lam)

    def offset(self, k: int, nk: int, lam: int) -> int:
        """eq. offset: sum over k_i = n_low .. n_k-1 of D(L_k, k_i) D(Gamma_k, n-lam-k_i)."""
        Q, Lk, g = self.Q, self.split[k], self.gamma[k]
        return sum(D(Q, Lk, j) * D(Q, g, self.n - lam - j)
                   for j in range(self.n_low(k, lam), nk))

    def stride(self, k: int, nk: int, lam: int) -> int:
        """eq. stride: D(Gamma_k, n - lam - n_k); 1 for the last subsystem."""
        return D(self.Q, self.gamma[k], self.n - lam - nk)

    def sub_digits(self, state: int, k: int):
        d = unpack(state, self.Q, self.L)
        return d[self.start[k]:self.start[k] + self.split[k]]

    def valid(self, state: int) -> bool:
        state = int(state)
        if state < 0 or state >> (self.nb * self.L):
            return False
        d = unpack(state, self.Q, self.L)
        return all(q < self.Q for q in d) and sum(d) == self.n

    def rank(self, state: int) -> int:
        """Alg. i / eq. index: sum of c_k = offset_k + stride_k * index_k; -1 if invalid."""
        if not self.valid(state):
            return -1
        idx, lam = 0, 0
        for k in range(self.N):
            w = self.sub_digits(state, k)
            nk = sum(w)
            ik = lex_rank(w, self.Q)
            idx += self.offset(k, nk, lam) + self.stride(k, nk, lam) * ik
            lam += nk
        return idx

    def unrank(self, index: int) -> int:
        """Alg. iii: peel off offset and stride subsystem by subsystem; None if out of range."""
        if not 0 <= index < self.dim:
            return None
        digits = []
        lam = 0
        for k in range(self.N - 1):
            Lk = self.split[k]
            lo, hi = self.n_low(k, lam), self.n_high(k, lam)
            nk = None
            for m in range(lo, hi + 1):
                start = self.offset(k, m, lam)
                end = start + D(self.Q, Lk, m) * self.stride(k, m, lam)
                if start <= index < end:
                    nk = m
                    break
            assert nk is not None
            index -= self.offset(k, nk, lam)
            st = self.stride(k, nk, lam)
            ik = index // st
            index -= ik * st
            digits += lex_unrank(ik, self.Q, Lk, nk)
            lam += nk
        digits += lex_unrank(index, self.Q, self.split[-1], self.n - lam)
        return pack(digits, self.Q)

    # -- increment, Alg. ii --------------------------------------------------
    def _minimal(self, length: int, m: int):
        """Word of given length and digit sum with index 0: digits packed to the right."""
        d = [0] * length
        rem = m
        for i in range(length - 1, -1, -1):
            q = min(self.Q - 1, rem)
            d[i] = q
            rem -= q
        assert rem == 0
        return d

    def increment(self, state: int):
        """Next state in canonical order (Alg. ii); None after the last state."""
        d = unpack(state, self.Q, self.L)
        lam, gam = 0, 0
        for k in range(self.N - 1, -1, -1):
            a, Lk = self.start[k], self.split[k]
            w = d[a:a + Lk]
            nk = sum(w)
            i = lex_rank(w, self.Q)
            if i + 1 < D(self.Q, Lk, nk):          # not maximal: step locally
                new = d[:a] + lex_unrank(i + 1, self.Q, Lk, nk) + self._minimal(gam, lam)
                return pack(new, self.Q)
            if lam > 0 and nk < (self.Q - 1) * Lk:  # move one particle into P_k
                new = d[:a] + self._minimal(Lk, nk + 1) + self._minimal(gam, lam - 1)
                return pack(new, self.Q)
            gam += Lk
            lam += nk
        return None

    def first(self) -> int:
        return pack(self._minimal(self.L, self.n), self.Q)

    # -- canonical order by nested generation (no offsets, no strides) --------
    def nested(self):
        """Yield the sector's states in canonical order by nested loops.

        Level k runs over its feasible local particle numbers in increasing
        order and, for each, over the words of P_k with that digit sum in lex
        order; the levels nest P_0 outermost.  Uses only digit sums.
        """
        Q, L = self.Q, self.L
        words_by_len = {}
        for Lk in set(self.split):
            ws = [list(t) for t in itertools.product(range(Q), repeat=Lk)]
            words_by_len[Lk] = ws

        def rec(k, lam, prefix):
            if k == self.N:
                yield pack(prefix, Q)
                return
            Lk = self.split[k]
            rest = L - self.start[k] - Lk
            r = self.n - lam
            for m in range(max(0, r - (Q - 1) * rest), min((Q - 1) * Lk, r) + 1):
                for w in words_by_len[Lk]:
                    if sum(w) == m:
                        yield from rec(k + 1, lam + m, prefix + w)

        yield from rec(0, 0, [])
