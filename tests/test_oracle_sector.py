"""Pins of the oracle's sector index against the paper's printed values, closed
forms, library routines and brute force.  CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import native
from oracle.sector import (BruteSector, D, Sector, cover_rank, default_split, dim_closed,
                           dim_poly, lex_rank, lex_unrank, pack, unpack)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def splits_of(L, N):
    """Most-equal split of L sites into N parts (shorter first) plus a few uneven ones."""
    base, extra = divmod(L, N)
    out = [[base] * (N - extra) + [base + 1] * extra]
    if N >= 2 and L >= N + 1:
        out.append([1] * (N - 1) + [L - N + 1])
        out.append([L - N + 1] + [1] * (N - 1))
    return out


# ---------------------------------------------------------------- dimension

@pytest.mark.parametrize("Q", [2, 3, 4, 5])
def test_dimension_closed_form_equals_polynomial(Q):
    for L in range(0, 11):
        tot = 0
        for n in range(0, (Q - 1) * L + 1):
            assert dim_closed(Q, L, n) == dim_poly(Q, L, n)
            tot += dim_poly(Q, L, n)
        assert tot == Q ** L


def test_dimension_binomial_and_worked_example():
    for L in range(0, 40):
        for n in range(0, L + 1):
            assert dim_poly(2, L, n) == math.comb(L, n)
    assert dim_closed(2, 9, 4) == gold("worked_example_L9.json")["dim"]
    # central trinomial coefficients are the spin-1 Sz=0 dimensions (OEIS A002426)
    assert [dim_poly(3, L, L) for L in range(0, 9)] == [1, 1, 3, 7, 19, 51, 141, 393, 1107]


def test_dimension_counts_words():
    for Q, L in [(2, 7), (3, 5), (4, 4)]:
        counts = {}
        for w in itertools.product(range(Q), repeat=L):
            counts[sum(w)] = counts.get(sum(w), 0) + 1
        for n, c in counts.items():
            assert D(Q, L, n) == c


# ---------------------------------------------------------------- printed values

def test_worked_example():
    g = gold("worked_example_L9.json")
    s = Sector(g["Q"], g["L"], g["n"], g["split"])
    st_ = pack(g["state_digits"], 2)
    assert s.dim == g["dim"]
    assert s.rank(st_) == g["index"]
    lam = 0
    for k, name in enumerate("ABC"):
        e = g[name]
        w = s.sub_digits(st_, k)
        assert sum(w) == e["n_k"] and lam == e["lambda"]
        assert lex_rank(w, 2) == e["local_index"]
        assert s.offset(k, e["n_k"], lam) == e["offset"]
        assert s.stride(k, e["n_k"], lam) == e["stride"]
        assert e["offset"] + e["stride"] * e["local_index"] == e["c"]
        lam += e["n_k"]
    assert s.unrank(g["index"]) == st_
    assert BruteSector(g["Q"], g["L"], g["n"], g["split"]).rank([st_])[0] == g["index"]
    ns = native.NativeSector(g["Q"], g["L"], g["n"], g["split"])
    assert int(ns.rank([st_])[0]) == g["index"]
    assert int(ns.unrank([g["index"]])[0]) == st_


def test_lookup_table():
    g = gold("lookup_table_L3.json")
    for e in g["entries"]:
        assert lex_rank(e["word"], g["Q"]) == e["index"]
        assert lex_unrank(e["index"], g["Q"], g["L_k"], e["n"]) == e["word"]
        # a one-subsystem sector of three sites numbers its states the same way
        ns = native.NativeSector(g["Q"], g["L_k"], e["n"], [g["L_k"]])
        assert int(ns.rank([pack(e["word"], 2)])[0]) == e["index"]


def test_cover_toy_set():
    g = gold("cover_toy.json")
    assert cover_rank(g["set"], g["word"]) == g["index"]
    S = [tuple(s) for s in g["set"]]
    for c in g["counts"]:
        p = tuple(c["prefix"])
        assert sum(1 for s in S if s[:len(p)] == p) == c["n_S"]
    # Cover's index of every element is its position in the (sorted) set
    for i, w in enumerate(sorted(S)):
        assert cover_rank(S, w) == i


def test_state_encoding():
    g = gold("state_encoding.json")
    assert pack(g["digits"], g["Q"]) == g["packed"]
    assert unpack(g["packed"], g["Q"], len(g["digits"])) == g["digits"]


# ---------------------------------------------------------------- library routines

@pytest.mark.parametrize("L,n", [(6, 3), (9, 4), (10, 1), (8, 8), (7, 0)])
def test_single_subsystem_is_reverse_combinations_order(L, n):
    """Q=2, N=1: the canonical order is lex order of words, i.e. the reverse of
    itertools.combinations order of the occupied sites."""
    combos = list(itertools.combinations(range(L), n))
    words = [pack([1 if i in c else 0 for i in range(L)], 2) for c in combos][::-1]
    s = Sector(2, L, n, [L])
    assert [s.unrank(i) for i in range(s.dim)] == words
    ns = native.NativeSector(2, L, n, [L])
    assert list(ns.unrank(np.arange(ns.dim))) == words


@pytest.mark.parametrize("Q,L,n", [(3, 5, 4), (4, 4, 5), (3, 4, 8), (5, 3, 6)])
def test_single_and_site_subsystems_are_lex_order(Q, L, n):
    """N=1 and N=L (the on-the-fly limit, eq. N=L) both give lex order over
    itertools.product."""
    words = [pack(w, Q) for w in itertools.product(range(Q), repeat=L) if sum(w) == n]
    for split in ([L], [1] * L):
        s = Sector(Q, L, n, split)
        assert [s.unrank(i) for i in range(s.dim)] == words
        assert [s.rank(w) for w in words] == list(range(len(words)))
        b = BruteSector(Q, L, n, split)
        assert [int(v) for v in b.states] == words


# ---------------------------------------------------------------- brute force

CASES = [(2, L, n, sp) for L in range(1, 9) for n in range(0, L + 1)
         for N in range(1, L + 1) for sp in splits_of(L, N)]
CASES += [(3, L, n, sp) for L in range(1, 6) for n in range(0, 2 * L + 1)
          for N in range(1, L + 1) for sp in splits_of(L, N)[:1]]
CASES += [(4, 4, n, sp) for n in range(0, 13) for sp in ([4], [2, 2], [1, 3], [1, 1, 1, 1])]


def test_closed_form_equals_sorted_order():
    for Q, L, n, sp in CASES:
        b = BruteSector(Q, L, n, sp)
        s = Sector(Q, L, n, sp)
        assert b.dim == s.dim == D(Q, L, n)
        ranks = [s.rank(int(v)) for v in b.states]
        assert ranks == list(range(b.dim)), (Q, L, n, sp)
        assert [s.unrank(i) for i in range(b.dim)] == [int(v) for v in b.states]


def test_native_equals_sorted_order_and_nested_generation():
    for Q, L, n, sp in CASES:
        b = BruteSector(Q, L, n, sp)
        ns = native.NativeSector(Q, L, n, sp)
        assert ns.dim == b.dim
        assert np.array_equal(ns.rank(b.states), np.arange(b.dim, dtype=np.uint64))
        assert np.array_equal(ns.unrank(np.arange(b.dim)), b.states)
        assert np.array_equal(np.concatenate(list(ns.iterate(7))), b.states)


def test_increment_walks_the_order():
    for Q, L, n, sp in CASES[::7]:
        s = Sector(Q, L, n, sp)
        b = BruteSector(Q, L, n, sp)
        seq, st_ = [], s.first()
        while st_ is not None:
            seq.append(st_)
            st_ = s.increment(st_)
        assert seq == [int(v) for v in b.states]
        assert list(s.nested()) == seq


def test_invalid_states_are_rejected():
    s = Sector(2, 9, 4, [3, 3, 3])
    ns = native.NativeSector(2, 9, 4, [3, 3, 3])
    bad = [pack([1] * 5 + [0] * 4, 2), 0, 1 << 9, (1 << 9) | 0b1111]
    for w in bad:
        assert s.rank(w) == -1
    assert np.all(ns.rank(bad) == np.uint64(2 ** 64 - 1))
    assert ns.unrank([126])[0] == np.uint64(2 ** 64 - 1)
    s3 = native.NativeSector(3, 4, 4, [2, 2])
    assert s3.rank([pack([3, 1, 0, 0], 4)])[0] == np.uint64(2 ** 64 - 1)   # digit 3 invalid at Q=3


def test_split_changes_order_not_set():
    a = BruteSector(2, 9, 4, [3, 3, 3])
    b = BruteSector(2, 9, 4, [9])
    assert set(a.states.tolist()) == set(b.states.tolist())
    # block-lex first differs from plain lex at position 2
    assert a.states[2] != b.states[2]
    assert unpack(int(a.states[2]), 2, 9) == [0, 0, 0, 1, 0, 0, 1, 1, 1]
    assert unpack(int(b.states[2]), 2, 9) == [0, 0, 0, 0, 1, 1, 0, 1, 1]


def test_default_split():
    assert default_split(2, 16) == [8, 8]
    assert default_split(2, 32) == [8, 8, 8, 8]
    assert default_split(2, 34) == [8, 8, 9, 9]
    assert default_split(2, 28) == [7, 7, 7, 7]
    assert default_split(2, 24) == [8, 8, 8]
    assert default_split(3, 16) == [4, 4, 4, 4]
    assert default_split(3, 13) == [3, 3, 3, 4]


@settings(max_examples=60, deadline=None)
@given(st.data())
def test_random_sectors_three_ways(data):
    Q = data.draw(st.integers(2, 4))
    L = data.draw(st.integers(1, {2: 10, 3: 6, 4: 5}[Q]))
    n = data.draw(st.integers(0, (Q - 1) * L))
    N = data.draw(st.integers(1, L))
    cuts = sorted(data.draw(st.lists(st.integers(1, L - 1), min_size=N - 1, max_size=N - 1,
                                     unique=True))) if N > 1 else []
    sp = [b - a for a, b in zip([0] + cuts, cuts + [L])]
    b = BruteSector(Q, L, n, sp)
    ns = native.NativeSector(Q, L, n, sp)
    assert np.array_equal(ns.rank(b.states), np.arange(b.dim, dtype=np.uint64))
    assert np.array_equal(ns.unrank(np.arange(b.dim)), b.states)
    s = Sector(Q, L, n, sp)
    pick = data.draw(st.lists(st.integers(0, b.dim - 1), min_size=1, max_size=8))
    for i in pick:
        assert s.rank(int(b.states[i])) == i


@pytest.mark.slow
def test_native_large_sector_bijection():
    """L=24, n=12, split 8/8/8 (2,704,156 states): nested generation (no offsets)
    equals the closed-form unrank, and rank inverts it."""
    ns = native.NativeSector(2, 24, 12, [8, 8, 8])
    assert ns.dim == math.comb(24, 12)
    pos = 0
    for chunk in ns.iterate(1 << 20):
        idx = np.arange(pos, pos + len(chunk), dtype=np.uint64)
        assert np.array_equal(ns.unrank(idx), chunk)
        assert np.array_equal(ns.rank(chunk), idx)
        pos += len(chunk)
    assert pos == ns.dim
