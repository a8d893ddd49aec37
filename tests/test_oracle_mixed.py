"""Pins of the mixed-dimension oracle (sites of different local dimensions, the
generalisation Sec. 5 names) against what the definitions and the mathematics fix:
the generating-function dimension, the single-Q oracle when all dimensions agree,
the whole-space tensor contraction, the spectrum of a spin-1/2 / spin-1 pair from
angular-momentum addition, and the ground-state spin of a ring of alternating spins
(Lieb-Mattis)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import mixed
from oracle.operators import apply_operator as apply_uniform
from oracle.operators import spin_matrices
from oracle.sector import BruteSector, dim_closed, nbits_for


@pytest.mark.parametrize("dims,n", [([2, 3], 1), ([3, 2, 4, 2], 3), ([2, 3, 2, 3, 2, 3], 4), ([4, 2, 5], 5),
                                    ([2, 2, 2, 3, 3], 0), ([2, 3, 4], 6)])
def test_dimension_and_states(dims, n):
    ms = mixed.MixedSector(dims, n)
    # dimension: the coefficient of x^n in prod (1 + ... + x^(q-1)), and a direct count
    direct = sum(1 for d in itertools.product(*[range(q) for q in dims]) if sum(d) == n)
    assert ms.dim == mixed.dim_poly(dims, n) == direct
    nb = nbits_for(max(dims))
    L = len(dims)
    seen = set()
    for s in ms.states:
        d = [(int(s) >> (nb * (L - 1 - i))) & ((1 << nb) - 1) for i in range(L)]
        assert all(di < q for di, q in zip(d, dims)) and sum(d) == n
        seen.add(int(s))
    assert len(seen) == ms.dim
    assert np.array_equal(ms.rank(ms.unrank(np.arange(ms.dim))), np.arange(ms.dim))


def test_invalid_digit_ranks_to_minus_one():
    ms = mixed.MixedSector([2, 3, 2], 2)
    # digit 2 on site 0 (local dimension 2) is outside the sector even though the sum is 2
    nb = 2
    bad = (2 << (2 * nb)) | 0
    assert ms.rank([bad])[0] == -1


@pytest.mark.parametrize("Q,L,n,split", [(2, 8, 3, [4, 4]), (3, 5, 4, [2, 3]), (4, 4, 5, None)])
def test_single_dimension_reduces_to_uniform_oracle(Q, L, n, split):
    ms = mixed.MixedSector([Q] * L, n, split)
    bs = BruteSector(Q, L, n, split)
    assert ms.dim == dim_closed(Q, L, n)
    assert np.array_equal(ms.states, bs.states)
    terms = [(0.7, (0, 2), synth.random_local_matrix(Q, 2, 5)), (-0.3, (L - 1,), synth.random_local_matrix(Q, 1, 6)),
             (1.1, (3, 1, 0), synth.random_local_matrix(Q, 3, 7, density=0.5))]
    x = np.random.default_rng(1).normal(size=ms.dim)
    assert np.allclose(mixed.apply_operator(ms, terms, x), apply_uniform(bs, terms, x), rtol=0, atol=1e-12)


@pytest.mark.parametrize("dims,n", [([2, 3, 2, 4], 4), ([3, 2, 3, 2, 2], 3)])
def test_push_form_matches_whole_space_matrix(dims, n):
    ms = mixed.MixedSector(dims, n)
    terms = []
    for t, sites in enumerate([(0, 1), (2,), (3, 0), (1, 2, 3)]):
        terms.append((0.4 + t, sites, synth.random_local_matrix_dims([dims[v] for v in sites], 30 + t, 0.8)))
    x = np.random.default_rng(2).normal(size=ms.dim)
    y = mixed.apply_operator(ms, terms, x)
    assert np.allclose(y, mixed.sector_matrix(ms, terms) @ x, rtol=0, atol=1e-12)
    # and with a complex vector
    xc = x + 1j * np.random.default_rng(3).normal(size=ms.dim)
    assert np.allclose(mixed.apply_operator(ms, terms, xc), mixed.sector_matrix(ms, terms) @ xc, rtol=0, atol=1e-12)


def heisenberg_pair(dims, i, j, J=1.0):
    """J S_i . S_j = J (Sz Sz + (S+ S- + S- S+) / 2) on sites of dims[i], dims[j]."""
    a, b = spin_matrices(dims[i]), spin_matrices(dims[j])
    M = np.kron(a["Sz"], b["Sz"]) + 0.5 * (np.kron(a["S+"], b["S-"]) + np.kron(a["S-"], b["S+"]))
    return (J, (i, j), M)


def test_spin_half_spin_one_dimer_spectrum():
    """S_1 . S_2 for s1 = 1/2, s2 = 1 equals (J(J+1) - 3/4 - 2) / 2 on total spin J:
    -1 for J = 1/2 and 1/2 for J = 3/2; each Sz sector holds the J that reach it."""
    dims = [2, 3]
    want = {0: [0.5], 1: [-1.0, 0.5], 2: [-1.0, 0.5], 3: [0.5]}  # n = Sz + 3/2
    for n, ev in want.items():
        ms = mixed.MixedSector(dims, n)
        H = mixed.sector_matrix(ms, [heisenberg_pair(dims, 0, 1)])
        assert np.allclose(np.linalg.eigvalsh(H), ev, atol=1e-12)


def test_alternating_ring_ground_state_spin():
    """Antiferromagnetic Heisenberg ring of alternating spin-1/2 and spin-1 sites (L = 6):
    by Lieb-Mattis the ground state has total spin |3 (1 - 1/2)| = 3/2, so the lowest
    energies of the sectors Sz = +-1/2, +-3/2 agree and lie below Sz = +-5/2."""
    dims = [2, 3] * 3
    L = len(dims)
    terms = [heisenberg_pair(dims, i, (i + 1) % L) for i in range(L)]
    smax = sum(q - 1 for q in dims) / 2.0
    e0 = {}
    for n in range(sum(q - 1 for q in dims) + 1):
        ms = mixed.MixedSector(dims, n)
        e0[n - smax] = np.linalg.eigvalsh(mixed.sector_matrix(ms, terms))[0]
    low = [e0[sz] for sz in (-1.5, -0.5, 0.5, 1.5)]
    assert max(low) - min(low) < 1e-10
    assert e0[2.5] > low[0] + 1e-3 and e0[-2.5] > low[0] + 1e-3
