"""Pins of the oracle's H*x: a push-built full-space matrix with no sector index,
exact spectra (magnons, free fermions, Majumdar-Ghosh, two-site spin-1, ferromagnetic
multiplets, Bethe ansatz), symmetries and split invariance.  CPU only."""
import itertools
import math

import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import native
from oracle.hamiltonian import (apply_h, full_basis_digit_sums, full_matrix, sector_matrix)
from oracle.lanczos import ground_state
from oracle.sector import BruteSector, default_split, pack, unpack


def restrict_full(Q, L, n, split, H_full):
    """Rows/columns of the full matrix for the sector's states, in canonical order."""
    b = BruteSector(Q, L, n, split)
    full_idx = []
    for s in b.states:
        d = unpack(int(s), Q, L)
        full_idx.append(sum(q * Q ** (L - 1 - i) for i, q in enumerate(d)))
    full_idx = np.array(full_idx)
    return b, H_full[np.ix_(full_idx, full_idx)]


@pytest.mark.parametrize("Q,L,split", [(2, 6, [3, 3]), (2, 8, [3, 2, 3]), (2, 7, [7]),
                                       (3, 4, [2, 2]), (3, 5, [1, 2, 2]), (4, 3, [1, 2])])
def test_sector_matrix_equals_restricted_full_matrix(Q, L, split):
    rng = np.random.default_rng(11)
    bonds = synth.chain_bonds(L, 1) + ([(0, 2), (1, L - 1)] if L > 4 else [])
    jxy = rng.uniform(-1, 1, len(bonds))
    jz = rng.uniform(-1, 1, len(bonds))
    h = rng.uniform(-1, 1, L)
    Hf = full_matrix(Q, L, bonds, jxy, jz, h)
    assert np.allclose(Hf, Hf.T, atol=0, rtol=0)
    sums = full_basis_digit_sums(Q, L)
    # H conserves the digit sum: no element connects different sums
    assert np.all(Hf[sums[:, None] != sums[None, :]] == 0)
    for n in range(0, (Q - 1) * L + 1):
        b, Hr = restrict_full(Q, L, n, split, Hf)
        Hs = sector_matrix(b, bonds, jxy, jz, h)
        assert np.array_equal(Hs, Hs.T)
        assert np.allclose(Hs, Hr, atol=1e-14, rtol=0), (Q, L, n)


def spectrum(Q, L, n, bonds, jxy, jz, split=None):
    b = BruteSector(Q, L, n, split or default_split(Q, L))
    return np.linalg.eigvalsh(sector_matrix(b, bonds, jxy, jz))


@pytest.mark.parametrize("L,J,Delta", [(8, 1.0, 1.0), (10, 0.7, 0.3), (9, 1.3, -0.5)])
def test_empty_sector_and_one_magnon(L, J, Delta):
    bonds, jxy, jz = synth.xxz_chain(L, J, Delta)
    assert np.allclose(spectrum(2, L, 0, bonds, jxy, jz), [J * Delta * L / 4])
    ks = 2 * np.pi * np.arange(L) / L
    expect = np.sort(J * (Delta * (L - 4) / 4 + np.cos(ks)))
    assert np.allclose(spectrum(2, L, 1, bonds, jxy, jz), expect, atol=1e-12)


@pytest.mark.parametrize("L,n", [(10, 3), (10, 4), (10, 5), (9, 4), (12, 6)])
def test_xx_chain_is_free_fermions(L, n):
    """Delta=0: Jordan-Wigner fermions with periodic (n odd) or antiperiodic (n even)
    momenta; every eigenvalue is a sum of n distinct J cos k."""
    J = 0.8
    bonds, jxy, jz = synth.xxz_chain(L, J, 0.0)
    phi = 0.0 if n % 2 else 0.5
    eps = J * np.cos(2 * np.pi * (np.arange(L) + phi) / L)
    sums = np.sort([sum(c) for c in itertools.combinations(eps, n)])
    assert np.allclose(spectrum(2, L, n, bonds, jxy, jz), sums, atol=1e-11)


@pytest.mark.parametrize("L", [8, 10, 12])
def test_majumdar_ghosh(L):
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    ev = spectrum(2, L, L // 2, bonds, jxy, jz)
    assert abs(ev[0] + 3 * L / 8) < 1e-11
    assert abs(ev[1] + 3 * L / 8) < 1e-11      # dimer states: two-fold degenerate
    assert ev[2] > ev[0] + 1e-3


def test_two_site_spin_one():
    """J S1.S2 with S=1: J/2 [S_t(S_t+1) - 4] for S_t = 0, 1, 2."""
    bonds, jxy, jz = [(0, 1)], [1.0], [1.0]
    assert np.allclose(spectrum(3, 2, 2, bonds, jxy, jz, [1, 1]), [-2.0, -1.0, 1.0])
    assert np.allclose(spectrum(3, 2, 1, bonds, jxy, jz, [1, 1]), [-1.0, 1.0])
    assert np.allclose(spectrum(3, 2, 0, bonds, jxy, jz, [2]), [1.0])
    # spin-1/2 singlet and triplet
    assert np.allclose(spectrum(2, 2, 1, bonds, jxy, jz, [1, 1]), [-0.75, 0.25])


@pytest.mark.parametrize("Q,L", [(2, 8), (3, 5), (4, 4)])
def test_heisenberg_multiplets(Q, L):
    """Delta=1 is SU(2) symmetric: the ferromagnetic multiplet J S^2 (#bonds) is the top
    level of every sector, and sector n contains the spectrum of sector n-1 below
    half filling."""
    S = (Q - 1) / 2
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    prev = None
    for n in range(0, (Q - 1) * L + 1):
        ev = spectrum(Q, L, n, bonds, jxy, jz)
        assert abs(ev[-1] - S * S * len(bonds)) < 1e-10
        if prev is not None and n <= (Q - 1) * L / 2:
            for e in prev:
                assert np.min(np.abs(ev - e)) < 1e-9
        prev = ev
        # particle-hole (spin flip) symmetry
        ev2 = spectrum(Q, L, (Q - 1) * L - n, bonds, jxy, jz)
        assert np.allclose(ev, ev2, atol=1e-10)


def test_split_invariance_of_y():
    Q, L, n = 2, 10, 4
    rng = np.random.default_rng(5)
    bonds, _, _ = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    jxy, jz = rng.normal(size=len(bonds)), rng.normal(size=len(bonds))
    a = BruteSector(Q, L, n, [10])
    b = BruteSector(Q, L, n, [3, 3, 4])
    xa = rng.normal(size=a.dim)
    perm = b.rank(a.states)                  # position of a's states in b's order
    xb = np.empty_like(xa)
    xb[perm] = xa
    ya = apply_h(a, bonds, jxy, jz, xa)
    yb = apply_h(b, bonds, jxy, jz, xb)
    assert np.allclose(yb[perm], ya, atol=1e-13)


def test_native_hx_equals_python():
    for Q, L, n, sp, k in [(2, 12, 5, [4, 4, 4], 1), (2, 11, 6, [5, 6], 3),
                           (3, 6, 6, [2, 2, 2], 2), (4, 5, 5, [2, 3], 1)]:
        b = BruteSector(Q, L, n, sp)
        ns = native.NativeSector(Q, L, n, sp)
        rng = np.random.default_rng(L)
        bonds, _, _ = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
        jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
        x = rng.normal(size=(b.dim, k)) if k > 1 else rng.normal(size=b.dim)
        t = native.NativeTerms(bonds, jxy, jz, h)
        y = apply_h(b, bonds, jxy, jz, x, h)
        assert np.allclose(native.hx_range(ns, t, x), y, atol=1e-13)
        rows = rng.integers(0, b.dim, 50)
        assert np.allclose(native.hx_rows(ns, t, x, rows), y[rows], atol=1e-13)
        y32 = native.hx_rows(ns, t, x.astype(np.float32), rows)
        assert np.allclose(y32, apply_h(b, bonds, jxy, jz, x.astype(np.float32).astype(np.float64), h)[rows],
                           atol=1e-12)


from oracle.closed_forms import bethe_e0 as bethe_ground_energy  # noqa: E402


@pytest.mark.parametrize("L", [8, 10, 12])
def test_majumdar_ghosh(L):
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    ev = spectrum(2, L, L // 2, bonds, jxy, jz)
    assert abs(ev[0] + 3 * L / 8) < 1e-11
    assert abs(ev[1] + 3 * L / 8) < 1e-11      # dimer states: two-fold degenerate
    assert ev[2] > ev[0] + 1e-3


def test_two_site_spin_one():
    """J S1.S2 with S=1: J/2 [S_t(S_t+1) - 4] for S_t = 0, 1, 2."""
    bonds, jxy, jz = [(0, 1)], [1.0], [1.0]
    assert np.allclose(spectrum(3, 2, 2, bonds, jxy, jz, [1, 1]), [-2.0, -1.0, 1.0])
    assert np.allclose(spectrum(3, 2, 1, bonds, jxy, jz, [1, 1]), [-1.0, 1.0])
    assert np.allclose(spectrum(3, 2, 0, bonds, jxy, jz, [2]), [1.0])
    # spin-1/2 singlet and triplet
    assert np.allclose(spectrum(2, 2, 1, bonds, jxy, jz, [1, 1]), [-0.75, 0.25])


@pytest.mark.parametrize("Q,L", [(2, 8), (3, 5), (4, 4)])
def test_heisenberg_multiplets(Q, L):
    """Delta=1 is SU(2) symmetric: the ferromagnetic multiplet J S^2 (#bonds) is the top
    level of every sector, and sector n contains the spectrum of sector n-1 below
    half filling."""
    S = (Q - 1) / 2
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    prev = None
    for n in range(0, (Q - 1) * L + 1):
        ev = spectrum(Q, L, n, bonds, jxy, jz)
        assert abs(ev[-1] - S * S * len(bonds)) < 1e-10
        if prev is not None and n <= (Q - 1) * L / 2:
            for e in prev:
                assert np.min(np.abs(ev - e)) < 1e-9
        prev = ev
        # particle-hole (spin flip) symmetry
        ev2 = spectrum(Q, L, (Q - 1) * L - n, bonds, jxy, jz)
        assert np.allclose(ev, ev2, atol=1e-10)


def test_split_invariance_of_y():
    Q, L, n = 2, 10, 4
    rng = np.random.default_rng(5)
    bonds, _, _ = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    jxy, jz = rng.normal(size=len(bonds)), rng.normal(size=len(bonds))
    a = BruteSector(Q, L, n, [10])
    b = BruteSector(Q, L, n, [3, 3, 4])
    xa = rng.normal(size=a.dim)
    perm = b.rank(a.states)                  # position of a's states in b's order
    xb = np.empty_like(xa)
    xb[perm] = xa
    ya = apply_h(a, bonds, jxy, jz, xa)
    yb = apply_h(b, bonds, jxy, jz, xb)
    assert np.allclose(yb[perm], ya, atol=1e-13)


def test_native_hx_equals_python():
    for Q, L, n, sp, k in [(2, 12, 5, [4, 4, 4], 1), (2, 11, 6, [5, 6], 3),
                           (3, 6, 6, [2, 2, 2], 2), (4, 5, 5, [2, 3], 1)]:
        b = BruteSector(Q, L, n, sp)
        ns = native.NativeSector(Q, L, n, sp)
        rng = np.random.default_rng(L)
        bonds, _, _ = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
        jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
        x = rng.normal(size=(b.dim, k)) if k > 1 else rng.normal(size=b.dim)
        t = native.NativeTerms(bonds, jxy, jz, h)
        y = apply_h(b, bonds, jxy, jz, x, h)
        assert np.allclose(native.hx_range(ns, t, x), y, atol=1e-13)
        rows = rng.integers(0, b.dim, 50)
        assert np.allclose(native.hx_rows(ns, t, x, rows), y[rows], atol=1e-13)
        y32 = native.hx_rows(ns, t, x.astype(np.float32), rows)
        assert np.allclose(y32, apply_h(b, bonds, jxy, jz, x.astype(np.float32).astype(np.float64), h)[rows],
                           atol=1e-12)


def bethe_ground_energy(L):
    """XXX chain, J=1, periodic, M=L/2: logarithmic Bethe equations
    2L arctan(2 l_j) = 2 pi I_j + 2 sum_k arctan(l_j - l_k),  E = L/4 - sum_j 2/(1+4 l_j^2)."""
    M = L // 2
    I = np.arange(M) - (M - 1) / 2.0

    def eqs(lam):
        d = lam[:, None] - lam[None, :]
        return 2 * L * np.arctan(2 * lam) - 2 * np.pi * I - 2 * np.arctan(d).sum(axis=1)

    lam0 = 0.5 * np.tan(np.pi * I / L)
    lam = scipy.optimize.fsolve(eqs, lam0, xtol=1e-13)
    assert np.max(np.abs(eqs(lam))) < 1e-11
    return L / 4 - np.sum(2 / (1 + 4 * lam ** 2))


@pytest.mark.parametrize("L", [8, 10, 12])
def test_bethe_ansatz_small(L):
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    assert abs(spectrum(2, L, L // 2, bonds, jxy, jz)[0] - bethe_ground_energy(L)) < 1e-10


def test_bethe_ansatz_sixteen_sites_lanczos():
    """The L=16, n=8 Heisenberg ground energy (the plain-method workload) from the
    C oracle's H*x and the oracle Lanczos equals the Bethe-ansatz energy."""
    L, n = 16, 8
    ns = native.NativeSector(2, L, n, [8, 8])
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    t = native.NativeTerms(bonds, jxy, jz)
    v0 = synth.vector(ns.dim, synth.SEED_V0)
    e0, psi, _, _ = ground_state(lambda v: native.hx_range(ns, t, v), v0, 100, ns.dim)
    assert abs(e0 - bethe_ground_energy(L)) < 1e-9
    r = native.hx_range(ns, t, psi) - e0 * psi
    assert np.linalg.norm(r) < 1e-6


def test_golden_bethe_values_match_the_oracle():
    """tests/golden/bethe_e0.json (read by the benchmark for the L=34 energy error)
    holds exactly what oracle.closed_forms.bethe_e0 gives."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bethe_e0.json")
    stored = json.load(open(path))["E0"]
    for L in (8, 16, 34):
        assert abs(stored[str(L)] - bethe_ground_energy(L)) <= 1e-12 * L
