"""Pins of the oracle's lowest states and expectation values (App. D): dense
diagonalisation of the full 2^L matrix built from Kronecker products of the
spin-1/2 matrices (no sector index, no oracle code), and free fermions for the
XX chain in a site-dependent field, where every eigenstate is a Slater
determinant of the L x L hopping matrix's orbitals.  CPU only."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sps

import synth
from oracle import native
from oracle.hamiltonian import apply_h
from oracle.observables import expectations, lowest_by_deflation, lowest_states
from oracle.sector import BruteSector, default_split

SZ = sps.csr_matrix(np.diag([-0.5, 0.5]))      # digit 0 -> m = -1/2, digit 1 -> m = +1/2
SP = sps.csr_matrix(np.array([[0.0, 0.0], [1.0, 0.0]]))  # S+ |d=0> = |d=1>
SM = SP.T.tocsr()


def site_op(L, ops):
    """Kronecker product with ops[i] at site i (site 0 the most significant factor)."""
    out = sps.identity(1, format="csr")
    for i in range(L):
        out = sps.kron(out, ops.get(i, sps.identity(2, format="csr")), format="csr")
    return out


def kron_terms(L, bonds):
    A = [0.5 * (site_op(L, {i: SP, j: SM}) + site_op(L, {i: SM, j: SP})) for i, j in bonds]
    Z = [site_op(L, {i: SZ, j: SZ}) for i, j in bonds]
    S = [site_op(L, {i: SZ}) for i in range(L)]
    return A, Z, S


def dense_sector(L, n, bonds, jxy, jz, h):
    A, Z, S = kron_terms(L, bonds)
    H = sum(a * M for a, M in zip(jxy, A)) + sum(c * M for c, M in zip(jz, Z))
    H = H + sum(c * M for c, M in zip(h, S))
    sel = np.array([x for x in range(2 ** L) if bin(x).count("1") == n])
    sub = lambda M: M[sel][:, sel].toarray()
    return sub(H), [sub(M) for M in A], [sub(M) for M in Z], [sub(M) for M in S]


@pytest.mark.parametrize("L,field", [(10, "tilted"), (12, "tilted"), (12, "random")])
def test_lowest_states_match_dense(L, field):
    n = L // 2
    bonds, jxy, jz, h = synth.tilted_field_chain(L)
    if field == "random":
        rng = np.random.default_rng(L)
        jxy, jz, h = rng.uniform(0.5, 1.5, len(bonds)), rng.uniform(0, 2, len(bonds)), rng.normal(size=L)
    H, A, Z, S = dense_sector(L, n, bonds, jxy, jz, h)
    ev, U = np.linalg.eigh(H)
    assert np.min(np.diff(ev[:5])) > 1e-6          # the four lowest are not degenerate
    b = BruteSector(2, L, n, default_split(2, L))
    apply = lambda v: apply_h(b, bonds, jxy, jz, v, h)
    v0 = synth.vector(b.dim, synth.SEED_V0)
    E, psi = lowest_states(apply, v0, 300, 4, b.dim)
    defl = lowest_by_deflation(apply, v0, 4, 300)
    for e in range(4):
        u = U[:, e]
        ref_sz = np.array([u @ M @ u for M in S])
        ref_xy = np.array([u @ M @ u for M in A])
        ref_z = np.array([u @ M @ u for M in Z])
        assert abs(E[e] - ev[e]) < 1e-10 * max(1, abs(ev[e]))
        assert abs(defl[e][0] - ev[e]) < 1e-10 * max(1, abs(ev[e]))
        for p in (psi[:, e], defl[e][1]):
            exy, ez, esz = expectations(b, bonds, p)
            np.testing.assert_allclose(esz, ref_sz, atol=1e-8)
            np.testing.assert_allclose(exy, ref_xy, atol=1e-8)
            np.testing.assert_allclose(ez, ref_z, atol=1e-8)
            # <H> from the term expectations is the energy
            assert abs(jxy @ exy + jz @ ez + h @ esz - ev[e]) < 1e-9 * max(1, abs(ev[e]))


def test_expectations_of_a_random_state_match_kron():
    L, n = 9, 4
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    H, A, Z, S = dense_sector(L, n, bonds, np.ones(len(bonds)), np.ones(len(bonds)), np.zeros(L))
    b = BruteSector(2, L, n, default_split(2, L))
    # the same state in both numberings: sector basis states sorted as in the
    # kron numbering (site 0 most significant) are the packed states in increasing order
    x = synth.vector(b.dim, 5)
    order = np.argsort(b.states)
    xk = x[order]
    exy, ez, esz = expectations(b, bonds, x)
    np.testing.assert_allclose(exy, [xk @ M @ xk for M in A], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ez, [xk @ M @ xk for M in Z], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(esz, [xk @ M @ xk for M in S], rtol=1e-12, atol=1e-12)
    # the C oracle's bond sums with g = x are the same numbers
    ns = native.NativeSector(2, L, n, default_split(2, L))
    gxy, gz, gh = native.bond_sums(ns, bonds, x, x, fields=True)
    np.testing.assert_allclose(gxy, exy, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gz, ez, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gh, esz, rtol=1e-12, atol=1e-12)


def test_lowest_states_free_fermions_in_a_field():
    """XX chain (Jz = 0), open, random field h_k: H = c^T T c - sum_k h_k / 2 with
    T tridiagonal (h_k on the diagonal, 1/2 beside it), so the many-body levels
    are sums of n of T's eigenvalues and <Sz_0> = sum_occupied |phi(0)|^2 - 1/2.
    (The linear field h_k = k gives a near-equidistant ladder of orbitals and
    degenerate many-body levels, so a random field is taken.)"""
    L, n = 16, 8
    bonds, jxy, jz, _ = synth.tilted_field_chain(L, jz=0.0)
    h = np.random.default_rng(16).normal(size=L)
    T = np.diag(h) + 0.5 * (np.eye(L, k=1) + np.eye(L, k=-1))
    eps, phi = np.linalg.eigh(T)
    levels = sorted((sum(eps[list(c)]) - h.sum() / 2, c) for c in itertools.combinations(range(L), n))
    E_ref = np.array([lv for lv, _ in levels[:5]])
    assert np.min(np.diff(E_ref)) > 1e-6
    ns = native.NativeSector(2, L, n, [8, 8])
    t = native.NativeTerms(bonds, jxy, jz, h)
    apply = lambda v: native.hx_range(ns, t, v)
    v0 = synth.vector(ns.dim, synth.SEED_V0)
    E, psi = lowest_states(apply, v0, 300, 4, ns.dim)
    defl = lowest_by_deflation(apply, v0, 4, 400)
    for e in range(4):
        occ = list(levels[e][1])
        sz_ref = (phi[:, occ] ** 2).sum(axis=1) - 0.5
        assert abs(E[e] - E_ref[e]) < 1e-10 * abs(E_ref[e])
        assert abs(defl[e][0] - E_ref[e]) < 1e-10 * abs(E_ref[e])
        for p in (psi[:, e], defl[e][1]):
            _, _, gh = native.bond_sums(ns, bonds, p, p, fields=True)
            np.testing.assert_allclose(gh, sz_ref, atol=1e-8)
