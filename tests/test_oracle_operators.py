"""Pins of the generic-operator oracle (Sec. 4.1 operator strings, App. C terms):
closed forms of the spin matrices, the XXZ Hamiltonian rebuilt from operator strings
against the XXZ oracle, and the push-form product against the operator built on the
whole Q^L space from tensor contractions alone."""
import numpy as np
import pytest

import synth
from oracle.hamiltonian import apply_h
from oracle.operators import apply_operator, sector_matrix, spin_matrices, string
from oracle.sector import BruteSector


@pytest.mark.parametrize("Q", [2, 3, 4, 5])
def test_spin_matrices_closed_forms(Q):
    m = spin_matrices(Q)
    S = (Q - 1) / 2
    sp, sm, sz = m["S+"], m["S-"], m["Sz"]
    assert np.allclose(sp.T, sm)
    assert np.allclose(sp @ sm - sm @ sp, 2 * sz)                      # [S+, S-] = 2 Sz
    assert np.allclose(sz @ sp - sp @ sz, sp)                          # [Sz, S+] = S+
    assert np.allclose((sp @ sm + sm @ sp) / 2 + sz @ sz, S * (S + 1) * np.eye(Q))  # Casimir
    assert np.allclose(np.diag(sz), np.arange(Q) - S)


def xxz_terms(Q, bonds, jxy, jz, h):
    terms = []
    for (i, j), a, z in zip(bonds, jxy, jz):
        terms.append(string(a / 2, (i, j), ("S+", "S-"), Q))
        terms.append(string(a / 2, (i, j), ("S-", "S+"), Q))
        terms.append(string(z, (i, j), ("Sz", "Sz"), Q))
    for i, hi in enumerate(h):
        terms.append(string(hi, (i,), ("Sz",), Q))
    return terms


@pytest.mark.parametrize("Q,L,n", [(2, 10, 5), (2, 9, 3), (3, 6, 6), (4, 5, 7)])
def test_xxz_from_operator_strings(Q, L, n):
    rng = np.random.default_rng(Q * 100 + L)
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
    bs = BruteSector(Q, L, n)
    x = rng.normal(size=bs.dim)
    y = apply_operator(bs, xxz_terms(Q, bonds, jxy, jz, h), x)
    assert np.allclose(y, apply_h(bs, bonds, jxy, jz, x, h=h), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("Q,L,n", [(2, 8, 4), (2, 7, 2), (3, 5, 4), (4, 4, 6)])
def test_push_form_against_full_space(Q, L, n):
    """Random conserving terms on 1, 2 and 3 sites, site lists in any order, matrices not
    symmetric: the sector block of the full-space operator times x."""
    rng = np.random.default_rng(Q * 10 + L)
    terms = [(1.5, (3,), synth.random_local_matrix(Q, 1, 1)),
             (-0.7, (L - 1, 1), synth.random_local_matrix(Q, 2, 2)),
             (0.3, (0, 2, L - 1), synth.random_local_matrix(Q, 3, 3, density=0.5)),
             (1.1, (2, 0), synth.random_local_matrix(Q, 2, 4))]
    bs = BruteSector(Q, L, n)
    x = rng.normal(size=bs.dim)
    assert np.allclose(apply_operator(bs, terms, x), sector_matrix(bs, terms) @ x, rtol=1e-12, atol=1e-12)


def test_nonconserving_term_rejected():
    bs = BruteSector(2, 6, 3)
    with pytest.raises(ValueError):
        apply_operator(bs, [string(1.0, (0,), ("S+",), 2)], np.ones(bs.dim))


def test_full_space_pin_catches_a_transposed_term():
    """The full-space construction distinguishes M from its transpose (a plausible
    mistake in either form)."""
    Q, L = 2, 6
    M = synth.random_local_matrix(Q, 2, 9)
    bs = BruteSector(Q, L, 3)
    x = np.random.default_rng(1).normal(size=bs.dim)
    a = sector_matrix(bs, [(1.0, (1, 4), M)]) @ x
    b = sector_matrix(bs, [(1.0, (1, 4), M.T)]) @ x
    assert not np.allclose(a, b)
    assert np.allclose(apply_operator(bs, [(1.0, (1, 4), M)], x), a, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("Q,L,n", [(2, 8, 4), (3, 5, 5)])
def test_complex_sy_strings_rebuild_the_real_xxz(Q, L, n):
    """Sx Sx + Sy Sy with the complex Sy = (S+ - S-)/(2i) equals (S+S- + S-S+)/2: the
    XXZ Hamiltonian built from Sx and Sy strings (complex matrices) has no imaginary
    part and equals the XXZ oracle on complex and real vectors."""
    rng = np.random.default_rng(Q + L)
    bonds = synth.chain_bonds(L, 1)
    jxy, jz = rng.normal(size=len(bonds)), rng.normal(size=len(bonds))
    terms = []
    for (i, j), a, z in zip(bonds, jxy, jz):
        # Sx Sx and Sy Sy each change the particle number; their sum does not
        xy = string(1.0, (i, j), ("Sx", "Sx"), Q)[2] + string(1.0, (i, j), ("Sy", "Sy"), Q)[2]
        terms += [(a, (i, j), xy), string(z, (i, j), ("Sz", "Sz"), Q)]
    assert any(np.iscomplexobj(M) for _, _, M in terms)
    bs = BruteSector(Q, L, n)
    xr, xi = rng.normal(size=bs.dim), rng.normal(size=bs.dim)
    y = apply_operator(bs, terms, xr + 1j * xi)
    assert np.allclose(y, apply_h(bs, bonds, jxy, jz, xr) + 1j * apply_h(bs, bonds, jxy, jz, xi),
                       rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("Q,L,n", [(2, 7, 3), (3, 5, 4)])
def test_complex_push_form_against_full_space(Q, L, n):
    """Complex conserving terms (random phases, a Dzyaloshinskii-Moriya-like
    i(S+S- - S-S+) term): the push form against the full-space tensor contraction, and
    the Hermitian part of the operator gives a Hermitian sector matrix."""
    rng = np.random.default_rng(L)
    M2 = synth.random_local_matrix(Q, 2, 3) * np.exp(1j * rng.uniform(0, 2 * np.pi, (Q * Q, Q * Q)))
    dm = 1j * (string(1.0, (0, 1), ("S+", "S-"), Q)[2] - string(1.0, (0, 1), ("S-", "S+"), Q)[2])
    terms = [(0.8, (1, L - 1), M2), (1.3, (2, 3), dm), (0.4, (0,), synth.random_local_matrix(Q, 1, 8) + 0j)]
    bs = BruteSector(Q, L, n)
    x = rng.normal(size=bs.dim) + 1j * rng.normal(size=bs.dim)
    A = sector_matrix(bs, terms)
    assert np.allclose(apply_operator(bs, terms, x), A @ x, rtol=1e-12, atol=1e-12)
    H = sector_matrix(bs, [(1.3, (2, 3), dm)])
    assert np.allclose(H, H.conj().T) and np.abs(H.imag).max() > 0


def test_lindbladian_dense_pins():
    """Trace and Hermiticity preservation; a pure dephasing channel A = Sz_i damps each
    element rho_ss' at the closed-form rate g/2 (m_i(s) - m_i(s'))^2; an eigenprojector
    of H is stationary without jumps."""
    from oracle.operators import lindbladian_dense
    Q, L, n = 2, 6, 3
    bs = BruteSector(Q, L, n)
    rng = np.random.default_rng(4)
    bonds = synth.chain_bonds(L, 1)
    h_terms = xxz_terms(Q, bonds, rng.uniform(0.5, 1.5, len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L))
    jumps = [(0.7, string(1.0, (2,), ("Sz",), Q)), (0.3, string(1.0, (0, 1), ("S+", "S-"), Q))]
    R = rng.normal(size=(bs.dim, bs.dim)) + 1j * rng.normal(size=(bs.dim, bs.dim))
    rho = R @ R.conj().T
    out = lindbladian_dense(bs, h_terms, jumps, rho)
    assert abs(np.trace(out)) < 1e-10 * np.abs(rho).sum()
    assert np.allclose(out, out.conj().T, atol=1e-12)
    g = 0.9
    deph = lindbladian_dense(bs, [], [(g, string(1.0, (3,), ("Sz",), Q))], rho)
    m = np.array([(int(st) >> (L - 1 - 3)) & 1 for st in bs.states]) - 0.5
    assert np.allclose(deph, -g / 2 * (m[:, None] - m[None, :]) ** 2 * rho, atol=1e-12)
    w, v = np.linalg.eigh(sector_matrix(bs, h_terms))
    P = np.outer(v[:, 0], v[:, 0].conj())
    assert np.abs(lindbladian_dense(bs, h_terms, [], P)).max() < 1e-12
