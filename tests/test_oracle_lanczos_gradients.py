"""Pins of the oracle Lanczos and gradients: dense diagonalisation of the full 2^L
matrix, free fermions, Majumdar-Ghosh, breakdown cases, finite differences
(exact for a linear map) and Hellmann-Feynman against finite differences of the
dense ground energy.  CPU only."""
import itertools

import numpy as np
import pytest

import synth
from oracle import native
from oracle.gradients import adjoint, chain_rule_j_delta, hellmann_feynman
from oracle.hamiltonian import apply_h, full_basis_digit_sums, full_matrix
from oracle.lanczos import ground_state, lanczos, ritz
from oracle.sector import BruteSector, default_split


@pytest.mark.parametrize("L,n", [(10, 5), (12, 6), (11, 3)])
def test_lanczos_matches_full_dense(L, n):
    rng = np.random.default_rng(L)
    bonds, _, _ = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    jxy, jz = rng.uniform(0.5, 1.5, len(bonds)), rng.uniform(0, 2, len(bonds))
    Hf = full_matrix(2, L, bonds, jxy, jz)
    sums = full_basis_digit_sums(2, L)
    sel = np.nonzero(sums == n)[0]
    ev_full = np.linalg.eigvalsh(Hf[np.ix_(sel, sel)])
    b = BruteSector(2, L, n, default_split(2, L))
    e0, psi, alpha, beta = ground_state(lambda v: apply_h(b, bonds, jxy, jz, v),
                                        synth.vector(b.dim, synth.SEED_V0), 120, b.dim)
    assert abs(e0 - ev_full[0]) < 1e-10 * max(1, abs(ev_full[0]))
    assert np.linalg.norm(apply_h(b, bonds, jxy, jz, psi) - e0 * psi) < 1e-6


def test_lanczos_majumdar_ghosh_16():
    ns = native.NativeSector(2, 16, 8, [8, 8])
    bonds, jxy, jz = synth.j1j2_chain(16, 1.0, 0.5, 1.0)
    t = native.NativeTerms(bonds, jxy, jz)
    a, bt, _ = lanczos(lambda v: native.hx_range(ns, t, v), synth.vector(ns.dim, 3), 120, ns.dim)
    assert abs(ritz(a, bt)[0] + 6.0) < 1e-10


@pytest.mark.slow
def test_lanczos_free_fermions_20():
    L, n = 20, 10
    ns = native.NativeSector(2, L, n, [6, 7, 7])
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 0.0)
    t = native.NativeTerms(bonds, jxy, jz)
    eps = np.sort(np.cos(2 * np.pi * (np.arange(L) + 0.5) / L))
    a, bt, _ = lanczos(lambda v: native.hx_range(ns, t, v), synth.vector(ns.dim, 3), 150, ns.dim)
    assert abs(ritz(a, bt)[0] - eps[:n].sum()) < 1e-9


def test_lanczos_breakdown_small_sectors():
    bonds, jxy, jz = synth.xxz_chain(8, 1.0, 1.0)
    b0 = BruteSector(2, 8, 0, [4, 4])
    a, bt, _ = lanczos(lambda v: apply_h(b0, bonds, jxy, jz, v), np.ones(1), 50, 1)
    assert len(a) == 1 and abs(a[0] - 2.0) < 1e-14
    b1 = BruteSector(2, 8, 1, [4, 4])
    a, bt, _ = lanczos(lambda v: apply_h(b1, bonds, jxy, jz, v), synth.vector(8, 3), 50, 8)
    assert len(a) <= 8
    ev = np.sort(1.0 * (1.0 * (8 - 4) / 4 + np.cos(2 * np.pi * np.arange(8) / 8)))
    assert abs(ritz(a, bt)[0] - ev[0]) < 1e-12


# ---------------------------------------------------------------- gradients

def _setup(L=8, n=4, seed=4):
    b = BruteSector(2, L, n, default_split(2, L))
    bonds, _, _ = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    J, Dl = synth.random_couplings(len(bonds), seed)
    return b, bonds, J, Dl


def test_adjoint_matches_finite_differences():
    b, bonds, J, Dl = _setup()
    jxy, jz = J, J * Dl
    rng = np.random.default_rng(9)
    x, g = rng.normal(size=b.dim), rng.normal(size=b.dim)
    h = rng.normal(size=b.L)
    gx, gj, gz, gh = adjoint(b, bonds, jxy, jz, x, g, h)

    def loss(jxy_, jz_, x_, h_):
        return float(g @ apply_h(b, bonds, jxy_, jz_, x_, h_))

    eps = 1e-3
    for k in range(len(bonds)):
        e = np.zeros(len(bonds))
        e[k] = eps
        fd = (loss(jxy + e, jz, x, h) - loss(jxy - e, jz, x, h)) / (2 * eps)
        assert abs(fd - gj[k]) < 1e-10
        fd = (loss(jxy, jz + e, x, h) - loss(jxy, jz - e, x, h)) / (2 * eps)
        assert abs(fd - gz[k]) < 1e-10
    for i in range(b.L):
        e = np.zeros(b.L)
        e[i] = eps
        fd = (loss(jxy, jz, x, h + e) - loss(jxy, jz, x, h - e)) / (2 * eps)
        assert abs(fd - gh[i]) < 1e-10
    u = rng.normal(size=b.dim)
    fd = (loss(jxy, jz, x + eps * u, h) - loss(jxy, jz, x - eps * u, h)) / (2 * eps)
    assert abs(fd - gx @ u) < 1e-9


def test_chain_rule_j_delta():
    b, bonds, J, Dl = _setup(seed=6)
    rng = np.random.default_rng(2)
    x, g = rng.normal(size=b.dim), rng.normal(size=b.dim)
    _, gj, gz, _ = adjoint(b, bonds, J, J * Dl, x, g)
    gJ, gD = chain_rule_j_delta(J, Dl, gj, gz)

    def loss(J_, D_):
        return float(g @ apply_h(b, bonds, J_, J_ * D_, x))

    eps = 1e-4
    for k in range(len(bonds)):
        e = np.zeros(len(bonds))
        e[k] = eps
        assert abs((loss(J + e, Dl) - loss(J - e, Dl)) / (2 * eps) - gJ[k]) < 1e-8
        assert abs((loss(J, Dl + e) - loss(J, Dl - e)) / (2 * eps) - gD[k]) < 1e-8


def test_hellmann_feynman_vs_dense_finite_differences():
    b, bonds, J, Dl = _setup(L=10, n=5, seed=8)
    jxy, jz = J, J * Dl
    sel = np.nonzero(full_basis_digit_sums(2, 10) == 5)[0]

    def e0(jxy_, jz_):
        return np.linalg.eigvalsh(full_matrix(2, 10, bonds, jxy_, jz_)[np.ix_(sel, sel)])[:2]

    ev = e0(jxy, jz)
    assert ev[1] - ev[0] > 1e-3          # non-degenerate: HF applies
    _, psi, _, _ = ground_state(lambda v: apply_h(b, bonds, jxy, jz, v),
                                synth.vector(b.dim, 3), 200, b.dim)
    gj, gz = hellmann_feynman(b, bonds, psi)
    eps = 1e-5
    for k in [0, 3, 7, 12, 19]:
        e = np.zeros(len(bonds))
        e[k] = eps
        fd = (e0(jxy + e, jz)[0] - e0(jxy - e, jz)[0]) / (2 * eps)
        assert abs(fd - gj[k]) < 1e-7
        fd = (e0(jxy, jz + e)[0] - e0(jxy, jz - e)[0]) / (2 * eps)
        assert abs(fd - gz[k]) < 1e-7


@pytest.mark.parametrize("Q,L,n,split,k", [(2, 12, 6, [4, 4, 4], 1), (2, 10, 4, [5, 5], 2),
                                           (3, 6, 6, [2, 2, 2], 4)])
def test_c_bond_sums_match_finite_differences(Q, L, n, split, k):
    """The C oracle's coupling and field sums (g . A_b x, g . Z_b x, g . Sz_i x, summed
    over rows and columns) against central differences of g . H(theta) x evaluated by
    the C oracle's own row-by-row product (exact for a map linear in theta)."""
    rng = np.random.default_rng(Q * L + k)
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    ns = native.NativeSector(Q, L, n, split)
    shape = (ns.dim, k) if k > 1 else (ns.dim,)
    x, g = rng.normal(size=shape), rng.normal(size=shape)
    jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
    gxy, gz, gh = native.bond_sums(ns, bonds, x, g, fields=True)

    def loss(a, b, f):
        return float(np.sum(g * native.hx_range(ns, native.NativeTerms(bonds, a, b, f), x)))

    eps = 0.5
    for q in range(len(bonds)):
        e = np.zeros(len(bonds))
        e[q] = eps
        fd_xy = (loss(jxy + e, jz, h) - loss(jxy - e, jz, h)) / (2 * eps)
        fd_z = (loss(jxy, jz + e, h) - loss(jxy, jz - e, h)) / (2 * eps)
        assert abs(fd_xy - gxy[q]) <= 1e-10 * max(1.0, abs(fd_xy)), (q, fd_xy, gxy[q])
        assert abs(fd_z - gz[q]) <= 1e-10 * max(1.0, abs(fd_z)), (q, fd_z, gz[q])
    for i in range(L):
        e = np.zeros(L)
        e[i] = eps
        fd_h = (loss(jxy, jz, h + e) - loss(jxy, jz, h - e)) / (2 * eps)
        assert abs(fd_h - gh[i]) <= 1e-10 * max(1.0, abs(fd_h)), (i, fd_h, gh[i])
