"""Host-side helpers of the generic operators, CPU only: the binding's local
operators against the oracle's spin matrices (two independent writings), and the
Lindblad superoperator terms on the doubled chain, assembled on the full space,
against the oracle's dense Lindbladian."""
import numpy as np
import pytest

import synth
from oracle.operators import full_space_matrix, lindbladian_dense, spin_matrices, string
from oracle.sector import BruteSector


def binding():
    try:
        import paper_2407_14591_amd as dq
    except Exception as e:  # the library is not built here
        pytest.skip(f"binding not importable: {e}")
    return dq


@pytest.mark.parametrize("Q", [2, 3, 4, 5])
def test_local_operators_match_the_oracle(Q):
    dq = binding()
    ref = spin_matrices(Q)
    for nm in ("Id", "Sz", "S+", "S-", "Sx", "Sy"):
        assert np.allclose(dq.local_operator(nm, Q), ref[nm], rtol=0, atol=1e-15), nm
    c, sites, M = dq.operator_string(0.5, (3, 1), ("S+", "Sy"), Q)
    c2, sites2, M2 = string(0.5, (3, 1), ("S+", "Sy"), Q)
    assert (c, sites) == (c2, sites2) and np.allclose(M, M2)
    with pytest.raises(ValueError):
        dq.local_operator("Sq", Q)


def test_lindbladian_terms_on_the_full_doubled_space():
    """The doubled-chain terms of a small Lindbladian (L = 4, n = 2: an XXZ chain from
    strings, dephasing and a hopping jump), summed on the full 2^8 space, restricted to
    the pairs (s, s') of the sector, act on vec(rho) as the dense Lindbladian."""
    dq = binding()
    Q, L, n = 2, 4, 2
    rng = np.random.default_rng(3)
    h = []
    for (i, j) in synth.chain_bonds(L, 1, periodic=False):
        a, z = rng.uniform(0.5, 1.5), rng.normal()
        h += [string(a / 2, (i, j), ("S+", "S-"), Q), string(a / 2, (i, j), ("S-", "S+"), Q),
              string(z, (i, j), ("Sz", "Sz"), Q)]
    jumps = [(0.8, string(1.0, (0,), ("Sz",), Q)), (0.3, string(1.0, (1, 2), ("S+", "S-"), Q))]
    F = full_space_matrix(Q, 2 * L, dq.lindbladian_terms(L, h, jumps))
    bs = BruteSector(Q, L, n)
    pairs = ((bs.states[:, None].astype(np.int64) << L) | bs.states[None, :].astype(np.int64)).ravel()
    R = rng.normal(size=(bs.dim, bs.dim)) + 1j * rng.normal(size=(bs.dim, bs.dim))
    rho = R @ R.conj().T
    v = np.zeros(2 ** (2 * L), dtype=np.complex128)
    v[pairs] = rho.ravel()
    got = (F @ v)[pairs].reshape(bs.dim, bs.dim)
    assert np.allclose(got, lindbladian_dense(bs, h, jumps, rho), rtol=1e-12, atol=1e-12)
