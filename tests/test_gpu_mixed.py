"""GPU sectors and operators on sites of different local dimensions (the
generalisation Sec. 5 names): rank / unrank / enumerate / sorted-list rank bit-exact
against the brute-force mixed oracle, properties of a 7.9-million-state sector, the
generic operators against the term-by-term oracle, Lanczos against dense
diagonalisation and against the Lieb-Mattis ground-state spin of an alternating
spin-1/2 / spin-1 ring, and the XXZ products refusing such sectors."""
import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, rel_err, say, to_dev, to_host_u64
from oracle import mixed
from oracle.operators import spin_matrices
from oracle.sector import canonical_keys, nbits_for

pytestmark = pytest.mark.gpu
BAD = np.uint64(2 ** 64 - 1)

CASES = [([2, 3] * 4, 5, [4, 4]), ([2, 3] * 4, 0, None), ([2, 3] * 4, 12, [2, 2, 2, 2]),
         ([3, 2, 4, 2, 3], 6, [2, 3]), ([2, 2, 3, 3, 4, 2, 2], 5, None), ([5, 2, 3, 4, 2], 7, [1, 2, 2]),
         ([2] * 6 + [3] * 6, 7, [6, 6]), ([4, 2, 2, 2, 2, 2, 2, 4], 6, [3, 5]), ([3, 2], 2, [1, 1])]


@pytest.mark.parametrize("bits", ["32", "64"])
def test_mixed_rank_unrank_enumerate(monkeypatch, bits):
    if bits == "64":
        monkeypatch.setenv("DCS_INDEX_BITS", "64")
    for dims, n, sp in CASES:
        ms = mixed.MixedSector(dims, n, sp)
        s = dq.Sector(len(dims), n, dims, sp)
        say("mixed sector", dims, n, s.split, bits, ms.dim)
        assert s.local_dims == dims and s.Q == max(dims)
        assert s.dim == ms.dim == mixed.dim_poly(dims, n)
        assert s.split == ms.split
        st = to_dev(ms.states)
        idx, bad = s.rank(st, count_invalid=True)
        assert np.array_equal(to_host_u64(idx), np.arange(ms.dim, dtype=np.uint64)) and int(bad.item()) == 0
        assert np.array_equal(to_host_u64(s.rank_search(st)), np.arange(ms.dim, dtype=np.uint64))
        back = s.unrank(to_dev(np.arange(ms.dim, dtype=np.uint64)))
        assert np.array_equal(to_host_u64(back), ms.states)
        assert np.array_equal(to_host_u64(s.enumerate(0, ms.dim)), ms.states)
        first = ms.dim // 3
        assert np.array_equal(to_host_u64(s.enumerate(first, ms.dim - first)), ms.states[first:])
        s.close()


def test_mixed_invalid_digits_flagged():
    """A digit at or above its site's dimension (but inside the packing width) is
    outside the sector, also when the digit sum is right."""
    dims, n = [2, 3, 2, 3], 2
    s = dq.Sector(4, n, dims, [2, 2])
    nb = 2
    pk = lambda d: sum(v << (nb * (3 - i)) for i, v in enumerate(d))
    states = np.array([pk([2, 0, 0, 0]), pk([0, 0, 2, 0]), pk([0, 2, 0, 0]), pk([1, 0, 0, 1]), pk([0, 3, 0, 0]),
                       pk([1, 1, 1, 0])], dtype=np.uint64)
    ref = mixed.MixedSector(dims, n, [2, 2]).rank(states)
    assert list(ref[:4] >= 0) == [False, False, True, True] and ref[4] == -1 and ref[5] == -1
    for f in (s.rank, s.rank_search):
        idx, cnt = f(to_dev(states), count_invalid=True)
        h = to_host_u64(idx)
        assert np.all(h[[0, 1, 4, 5]] == BAD) and int(cnt.item()) == 4
        assert np.array_equal(h[[2, 3]].astype(np.int64), ref[[2, 3]])


def test_mixed_large_sector_properties():
    """Alternating spin-1/2, spin-1 sites, L = 20, Sz = 0 (7,873,260 states): the
    dimension from the generating function, every enumerated state valid and in
    strictly increasing canonical order, rank of the enumeration = 0..D-1, unrank
    the enumeration back."""
    dims = [2, 3] * 10
    n = 15
    s = dq.Sector(20, n, dims)
    assert s.dim == mixed.dim_poly(dims, n)
    say("mixed large", s.dim, s.split)
    st = s.enumerate(0, s.dim)
    h = to_host_u64(st)
    nb = nbits_for(3)
    dig = np.stack([((h >> np.uint64(nb * (19 - i))) & np.uint64(3)).astype(np.int64) for i in range(20)], axis=1)
    assert np.all(dig < np.array(dims)) and np.all(dig.sum(axis=1) == n)
    keys = canonical_keys(h, 3, s.split)
    # strictly increasing in the canonical order: lexicographic comparison of consecutive key rows
    diff = keys[1:] - keys[:-1]
    first_nz = np.argmax(diff != 0, axis=1)
    assert np.all(diff[np.arange(len(diff)), first_nz] > 0)
    ar = torch.arange(s.dim, device=DEV, dtype=torch.int64)
    assert torch.equal(s.rank(st), ar)
    assert torch.equal(s.unrank(ar), st)
    s.close()


def random_terms(dims, seed, cplx=False):
    rng = np.random.default_rng(seed)
    L = len(dims)
    terms = []
    for t in range(2 * L):
        m = 1 + t % 3
        sites = tuple(int(v) for v in rng.choice(L, size=m, replace=False))
        M = synth.random_local_matrix_dims([dims[v] for v in sites], seed * 100 + t, density=0.7)
        if cplx:
            M = M + 1j * np.where(M != 0, synth.random_local_matrix_dims([dims[v] for v in sites], seed * 100 + t + 50), 0)
        terms.append((float(rng.normal()), sites, M))
    return terms


@pytest.mark.parametrize("dims,n,split", [([2, 3] * 4, 5, [4, 4]), ([3, 2, 4, 2, 3], 6, [2, 3]),
                                         ([2, 2, 3, 3, 4, 2, 2], 5, None)])
@pytest.mark.parametrize("cluster", [1, 2, 4])
def test_mixed_operator_matches_oracle(dims, n, split, cluster):
    L = len(dims)
    terms = random_terms(dims, 11 + L)
    op = dq.Operator(dims, L, terms, cluster_sites=cluster)
    ms = mixed.MixedSector(dims, n, split)
    s = dq.Sector(L, n, dims, split)
    x = np.random.default_rng(L).normal(size=ms.dim)
    ref = mixed.apply_operator(ms, terms, x)
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        y = dq.operator_apply(s, op, torch.tensor(x, device=DEV).to(dt))
        err = rel_err(y.double().cpu().numpy(), ref)
        say("mixed operator", dims, n, cluster, dt, op.num_clusters, op.nnz, err)
        assert err <= tol
    # a block of 4 real columns
    X = np.random.default_rng(L + 1).normal(size=(ms.dim, 4))
    Y = dq.operator_apply(s, op, torch.tensor(X, device=DEV)).cpu().numpy()
    for c in range(4):
        assert rel_err(Y[:, c], mixed.apply_operator(ms, terms, X[:, c])) <= 1e-12


def test_mixed_complex_operator():
    dims, n = [3, 2, 2, 3, 2, 4], 6
    L = len(dims)
    terms = random_terms(dims, 5, cplx=True)
    op = dq.Operator(dims, L, terms, cluster_sites=3)
    assert op.is_complex
    ms = mixed.MixedSector(dims, n)
    s = dq.Sector(L, n, dims)
    rng = np.random.default_rng(9)
    x = rng.normal(size=ms.dim) + 1j * rng.normal(size=ms.dim)
    ref = mixed.apply_operator(ms, terms, x)
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        y = dq.operator_apply(s, op, torch.tensor(x, device=DEV).to(dt))
        err = rel_err(y.cpu().numpy(), ref)
        say("mixed complex operator", dt, err)
        assert err <= tol


def heisenberg_ring(dims):
    L = len(dims)
    terms = []
    for i in range(L):
        j = (i + 1) % L
        for nm in ("Sz", "S+", "S-"):
            other = {"Sz": "Sz", "S+": "S-", "S-": "S+"}[nm]
            terms.append(dq.operator_string(1.0 if nm == "Sz" else 0.5, (i, j), (nm, other), dims))
    return terms


def test_mixed_lanczos_against_dense():
    dims = [2, 3] * 4
    L, n = 8, 6
    terms = heisenberg_ring(dims)
    op = dq.Operator(dims, L, terms, cluster_sites=4)
    s = dq.Sector(L, n, dims)
    ms = mixed.MixedSector(dims, n, s.split)
    ev = np.linalg.eigvalsh(mixed.sector_matrix(ms, terms))
    v0 = torch.tensor(synth.vector(s.dim, synth.SEED_V0), device=DEV)
    r = dq.lanczos(s, op, None, None, v0, min(s.dim, 120), reorth="full", num_eig=3)
    say("mixed lanczos L8", r["eig"][:3], ev[:3])
    assert np.allclose(r["eig"][:3], ev[:3], atol=1e-9)


def test_mixed_ring_lieb_mattis():
    """Alternating spin-1/2, spin-1 Heisenberg ring, L = 16: total ground-state spin
    8 (1 - 1/2) = 4, so the Sz = 0 and Sz = 4 sectors share the lowest energy and
    Sz = 5 lies above it."""
    dims = [2, 3] * 8
    L = 16
    smax = sum(q - 1 for q in dims) // 2  # Sz = n - 12
    op = dq.Operator(dims, L, heisenberg_ring(dims), cluster_sites=4)
    e = {}
    for sz in (0, 4, 5):
        s = dq.Sector(L, smax + sz, dims)
        v0 = torch.tensor(synth.vector(s.dim, synth.SEED_V0), device=DEV)
        r = dq.lanczos(s, op, None, None, v0, 200, reorth="local", num_eig=1)
        e[sz] = r["eig"][0]
        say("mixed ring", sz, s.dim, e[sz], r["steps_done"])
        s.close()
    assert abs(e[0] - e[4]) <= 1e-8
    assert e[5] > e[4] + 1e-3


def test_mixed_refusals():
    dims = [2, 3, 2, 3, 2, 3]
    s = dq.Sector(6, 4, dims)
    t = dq.Terms(synth.chain_bonds(6, 1))
    j = torch.ones(6, dtype=torch.float64, device=DEV)
    x = torch.zeros(s.dim, dtype=torch.float64, device=DEV)
    with pytest.raises(dq.DcsError) as e:
        dq.hamiltonian_apply(s, t, j, j, x)
    assert e.value.code == dq._lib.DCS_EUNSUPPORTED
    with pytest.raises(dq.DcsError):
        dq.hamiltonian_apply_adjoint(s, t, j, j, x, x)
    with pytest.raises(dq.DcsError):
        dq.Plan([(s, t, j, j)])
    with pytest.raises(dq.DcsError):
        dq.lanczos(s, t, j, j, x + 1, 5)
    # an operator for other local dimensions
    for Q in (3, [3, 2, 3, 2, 3, 2]):
        op = dq.Operator(Q, 6, [dq.operator_string(1.0, (0, 1), ("S+", "S-"), Q)])
        with pytest.raises(dq.DcsError) as e:
            dq.operator_apply(s, op, x)
        assert e.value.code == dq._lib.DCS_EINVAL
    # one dimension everywhere through the mixed entry point: the uniform sector
    u = dq.Sector(8, 4, [2] * 8, [4, 4])
    v = dq.Sector(8, 4, 2, [4, 4])
    assert u.dim == v.dim and torch.equal(u.enumerate(0, u.dim), v.enumerate(0, v.dim))


@pytest.mark.parametrize("dims,n", [([2, 3] * 4, 5), ([3, 2, 4, 2, 3], 6), ([5, 2, 3, 4, 2], 7), ([2, 3], 2),
                                    ([4, 2, 2, 3, 2, 2, 4], 0), ([2, 3, 2, 3, 2, 3], 9)])
def test_mixed_on_the_fly_full(dims, n):
    """The on-the-fly container (N = L, no tables of states) with a local dimension per
    site: every state in the order of L one-site subsystems (the brute-force mixed oracle)
    against rank and unrank; a digit above its site's dimension ranked out."""
    L = len(dims)
    ms = mixed.MixedSector(dims, n, [1] * L)
    ar = np.arange(ms.dim, dtype=np.uint64)
    idx, bad = dq.lex_rank(L, n, to_dev(ms.states), count_invalid=True, Q=dims)
    assert int(bad.item()) == 0 and np.array_equal(to_host_u64(idx), ar)
    back, bad = dq.lex_unrank(L, n, to_dev(ar), count_invalid=True, Q=dims)
    assert int(bad.item()) == 0 and np.array_equal(to_host_u64(back), ms.states)
    if min(dims) == 2 and max(dims) > 2:  # site with dimension 2 holding digit 2
        nb = nbits_for(max(dims))
        i2 = dims.index(2)
        s = np.uint64(2) << np.uint64(nb * (L - 1 - i2))
        _, cnt = dq.lex_rank(L, 2, to_dev(np.array([s], dtype=np.uint64)), count_invalid=True, Q=dims)
        assert int(cnt.item()) == 1


def test_mixed_on_the_fly_large():
    """Alternating spin-1/2, spin-1 sites, L = 32, Sz = 0 (64 packed bits): 2^20 random
    indices unrank to valid states whose numeric order is the index order (the
    lexicographic order of L one-site subsystems), rank back to themselves; indices >= D
    are counted."""
    dims = [2, 3] * 16
    L, n = 32, 24
    dim = mixed.dim_poly(dims, n)
    ids = np.sort(np.random.default_rng(4).integers(0, dim, size=1 << 20, dtype=np.int64)).astype(np.uint64)
    ids = np.unique(ids)
    st = dq.lex_unrank(L, n, to_dev(ids), Q=dims)
    h = to_host_u64(st)
    assert np.all(np.diff(h.astype(object)) > 0) if len(h) < 1000 else np.all(h[1:] > h[:-1])
    dig = np.stack([((h >> np.uint64(2 * (L - 1 - i))) & np.uint64(3)).astype(np.int64) for i in range(L)], axis=1)
    assert np.all(dig < np.array(dims)) and np.all(dig.sum(axis=1) == n)
    assert np.array_equal(to_host_u64(dq.lex_rank(L, n, st, Q=dims)), ids)
    _, cnt = dq.lex_unrank(L, n, to_dev(np.array([dim - 1, dim, dim + 5], dtype=np.uint64)), count_invalid=True, Q=dims)
    assert int(cnt.item()) == 2


def test_mixed_tables_in_device_memory(monkeypatch):
    """The same sectors with their tables read in device memory (the kernels' global-table
    path): rank, sorted-list rank, unrank, enumerate and an operator product."""
    monkeypatch.setenv("DCS_GLOBAL_TABLES", "1")
    for dims, n, sp in [([2, 3] * 4, 5, [4, 4]), ([3, 2, 4, 2, 3], 6, [2, 3]), ([2] * 6 + [3] * 6, 7, [6, 6])]:
        ms = mixed.MixedSector(dims, n, sp)
        s = dq.Sector(len(dims), n, dims, sp)
        assert s.tables_in_device_memory
        st = to_dev(ms.states)
        ar = np.arange(ms.dim, dtype=np.uint64)
        assert np.array_equal(to_host_u64(s.rank(st)), ar)
        assert np.array_equal(to_host_u64(s.rank_search(st)), ar)
        assert np.array_equal(to_host_u64(s.unrank(to_dev(ar))), ms.states)
        assert np.array_equal(to_host_u64(s.enumerate(0, ms.dim)), ms.states)
        terms = random_terms(dims, 40 + len(dims))
        op = dq.Operator(dims, len(dims), terms, cluster_sites=4)
        x = np.random.default_rng(6).normal(size=ms.dim)
        err = rel_err(dq.operator_apply(s, op, torch.tensor(x, device=DEV)).cpu().numpy(),
                      mixed.apply_operator(ms, terms, x))
        say("mixed global tables", dims, n, err)
        assert err <= 1e-12
        s.close()


def test_mixed_ring_full_size_properties():
    """The bench's mixed-dimension workload at its size (alternating spin-1/2 / spin-1
    Heisenberg ring, L = 24, Sz = 0, 259,258,780 states), by properties that hold at any
    size: the operator is symmetric (<u, H v> = <H u, v> to 1e-12), the FP32 product
    agrees with the FP64 one to 1e-5, and the expectation call equals x . (H x)."""
    dims = [2, 3] * 12
    L, n = 24, 18
    op = dq.Operator(dims, L, heisenberg_ring(dims), cluster_sites=4)
    s = dq.Sector(L, n, dims)
    assert s.dim == mixed.dim_poly(dims, n) == 259258780
    g = torch.Generator(device=DEV)
    g.manual_seed(17)
    u = torch.randn(s.dim, generator=g, device=DEV, dtype=torch.float64)
    v = torch.randn(s.dim, generator=g, device=DEV, dtype=torch.float64)
    hv = dq.operator_apply(s, op, v)
    hu = dq.operator_apply(s, op, u)
    lhs, rhs = torch.dot(u, hv).item(), torch.dot(hu, v).item()
    scale = torch.linalg.vector_norm(u).item() * torch.linalg.vector_norm(hv).item()
    say("mixed ring L24 symmetry", lhs, rhs, scale)
    assert abs(lhs - rhs) <= 1e-12 * scale
    hv32 = dq.operator_apply(s, op, v.float()).double()
    err = (torch.linalg.vector_norm(hv32 - hv) / torch.linalg.vector_norm(hv)).item()
    assert err <= 1e-5
    e = dq.operator_expectation(s, op, u).item()
    assert abs(e - torch.dot(u, hu).item()) <= 1e-12 * torch.linalg.vector_norm(u).item() * torch.linalg.vector_norm(hu).item()
    del u, v, hu, hv, hv32
    s.close()
