"""Sectors whose index tables stay in device memory (table placement, Sec. 4.2
containers and Sec. 4.3's choice of the number of subsystems): the 16/16 and
10/11/11 splits of L = 32, whose tables exceed the on-chip budget, and small
sectors forced there (DCS_GLOBAL_TABLES=1 at creation).  Against the C oracle:
rank and unrank bit-exact on 2^20 random states; H*x on sampled rows at L = 32
and on all rows at L = 24; the adjoint on the split tables; the calls that need
tables in LDS refuse with DcsError."""
import itertools

import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, rel_err, say, to_dev, to_host_u64
from oracle import native

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def sampled_rows(dim, count, seed):
    rng = np.random.default_rng(seed)
    parts = [np.arange(0, 4096, dtype=np.uint64), np.arange(dim - 4096, dim, dtype=np.uint64),
             rng.integers(0, dim, count).astype(np.uint64)]
    return np.unique(np.concatenate(parts))


@pytest.fixture(scope="module")
def x32():
    """The L=32, n=16 FP64 input (one seeded vector; each split reads it in its own order)."""
    return synth.vector(601080390, synth.SEED_X, np.float64)


@pytest.mark.parametrize("split", [[16, 16], [10, 11, 11]])
def test_device_tables_L32_rank_unrank(split):
    L, n = 32, 16
    s = dq.Sector(L, n, 2, split)
    assert s.dim == 601080390
    ns = native.NativeSector(2, L, n, split)
    st = synth.pack_digits(synth.random_states(2, L, n, 1 << 20, seed=11), 2)
    ref = ns.rank(st)
    idx = s.rank(to_dev(st))
    got = to_host_u64(idx)
    say("rank", split, int((got != ref).sum()))
    assert np.array_equal(got, ref)
    back = s.unrank(idx)
    assert np.array_equal(to_host_u64(back), st)
    # the ends of the canonical order and a ragged enumeration
    ends = np.array([0, 1, s.dim - 2, s.dim - 1], dtype=np.uint64)
    assert np.array_equal(to_host_u64(s.unrank(to_dev(ends))), ns.unrank(ends))
    first = s.dim - 1000
    assert np.array_equal(to_host_u64(s.enumerate(first, 1000)), ns.unrank(np.arange(first, s.dim, dtype=np.uint64)))
    # states outside the sector
    bad = st.copy()
    bad[:100] ^= np.uint64(1)  # one site flipped: digit sum n +- 1
    _, nbad = s.rank(to_dev(bad), count_invalid=True)
    assert int(nbad.item()) == 100


@pytest.mark.parametrize("split", [[16, 16], [10, 11, 11]])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_device_tables_L32_product_sampled(x32, split, dt):
    """J1-J2 (J2 = 0.5), k = 1: 16/16 runs the split product, 10/11/11 (runs of up
    to 705,432 rows) the one-pass kernel reading its tables in device memory."""
    L, n = 32, 16
    s = dq.Sector(L, n, 2, split)
    ns = native.NativeSector(2, L, n, split)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    t = dq.Terms(bonds)
    rows = sampled_rows(s.dim, 200_000, 9)
    y_ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), x32, rows)
    y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), torch.from_numpy(x32).to(DEV).to(dt))
    got = y[torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
    err = rel_err(got, y_ref)
    say("L32", split, dt, dq.hamiltonian_form(s, t, dt, 1), "rel err", err)
    assert err <= TOL[dt]


@pytest.mark.parametrize("split", [[12, 12], [8, 8, 8], [6, 6, 6, 6]])
@pytest.mark.parametrize("k", [1, 8])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_forced_device_tables_L24_all_rows(monkeypatch, split, k, dt):
    """L = 24, n = 12 with tables forced into device memory, every row against the
    oracle; k = 8 needs the split product, which every split here has."""
    monkeypatch.setenv("DCS_GLOBAL_TABLES", "1")
    L, n = 24, 12
    s = dq.Sector(L, n, 2, split)
    ns = native.NativeSector(2, L, n, split)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    h = np.linspace(-0.5, 0.5, L)
    x = synth.vector(s.dim, synth.SEED_X, np.float64, k=k)
    y_ref = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz, h), x)
    y = dq.hamiltonian_apply(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), torch.from_numpy(x).to(DEV).to(dt),
                             h=dev_f64(h))
    err = rel_err(y.double().cpu().numpy(), y_ref)
    say("L24 device tables", split, k, dt, "rel err", err)
    assert err <= TOL[dt]
    st = synth.pack_digits(synth.random_states(2, L, n, 1 << 16, seed=5), 2)
    assert np.array_equal(to_host_u64(s.rank(to_dev(st))), ns.rank(st))


def test_device_tables_adjoint_and_refusals(monkeypatch):
    """The adjoint with tables in device memory (FP32 and FP64, k = 1, every way the
    autotuner times; the split view exists from 2^20 rows) against the oracle; the
    calls that need tables in LDS raise DcsError instead of running."""
    monkeypatch.setenv("DCS_GLOBAL_TABLES", "1")
    L, n, split = 24, 12, [12, 12]
    s = dq.Sector(L, n, 2, split)
    ns = native.NativeSector(2, L, n, split)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    t = dq.Terms(bonds)
    x = synth.vector(s.dim, synth.SEED_X, np.float32).astype(np.float64)
    g = synth.vector(s.dim, synth.SEED_G, np.float32).astype(np.float64)
    gx_ref = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz), g)
    gj_ref, gz_ref, _ = native.bond_sums(ns, bonds, x, g)
    xd, gd = (torch.from_numpy(v).to(DEV).float() for v in (x, g))
    gx, gj, gz, _ = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz), xd, gd)
    errs = [rel_err(gx.double().cpu().numpy(), gx_ref), rel_err(gj.cpu().numpy(), gj_ref),
            rel_err(gz.cpu().numpy(), gz_ref)]
    say("adjoint on device tables", errs)
    assert max(errs) <= 1e-5
    gx, gj, gz, _ = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz), xd.double(), gd.double())
    errs = [rel_err(gx.cpu().numpy(), gx_ref), rel_err(gj.cpu().numpy(), gj_ref), rel_err(gz.cpu().numpy(), gz_ref)]
    say("FP64 adjoint on device tables", errs)
    assert max(errs) <= 1e-12
    xb = torch.stack([xd, gd], dim=1).repeat(1, 4).contiguous()
    with pytest.raises(dq.DcsError):  # a block's sums pass needs the tables in LDS
        dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz), xb, xb)
    with pytest.raises(dq.DcsError):  # a plan needs LDS tables for sectors without a split view
        dq.Plan([(dq.Sector(9, 4, 3, [3, 3, 3]), dq.Terms(synth.chain_bonds(9, 1)),
                  dev_f64(np.ones(9)), dev_f64(np.ones(9)))])


@pytest.mark.parametrize("L,n,split,min_dim", [(24, 12, [2, 2, 7, 7, 6], None), (22, 11, [1, 1, 10, 10], "0")])
@pytest.mark.parametrize("k,dt", [(1, torch.float32), (1, torch.float64), (2, torch.float64), (8, torch.float32)])
@pytest.mark.parametrize("fused", ["0", "1"])
def test_split_long_runs_all_rows(monkeypatch, L, n, split, min_dim, k, dt, fused):
    """Cuts that leave runs of 65,535 rows or more (C(20, 10) = 184,756 here): the
    split product with 32-bit target offsets, every row against the oracle, in the
    default form and in the fused one."""
    if min_dim is not None:
        monkeypatch.setenv("DCS_SPLIT_MIN_DIM", min_dim)
    monkeypatch.setenv("DCS_AUTOTUNE", "0")
    monkeypatch.setenv("DCS_SPLIT_FUSED", fused)
    s = dq.Sector(L, n, 2, split)
    ns = native.NativeSector(2, L, n, split)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    h = np.linspace(-0.3, 0.4, L)
    t = dq.Terms(bonds)
    x = synth.vector(s.dim, synth.SEED_X, np.float64, k=k)
    y_ref = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz, h), x)
    y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), torch.from_numpy(x).to(DEV).to(dt), h=dev_f64(h))
    form = dq.hamiltonian_form(s, t, dt, k)
    err = rel_err(y.double().cpu().numpy(), y_ref)
    say("long runs", L, split, k, dt, form, "rel err", err)
    assert form == ("split_fused" if fused == "1" else "split_staged")
    assert err <= TOL[dt]


def test_split_long_runs_L32_sampled(x32):
    """L=32 split 6/6/6/7/7 (cut 12 | 20, runs up to 184,756 rows), FP32 k=1 in the
    autotuner's form, sampled rows against the oracle."""
    L, n, split = 32, 16, [6, 6, 6, 7, 7]
    s = dq.Sector(L, n, 2, split)
    ns = native.NativeSector(2, L, n, split)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    t = dq.Terms(bonds)
    rows = sampled_rows(s.dim, 200_000, 10)
    y_ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), x32, rows)
    y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), torch.from_numpy(x32).to(DEV).float())
    got = y[torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
    err = rel_err(got, y_ref)
    form = dq.hamiltonian_form(s, t, torch.float32, 1)
    say("L32 6/6/6/7/7", form, "rel err", err)
    assert err <= TOL[torch.float32]


@pytest.mark.parametrize("L,n", [(1, 0), (1, 1), (12, 0), (12, 12), (16, 8), (20, 7), (24, 12), (64, 1), (64, 63)])
def test_lex_rank_unrank_full(L, n):
    """The table-free N = L order (Alg. on-the-fly) is the numeric order of the packed
    states: every state of the sector, sorted by brute force, against rank and unrank."""
    if L <= 24:
        st = np.array(sorted(sum(1 << b for b in c) for c in itertools.combinations(range(L), n)),
                      dtype=np.uint64) if L <= 16 else _all_states(L, n)
    else:  # L = 64 with one particle or one hole
        bits = [1 << b for b in range(64)]
        st = np.array(sorted(bits if n == 1 else [(2 ** 64 - 1) ^ b for b in bits]), dtype=np.uint64)
    idx, bad = dq.lex_rank(L, n, to_dev(st), count_invalid=True)
    assert int(bad.item()) == 0
    assert np.array_equal(to_host_u64(idx), np.arange(len(st), dtype=np.uint64))
    back, bad = dq.lex_unrank(L, n, to_dev(np.arange(len(st), dtype=np.uint64)), count_invalid=True)
    assert np.array_equal(to_host_u64(back), st) and int(bad.item()) == 0


def _all_states(L, n):
    """All L-bit words with n ones in increasing numeric order (numpy, by popcount filter)."""
    w = np.arange(1 << L, dtype=np.uint64)
    pc = np.zeros(len(w), dtype=np.int64)
    v = w.copy()
    for _ in range(L):
        pc += (v & np.uint64(1)).astype(np.int64)
        v >>= np.uint64(1)
    return w[pc == n]


def test_lex_rank_L32_against_oracle():
    """L = 32, n = 16: 2^20 random states round-trip; 4096 of them against the oracle's
    lexicographic rank (eq. N=L, written from the paper); invalid states and indices counted."""
    from oracle.sector import lex_rank as o_lex_rank
    L, n = 32, 16
    dig = synth.random_states(2, L, n, 1 << 20, seed=21)
    st = synth.pack_digits(dig, 2)
    idx = dq.lex_rank(L, n, to_dev(st))
    got = to_host_u64(idx)
    ref = np.array([o_lex_rank(list(d), 2) for d in dig[:4096]], dtype=np.uint64)
    assert np.array_equal(got[:4096], ref)
    assert np.array_equal(to_host_u64(dq.lex_unrank(L, n, idx)), st)
    assert int(got.max()) < 601080390
    bad = st.copy()
    bad[:50] ^= np.uint64(1 << 40)  # a bit above L
    bad[50:80] ^= np.uint64(1)      # the wrong particle number
    _, nb = dq.lex_rank(L, n, to_dev(bad), count_invalid=True)
    assert int(nb.item()) == 80
    _, nb = dq.lex_unrank(L, n, to_dev(np.array([601080389, 601080390, 2 ** 40], dtype=np.uint64)),
                          count_invalid=True)
    assert int(nb.item()) == 2


@pytest.mark.parametrize("Q,L,n", [(3, 1, 2), (3, 6, 6), (3, 8, 3), (3, 9, 0), (3, 9, 18), (4, 5, 7), (5, 4, 8),
                                   (7, 3, 9), (16, 3, 20), (2, 12, 6)])
def test_lex_rank_any_q_full(Q, L, n):
    """Any Q (eq. N=L with D_Q): every state of the sector in the canonical order of L
    one-site subsystems (the brute-force oracle's sort) against rank and unrank."""
    from oracle.sector import BruteSector
    bs = BruteSector(Q, L, n, [1] * L)
    st = to_dev(bs.states)
    ar = np.arange(bs.dim, dtype=np.uint64)
    if Q == 2:  # the any-Q kernels through the C ABI, beside the binomial ones
        out = torch.empty_like(st)
        dq._lib.call("dcs_lex_rank_q", L, n, 2, st.data_ptr(), out.data_ptr(), bs.dim, None, None)
        assert np.array_equal(to_host_u64(out), ar)
    idx, bad = dq.lex_rank(L, n, st, count_invalid=True, Q=Q)
    assert int(bad.item()) == 0 and np.array_equal(to_host_u64(idx), ar)
    back, bad = dq.lex_unrank(L, n, to_dev(ar), count_invalid=True, Q=Q)
    assert int(bad.item()) == 0 and np.array_equal(to_host_u64(back), bs.states)


@pytest.mark.parametrize("Q,L,n", [(3, 32, 32), (5, 21, 42)])
def test_lex_rank_any_q_against_oracle(Q, L, n):
    """2^16 random states of a large sector round-trip; 1024 of them against the oracle's
    lexicographic rank; digits >= Q, bits above the fields, other digit sums and indices
    >= D are counted."""
    from oracle.sector import dim_closed
    from oracle.sector import lex_rank as o_lex_rank
    dig = synth.random_states(Q, L, n, 1 << 16, seed=23)
    st = synth.pack_digits(dig, Q)
    idx = dq.lex_rank(L, n, to_dev(st), Q=Q)
    got = to_host_u64(idx)
    ref = np.array([o_lex_rank(list(int(v) for v in d), Q) for d in dig[:1024]], dtype=np.uint64)
    assert np.array_equal(got[:1024], ref)
    assert np.array_equal(to_host_u64(dq.lex_unrank(L, n, idx, Q=Q)), st)
    dim = dim_closed(Q, L, n)
    assert int(got.max()) < dim
    nb = (Q - 1).bit_length()
    bad = st.copy()
    bad[:40] ^= np.uint64(1 << (nb * L)) if nb * L < 64 else np.uint64(0)  # a bit above the fields
    hi = np.uint64((1 << nb) - 1)
    # a digit >= Q at site 0 (all ones in its field) where the field allows one
    bad[40:60] = (bad[40:60] & ~(hi << np.uint64(nb * (L - 1)))) | (hi << np.uint64(nb * (L - 1)))
    bad[60:90] ^= np.uint64(1)  # another digit sum, or a digit >= Q
    _, cnt = dq.lex_rank(L, n, to_dev(bad), count_invalid=True, Q=Q)
    want = (40 if nb * L < 64 else 0) + 20 + 30
    assert int(cnt.item()) == want
    _, cnt = dq.lex_unrank(L, n, to_dev(np.array([dim - 1, dim, 2 ** 62], dtype=np.uint64)), count_invalid=True, Q=Q)
    assert int(cnt.item()) == 2
    with pytest.raises(dq.DcsError):
        dq.lex_rank(L + 64, n, to_dev(st[:4]), Q=Q)


def test_lex_rank_L64_half_filling():
    """L = 64, n = 32 (1.8e18 states, the largest spin-1/2 sector of 64 sites): 2^16
    random states round-trip, 256 of them against the oracle's lexicographic rank, and
    the first and last states rank to 0 and D - 1."""
    import math
    from oracle.sector import lex_rank as o_lex_rank
    L, n = 64, 32
    dim = math.comb(L, n)
    dig = synth.random_states(2, L, n, 1 << 16, seed=29)
    st = synth.pack_digits(dig, 2)
    idx = dq.lex_rank(L, n, to_dev(st))
    got = to_host_u64(idx)
    ref = np.array([o_lex_rank(list(int(v) for v in d), 2) for d in dig[:256]], dtype=np.uint64)
    assert np.array_equal(got[:256], ref)
    assert int(got.max()) < dim
    assert np.array_equal(to_host_u64(dq.lex_unrank(L, n, idx)), st)
    ends = np.array([(1 << 32) - 1, ((1 << 32) - 1) << 32], dtype=np.uint64)  # first and last states
    assert to_host_u64(dq.lex_rank(L, n, to_dev(ends))).tolist() == [0, dim - 1]
