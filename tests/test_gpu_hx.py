"""GPU parity of Y = H X against the FP64 oracle.

Tolerances (norm-wise relative error |y - y_ref| / |y_ref|): FP64 1e-12,
FP32 1e-5, against the oracle run in FP64 on the FP64 input.
"""
import math

import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, rel_err, say, to_dev
from oracle import native
from oracle.hamiltonian import apply_h
from oracle.sector import BruteSector

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def random_graph(L, nb, rng):
    bonds = set()
    while len(bonds) < nb:
        i, j = rng.integers(0, L, 2)
        if i != j and (j, i) not in bonds:
            bonds.add((int(i), int(j)))
    return sorted(bonds)


SMALL = [
    # Q, L, n, split, topology
    (2, 10, 5, [5, 5], "j1j2"),
    (2, 12, 5, [4, 4, 4], "j1j2"),
    (2, 12, 6, None, "graph"),
    (2, 9, 4, [3, 3, 3], "j1j2"),
    (2, 11, 4, [1, 2, 3, 1, 2, 1, 1], "graph"),
    (2, 10, 3, [1] * 7 + [3], "j1j2"),
    (2, 13, 6, [13], "chain"),
    (2, 8, 0, [4, 4], "chain"),
    (2, 8, 8, [4, 4], "chain"),
    (2, 8, 1, [2, 6], "graph"),
    (3, 6, 6, [2, 2, 2], "chain"),
    (3, 7, 5, [3, 4], "graph"),
    (3, 5, 7, [1, 1, 1, 2], "j1j2"),
    (4, 5, 7, [2, 3], "chain"),
    (5, 4, 6, [2, 2], "chain"),
]


def topology(kind, L, rng):
    if kind == "chain":
        return synth.chain_bonds(L, 1)
    if kind == "j1j2":
        return synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    return random_graph(L, 2 * L, rng)


@pytest.mark.parametrize("bits", ["32", "64"])
def test_small_sectors_all_dtypes_and_k(monkeypatch, bits):
    if bits == "64":
        monkeypatch.setenv("DCS_INDEX_BITS", "64")
    rng = np.random.default_rng(1)
    for Q, L, n, sp, kind in SMALL:
        b = BruteSector(Q, L, n, sp)
        bonds = topology(kind, L, rng)
        jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
        s = dq.Sector(L, n, Q, sp)
        t = dq.Terms(bonds)
        for use_h in (False, True):
            for k in (1, 2, 4, 8):
                x = rng.normal(size=(b.dim, k)) if k > 1 else rng.normal(size=b.dim)
                y_ref = apply_h(b, bonds, jxy, jz, x, h if use_h else None)
                for dt in (torch.float64, torch.float32):
                    say("hx", Q, L, n, s.split, kind, k, dt, use_h, bits)
                    xd = torch.tensor(x, device=DEV).to(dt)
                    y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xd,
                                             h=dev_f64(h) if use_h else None)
                    assert rel_err(y.cpu().double().numpy(), y_ref) <= TOL[dt], (Q, L, n, k, dt)


def test_bitwise_reproducible():
    L, n = 20, 10
    s = dq.Sector(L, n, 2, [6, 7, 7])
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    t = dq.Terms(bonds)
    x = torch.tensor(synth.vector(s.dim), device=DEV, dtype=torch.float32)
    y1 = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), x)
    y2 = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), x)
    assert torch.equal(y1, y2)


def test_plain_workload_L16_full():
    """L=16, n=8, 8/8 Heisenberg chain: every row against the C oracle."""
    L, n, sp = 16, 8, [8, 8]
    s = dq.Sector(L, n, 2, sp)
    ns = native.NativeSector(2, L, n, sp)
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    t = dq.Terms(bonds)
    x = synth.vector(s.dim)
    y_ref = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz), x)
    for dt in (torch.float64, torch.float32):
        y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), torch.tensor(x, device=DEV).to(dt))
        assert rel_err(y.cpu().double().numpy(), y_ref) <= TOL[dt]


def test_differentiable_workload_L24_full():
    """L=24, n=12, 8/8/8 with per-bond J_b ~ U(0.5,1.5), Delta_b ~ U(0,2): all rows."""
    L, n, sp = 24, 12, [8, 8, 8]
    s = dq.Sector(L, n, 2, sp)
    ns = native.NativeSector(2, L, n, sp)
    bonds = synth.chain_bonds(L, 1)
    J, D = synth.random_couplings(len(bonds))
    jxy, jz = J, J * D
    t = dq.Terms(bonds)
    x = synth.vector(s.dim)
    y_ref = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz), x)
    y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), torch.tensor(x, device=DEV))
    assert rel_err(y.cpu().numpy(), y_ref) <= 1e-12


def sampled_rows(dim, count, seed):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, dim, count).astype(np.uint64)
    edge = np.concatenate([np.arange(0, 4096), np.arange(dim - 4096, dim)]).astype(np.uint64)
    return np.concatenate([edge, rows])


def test_k8_block_L28_sampled():
    """L=28, n=14 (7/7/7/7), k=8 FP32 block: 200k sampled rows against the oracle."""
    L, n, sp = 28, 14, [7, 7, 7, 7]
    s = dq.Sector(L, n, 2, sp)
    ns = native.NativeSector(2, L, n, sp)
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    x64 = synth.vector(s.dim, synth.SEED_X, np.float64, k=8)
    rows = sampled_rows(s.dim, 200_000, 5)
    y_ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), x64, rows)
    xd = torch.tensor(x64, device=DEV, dtype=torch.float32)
    del x64
    y = dq.hamiltonian_apply(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), xd)
    got = y[torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
    assert rel_err(got, y_ref) <= 1e-5


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_headline_workload_L32_sampled(dt):
    """L=32, n=16 (601,080,390 states, 8/8/8/8), J1-J2 with J2=0.5, Delta=1: the
    launch the bench times, checked on 300k sampled rows (plus the first and last 4096)."""
    L, n, sp = 32, 16, [8, 8, 8, 8]
    s = dq.Sector(L, n, 2, sp)
    ns = native.NativeSector(2, L, n, sp)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    say("generating x", s.dim)
    xh = synth.vector(s.dim, synth.SEED_X, np.float64)
    rows = sampled_rows(s.dim, 300_000, 6)
    say("oracle rows")
    y_ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), xh, rows)
    xd = torch.from_numpy(xh).to(DEV).to(dt)
    del xh
    y = dq.hamiltonian_apply(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), xd)
    got = y[torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
    err = rel_err(got, y_ref)
    say("rel err", err)
    assert err <= TOL[dt]


@pytest.mark.parametrize("L,n,split,k,dt", [
    (12, 6, [3, 3, 3, 3], 1, torch.float64), (12, 5, [4, 4, 4], 8, torch.float32),
    (14, 7, [3, 4, 3, 4], 4, torch.float32), (16, 8, [8, 8], 2, torch.float64),
    (13, 6, [2, 2, 2, 2, 2, 3], 1, torch.float32), (15, 7, [3, 3, 3, 3, 3], 8, torch.float64),
    (12, 0, [6, 6], 1, torch.float64), (12, 12, [6, 6], 2, torch.float32),
    (12, 1, [4, 4, 4], 4, torch.float64), (13, 12, [3, 3, 3, 4], 1, torch.float32),
    (14, 2, [7, 7], 8, torch.float32), (16, 8, [4, 4, 4, 4], 2, torch.float32)])
@pytest.mark.parametrize("staged", ["1", "0", "fused"])
def test_split_small(monkeypatch, L, n, split, k, dt, staged):
    """The split product (rows for the bonds right of and across the cut, column
    chunks for the bonds left of it; or the fused form, whose row pass also
    applies the bonds left of the cut) forced on small sectors, against the
    oracle; random bond graphs put many bonds across the cut, and n = 0, 1, L-1,
    L give runs of length one."""
    monkeypatch.setenv("DCS_SPLIT_MIN_DIM", "0")
    monkeypatch.setenv("DCS_SPLIT_LDS", "1" if staged == "fused" else staged)
    monkeypatch.setenv("DCS_SPLIT_FUSED", "1" if staged == "fused" else "0")
    monkeypatch.setenv("DCS_AUTOTUNE", "0")  # keep the split form (the tuner may pick another)
    rng = np.random.default_rng(L + k)
    b = BruteSector(2, L, n, split)
    bonds = random_graph(L, 2 * L, rng) + synth.chain_bonds(L, 1)
    jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
    s, t = dq.Sector(L, n, 2, split), dq.Terms(bonds)
    for x in (rng.normal(size=(b.dim, k)) if k > 1 else rng.normal(size=b.dim),):
        for use_h in (False, True):
            y_ref = apply_h(b, bonds, jxy, jz, x, h if use_h else None)
            y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), torch.tensor(x, device=DEV).to(dt),
                                     h=dev_f64(h) if use_h else None)
            assert rel_err(y.cpu().double().numpy(), y_ref) <= TOL[dt], (L, n, split, k, dt, use_h)


@pytest.mark.parametrize("staged", ["1", "0", "fused"])
def test_split_L26_all_rows(monkeypatch, staged):
    """L=26, n=13 (10,400,600 states, split 8/9/9): the split product on every row,
    with and without the runs of x staged in LDS, and the fused form."""
    monkeypatch.setenv("DCS_SPLIT_LDS", "1" if staged == "fused" else staged)
    monkeypatch.setenv("DCS_SPLIT_FUSED", "1" if staged == "fused" else "0")
    monkeypatch.setenv("DCS_AUTOTUNE", "0")
    L, n, sp = 26, 13, [8, 9, 9]
    s = dq.Sector(L, n, 2, sp)
    ns = native.NativeSector(2, L, n, sp)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    x = synth.vector(s.dim)
    y_ref = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz), x)
    for dt in (torch.float64, torch.float32):
        y = dq.hamiltonian_apply(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz),
                                 torch.tensor(x, device=DEV).to(dt))
        assert rel_err(y.cpu().double().numpy(), y_ref) <= TOL[dt]


@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_split_matches_single_pass_L24(monkeypatch, k):
    """L=24, n=12 (2,704,156 states) with the split view forced on: the split product
    (staged and unstaged runs, fused form) against the single pass, in FP64 and FP32."""
    monkeypatch.setenv("DCS_SPLIT_MIN_DIM", "0")
    monkeypatch.setenv("DCS_AUTOTUNE", "0")
    L, n = 24, 12
    s = dq.Sector(L, n, 2, [6, 6, 6, 6])
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    t = dq.Terms(bonds)
    h = synth.gaussian(L, synth.SEED_G)
    g = torch.Generator(device=DEV)
    g.manual_seed(k)
    for dt in (torch.float64, torch.float32):
        x = torch.randn((s.dim, k) if k > 1 else (s.dim,), generator=g, device=DEV,
                        dtype=torch.float64).to(dt)
        out = {}
        for mode, env in (("single", {"DCS_SPLIT": "0"}), ("staged", {"DCS_SPLIT_LDS": "1"}),
                          ("global", {"DCS_SPLIT_LDS": "0"}), ("fused", {"DCS_SPLIT_FUSED": "1"})):
            for key in ("DCS_SPLIT", "DCS_SPLIT_LDS", "DCS_SPLIT_FUSED"):
                monkeypatch.delenv(key, raising=False)
            for key, v in env.items():
                monkeypatch.setenv(key, v)
            out[mode] = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), x,
                                             h=dev_f64(h)).double().cpu().numpy()
        for mode in ("staged", "global", "fused"):
            assert rel_err(out[mode], out["single"]) <= TOL[dt], (k, dt, mode)


def test_large_workload_L34_sampled():
    """L=34, n=17 (2,333,606,220 states, 8/8/9/9), Heisenberg chain, FP32 vectors: the
    product (rows of 18-site right halves, runs up to 48,620 rows) on 200k sampled
    rows plus the first and last 4096, against the FP64 oracle on the FP64 draws (the
    FP32 vector is those draws rounded)."""
    L, n, sp = 34, 17, [8, 8, 9, 9]
    s = dq.Sector(L, n, 2, sp)
    assert s.dim == 2_333_606_220
    ns = native.NativeSector(2, L, n, sp)
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    say("generating x", s.dim)
    xh = synth.vector(s.dim, synth.SEED_X, np.float64)
    xd = torch.empty(s.dim, dtype=torch.float32, device=DEV)
    step = 1 << 27
    for a in range(0, s.dim, step):
        xd[a:a + step] = torch.from_numpy(xh[a:a + step]).to(DEV).float()
    rows = sampled_rows(s.dim, 200_000, 8)
    say("oracle rows")
    y_ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), xh, rows)
    del xh
    y = dq.hamiltonian_apply(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), xd)
    got = y[torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
    err = rel_err(got, y_ref)
    say("rel err", err)
    assert err <= TOL[torch.float32]


def test_split_tables_cache_and_couplings(monkeypatch):
    """One split sector with six terms objects (more than the four cached table sets,
    so sets are evicted and rebuilt) and couplings changed between calls: every
    product equals the single pass on the same input (FP64)."""
    monkeypatch.setenv("DCS_SPLIT_MIN_DIM", "0")
    monkeypatch.setenv("DCS_AUTOTUNE", "0")
    L, n = 18, 9
    s = dq.Sector(L, n, 2, [5, 4, 5, 4])
    rng = np.random.default_rng(11)
    x = torch.tensor(rng.normal(size=s.dim), device=DEV)
    graphs = [random_graph(L, L + 3 * i, rng) + synth.chain_bonds(L, 1) for i in range(6)]
    terms = [dq.Terms(b) for b in graphs]
    for rep in range(2):
        for b, t in zip(graphs, terms):
            for _ in range(2):  # same tables, new couplings
                jxy, jz = dev_f64(rng.normal(size=len(b))), dev_f64(rng.normal(size=len(b)))
                h = dev_f64(rng.normal(size=L))
                monkeypatch.delenv("DCS_SPLIT", raising=False)
                y_split = dq.hamiltonian_apply(s, t, jxy, jz, x, h=h)
                monkeypatch.setenv("DCS_SPLIT", "0")
                y_one = dq.hamiltonian_apply(s, t, jxy, jz, x, h=h)
                assert rel_err(y_split.cpu().numpy(), y_one.cpu().numpy()) <= 1e-12, rep
    monkeypatch.delenv("DCS_SPLIT", raising=False)


@pytest.mark.parametrize("k,dt", [(1, torch.float32), (8, torch.float32), (1, torch.float64)])
def test_autotuned_form(monkeypatch, k, dt):
    """With the autotuner on, the first product of a (terms, dtype, k) times the launch
    forms and returns the fastest one's Y: it matches the oracle, and later calls are
    bitwise equal to it; each form on its own also matches the oracle."""
    monkeypatch.setenv("DCS_SPLIT_MIN_DIM", "0")
    L, n, sp = 20, 10, [5, 5, 5, 5]
    s = dq.Sector(L, n, 2, sp)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    t = dq.Terms(bonds)
    x = synth.vector(s.dim, synth.SEED_X, k=k)
    y_ref = native.hx_range(native.NativeSector(2, L, n, sp), native.NativeTerms(bonds, jxy, jz), x)
    xd = torch.tensor(x, device=DEV).to(dt)
    monkeypatch.delenv("DCS_AUTOTUNE", raising=False)
    y1 = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xd)
    y2 = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xd)
    assert torch.equal(y1, y2)
    assert rel_err(y1.double().cpu().numpy(), y_ref) <= TOL[dt]
    monkeypatch.setenv("DCS_AUTOTUNE", "0")
    for env in ({"DCS_SPLIT_LDS": "1"}, {"DCS_SPLIT_LDS": "0"}, {"DCS_SPLIT_FUSED": "1"}, {"DCS_SPLIT": "0"}):
        for key in ("DCS_SPLIT", "DCS_SPLIT_LDS", "DCS_SPLIT_FUSED"):
            monkeypatch.delenv(key, raising=False)
        for key, v in env.items():
            monkeypatch.setenv(key, v)
        y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xd)
        assert rel_err(y.double().cpu().numpy(), y_ref) <= TOL[dt], env


@pytest.mark.parametrize("L,n,split,k,dt", [
    (24, 12, [6, 6, 6, 6], 8, torch.float32), (24, 12, [6, 6, 6, 6], 4, torch.float32),
    (24, 12, [6, 6, 6, 6], 2, torch.float64), (24, 11, [6, 6, 6, 6], 8, torch.float64),
    (26, 13, [5, 5, 4, 12], 8, torch.float32), (26, 13, [5, 5, 4, 12], 8, torch.float64),
    (24, 12, [6, 4, 14], 8, torch.float64), (22, 10, [4, 4, 4, 5, 5], 4, torch.float64)])
def test_block_tiled_rows(monkeypatch, L, n, split, k, dt):
    """The row pass that stages whole n_K blocks of a run in LDS (the split_tiled form,
    rows of 16 bytes and more), in both tile orders, against the oracle on every row,
    and the staged form beside it.  The splits include n_K blocks larger than one tile (whole
    sub-runs of equal P_K word per tile: 4/12 right halves) and sub-runs larger than
    a tile (a 14-site last subsystem at 64-byte rows, 6/4/14)."""
    monkeypatch.setenv("DCS_SPLIT_MIN_DIM", "0")
    monkeypatch.setenv("DCS_AUTOTUNE", "0")
    s = dq.Sector(L, n, 2, split)
    ns = native.NativeSector(2, L, n, split)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    hf = synth.gaussian(L, 9)
    t = dq.Terms(bonds)
    x = synth.vector(s.dim, synth.SEED_X, k=k)
    y_ref = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz, hf), x)
    xd = torch.tensor(x, device=DEV).to(dt)
    out = {}
    for name, env in (("groups", {"DCS_SPLIT_TILED": "1"}),
                      ("rows", {"DCS_SPLIT_TILED": "1", "DCS_ROW_ORDER": "rows"}), ("untiled", {})):
        for key in ("DCS_ROW_ORDER", "DCS_SPLIT_TILED"):
            monkeypatch.delenv(key, raising=False)
        for key, v in env.items():
            monkeypatch.setenv(key, v)
        out[name] = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xd, h=dev_f64(hf))
        e = rel_err(out[name].double().cpu().numpy(), y_ref)
        say("tiled rows", L, n, split, k, dt, name, e)
        assert e <= TOL[dt], (name, e)
    # the tile order changes which workgroup computes a row, not the row's arithmetic
    assert torch.equal(out["groups"], out["rows"])
