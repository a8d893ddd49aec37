"""Many sectors in one launch (dcs_plan_*): parity with the oracle and with the
one-sector launches."""
import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, rel_err, say
from oracle import native
from oracle.hamiltonian import apply_h
from oracle.sector import BruteSector, default_split

pytestmark = pytest.mark.gpu


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def test_mixed_small_plan():
    rng = np.random.default_rng(4)
    specs = [(2, 10, n, None) for n in range(0, 11)] + [(3, 6, n, [2, 2, 2]) for n in (0, 3, 6, 12)] + \
            [(4, 5, 7, [2, 3]), (2, 12, 6, [1, 2, 3, 4, 1, 1])]
    items, refs, xs = [], [], []
    for Q, L, n, sp in specs:
        b = BruteSector(Q, L, n, sp or default_split(Q, L))
        bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
        jxy, jz = rng.normal(size=len(bonds)), rng.normal(size=len(bonds))
        x = rng.normal(size=b.dim)
        refs.append(apply_h(b, bonds, jxy, jz, x))
        items.append((dq.Sector(L, n, Q, sp), dq.Terms(bonds), dev_f64(jxy), dev_f64(jz)))
        xs.append(x)
    plan = dq.Plan(items)
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        ys = plan.apply([torch.tensor(x, device=DEV).to(dt) for x in xs])
        for (s, _, _, _), y, r in zip(items, ys, refs):
            assert rel_err(y.double().cpu().numpy(), r) <= tol, (s.L, s.n, s.Q)
        # second apply with new vectors reuses the plan
        ys2 = plan.apply([torch.tensor(2 * x, device=DEV).to(dt) for x in xs])
        for y, y2 in zip(ys, ys2):
            assert torch.allclose(2 * y, y2, rtol=1e-6 if dt == torch.float32 else 1e-14, atol=1e-5)


def batched_workload():
    """Every sector n = 0..L of periodic spin-1/2 XXZ chains L = 20, 22, 24, 26 and the
    spin-1 chains L = 12..16 at total Sz = 0 (n = L), J = Delta = 1."""
    specs = [(2, L, n) for L in (20, 22, 24, 26) for n in range(0, L + 1)]
    specs += [(3, L, L) for L in range(12, 17)]
    return specs


def test_batched_workload_one_launch(monkeypatch):
    # one-pass products for the bitwise comparison with the plan (same summation order)
    monkeypatch.setenv("DCS_SPLIT_MIN_DIM", str(1 << 62))
    specs = batched_workload()
    items, xs = [], []
    total = 0
    for Q, L, n in specs:
        bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
        s = dq.Sector(L, n, Q)
        items.append((s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz)))
        g = torch.Generator(device=DEV)
        g.manual_seed(1000 * L + 10 * n + Q)
        xs.append(torch.randn(s.dim, generator=g, device=DEV, dtype=torch.float32))
        total += s.dim
    assert len(items) == 101 and total == 97_016_151
    plan = dq.Plan(items)
    ys = plan.apply(xs)
    torch.cuda.synchronize()
    # the one-launch result equals the per-sector launches bit for bit
    for (s, t, j, z), x, y in zip(items, xs, ys):
        y1 = dq.hamiltonian_apply(s, t, j, z, x)
        assert torch.equal(y, y1), (s.L, s.n, s.Q)
    # and the oracle on sampled rows of a few sectors
    rng = np.random.default_rng(2)
    for idx in (0, 30, 60, 95, 96, 100):
        (s, _, _, _), x, y = items[idx], xs[idx], ys[idx]
        Q, L, n = specs[idx]
        bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
        ns = native.NativeSector(Q, L, n, s.split)
        rows = rng.integers(0, s.dim, min(s.dim, 20000)).astype(np.uint64)
        ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), x.cpu().numpy(), rows)
        got = y[torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
        say("plan sector", Q, L, n, rel_err(got, ref))
        assert rel_err(got, ref) <= 1e-5


@pytest.mark.parametrize("hybrid", [False, True])
def test_batched_workload_with_split_sectors(monkeypatch, hybrid):
    """The batched workload with the default split threshold.  By default every
    sector is in the one launch; every sector's y equals its one-pass product
    (DCS_SPLIT=0) bit for bit.  With DCS_PLAN_HYBRID=1 the sectors of at least 2^20
    states run their own split product beside the launch; every sector's y equals
    its own product bit for bit.  Sampled rows of those sectors match the oracle."""
    if hybrid:
        monkeypatch.setenv("DCS_PLAN_HYBRID", "1")
    specs = batched_workload()
    items, xs = [], []
    for Q, L, n in specs:
        bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
        s = dq.Sector(L, n, Q)
        items.append((s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz)))
        g = torch.Generator(device=DEV)
        g.manual_seed(7 * L + n + Q)
        xs.append(torch.randn(s.dim, generator=g, device=DEV, dtype=torch.float32))
    plan = dq.Plan(items)
    ys = plan.apply(xs)
    ys2 = plan.apply(xs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    if not hybrid:
        monkeypatch.setenv("DCS_SPLIT", "0")  # the per-sector products in the launch's (one-pass) form
    for idx, ((s, t, j, z), x, y, y2) in enumerate(zip(items, xs, ys, ys2)):
        assert torch.equal(y, y2)
        assert torch.equal(y, dq.hamiltonian_apply(s, t, j, z, x)), specs[idx]
        Q, L, n = specs[idx]
        if s.dim >= (1 << 20):
            bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
            ns = native.NativeSector(Q, L, n, s.split)
            rows = rng.integers(0, s.dim, 20000).astype(np.uint64)
            ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), x.cpu().numpy(), rows)
            got = y[torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
            assert rel_err(got, ref) <= 1e-5, specs[idx]


def test_split_sectors_alternating_dtypes(monkeypatch):
    """Applies of one plan (DCS_PLAN_HYBRID=1) alternating FP32 and FP64 (the first
    of each dtype on the caller's stream, later ones with the split sectors on the
    plan's streams): every sector's y equals its own product bit for bit, every time."""
    monkeypatch.setenv("DCS_PLAN_HYBRID", "1")
    specs = [(2, 24, n) for n in (9, 12, 15)] + [(2, 22, n) for n in range(0, 23, 4)] + [(3, 12, 12)]
    items = []
    for Q, L, n in specs:
        bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
        items.append((dq.Sector(L, n, Q), dq.Terms(bonds), dev_f64(jxy), dev_f64(jz)))
    assert sum(1 for s, _, _, _ in items if s.dim >= (1 << 20)) == 3
    plan = dq.Plan(items)
    g = torch.Generator(device=DEV)
    g.manual_seed(11)
    xs64 = [torch.randn(s.dim, generator=g, device=DEV, dtype=torch.float64) for s, _, _, _ in items]
    for rep, dt in enumerate((torch.float32, torch.float64, torch.float32, torch.float64, torch.float32)):
        xs = [x.to(dt) for x in xs64]
        ys = plan.apply(xs)
        torch.cuda.synchronize()
        for (s, t, j, z), x, y in zip(items, xs, ys):
            assert torch.equal(y, dq.hamiltonian_apply(s, t, j, z, x)), (rep, dt, s.L, s.n)


def test_repeated_split_sector_in_hybrid_plan(monkeypatch):
    """One split sector listed three times (twice with one Terms object and different
    couplings, once with its own Terms), beside a second split sector, with
    DCS_PLAN_HYBRID=1: the repeated products share the sector's tile queue and split
    tables, so the plan runs them on one stream.  Three applies; every y equals the
    sector's own product bit for bit, and sampled rows match the oracle."""
    monkeypatch.setenv("DCS_PLAN_HYBRID", "1")
    L, n = 24, 12
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    s, s2 = dq.Sector(L, n, 2), dq.Sector(L, 11, 2)
    t, t_other = dq.Terms(bonds), dq.Terms(bonds)
    rng = np.random.default_rng(17)
    cpl = [(jxy * rng.uniform(0.5, 1.5, len(bonds)), jz * rng.uniform(0.5, 1.5, len(bonds))) for _ in range(4)]
    items = [(s, t, dev_f64(cpl[0][0]), dev_f64(cpl[0][1])), (s2, t_other, dev_f64(cpl[1][0]), dev_f64(cpl[1][1])),
             (s, t, dev_f64(cpl[2][0]), dev_f64(cpl[2][1])), (s, t_other, dev_f64(cpl[3][0]), dev_f64(cpl[3][1]))]
    plan = dq.Plan(items)
    g = torch.Generator(device=DEV)
    g.manual_seed(23)
    xs = [torch.randn(sec.dim, generator=g, device=DEV, dtype=torch.float32) for sec, _, _, _ in items]
    for rep in range(3):
        ys = plan.apply(xs)
        torch.cuda.synchronize()
        for i, ((sec, tt, j, z), x, y) in enumerate(zip(items, xs, ys)):
            assert torch.equal(y, dq.hamiltonian_apply(sec, tt, j, z, x)), (rep, i)
    ns = native.NativeSector(2, L, n, s.split)
    rows = rng.integers(0, s.dim, 20000).astype(np.uint64)
    for i in (0, 2, 3):
        ref = native.hx_rows(ns, native.NativeTerms(bonds, cpl[i][0], cpl[i][1]), xs[i].cpu().numpy(), rows)
        got = ys[i][torch.tensor(rows.astype(np.int64), device=DEV)].double().cpu().numpy()
        assert rel_err(got, ref) <= 1e-5, i
