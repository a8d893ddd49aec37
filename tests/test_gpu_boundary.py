"""The Python binding rejects every wrong-sized, wrong-typed or misplaced tensor
before anything reaches a kernel (each check raises ValueError or TypeError), and a
plan that lists one split-view sector several times serialises that sector's
products (they share its tile counters, tables and diagonal buffer)."""
import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, rel_err

pytestmark = pytest.mark.gpu


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


@pytest.fixture(scope="module")
def small():
    L, n = 10, 5
    s = dq.Sector(L, n, 2, [5, 5])
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    return s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz)


def test_apply_rejects_bad_shapes(small):
    s, t, j, z = small
    D = s.dim
    ok = torch.zeros(D, dtype=torch.float64, device=DEV)
    for bad in (torch.zeros(D - 1, dtype=torch.float64, device=DEV),
                torch.zeros(D, 3, dtype=torch.float64, device=DEV),
                torch.zeros(D, 2, 2, dtype=torch.float64, device=DEV),
                torch.zeros(D, 16, dtype=torch.float64, device=DEV)):
        with pytest.raises(ValueError):
            dq.hamiltonian_apply(s, t, j, z, bad)
    with pytest.raises(TypeError):
        dq.hamiltonian_apply(s, t, j, z, ok.to(torch.float16))
    with pytest.raises(ValueError):
        dq.hamiltonian_apply(s, t, j, z, ok.cpu())
    with pytest.raises(ValueError):
        dq.hamiltonian_apply(s, t, j, z, torch.zeros(D, 2, dtype=torch.float64, device=DEV)[:, 0])
    for bad_out in (torch.empty(D - 1, dtype=torch.float64, device=DEV),
                    torch.empty(D, 2, dtype=torch.float64, device=DEV)):
        with pytest.raises(ValueError):
            dq.hamiltonian_apply(s, t, j, z, ok, out=bad_out)
    with pytest.raises(TypeError):
        dq.hamiltonian_apply(s, t, j, z, ok, out=torch.empty(D, dtype=torch.float32, device=DEV))
    with pytest.raises(ValueError):
        dq.hamiltonian_apply(s, t, j[:-1].contiguous(), z, ok)


def test_adjoint_rejects_bad_sizes(small):
    s, t, j, z = small
    D = s.dim
    x = torch.zeros(D, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):  # block and vector mixed
        dq.hamiltonian_apply_adjoint(s, t, j, z, torch.zeros(D, 2, dtype=torch.float64, device=DEV),
                                     torch.zeros(D, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):  # 3 columns
        dq.hamiltonian_apply_adjoint(s, t, j, z, torch.zeros(D, 3, dtype=torch.float64, device=DEV),
                                     torch.zeros(D, 3, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        dq.hamiltonian_apply_adjoint(s, t, j, z, x, torch.zeros(D - 1, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        dq.hamiltonian_apply_adjoint(s, t, j, z, x[:-1].contiguous(), x[:-1].contiguous())
    with pytest.raises(TypeError):
        dq.hamiltonian_apply_adjoint(s, t, j, z, x, x.float())



def test_index_and_lanczos_reject_bad_sizes(small):
    s, t, j, z = small
    st = s.enumerate(0, 8)
    with pytest.raises(ValueError):
        s.rank(st, out=torch.empty(7, dtype=torch.int64, device=DEV))
    with pytest.raises(ValueError):
        s.unrank(st, out=torch.empty(9, dtype=torch.int64, device=DEV))
    with pytest.raises(TypeError):
        s.rank(st, out=torch.empty(8, dtype=torch.int32, device=DEV))
    with pytest.raises(ValueError):
        s.enumerate(0, 8, out=torch.empty(4, dtype=torch.int64, device=DEV))
    with pytest.raises(ValueError):
        dq.lanczos(s, t, j, z, torch.ones(s.dim - 1, dtype=torch.float64, device=DEV), 10)
    with pytest.raises(ValueError):
        dq.lanczos(s, t, j, z, torch.ones(s.dim, 2, dtype=torch.float64, device=DEV), 10)


def test_plan_rejects_bad_outputs(small):
    s, t, j, z = small
    plan = dq.Plan([(s, t, j, z)])
    x = torch.zeros(s.dim, dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        plan.apply([x], [torch.empty(s.dim - 1, dtype=torch.float32, device=DEV)])
    with pytest.raises(TypeError):
        plan.apply([x], [torch.empty(s.dim, dtype=torch.float64, device=DEV)])
    with pytest.raises(ValueError):
        plan.apply([x], [])


def test_plan_repeated_split_sector(monkeypatch):
    """One split-view sector listed three times (two terms objects, three coupling sets)
    next to an ordinary sector, with the split products beside the launch
    (DCS_PLAN_HYBRID=1); from the second apply on they run on the plan's side
    streams.  Every apply equals the one-sector products bit for bit."""
    monkeypatch.setenv("DCS_PLAN_HYBRID", "1")
    monkeypatch.setenv("DCS_SPLIT_MIN_DIM", "0")
    L, n = 20, 10
    s = dq.Sector(L, n, 2, [5, 5, 5, 5])
    other = dq.Sector(12, 6, 2, [6, 6])
    monkeypatch.delenv("DCS_SPLIT_MIN_DIM")
    b1, j1, z1 = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    b2, j2, z2 = synth.xxz_chain(L, 1.0, 0.7)
    t1, t2 = dq.Terms(b1), dq.Terms(b2)
    bo, jo, zo = synth.xxz_chain(12, 1.0, 1.0)
    items = [(s, t1, dev_f64(j1), dev_f64(z1)), (other, dq.Terms(bo), dev_f64(jo), dev_f64(zo)),
             (s, t2, dev_f64(j2), dev_f64(z2)), (s, t1, dev_f64(2 * j1), dev_f64(-z1))]
    plan = dq.Plan(items)
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    for dt in (torch.float64, torch.float32):
        for rep in range(3):
            xs = [torch.randn(it[0].dim, generator=g, device=DEV, dtype=torch.float64).to(dt)
                  for it in items]
            ys = plan.apply(xs)
            torch.cuda.synchronize()
            for (sec, tt, jj, zz), x, y in zip(items, xs, ys):
                y1 = dq.hamiltonian_apply(sec, tt, jj, zz, x)
                assert torch.equal(y, y1), (rep, dt, sec.L)
