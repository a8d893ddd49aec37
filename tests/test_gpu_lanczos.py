"""GPU Lanczos (FP64 scalars; FP64 or FP32 vectors) against the oracle Lanczos,
closed forms and the Bethe ansatz, plus the device tridiagonal eigensolver."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, say
from oracle import native
from oracle.closed_forms import bethe_e0
from oracle.lanczos import lanczos as o_lanczos, ritz

pytestmark = pytest.mark.gpu


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def test_tridiagonal_eigensolver():
    rng = np.random.default_rng(3)
    for m in (1, 2, 5, 50, 200):
        a, b = rng.normal(size=m), rng.uniform(0.01, 2, size=max(m - 1, 0))
        ref = np.sort(scipy.linalg.eigvalsh_tridiagonal(a, b)) if m > 1 else a
        num = min(m, 8)
        got = dq.tridiag_eigvals(list(a), list(b), num)
        assert np.allclose(got, ref[:num], atol=1e-12 * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("reorth", ["full", "local", "none"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_plain_workload_L16(reorth, dt):
    """L=16, n=8, 8/8 Heisenberg chain, 100 steps: E0 against the oracle Lanczos
    (same start vector) and the Bethe-ansatz energy."""
    L, n, sp = 16, 8, [8, 8]
    s = dq.Sector(L, n, 2, sp)
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    v0 = synth.vector(s.dim, synth.SEED_V0)
    ns = native.NativeSector(2, L, n, sp)
    t = native.NativeTerms(bonds, jxy, jz)
    a, b, _ = o_lanczos(lambda v: native.hx_range(ns, t, v), v0, 100, ns.dim)
    e_oracle = ritz(a, b)[0]
    e_bethe = bethe_e0(L)
    assert abs(e_oracle - e_bethe) < 1e-9
    res = dq.lanczos(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz),
                     torch.tensor(v0, device=DEV).to(dt), 100, reorth=reorth, num_eig=3,
                     want_vector=True)
    e0 = res["eig"][0]
    err = abs(e0 - e_oracle) / abs(e_oracle)
    say("L16", reorth, dt, res["steps_done"], e0, e_oracle, "rel err", err)
    assert err <= (1e-10 if dt == torch.float64 else 1e-5)
    psi = res["vector"]
    hpsi = dq.hamiltonian_apply(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), psi)
    r = (hpsi.double() - e0 * psi.double()).norm().item()
    assert r < (1e-5 if (dt == torch.float64 and reorth != "none") else 1e-2)
    if dt == torch.float64 and reorth == "full":
        # the first coefficients agree with the oracle run
        assert np.allclose(res["alpha"][:10], a[:10], rtol=1e-10, atol=1e-10)
        assert np.allclose(res["beta"][:10], b[:10], rtol=1e-10, atol=1e-10)


def test_breakdown_and_tiny_sectors():
    L = 10
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 0.7)
    t = dq.Terms(bonds)
    s0 = dq.Sector(L, 0, 2)
    res = dq.lanczos(s0, t, dev_f64(jxy), dev_f64(jz), torch.ones(1, device=DEV, dtype=torch.float64),
                     50, reorth="full")
    assert res["steps_done"] == 1 and abs(res["eig"][0] - 0.7 * L / 4) < 1e-14
    s1 = dq.Sector(L, 1, 2)
    v0 = torch.tensor(synth.vector(L, 3), device=DEV)
    res = dq.lanczos(s1, t, dev_f64(jxy), dev_f64(jz), v0, 50, reorth="full", num_eig=L)
    ks = 2 * np.pi * np.arange(L) / L
    ev = np.unique(np.round(1.0 * (0.7 * (L - 4) / 4 + np.cos(ks)), 12))
    assert res["steps_done"] <= L
    assert abs(res["eig"][0] - ev[0]) < 1e-12


def test_majumdar_ghosh_L16():
    L = 16
    s = dq.Sector(L, 8, 2, [8, 8])
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    res = dq.lanczos(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz),
                     torch.tensor(synth.vector(s.dim, 3), device=DEV), 120, reorth="full")
    assert abs(res["eig"][0] + 6.0) < 1e-10


def test_differentiable_workload_L24():
    """L=24, n=12 random couplings, FP64: 80 steps, E0 against the oracle run."""
    L, n, sp = 24, 12, [8, 8, 8]
    bonds = synth.chain_bonds(L, 1)
    J, D = synth.random_couplings(len(bonds))
    jxy, jz = J, J * D
    ns = native.NativeSector(2, L, n, sp)
    t = native.NativeTerms(bonds, jxy, jz)
    v0 = synth.vector(ns.dim, synth.SEED_V0)
    a, b, _ = o_lanczos(lambda v: native.hx_range(ns, t, v), v0, 80, ns.dim)
    e_oracle = ritz(a, b)[:2]
    s = dq.Sector(L, n, 2, sp)
    res = dq.lanczos(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), torch.tensor(v0, device=DEV),
                     80, reorth="full", num_eig=2)
    say("L24", res["eig"], e_oracle)
    assert abs(res["eig"][0] - e_oracle[0]) < 1e-9 * abs(e_oracle[0])


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_headline_workload_L32_majumdar_ghosh(dt):
    """L=32, n=16, J1-J2 at J2 = J1/2 (Majumdar-Ghosh): the exact ground energy is
    -3L/8 = -12.  200 steps, local re-orthogonalisation, FP64 scalars."""
    L, n, sp = 32, 16, [8, 8, 8, 8]
    s = dq.Sector(L, n, 2, sp)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    g = torch.Generator(device=DEV)
    g.manual_seed(synth.SEED_V0)
    v0 = torch.randn(s.dim, generator=g, device=DEV, dtype=torch.float64).to(dt)
    res = dq.lanczos(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), v0, 200, reorth="local")
    e0 = res["eig"][0]
    err = abs(e0 + 12.0) / 12.0
    say("L32 MG", dt, res["steps_done"], e0, "rel err", err)
    assert err <= (1e-9 if dt == torch.float64 else 1e-5)


def test_large_workload_L34():
    """L=34, n=17 (2,333,606,220 states, 8/8/9/9) Heisenberg chain: 150 steps with FP32
    vectors and FP64 scalars (local re-orthogonalisation); E0 against the Bethe ansatz."""
    L, n = 34, 17
    s = dq.Sector(L, n, 2, [8, 8, 9, 9])
    bonds, jxy, jz = synth.xxz_chain(L, 1.0, 1.0)
    g = torch.Generator(device=DEV)
    g.manual_seed(synth.SEED_V0)
    v0 = torch.randn(s.dim, generator=g, device=DEV, dtype=torch.float32)
    res = dq.lanczos(s, dq.Terms(bonds), dev_f64(jxy), dev_f64(jz), v0, 150, reorth="local")
    e_b = bethe_e0(L)
    say("L34", res["steps_done"], res["eig"][0], e_b)
    assert res["steps_done"] == 150
    assert abs(res["eig"][0] - e_b) <= 1e-6 * abs(e_b)


@pytest.mark.parametrize("split_view", [False, True])
@pytest.mark.parametrize("reorth", ["local", "none"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_captured_steps_match_eager(monkeypatch, split_view, reorth, dt):
    """Steps 2.. replayed from two captured HIP graphs give the same alpha, beta and
    Ritz values, bit for bit, as launching every step eagerly; the captured run is
    repeated with eager products in between (single pass and split product)."""
    if split_view:
        monkeypatch.setenv("DCS_SPLIT_MIN_DIM", "0")
        monkeypatch.setenv("DCS_AUTOTUNE", "0")
    L, n = 20, 10
    s = dq.Sector(L, n, 2, [5, 5, 5, 5])
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.3, 0.8)
    t = dq.Terms(bonds)
    jd, zd = dev_f64(jxy), dev_f64(jz)
    v0 = torch.tensor(synth.vector(s.dim, synth.SEED_V0), device=DEV).to(dt)
    monkeypatch.setenv("DCS_LANCZOS_GRAPH", "0")
    ref = dq.lanczos(s, t, jd, zd, v0, 60, reorth=reorth, num_eig=3)
    monkeypatch.delenv("DCS_LANCZOS_GRAPH")
    for rep in range(3):
        got = dq.lanczos(s, t, jd, zd, v0, 60, reorth=reorth, num_eig=3)
        assert got["steps_done"] == ref["steps_done"]
        assert got["alpha"] == ref["alpha"] and got["beta"] == ref["beta"], rep
        assert got["eig"] == ref["eig"], rep
        y = dq.hamiltonian_apply(s, t, jd, zd, v0)  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
