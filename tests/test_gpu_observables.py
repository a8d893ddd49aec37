"""GPU lowest states and expectation values (App. D's example) against the
oracle: several Ritz vectors from one Lanczos run (stored basis and replay),
the expectation values of every bond term and site field, and the L = 28,
n = 14 run of the example against values the oracle wrote (tests/golden)."""
import json
import os

import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, say
from oracle import native
from oracle.observables import lowest_states

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def tilted(L):
    bonds, jxy, jz, h = synth.tilted_field_chain(L)
    return bonds, jxy, jz, h, dq.Terms(bonds)


@pytest.mark.parametrize("L,split", [(20, [10, 10]), (22, [7, 7, 8])])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_expectation_values_match_oracle(L, split, dt):
    """<x|term|x> for two seeded vectors (not normalised) against the oracle's bond sums."""
    n = L // 2
    s = dq.Sector(L, n, 2, split)
    bonds, _, _, _, terms = tilted(L)
    ns = native.NativeSector(2, L, n, split)
    X = np.stack([synth.vector(s.dim, synth.SEED_X), synth.vector(s.dim, synth.SEED_G)])
    if dt == torch.float32:
        X = X.astype(np.float32).astype(np.float64)   # the values the FP32 call sees
    got = dq.expectation_values(s, terms, torch.tensor(X, device=DEV).to(dt))
    tol = 1e-12 if dt == torch.float64 else 2e-5
    for e in range(2):
        gxy, gz, gh = native.bond_sums(ns, bonds, X[e], X[e], fields=True)
        scale = float(X[e] @ X[e])
        say("expect", L, split, dt, e, np.abs(got["sz"][e].cpu().numpy() - gh).max() / scale)
        np.testing.assert_allclose(got["xy"][e].cpu().numpy(), gxy, atol=tol * scale, rtol=0)
        np.testing.assert_allclose(got["z"][e].cpu().numpy(), gz, atol=tol * scale, rtol=0)
        np.testing.assert_allclose(got["sz"][e].cpu().numpy(), gh, atol=tol * scale, rtol=0)


def test_expectation_values_edge_cases():
    L = 12
    s = dq.Sector(L, 6, 2, [6, 6])
    bonds, _, _, _, terms = tilted(L)
    empty = torch.zeros((0, s.dim), dtype=torch.float64, device=DEV)
    out = dq.expectation_values(s, terms, empty)
    assert out["xy"].shape == (0, len(bonds))
    with pytest.raises(ValueError):
        dq.expectation_values(s, terms, torch.zeros(s.dim + 1, dtype=torch.float64, device=DEV))
    # a basis state: <A_b> = 0, <Z_b> = m_i m_j, <Sz_i> = m_i
    dig = synth.random_states(2, L, 6, 1, seed=4)
    idx = native.NativeSector(2, L, 6, [6, 6]).rank(synth.pack_digits(dig, 2))[0]
    e = torch.zeros(s.dim, dtype=torch.float64, device=DEV)
    e[int(idx)] = 1.0
    out = dq.expectation_values(s, terms, e)
    m = dig[0].astype(np.float64) - 0.5
    assert np.all(out["xy"].cpu().numpy() == 0.0)
    assert np.array_equal(out["z"][0].cpu().numpy(), np.array([m[i] * m[j] for i, j in bonds]))
    assert np.array_equal(out["sz"][0].cpu().numpy(), m)


@pytest.mark.parametrize("reorth,L,steps,num", [("full", 20, 170, 4), ("local", 16, 100, 3)])
def test_lowest_states_match_oracle(reorth, L, steps, num):
    """The num lowest Ritz pairs of one run (stored basis / replayed recurrence)
    against the oracle's fully re-orthogonalised run from the same start vector,
    and each state's site magnetisations."""
    n = L // 2
    split = [L // 2, L - L // 2]
    s = dq.Sector(L, n, 2, split)
    bonds, jxy, jz, h, terms = tilted(L)
    ns = native.NativeSector(2, L, n, split)
    t = native.NativeTerms(bonds, jxy, jz, h)
    v0 = synth.vector(s.dim, synth.SEED_V0)
    E_o, psi_o = lowest_states(lambda v: native.hx_range(ns, t, v), v0, steps, num, ns.dim)
    res = dq.lanczos(s, terms, dev_f64(jxy), dev_f64(jz), torch.tensor(v0, device=DEV), steps,
                     reorth=reorth, num_eig=num, num_vec=num, h=dev_f64(h))
    psi = res["vectors"]
    assert psi.shape == (num, s.dim)
    ex = dq.expectation_values(s, terms, psi)
    for e in range(num):
        pg = psi[e].cpu().numpy()
        ov = abs(float(pg @ psi_o[:, e]))
        _, _, sz_o = native.bond_sums(ns, bonds, psi_o[:, e], psi_o[:, e], fields=True)
        dsz = np.abs(ex["sz"][e].cpu().numpy() - sz_o).max()
        say("lowest", reorth, L, e, res["eig"][e], E_o[e], "1-overlap", 1 - ov, "dsz", dsz)
        assert abs(res["eig"][e] - E_o[e]) <= 1e-10 * abs(E_o[e])
        assert 1 - ov < 1e-8
        assert dsz < 1e-7
        # <H> from the term expectations is the Ritz value
        eh = (jxy @ ex["xy"][e].cpu().numpy() + jz @ ex["z"][e].cpu().numpy()
              + h @ ex["sz"][e].cpu().numpy())
        assert abs(eh - res["eig"][e]) <= 1e-9 * abs(E_o[e])


def test_app_d_L28():
    """App. D's example at its size: L = 28, n = 14, the four lowest states of the
    open chain in the field h_k = k, with <Sz_0> (and every site) of each, against
    the oracle's deflated Lanczos values; the Lanczos arguments are the bench's."""
    path = os.path.join(GOLDEN, "appd_L28.json")
    ref = json.load(open(path))
    L, n = ref["L"], ref["n"]
    s = dq.Sector(L, n, 2, [7, 7, 7, 7])  # energies and expectation values do not depend on the split
    bonds, jxy, jz, h, terms = tilted(L)
    assert [list(b) for b in bonds] == ref["bonds"] and s.dim == ref["dim"]
    v0 = torch.tensor(synth.vector(s.dim, synth.SEED_V0), device=DEV)
    num = len(ref["states"])
    res = dq.lanczos(s, terms, dev_f64(jxy), dev_f64(jz), v0, 240, reorth="full",
                     num_eig=num + 1, num_vec=num, h=dev_f64(h))
    ex = dq.expectation_values(s, terms, res["vectors"])
    # The oracle's vectors carry residuals r = |H psi - E psi| of 1e-8..1e-7: a vector
    # error of at most r / gap, gap the distance to the nearest other level (from the
    # num + 1 lowest Ritz values), moves each <Sz_i> by at most 2 r / gap; the
    # energies (Rayleigh quotients) by r^2 / gap.
    E = np.array(res["eig"])
    for e, st in enumerate(ref["states"]):
        gap = np.min(np.abs(np.delete(E, e) - E[e]))
        assert gap > 0.1
        dsz = np.abs(ex["sz"][e].cpu().numpy() - np.array(st["sz"])).max()
        say("appd", e, res["eig"][e], st["E"], "dsz", dsz, "oracle residual", st["residual_norm"],
            "gap", gap, "steps", res["steps_done"])
        assert abs(res["eig"][e] - st["E"]) <= 1e-10 * abs(st["E"])
        assert dsz <= 2 * st["residual_norm"] / gap + 1e-9
