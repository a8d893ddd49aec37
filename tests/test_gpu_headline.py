"""Parity of exactly the launches the benchmark times, at its full sizes.

The benchmark's headline is the FP32 block of k = 8 columns on the L=32, n=16 J1-J2
sector (601,080,390 states, split 8/8/8/8).  These tests run that product in the
form the autotuner keeps (the form bench.py times) and in the default two-pass split
form, and compare against the FP64 C oracle evaluated on the FP64 draws (the FP32
block is those draws rounded), on sampled rows that include every row of the first
and last run of each left particle-number block of the split view.  The FP32 adjoint
on the same sector is checked the same way (grad_x rows and the coupling and field
sums), and the k = 8 block column by column against the k = 1 product on all rows.

Tolerance: norm-wise relative error 1e-5 (FP32) against the FP64 oracle on the FP64
input.  Host memory: the FP64 k = 8 block is 38.5 GB.
"""
import math
import os

import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, rel_err, say
from oracle import native

pytestmark = pytest.mark.gpu

L, N_UP, SPLIT = 32, 16, [8, 8, 8, 8]


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def to_dev_f32(xh: np.ndarray) -> torch.Tensor:
    """FP64 host array -> FP32 device tensor, in slices (no FP64 copy on the device)."""
    out = torch.empty(xh.shape, dtype=torch.float32, device=DEV)
    step = 1 << 26
    for a in range(0, xh.shape[0], step):
        out[a:a + step] = torch.from_numpy(xh[a:a + step]).to(DEV).float()
    return out


def edge_runs(ns: native.NativeSector, half: int):
    """Rows of the first and last run of every left particle-number block: the left
    configuration is the word of the first `half` sites, its run is the rows sharing
    it; run start = oracle rank of the left word followed by the first right word in
    canonical order (fewest particles on the first right subsystem, each subsystem's
    particles on its last sites)."""
    words = np.arange(1 << half, dtype=np.uint64)
    pop = np.array([bin(int(w)).count("1") for w in words])
    rows = []
    rsub = [s for s in ns.split[len(ns.split) // 2:]]
    assert sum(rsub) == L - half
    for m in range(0, min(half, N_UP) + 1):
        mr = N_UP - m
        if mr > L - half or mr < 0:
            continue
        # first right configuration: lowest particle count on each subsystem from the left
        right = 0
        left_over = mr
        counts = []
        for i, ls in enumerate(rsub):
            rest = sum(rsub[i + 1:])
            c = max(0, left_over - rest)
            counts.append(c)
            left_over -= c
        for ls, c in zip(rsub, counts):
            right = (right << ls) | ((1 << c) - 1)
        sel = words[pop == m]
        states = (sel << np.uint64(L - half)) | np.uint64(right)
        starts = ns.rank(states)
        run = math.comb(L - half, mr)
        for st in (starts.min(), starts.max()):
            rows.append(np.arange(int(st), int(st) + run, dtype=np.uint64))
    return np.concatenate(rows)


def sampled_rows(dim, count, seed, extra=None):
    rng = np.random.default_rng(seed)
    parts = [np.arange(0, 4096, dtype=np.uint64), np.arange(dim - 4096, dim, dtype=np.uint64),
             rng.integers(0, dim, count).astype(np.uint64)]
    if extra is not None:
        parts.append(extra)
    return np.unique(np.concatenate(parts))


@pytest.fixture(scope="module")
def headline():
    s = dq.Sector(L, N_UP, 2, SPLIT)
    ns = native.NativeSector(2, L, N_UP, SPLIT)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 1.0)
    return s, ns, bonds, jxy, jz


@pytest.mark.parametrize("autotune", ["1", "0"])
def test_timed_product_L32_f32_k8(monkeypatch, headline, autotune):
    """The bench's headline product: FP32, k = 8, in the autotuner's form (autotune=1,
    what bench.py times) and in the default split form (autotune=0), against the FP64
    oracle on >= 300k sampled rows plus every row of the first and last run of each
    left block; then every column against the k = 1 product of that column."""
    s, ns, bonds, jxy, jz = headline
    monkeypatch.setenv("DCS_AUTOTUNE", autotune)
    t = dq.Terms(bonds)  # a fresh terms object: a fresh autotuner record
    say("generating the FP64 k=8 block", s.dim)
    x64 = synth.vector(s.dim, synth.SEED_X, np.float64, k=8)
    xd = to_dev_f32(x64)
    rows = sampled_rows(s.dim, 300_000, 21, edge_runs(ns, 16))
    say("oracle rows", len(rows))
    y_ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), x64, rows)
    del x64
    y = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xd)
    form = dq.hamiltonian_form(s, t, torch.float32, 8)
    say("form", form)
    assert form in ("split_staged", "split_global", "split_fused", "single")
    if autotune == "0":
        assert form == "split_staged"
    got = y[torch.from_numpy(rows.astype(np.int64)).to(DEV)].double().cpu().numpy()
    err = rel_err(got, y_ref)
    say("k=8 rel err vs oracle", err)
    assert err <= 1e-5
    y2 = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xd)
    assert torch.equal(y, y2)  # later calls: same form, bitwise
    del y2
    worst = 0.0
    for c in range(8):
        xc = xd[:, c].contiguous()
        yc = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), xc)
        d = (y[:, c].double() - yc.double()).norm().item() / yc.double().norm().item()
        worst = max(worst, d)
        del xc, yc
    say("k=8 columns vs k=1 products, worst rel diff", worst)
    assert worst <= 1e-5


def test_timed_adjoint_L32_f32(headline):
    """FP32 adjoint on the L=32 sector: grad_x = H g on sampled rows against the FP64
    oracle, and the coupling sums of four bonds (one left of the cut, one right, two
    across) plus all field sums against the oracle's sums over every row."""
    s, ns, bonds, jxy, jz = headline
    t = dq.Terms(bonds)
    say("generating x, g", s.dim)
    x64 = synth.vector(s.dim, synth.SEED_X)
    g64 = synth.vector(s.dim, synth.SEED_G)
    xd, gd = to_dev_f32(x64), to_dev_f32(g64)
    gx, gj, gz, gh = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz), xd, gd,
                                                  want_grad_h=True)
    rows = sampled_rows(s.dim, 300_000, 22)
    say("oracle grad_x rows")
    ref = native.hx_rows(ns, native.NativeTerms(bonds, jxy, jz), g64, rows)
    got = gx[torch.from_numpy(rows.astype(np.int64)).to(DEV)].double().cpu().numpy()
    err = rel_err(got, ref)
    say("grad_x rel err", err)
    assert err <= 1e-5
    sel = [0, 15, 20, 47]  # (0,1) left; (15,16) across; (20,21) right; (15,17) across
    say("oracle bond sums", [bonds[b] for b in sel])
    rxy, rz, rh = native.bond_sums(ns, [bonds[b] for b in sel], x64, g64, fields=True)
    for b, a, r in zip(sel, gj.cpu().numpy()[sel], rxy):
        say("jxy", b, a, r)
    assert rel_err(gj.cpu().numpy()[sel], rxy) <= 1e-5
    assert rel_err(gz.cpu().numpy()[sel], rz) <= 1e-5
    assert rel_err(gh.cpu().numpy(), rh) <= 1e-5
