#!/usr/bin/env python3
"""Benchmark of the matrix-free product y = H x on one particle-number sector.

Workload: periodic spin-1/2 J1-J2 XXZ chain, L=32 sites, n=16 up spins
(601,080,390 states), J1=1, J2=0.5, Delta=1, index split 8/8/8/8; x ~ N(0,1)
from a seeded device generator (synthetic data).  One step is one H*X over the
whole sector: every row decoded (Alg. iii), every bond applied, every reached
state ranked (eq. index), x gathered, y written.

Three forms are timed: the batched FP32 block of k=8 columns (the headline
`value`), FP32 k=1, and the plain FP64 k=1 product.  `value` is sector states per
second, dim / t, with t the median of the timed products (HIP events between
consecutive products on the launch stream); the per-column rate dim * k / t is
reported next to it.  One product is one call of dcs_hamiltonian_apply: on this
sector the split product's launches (diagonal per side configuration, row pass,
column pass, in the form the autotuner keeps; `roofline.kernel` names it).

Besides the headline, `workloads` times the other measured cases of the
method (skipped with --no-extras): rank and unrank of 2^24 random states of the
L=32 sector, the k=8 FP32 block on L=28 n=14, the fused
adjoint on L=24 n=12 with per-bond couplings, all 101 sectors of the batched
workload in one launch, 200 Lanczos steps on the L=32 sector with FP32
and with FP64 vectors (FP64 scalars; E0 = -12 exactly at this coupling ratio,
the Majumdar-Ghosh point), and on L=34, n=17 (2,333,606,220 states) the FP32
product and 150 Lanczos steps.  One JSON line is printed.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·x sector states/s + HBM GB/s, XXZ L=32 N=16; FP32 batched vs plain FP64"
PEAK_HBM_GBS = 8000.0
L, N_UP, SPLIT = 32, 16, [8, 8, 8, 8]
J1, J2, DELTA = 1.0, 0.5, 1.0
KERNEL_SOURCES = ["split_impl.h", "split.cpp", "hx_impl.h", "device_common.h", "dcs_internal.h",
                  "hx_dispatch.hip"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "hx_L32_counters.md")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2407_14591_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(variant: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE, WRITE_SIZE),
    valid only while the kernel sources are unchanged since the measurement."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    txt = open(COUNTERS_FILE).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(rf"traffic_bytes_per_launch\[{variant}\]:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def time_variant(fn, stream, steps: int, warmup: int):
    """Seconds of `steps` back-to-back launches of fn on `stream` (HIP events around
    the whole loop), after `warmup` untimed launches."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3  # seconds for `steps` launches


def time_steps(fn, stream, steps: int, warmup: int):
    """Per-launch seconds of `steps` launches of fn: an event is recorded on `stream`
    between consecutive launches, so every interval is one launch's device time."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(steps)]


def median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def extra_workloads(dq, synth, torch, steps: int, warmup: int):
    """The other measured cases (dict of results); every input is seeded and synthetic.
    Times are medians of per-launch HIP-event intervals."""
    import numpy as np

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}

    def timed(fn, n=steps, w=warmup):
        return median(time_steps(fn, stream, max(n, 3), w))

    # rank and unrank of 2^24 uniformly random states of the L=32, n=16 sector (the paper's
    # random trial states: a uniform n-subset of the sites per state, drawn on the device)
    s = dq.Sector(L, N_UP, 2, SPLIT, device=0)
    cnt = 1 << 24
    g = torch.Generator(device=dev)
    g.manual_seed(synth.SEED_X)
    occ = torch.rand((cnt, L), generator=g, device=dev).argsort(dim=1)[:, :N_UP]
    states = (torch.ones(cnt, N_UP, dtype=torch.int64, device=dev) << (L - 1 - occ)).sum(dim=1)
    del occ
    idx = torch.empty_like(states)
    back = torch.empty_like(states)
    per_r = timed(lambda: s.rank(states, out=idx))
    per_u = timed(lambda: s.unrank(idx, out=back))
    assert torch.equal(back, states)
    idx2 = torch.empty_like(states)
    per_rs = timed(lambda: s.rank_search(states, out=idx2))  # the sorted-list container
    assert torch.equal(idx2, idx)
    out["rank_unrank_L32"] = {"states": cnt, "rank_ms": per_r * 1e3, "unrank_ms": per_u * 1e3,
                              "rank_per_s": cnt / per_r, "unrank_per_s": cnt / per_u,
                              "rank_GBs": cnt * 16 / per_r / 1e9, "unrank_GBs": cnt * 16 / per_u / 1e9,
                              "rank_search_ms": per_rs * 1e3, "rank_search_per_s": cnt / per_rs}
    del idx2
    del states, idx, back

    # FP32 adjoint on the L=32 sector: grad_x = H g and the 64 coupling sums
    bonds, jxy, jz = synth.j1j2_chain(L, J1, J2, DELTA)
    t = dq.Terms(bonds)
    jd, zd = torch.tensor(jxy, device=dev), torch.tensor(jz, device=dev)
    x = torch.randn(s.dim, generator=g, device=dev, dtype=torch.float32)
    gv = torch.randn(s.dim, generator=g, device=dev, dtype=torch.float32)
    per_f = timed(lambda: dq.hamiltonian_apply(s, t, jd, zd, x), n=max(3, steps // 2))
    per_a = timed(lambda: dq.hamiltonian_apply_adjoint(s, t, jd, zd, x, gv), n=max(3, steps // 2))
    out["adjoint_L32_f32"] = {"forward_ms": per_f * 1e3, "adjoint_ms": per_a * 1e3,
                              "adjoint_over_forward": per_a / per_f,
                              "adjoint_states_per_s": s.dim / per_a,
                              "compulsory_bytes": s.dim * 12,
                              "adjoint_compulsory_GBs": s.dim * 12 / per_a / 1e9,
                              "frac_of_peak": s.dim * 12 / per_a / 1e9 / PEAK_HBM_GBS}
    del x, gv
    torch.cuda.empty_cache()

    # the batched FP32 form's adjoint on the same sector: a block of k=8 columns
    xb = torch.randn((s.dim, 8), generator=g, device=dev, dtype=torch.float32)
    gb = torch.randn((s.dim, 8), generator=g, device=dev, dtype=torch.float32)
    per_f = timed(lambda: dq.hamiltonian_apply(s, t, jd, zd, xb), n=3, w=1)
    per_a = timed(lambda: dq.hamiltonian_apply_adjoint(s, t, jd, zd, xb, gb), n=3, w=1)
    out["adjoint_L32_f32k8"] = {"forward_ms": per_f * 1e3, "adjoint_ms": per_a * 1e3,
                                "adjoint_over_forward": per_a / per_f,
                                "adjoint_states_per_s": s.dim / per_a,
                                "compulsory_bytes": s.dim * 8 * 12,
                                "adjoint_compulsory_GBs": s.dim * 8 * 12 / per_a / 1e9,
                                "frac_of_peak": s.dim * 8 * 12 / per_a / 1e9 / PEAK_HBM_GBS}
    del xb, gb, s, t
    torch.cuda.empty_cache()

    # k=8 FP32 block on L=28, n=14 (40,116,600 rows), XXZ J = Delta = 1
    s = dq.Sector(28, 14, 2, [7, 7, 7, 7], device=0)
    bonds, jxy, jz = synth.xxz_chain(28, 1.0, 1.0)
    t = dq.Terms(bonds)
    jd, zd = torch.tensor(jxy, device=dev), torch.tensor(jz, device=dev)
    x = torch.randn((s.dim, 8), generator=g, device=dev, dtype=torch.float32)
    y = torch.empty_like(x)
    per = timed(lambda: dq.hamiltonian_apply(s, t, jd, zd, x, out=y))
    out["hx_L28_f32k8"] = {"ms": per * 1e3, "states_per_s": s.dim / per,
                           "columns_per_s": s.dim * 8 / per,
                           "achieved_GBs": s.dim * 8 * 2 * 4 / per / 1e9,
                           "form": dq.hamiltonian_form(s, t, torch.float32, 8)}
    del x, y, s, t

    # fused adjoint on L=24, n=12, per-bond J_b, Delta_b (24 bonds), FP64
    s = dq.Sector(24, 12, 2, [8, 8, 8], device=0)
    bonds = synth.chain_bonds(24, 1)
    J, D = synth.random_couplings(len(bonds))
    t = dq.Terms(bonds)
    jd, zd = torch.tensor(J, device=dev), torch.tensor(J * D, device=dev)
    x = torch.randn(s.dim, generator=g, device=dev, dtype=torch.float64)
    gv = torch.randn(s.dim, generator=g, device=dev, dtype=torch.float64)
    per_f = timed(lambda: dq.hamiltonian_apply(s, t, jd, zd, x))
    per_a = timed(lambda: dq.hamiltonian_apply_adjoint(s, t, jd, zd, x, gv))
    out["adjoint_L24_f64"] = {"forward_ms": per_f * 1e3, "adjoint_ms": per_a * 1e3,
                              "adjoint_states_per_s": s.dim / per_a,
                              "adjoint_compulsory_GBs": s.dim * 24 / per_a / 1e9,
                              "frac_of_peak": s.dim * 24 / per_a / 1e9 / PEAK_HBM_GBS}
    del x, gv, s, t

    # all sectors of L = 20..26 (spin 1/2, n = 0..L) and spin-1 L = 12..16 at Sz = 0, one call
    items, xs, total = [], [], 0
    specs = [(2, ls, ns) for ls in (20, 22, 24, 26) for ns in range(ls + 1)]
    specs += [(3, ls, ls) for ls in range(12, 17)]
    for q_, ls, ns in specs:
        b, j_, z_ = synth.xxz_chain(ls, 1.0, 1.0)
        sec = dq.Sector(ls, ns, q_, device=0)
        items.append((sec, dq.Terms(b), torch.tensor(j_, device=dev), torch.tensor(z_, device=dev)))
        xs.append(torch.randn(sec.dim, generator=g, device=dev, dtype=torch.float32))
        total += sec.dim
    plan = dq.Plan(items)
    ys = [torch.empty_like(v) for v in xs]
    per = timed(lambda: plan.apply(xs, ys))
    out["plan_101_sectors_f32"] = {"sectors": len(items), "rows": total, "ms": per * 1e3,
                                   "states_per_s": total / per,
                                   "achieved_GBs": total * 8 / per / 1e9,
                                   "frac_of_peak": total * 8 / per / 1e9 / PEAK_HBM_GBS,
                                   "note": "every sector in the one persistent launch"}
    del plan
    # the same sectors with the 18 of >= 2^20 rows on their own split products beside the launch
    os.environ["DCS_PLAN_HYBRID"] = "1"
    try:
        plan1 = dq.Plan(items)
    finally:
        os.environ.pop("DCS_PLAN_HYBRID", None)
    per1 = timed(lambda: plan1.apply(xs, ys))
    out["plan_101_sectors_f32_hybrid"] = {"sectors": len(items), "rows": total, "ms": per1 * 1e3,
                                          "states_per_s": total / per1,
                                          "achieved_GBs": total * 8 / per1 / 1e9,
                                          "frac_of_peak": total * 8 / per1 / 1e9 / PEAK_HBM_GBS,
                                          "hybrid_over_one_launch": per1 / per}
    del plan1, items, xs, ys

    # 200 Lanczos steps on the L=32, n=16 J1-J2 sector (J2/J1 = 1/2: E0 = -3L/8 = -12)
    s = dq.Sector(L, N_UP, 2, SPLIT, device=0)
    bonds, jxy, jz = synth.j1j2_chain(L, J1, J2, DELTA)
    t = dq.Terms(bonds)
    jd, zd = torch.tensor(jxy, device=dev), torch.tensor(jz, device=dev)
    for dt, name in ((torch.float32, "lanczos_L32_f32vec"), (torch.float64, "lanczos_L32_f64vec")):
        v0 = torch.randn(s.dim, generator=g, device=dev, dtype=torch.float64).to(dt)
        dq.hamiltonian_apply(s, t, jd, zd, v0)  # builds this terms object's tables before the clock
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = dq.lanczos(s, t, jd, zd, v0, 200, reorth="local")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"steps": r["steps_done"], "seconds": el, "ms_per_step": el / r["steps_done"] * 1e3,
                     "reorth": r["reorth"], "E0": r["eig"][0], "E0_exact": -12.0,
                     "E0_error_vs_exact": r["eig"][0] + 12.0}
        del v0
        torch.cuda.empty_cache()
    del s, t

    # L=34, n=17 (2,333,606,220 rows, 8/8/9/9) Heisenberg chain, FP32 vectors: H*x and 150 Lanczos steps
    s = dq.Sector(34, 17, 2, [8, 8, 9, 9], device=0)
    bonds, jxy, jz = synth.xxz_chain(34, 1.0, 1.0)
    t = dq.Terms(bonds)
    jd, zd = torch.tensor(jxy, device=dev), torch.tensor(jz, device=dev)
    x = torch.randn(s.dim, generator=g, device=dev, dtype=torch.float32)
    y = torch.empty_like(x)
    per = timed(lambda: dq.hamiltonian_apply(s, t, jd, zd, x, out=y), n=max(3, steps // 4), w=1)
    out["hx_L34_f32k1"] = {"ms": per * 1e3, "states_per_s": s.dim / per,
                           "achieved_GBs": s.dim * 2 * 4 / per / 1e9,
                           "form": dq.hamiltonian_form(s, t, torch.float32, 1)}
    del y
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = dq.lanczos(s, t, jd, zd, x, 150, reorth="local")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    e_bethe = json.load(open(os.path.join(ROOT, "tests", "golden", "bethe_e0.json")))["E0"]["34"]
    out["lanczos_L34_f32vec"] = {"steps": r["steps_done"], "seconds": el,
                                 "ms_per_step": el / r["steps_done"] * 1e3, "reorth": r["reorth"],
                                 "E0": r["eig"][0], "E0_bethe_ansatz": e_bethe,
                                 "E0_error_vs_bethe": r["eig"][0] - e_bethe}
    del x, s, t
    torch.cuda.empty_cache()

    # App. D's example: open L=28, n=14 chain in the field h_k = k, the four lowest
    # states (240 Lanczos steps, stored basis, FP64) and <Sz_0> of each, against the
    # values the oracle's deflated Lanczos wrote to tests/golden/appd_L28.json
    s = dq.Sector(28, 14, 2, [7, 7, 7, 7], device=0)
    bonds, jxy, jz, h = synth.tilted_field_chain(28)
    t = dq.Terms(bonds)
    jd, zd, hd = (torch.tensor(a, device=dev) for a in (jxy, jz, h))
    v0 = torch.tensor(synth.vector(s.dim, synth.SEED_V0), device=dev)
    dq.hamiltonian_apply(s, t, jd, zd, v0, h=hd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = dq.lanczos(s, t, jd, zd, v0, 240, reorth="full", num_eig=4, num_vec=4, h=hd)
    t1 = time.perf_counter()
    ex = dq.expectation_values(s, t, r["vectors"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "appd_L28.json")))["states"]
    sz0 = ex["sz"][:, 0].cpu().tolist()
    out["appd_L28_lowest4"] = {
        "steps": r["steps_done"], "reorth": r["reorth"], "lanczos_s": t1 - t0,
        "expectation_s": t2 - t1, "ms_per_step": (t1 - t0) / r["steps_done"] * 1e3,
        "E": r["eig"], "Sz0": sz0,
        "E_error_vs_oracle": [r["eig"][e] - ref[e]["E"] for e in range(len(ref))],
        "Sz_max_error_vs_oracle": max(
            float(np.abs(ex["sz"][e].cpu().numpy() - np.array(ref[e]["sz"])).max())
            for e in range(len(ref)))}
    del r, ex, v0

    del s, t, jd, zd, hd
    torch.cuda.empty_cache()
    out.update(operator_workloads(dq, synth, torch, steps, warmup))
    return out


def operator_workloads(dq, synth, torch, steps: int, warmup: int):
    """Generic operators (Sec. 4.1, App. C), the Lindbladian, sites of different local
    dimensions (Sec. 5) and the on-the-fly container for Q = 3: the bench's workloads of
    the operator class (run alone with --operator-workloads-only)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}

    def timed(fn, n=steps, w=warmup):
        return median(time_steps(fn, stream, max(n, 3), w))

    g = torch.Generator(device=dev)
    g.manual_seed(synth.SEED_X)
    s = dq.Sector(28, 14, 2, [7, 7, 7, 7], device=0)
    bonds, jxy, jz, h = synth.tilted_field_chain(28)
    t = dq.Terms(bonds)
    jd, zd, hd = (torch.tensor(a, device=dev) for a in (jxy, jz, h))
    # the same Hamiltonian as a generic operator (Sec. 4.1 strings S+S-, S-S+, SzSz, Sz;
    # App. C clusters of 4 sites): one product per dtype against the XXZ product,
    # and the largest difference between the two
    terms = []
    for (i, j), a, z in zip(bonds, jxy, jz):
        terms += [dq.operator_string(a / 2, (i, j), ("S+", "S-"), 2),
                  dq.operator_string(a / 2, (i, j), ("S-", "S+"), 2),
                  dq.operator_string(z, (i, j), ("Sz", "Sz"), 2)]
    terms += [dq.operator_string(hv, (i,), ("Sz",), 2) for i, hv in enumerate(h)]
    op = dq.Operator(2, 28, terms, cluster_sites=4)
    for dt, tag, es in ((torch.float64, "f64", 8), (torch.float32, "f32", 4)):
        x = torch.randn(s.dim, generator=g, device=dev, dtype=dt)
        y = torch.empty_like(x)
        y2 = torch.empty_like(x)
        per_o = timed(lambda: dq.operator_apply(s, op, x, out=y), n=max(3, steps // 4), w=1)
        per_h = timed(lambda: dq.hamiltonian_apply(s, t, jd, zd, x, h=hd, out=y2), n=max(3, steps // 4), w=1)
        out[f"operator_L28_appd_{tag}"] = {
            "ms": per_o * 1e3, "xxz_product_ms": per_h * 1e3, "over_xxz": per_o / per_h,
            "clusters": op.num_clusters, "nnz": op.nnz, "states_per_s": s.dim / per_o,
            "achieved_GBs": s.dim * 2 * es / per_o / 1e9,
            "frac_of_peak": s.dim * 2 * es / per_o / 1e9 / PEAK_HBM_GBS,
            "max_rel_diff_vs_xxz": float(((y - y2).abs().max() / y2.abs().max()).item())}
        if tag == "f64":  # <x|H|x> without storing H x (reads x once, writes nothing)
            per_e = timed(lambda: dq.operator_expectation(s, op, x), n=max(3, steps // 4), w=1)
            out["operator_L28_appd_f64"]["expectation_ms"] = per_e * 1e3
            out["operator_L28_appd_f64"]["expectation_rel_diff"] = float(
                abs(dq.operator_expectation(s, op, x).item() - torch.dot(x, y).item()) / abs(torch.dot(x, y).item()))
        del x, y, y2
    # complex128 vectors (a real operator on the real and imaginary parts at once)
    xc = torch.complex(torch.randn(s.dim, generator=g, device=dev, dtype=torch.float64),
                       torch.randn(s.dim, generator=g, device=dev, dtype=torch.float64))
    yc = torch.empty_like(xc)
    per_c = timed(lambda: dq.operator_apply(s, op, xc, out=yc), n=max(3, steps // 4), w=1)
    out["operator_L28_appd_c128"] = {"ms": per_c * 1e3, "states_per_s": s.dim / per_c,
                                     "achieved_GBs": s.dim * 32 / per_c / 1e9,
                                     "frac_of_peak": s.dim * 32 / per_c / 1e9 / PEAK_HBM_GBS}
    del xc, yc
    # a block of 8 FP32 columns (one unrank and one rank per reached state serve all 8)
    xb = torch.randn((s.dim, 8), generator=g, device=dev, dtype=torch.float32)
    yb = torch.empty_like(xb)
    per_b = timed(lambda: dq.operator_apply(s, op, xb, out=yb), n=max(3, steps // 4), w=1)
    out["operator_L28_appd_f32k8"] = {"ms": per_b * 1e3, "columns_per_s": s.dim * 8 / per_b,
                                      "achieved_GBs": s.dim * 8 * 8 / per_b / 1e9,
                                      "frac_of_peak": s.dim * 8 * 8 / per_b / 1e9 / PEAK_HBM_GBS}
    del xb, yb
    del op, s, t

    # Sec. 4.1's Lindbladian example at L=12, n=6 (Heisenberg chain from Sx, Sy, Sz strings,
    # dephasing on site 0) on the doubled chain of 24 sites and 12 particles, complex128
    Lh, nh = 12, 6
    hterms = [dq.operator_string(1.0, (i, i + 1), (nm, nm), 2) for i in range(Lh - 1) for nm in ("Sx", "Sy", "Sz")]
    lop = dq.Operator(2, 2 * Lh, dq.lindbladian_terms(Lh, hterms, [(1.0, dq.operator_string(1.0, (0,), ("Sz",), 2))]),
                      cluster_sites=4)
    big = dq.Sector(2 * Lh, 2 * nh, 2, device=0)
    xc = torch.complex(torch.randn(big.dim, generator=g, device=dev, dtype=torch.float64),
                       torch.randn(big.dim, generator=g, device=dev, dtype=torch.float64))
    yc = torch.empty_like(xc)
    per_l = timed(lambda: dq.operator_apply(big, lop, xc, out=yc), n=max(3, steps // 4), w=1)
    out["lindbladian_L12_c128"] = {"ms": per_l * 1e3, "doubled_sector_dim": big.dim,
                                   "clusters": lop.num_clusters, "nnz": lop.nnz,
                                   "states_per_s": big.dim / per_l,
                                   "achieved_GBs": big.dim * 32 / per_l / 1e9,
                                   "frac_of_peak": big.dim * 32 / per_l / 1e9 / PEAK_HBM_GBS}
    del xc, yc, lop, big

    # sites of different local dimensions (Sec. 5's generalisation): the antiferromagnetic
    # Heisenberg ring of alternating spin-1/2 and spin-1 sites, L=24, Sz=0 (n=18), as
    # operator strings; one FP64 and one FP32 product, and rank / unrank of 2^24 states
    dims = [2, 3] * 12
    mterms = []
    for i in range(24):
        j = (i + 1) % 24
        mterms += [dq.operator_string(1.0, (i, j), ("Sz", "Sz"), dims),
                   dq.operator_string(0.5, (i, j), ("S+", "S-"), dims),
                   dq.operator_string(0.5, (i, j), ("S-", "S+"), dims)]
    mop = dq.Operator(dims, 24, mterms, cluster_sites=4)
    ms = dq.Sector(24, 18, dims, device=0)
    entry = {"dim": ms.dim, "split": ms.split, "clusters": mop.num_clusters, "nnz": mop.nnz}
    for tag, dt, vb in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        xm = torch.randn(ms.dim, generator=g, device=dev, dtype=torch.float64).to(dt)
        ym = torch.empty_like(xm)
        per_m = timed(lambda: dq.operator_apply(ms, mop, xm, out=ym), n=max(3, steps // 4), w=1)
        entry[f"{tag}_ms"] = per_m * 1e3
        entry[f"{tag}_states_per_s"] = ms.dim / per_m
        entry[f"{tag}_frac_of_peak"] = ms.dim * 2 * vb / per_m / 1e9 / PEAK_HBM_GBS
        del xm, ym
    nr = 1 << 24
    ids = torch.randint(0, ms.dim, (nr,), generator=g, device=dev, dtype=torch.int64)
    sts = ms.unrank(ids)
    back = torch.empty_like(ids)
    per_u = timed(lambda: ms.unrank(ids, out=sts), n=max(3, steps // 4), w=1)
    per_r = timed(lambda: ms.rank(sts, out=back), n=max(3, steps // 4), w=1)
    if not torch.equal(back, ids):
        raise RuntimeError("mixed sector: rank(unrank(i)) != i")
    entry["unrank_per_s"] = nr / per_u
    entry["rank_per_s"] = nr / per_r
    out["mixed_ring_L24_operator"] = entry
    del ids, sts, back, mop, ms

    # the on-the-fly limit (eq. N=L) for Q = 3, L = 32, n = 32 (1.6e14 states): unrank 2^24
    # random indices and rank them back, with no tables of states
    d3 = dq.Sector(32, 32, 3, device=0).dim
    ids = torch.randint(0, d3, (nr,), generator=g, device=dev, dtype=torch.int64)
    sts = dq.lex_unrank(32, 32, ids, Q=3)
    back = torch.empty_like(ids)
    per_u = timed(lambda: dq.lex_unrank(32, 32, ids, out=sts, Q=3), n=max(3, steps // 4), w=1)
    per_r = timed(lambda: dq.lex_rank(32, 32, sts, out=back, Q=3), n=max(3, steps // 4), w=1)
    if not torch.equal(back, ids):
        raise RuntimeError("on-the-fly Q=3: rank(unrank(i)) != i")
    out["onthefly_Q3_L32"] = {"dim": d3, "unrank_per_s": nr / per_u, "rank_per_s": nr / per_r}
    del ids, sts, back
    torch.cuda.empty_cache()
    return out


def split_sweep(dq, synth, torch, steps: int, warmup: int):
    """Rank, unrank and FP32 H*x throughput on the L=32, n=16 sector versus the number
    of subsystems (most-equal splits, shorter parts first) and the placement of the
    index tables: the paper's question of the best split, asked of the GPU kernels.
    Tables up to the on-chip budget go to LDS ("lds"); larger ones (16/16, 10/11/11)
    stay in device memory ("device"), and every split that fits LDS is run a second
    time with its tables forced into device memory.  H*x is timed in the form the
    autotuner keeps and, where that is the split product, also as the one-pass
    kernel (DCS_SPLIT=0)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    cnt = 1 << 24
    g = torch.Generator(device=dev)
    g.manual_seed(synth.SEED_X)
    occ = torch.rand((cnt, L), generator=g, device=dev).argsort(dim=1)[:, :N_UP]
    states = (torch.ones(cnt, N_UP, dtype=torch.int64, device=dev) << (L - 1 - occ)).sum(dim=1)
    del occ
    bonds, jxy, jz = synth.j1j2_chain(L, J1, J2, DELTA)
    jd, zd = torch.tensor(jxy, device=dev), torch.tensor(jz, device=dev)
    x = torch.randn(601080390, generator=g, device=dev, dtype=torch.float32)
    y = torch.empty_like(x)
    out = {}

    def run(sizes, force_device):
        old = os.environ.get("DCS_GLOBAL_TABLES")
        if force_device:
            os.environ["DCS_GLOBAL_TABLES"] = "1"
        try:
            s = dq.Sector(L, N_UP, 2, sizes, device=0)
        except Exception as e:
            return {"supported": False, "reason": str(e).splitlines()[0][:160]}
        finally:
            if force_device:
                if old is None:
                    os.environ.pop("DCS_GLOBAL_TABLES", None)
                else:
                    os.environ["DCS_GLOBAL_TABLES"] = old
        idx = torch.empty_like(states)
        back = torch.empty_like(states)
        per_r = median(time_steps(lambda: s.rank(states, out=idx), stream, steps, warmup))
        per_u = median(time_steps(lambda: s.unrank(idx, out=back), stream, steps, warmup))
        ok = bool(torch.equal(back, states))
        per_rs = median(time_steps(lambda: s.rank_search(states, out=back), stream, steps, warmup))
        ok = ok and bool(torch.equal(back, idx))
        t = dq.Terms(bonds)
        per_h = median(time_steps(lambda: dq.hamiltonian_apply(s, t, jd, zd, x, out=y), stream,
                                  max(3, steps // 4), 1))
        form = dq.hamiltonian_form(s, t, torch.float32, 1)
        rec = {"supported": True, "tables": "device" if s.tables_in_device_memory else "lds",
               "table_bytes": s.table_bytes, "rank_per_s": cnt / per_r, "unrank_per_s": cnt / per_u,
               "rank_search_per_s": cnt / per_rs,
               "roundtrip_ok": ok, "hx_f32k1_ms": per_h * 1e3, "hx_states_per_s": s.dim / per_h,
               "form": form}
        if form != "single":
            os.environ["DCS_SPLIT"] = "0"
            try:
                per_1 = median(time_steps(lambda: dq.hamiltonian_apply(s, t, jd, zd, x, out=y), stream,
                                          max(3, steps // 4), 1))
                rec["hx_f32k1_one_pass_ms"] = per_1 * 1e3
            except Exception as e:
                rec["hx_f32k1_one_pass_ms"] = None
                rec["one_pass_reason"] = str(e).splitlines()[0][:160]
            finally:
                os.environ.pop("DCS_SPLIT", None)
        del idx, back, s, t
        return rec

    for nsub in (2, 3, 4, 5, 6, 7, 8):
        sizes = [L // nsub + (1 if i >= nsub - L % nsub else 0) for i in range(nsub)]
        key = "/".join(map(str, sizes))
        out[key] = run(sizes, False)
        if out[key].get("tables") == "lds":
            out[key + " (device tables)"] = run(sizes, True)
    # N = L: the on-the-fly order without tables (rank and unrank only; no sector object)
    idx = torch.empty_like(states)
    back = torch.empty_like(states)
    per_r = median(time_steps(lambda: dq.lex_rank(L, N_UP, states, out=idx), stream, steps, warmup))
    per_u = median(time_steps(lambda: dq.lex_unrank(L, N_UP, idx, out=back), stream, steps, warmup))
    out["1x32 (N=L, on the fly)"] = {"supported": True, "tables": "none", "table_bytes": 0,
                                     "rank_per_s": cnt / per_r, "unrank_per_s": cnt / per_u,
                                     "roundtrip_ok": bool(torch.equal(back, states))}
    return out


def cpu_baseline(x_host, checks, runs: int = 3, target_s: float = 4.0, one_core_s: float = 6.0):
    """The oracle leg: the FP64 C oracle (OpenMP over contiguous row blocks, as the
    paper's workers) timed on a contiguous block of rows from the middle of the
    sector, median of `runs` runs on all host threads and one run on one thread;
    and the errors of the timed GPU variants against the oracle on their sampled
    rows (`checks`: variant -> (host FP64 x, rows, GPU rows of y))."""
    import numpy as np
    import synth
    from oracle import native
    ns = native.NativeSector(2, L, N_UP, SPLIT)
    bonds, jxy, jz = synth.j1j2_chain(L, J1, J2, DELTA)
    t = native.NativeTerms(bonds, jxy, jz)
    errors = {}
    for v, (xh, rows, got) in checks.items():
        ref = native.hx_rows(ns, t, xh, rows)
        den = np.abs(ref).sum(axis=-1) if ref.ndim > 1 else np.abs(ref)
        errors[v] = {"rows": int(len(rows)),
                     "rel_err": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                     "max_abs_err": float(np.abs(got - ref).max()),
                     "max_row_err_over_row_norm": float((np.abs(got - ref).reshape(len(rows), -1).sum(axis=1)
                                                         / np.maximum(den.reshape(len(rows), -1).sum(axis=1),
                                                                      1e-300)).max())}
    threads = native.num_threads()
    probe = 1 << 18
    first = (ns.dim - probe) // 2
    t0 = time.perf_counter()
    native.hx_range(ns, t, x_host, first, probe)
    rate = probe / (time.perf_counter() - t0)
    rows = int(min(ns.dim, max(probe, rate * target_s)))
    first = (ns.dim - rows) // 2
    secs = []
    for _ in range(runs):
        t0 = time.perf_counter()
        native.hx_range(ns, t, x_host, first, rows)
        secs.append(time.perf_counter() - t0)
    el = median(secs)
    native.set_threads(1)
    try:
        rows1 = int(max(1 << 14, rate / threads * one_core_s))
        first1 = (ns.dim - rows1) // 2
        t0 = time.perf_counter()
        native.hx_range(ns, t, x_host, first1, rows1)
        el1 = time.perf_counter() - t0
    finally:
        native.set_threads(threads)
    return {"value": rows / el, "unit": "sector states/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 y=Hx on {rows} contiguous rows [{first}, {first + rows}) of the "
                      f"L=32 n=16 sector, median of {runs} runs ({el:.2f} s each), OpenMP static "
                      f"row blocks on {threads} threads; one thread: {rows1} rows in {el1:.2f} s",
            "seconds": el, "runs_seconds": secs,
            "one_core": {"value": rows1 / el1, "unit": "sector states/s", "cores": 1, "rows": rows1,
                         "seconds": el1},
            "variant_errors_vs_oracle": errors}


FORM_KERNELS = {
    "split_staged": "split_diag + split_rows (runs staged in LDS where they fit) + split_cols",
    "split_global": "split_diag + split_rows + split_cols",
    "split_fused": "split_diag + split_rows (left family fused in)",
    "split_tiled": "split_diag + split_rows_tiled (whole n_K blocks of a run staged in LDS) + split_cols",
    "single": "hx_kernel (one pass)",
}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variants", default="f32k8,f32k1,f64k1",
                    help="comma list; the first is the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU timing and the variants' errors vs the oracle)")
    ap.add_argument("--no-extras", action="store_true", help="time the headline product only")
    ap.add_argument("--operator-workloads-only", action="store_true",
                    help="of the other workloads, time only those of the operator class")
    ap.add_argument("--split-sweep", action="store_true",
                    help="also time rank, unrank and H*x versus the number of subsystems")
    ap.add_argument("--no-copy", action="store_true",
                    help="skip the device copy of the FP32 vector size (the reference kernel for "
                         "the achievable bandwidth and for scaling the HBM byte counters)")
    ap.add_argument("--check-rows", type=int, default=100_000,
                    help="sampled rows per variant checked against the oracle")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU row sharding is a design, see the design notes)", file=sys.stderr)
        return 2
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one process only", file=sys.stderr)
        return 2
    if args.steps < 10:
        print("bench.py: note: fewer than 10 timed steps; the median is less stable", file=sys.stderr)

    import numpy as np
    import torch
    import paper_2407_14591_amd as dq
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = dq.Sector(L, N_UP, 2, SPLIT, device=0)
    bonds, jxy, jz = synth.j1j2_chain(L, J1, J2, DELTA)
    terms = dq.Terms(bonds)
    jxy_d = torch.tensor(jxy, device=dev)
    jz_d = torch.tensor(jz, device=dev)
    D = s.dim
    stream = torch.cuda.current_stream(dev)
    results = {}
    copy_info = None
    if not args.no_copy:
        gen = torch.Generator(device=dev)
        gen.manual_seed(synth.SEED_G)
        a = torch.empty(D, dtype=torch.float32, device=dev).normal_(generator=gen)
        b = torch.empty_like(a)
        per = median(time_steps(lambda: b.copy_(a), stream, max(args.steps, 10), args.warmup))
        copy_info = {"bytes_per_copy": 2 * a.numel() * 4, "read_bytes": a.numel() * 4,
                     "write_bytes": a.numel() * 4, "ms": per * 1e3,
                     "GBs": 2 * a.numel() * 4 / per / 1e9}
        del a, b
        torch.cuda.empty_cache()
    want_check = not args.no_cpu_baseline
    rows = np.unique(np.concatenate([np.arange(4096), np.arange(D - 4096, D),
                                     np.random.default_rng(31).integers(0, D, args.check_rows)])).astype(np.uint64)
    rows_d = torch.from_numpy(rows.astype(np.int64)).to(dev)
    checks = {}
    x_host_k1 = None
    for v in args.variants.split(","):
        dt = torch.float32 if v.startswith("f32") else torch.float64
        k = int(v.split("k")[1])
        shape = (D,) if k == 1 else (D, k)
        gen = torch.Generator(device=dev)
        gen.manual_seed(synth.SEED_X)
        x64 = torch.randn(shape, generator=gen, device=dev, dtype=torch.float64)
        x = x64.to(dt)
        xh = None
        if want_check:
            if k == 1 and x_host_k1 is not None:
                xh = x_host_k1
            else:
                xh = x64.cpu().numpy()
                if k == 1:
                    x_host_k1 = xh
        del x64
        y = torch.empty_like(x)

        def step():
            dq.hamiltonian_apply(s, terms, jxy_d, jz_d, x, out=y)

        per_steps = time_steps(step, stream, args.steps, args.warmup)
        per = median(per_steps)
        es = 4 if dt == torch.float32 else 8
        bytes_alg = D * k * 2 * es  # read x once, write y once
        results[v] = {"k": k, "dtype": "f32" if es == 4 else "f64", "seconds_per_step": per,
                      "mean_seconds": sum(per_steps) / len(per_steps),
                      "min_seconds": min(per_steps), "max_seconds": max(per_steps),
                      "states_per_s": D / per, "columns_per_s": D * k / per,
                      "algorithmic_bytes": bytes_alg, "achieved_GBs": bytes_alg / per / 1e9,
                      "form": dq.hamiltonian_form(s, terms, dt, k)}
        if want_check:
            checks[v] = (xh, rows, y[rows_d].double().cpu().numpy())
        del x, y, xh
        torch.cuda.empty_cache()

    head = args.variants.split(",")[0]
    r = results[head]
    traffic = read_traffic(head)
    per = r["seconds_per_step"]
    roofline = {"bound": "hbm", "achieved": r["achieved_GBs"], "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": r["achieved_GBs"] / PEAK_HBM_GBS, "traffic": traffic,
                "kernel": f"one H*X product, form {r['form']}: {FORM_KERNELS.get(r['form'], r['form'])}; "
                          f"algorithmic bytes = dim*k*(4+4) = {r['algorithmic_bytes']}: read X once, "
                          f"write Y once; achieved = those bytes / median product time",
                "byte_model": "compulsory"}
    if traffic:
        roofline["traffic_GBs"] = traffic / per / 1e9
        roofline["traffic_frac"] = traffic / per / 1e9 / PEAK_HBM_GBS
        roofline["amplification"] = traffic / r["algorithmic_bytes"]
    if copy_info:
        roofline["copy_GBs"] = copy_info["GBs"]
        roofline["frac_of_copy"] = r["achieved_GBs"] / copy_info["GBs"]
    out = {
        "metric": METRIC,
        "value": r["states_per_s"],
        "unit": "sector states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dtype"],
        "data": "synthetic",
        "config": {"workload": "J1-J2 XXZ chain L=32 n=16 periodic, J1=1 J2=0.5 Delta=1, split 8/8/8/8",
                   "dim": D, "k": r["k"], "vector_dtype": r["dtype"], "variant": head,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "columns_per_s": r["columns_per_s"],
        "variants": {k_: {"states_per_s": v_["states_per_s"], "columns_per_s": v_["columns_per_s"],
                          "ms": v_["seconds_per_step"] * 1e3, "ms_mean": v_["mean_seconds"] * 1e3,
                          "achieved_GBs": v_["achieved_GBs"],
                          "frac_of_peak": v_["achieved_GBs"] / PEAK_HBM_GBS,
                          "traffic": read_traffic(k_), "form": v_["form"]}
                     for k_, v_ in results.items()},
    }
    for k_, v_ in out["variants"].items():
        if v_["traffic"]:
            v_["amplification"] = v_["traffic"] / results[k_]["algorithmic_bytes"]
            v_["traffic_GBs"] = v_["traffic"] / results[k_]["seconds_per_step"] / 1e9
    if copy_info:
        out["copy_calibration"] = copy_info
    if "f64k1" in results:
        out["speedup_vs_plain_f64_per_column"] = r["columns_per_s"] / results["f64k1"]["columns_per_s"]
    if not args.no_extras:
        out["workloads"] = (operator_workloads(dq, synth, torch, args.steps, args.warmup)
                            if args.operator_workloads_only else
                            extra_workloads(dq, synth, torch, args.steps, args.warmup))
    if args.split_sweep:
        out["split_sweep"] = split_sweep(dq, synth, torch, args.steps, args.warmup)
    if want_check and x_host_k1 is not None:
        cb = cpu_baseline(x_host_k1, checks)
        for k_, e in cb.pop("variant_errors_vs_oracle").items():
            out["variants"][k_]["error_vs_oracle"] = e
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
