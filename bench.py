#!/usr/bin/env python3
"""Benchmark of the matrix-free product y = H x on one particle-number sector.

Workload: periodic spin-1/2 J1-J2 XXZ chain, L=32 sites, n=16 up spins
(601,080,390 states), J1=1, J2=0.5, Delta=1, index split 8/8/8/8; x ~ N(0,1)
from a seeded device generator (synthetic data).  One step is one H*X over the
whole sector: every row decoded (Alg. iii), every bond applied, every reached
state ranked (eq. index), x gathered, y written.

Three forms are timed: the batched FP32 block of k=8 columns (the headline
`value`), FP32 k=1, and the plain FP64 k=1 product.  `value` counts sector
states per second per column (dim * k / time).  One product is one call of
dcs_hamiltonian_apply: on this sector the split product's launches (diagonal
per side configuration, row pass, column pass).

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


def extra_workloads(dq, synth, torch, steps: int, warmup: int):
    """The other measured cases (dict of results); every input is seeded and synthetic."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}

    def timed(fn, n=steps, w=warmup):
        return time_variant(fn, stream, n, w) / n

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
    out["rank_unrank_L32"] = {"states": cnt, "rank_ms": per_r * 1e3, "unrank_ms": per_u * 1e3,
                              "rank_per_s": cnt / per_r, "unrank_per_s": cnt / per_u}
    del states, idx, back, s

    # k=8 FP32 block on L=28, n=14 (40,116,600 rows), XXZ J = Delta = 1
    s = dq.Sector(28, 14, 2, [7, 7, 7, 7], device=0)
    bonds, jxy, jz = synth.xxz_chain(28, 1.0, 1.0)
    t = dq.Terms(bonds)
    jd, zd = torch.tensor(jxy, device=dev), torch.tensor(jz, device=dev)
    x = torch.randn((s.dim, 8), generator=g, device=dev, dtype=torch.float32)
    y = torch.empty_like(x)
    per = timed(lambda: dq.hamiltonian_apply(s, t, jd, zd, x, out=y))
    out["hx_L28_f32k8"] = {"ms": per * 1e3, "states_per_s": s.dim * 8 / per,
                           "achieved_GBs": s.dim * 8 * 2 * 4 / per / 1e9}
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
                              "adjoint_compulsory_GBs": s.dim * 24 / per_a / 1e9}
    del x, gv, s, t

    # all sectors of L = 20..26 (spin 1/2, n = 0..L) and spin-1 L = 12..16 at Sz = 0, one launch
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
                                   "states_per_s": total / per}
    del plan, items, xs, ys

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
                     "reorth": r["reorth"], "E0": r["eig"][0], "E0_error_vs_exact": r["eig"][0] + 12.0}
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
                           "achieved_GBs": s.dim * 2 * 4 / per / 1e9}
    del y
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = dq.lanczos(s, t, jd, zd, x, 150, reorth="local")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["lanczos_L34_f32vec"] = {"steps": r["steps_done"], "seconds": el,
                                 "ms_per_step": el / r["steps_done"] * 1e3, "reorth": r["reorth"],
                                 "E0": r["eig"][0]}
    del x
    torch.cuda.empty_cache()
    return out


def split_sweep(dq, synth, torch, steps: int, warmup: int):
    """Rank, unrank and FP32 H*x throughput on the L=32, n=16 sector versus the number
    of subsystems (most-equal splits, shorter parts first): the paper's question of
    the best split, asked of the GPU kernels.  Splits whose tables exceed on-chip
    memory are reported as unsupported."""
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
    for nsub in (2, 3, 4, 5, 6, 7, 8):
        sizes = [L // nsub + (1 if i >= nsub - L % nsub else 0) for i in range(nsub)]
        key = "/".join(map(str, sizes))
        try:
            s = dq.Sector(L, N_UP, 2, sizes, device=0)
        except Exception as e:  # tables beyond the on-chip budget
            out[key] = {"supported": False, "reason": str(e).splitlines()[0][:160]}
            continue
        idx = torch.empty_like(states)
        back = torch.empty_like(states)
        per_r = time_variant(lambda: s.rank(states, out=idx), stream, steps, warmup) / steps
        per_u = time_variant(lambda: s.unrank(idx, out=back), stream, steps, warmup) / steps
        ok = bool(torch.equal(back, states))
        t = dq.Terms(bonds)
        per_h = time_variant(lambda: dq.hamiltonian_apply(s, t, jd, zd, x, out=y), stream,
                             max(2, steps // 4), 1) / max(2, steps // 4)
        out[key] = {"supported": True, "rank_per_s": cnt / per_r, "unrank_per_s": cnt / per_u,
                    "roundtrip_ok": ok, "hx_f32k1_ms": per_h * 1e3, "hx_states_per_s": s.dim / per_h}
        del idx, back, s, t
    return out


def cpu_baseline(x_host, target_s: float = 15.0):
    """The FP64 C oracle (OpenMP over contiguous row blocks, as the paper's
    workers) timed on a contiguous block of rows from the middle of the sector."""
    import numpy as np
    import synth
    from oracle import native
    ns = native.NativeSector(2, L, N_UP, SPLIT)
    bonds, jxy, jz = synth.j1j2_chain(L, J1, J2, DELTA)
    t = native.NativeTerms(bonds, jxy, jz)
    probe = 1 << 18
    first = (ns.dim - probe) // 2
    t0 = time.perf_counter()
    native.hx_range(ns, t, x_host, first, probe)
    rate = probe / (time.perf_counter() - t0)
    rows = int(min(ns.dim, max(probe, rate * target_s)))
    first = (ns.dim - rows) // 2
    t0 = time.perf_counter()
    native.hx_range(ns, t, x_host, first, rows)
    el = time.perf_counter() - t0
    return {"value": rows / el, "unit": "sector states/s", "cores": native.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 y=Hx on {rows} contiguous rows [{first}, {first + rows}) of the "
                      f"L=32 n=16 sector ({el:.1f} s, OpenMP static row blocks)",
            "seconds": el}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variants", default="f32k8,f32k1,f64k1",
                    help="comma list; the first is the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="time the headline product only")
    ap.add_argument("--split-sweep", action="store_true",
                    help="also time rank, unrank and H*x versus the number of subsystems")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also time a plain device copy of the FP32 vector size (the reference "
                         "kernel for scaling the HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU row sharding is a design, see the design notes)", file=sys.stderr)
        return 2
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one process only", file=sys.stderr)
        return 2

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
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED_X)
    stream = torch.cuda.current_stream(dev)
    results = {}
    x_host = None
    copy_info = None
    if args.calibrate_copy:
        a = torch.empty(D, dtype=torch.float32, device=dev).normal_(generator=gen)
        b = torch.empty_like(a)
        el = time_variant(lambda: b.copy_(a), stream, args.steps, args.warmup)
        copy_info = {"bytes_per_copy": 2 * a.numel() * 4, "read_bytes": a.numel() * 4,
                     "write_bytes": a.numel() * 4,
                     "GBs": 2 * a.numel() * 4 * args.steps / el / 1e9}
        del a, b
        torch.cuda.empty_cache()
    for v in args.variants.split(","):
        dt = torch.float32 if v.startswith("f32") else torch.float64
        k = int(v.split("k")[1])
        shape = (D,) if k == 1 else (D, k)
        x = torch.randn(shape, generator=gen, device=dev, dtype=torch.float64)
        if v == "f64k1" and not args.no_cpu_baseline:
            x_host = x.cpu().numpy()
        x = x.to(dt)
        y = torch.empty_like(x)

        def step():
            dq.hamiltonian_apply(s, terms, jxy_d, jz_d, x, out=y)

        el = time_variant(step, stream, args.steps, args.warmup)
        per = el / args.steps
        es = 4 if dt == torch.float32 else 8
        bytes_alg = D * k * 2 * es  # read x once, write y once
        results[v] = {"k": k, "dtype": "f32" if es == 4 else "f64", "seconds_per_step": per,
                      "states_per_s": D * k / per, "algorithmic_bytes": bytes_alg,
                      "achieved_GBs": bytes_alg / per / 1e9}
        del x, y
        torch.cuda.empty_cache()

    head = args.variants.split(",")[0]
    r = results[head]
    traffic = read_traffic(head)
    out = {
        "metric": METRIC,
        "value": r["states_per_s"],
        "unit": "sector states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["seconds_per_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dtype"],
        "data": "synthetic",
        "config": {"workload": "J1-J2 XXZ chain L=32 n=16 periodic, J1=1 J2=0.5 Delta=1, split 8/8/8/8",
                   "dim": D, "k": r["k"], "vector_dtype": r["dtype"], "variant": head,
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBs"], "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": r["achieved_GBs"] / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "kernel": "one H*X product (split_diag + split_rows + split_cols launches); "
                               "algorithmic bytes = dim*k*(4+4): read X once, write Y once"},
        "variants": {k_: {"states_per_s": v_["states_per_s"], "ms": v_["seconds_per_step"] * 1e3,
                          "achieved_GBs": v_["achieved_GBs"]} for k_, v_ in results.items()},
    }
    if copy_info:
        out["copy_calibration"] = copy_info
    if "f64k1" in results:
        out["speedup_vs_plain_f64_per_column"] = r["states_per_s"] / results["f64k1"]["states_per_s"]
    if not args.no_extras:
        out["workloads"] = extra_workloads(dq, synth, torch, args.steps, args.warmup)
    if args.split_sweep:
        out["split_sweep"] = split_sweep(dq, synth, torch, args.steps, args.warmup)
    if x_host is not None:
        out["cpu_baseline"] = cpu_baseline(x_host)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
