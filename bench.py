"""Benchmark of the closed-shell (T) energy on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C3] [--precision bf16x3]

One step = one complete E(T) evaluation (pack, both contraction passes, the
energy kernel and every reduction) over synthetic inputs already resident in
HBM.  Prints one JSON line.  The metric is algorithmic GFLOP/s, with
F = (o^3 - o)(2 v^4 + 2 o v^3) the distinct contraction flops under i<=j<=k.

roofline: the dominant kernel is the contraction (both passes, all six
permutation terms of W).  Its algorithmic flops per launch are the flops of
the triples it processes, m (2 v^4 + 2 o v^3) per triple; for BF16X3 every
useful multiply-add issues three bf16 MFMA products, so the MFMA flops are
three times that and are compared with the dense bf16 peak.  Durations come from HIP events the library
records around every launch on the launch stream.

cpu_baseline: the CPU oracle (test infrastructure) on a fixed sample of
triples of the same workload, timed on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
MFMA_FACTOR = {"fp64": 1.0, "fp32": 1.0, "bf16x3": 3.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(key):
    """HBM bytes per launch of the dominant kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes recorded in profiles/traffic.json (scaled by a plain copy's
    counter readings), or None when absent or taken on other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def blas_reference():
    """Vendor-library BF16 rates on this device (random N(0,1) operands, FP32
    accumulation, contiguous operands): square products, and batched products
    of the shape of one contraction pass at C3 (v x v outputs, K = Kp)."""
    import torch
    torch.manual_seed(0)

    def rate(fn, flops, reps=10):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return flops * reps / (time.perf_counter() - t0) / 1e12

    out = {}
    for n in (4096, 8192, 16384):
        a = torch.randn(n, n, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(n, n, device="cuda", dtype=torch.bfloat16)
        out[f"matmul {n}x{n}x{n}"] = rate(lambda: a @ b, 2.0 * n ** 3)
        log(f"blas reference: square {n} done")
        del a, b
    for (bt, m, n, k) in [(600, 600, 600, 640), (300, 1200, 600, 640), (64, 4800, 600, 640)]:
        a = torch.randn(bt, m, k, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(bt, k, n, device="cuda", dtype=torch.bfloat16)
        out[f"bmm {bt}x({m}x{k})x({k}x{n})"] = rate(lambda: torch.bmm(a, b), 2.0 * bt * m * n * k)
        log(f"blas reference: batched {bt} done")
        del a, b
    print(json.dumps({"blas_reference_tflops": out, "peak_bf16_tflops": 2500.0}), flush=True)


def triple_flops(o, v, m):
    return m * (2.0 * v ** 4 + 2.0 * o * v ** 3)


class _SliceStore:
    """vvvo stand-in for the oracle: serves vvvo[:, :, :, p] for the sampled p."""

    def __init__(self, slices):
        self.slices = slices

    def __getitem__(self, key):
        p = key[-1]
        return self.slices[p]


def ctx_energy(ctx, dev, prec, stream):
    return ctx.energy(dev, prec, stream)


def ctx_energy_df(ctx, dev, prec, stream):
    return ctx.energy_df(dev, prec, stream)


def cpu_baseline(dev, sample):
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    host = {f: dev[f].cpu().numpy() for f in ("eps_o", "eps_v", "t1", "t2", "ovoo", "ovov")}
    ps = sorted({p for t in sample for p in t})
    o, v = dev["nocc"], dev["nvirt"]
    t0 = time.perf_counter()
    if "vvvo" in dev:
        host["vvvo"] = _SliceStore({p: np.ascontiguousarray(dev["vvvo"][..., p].cpu().numpy()) for p in ps})
        t0 = time.perf_counter()
    else:
        # density-fitted input: the oracle assembles the needed (vv|vo) slices
        # itself (timed as part of the baseline)
        bvv, bvo = dev["bvv"].cpu().numpy(), dev["bvo"].cpu().numpy()
        t0 = time.perf_counter()
        host["vvvo"] = _SliceStore({p: oracle.vvvo_from_df(bvv, np.ascontiguousarray(bvo[:, p:p + 1, :]))[..., 0]
                                    for p in ps})
    res = []
    for t in sample:
        res.append(oracle.triple_restricted(*t, host["eps_o"], host["eps_v"], host["t1"], host["t2"],
                                            host["vvvo"], host["ovoo"], host["ovov"]))
    dt = time.perf_counter() - t0
    fl = sum(triple_flops(o, v, oracle.multiplicity(*t)) for t in sample)
    return res, dt, fl, threads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed full steps before the timed ones (an untimed prime pass over "
                         "four triples always runs first: it allocates every workspace buffer at "
                         "full size and loads the kernels)")
    ap.add_argument("--config", default="C3", choices=["C0", "C1", "C2", "C3", "batch", "M0", "M1"],
                    help="C0..C3: one (T) problem of the named size; batch: 64 uneven (T) problems "
                         "(o ~ U{4..16}, v ~ U{40..160}) per step through one captured graph; "
                         "M0, M1: RI-MP2 energy (M1: o=119, v=2546, naux=5852)")
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--input", default="eri", choices=["eri", "df", "host"],
                    help="eri: the (vv|vo) block is an input in HBM; df: density-fitting factors are the input "
                         "and the library assembles the (vv|vo) operand on the GPU; host: the (vv|vo) block is "
                         "in pinned host memory and streamed by the library (PCIe-inclusive)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sample", default="0,1,2",
                    help="triples for the CPU baseline and the sampled parity, as i,j,k[;i,j,k]")
    ap.add_argument("--partial-triples", type=int, default=0, metavar="N",
                    help="profiling aid: instead of a step, evaluate the N distinct triples (0, 1, 2..N+1) "
                         "twice (kernel loading, then the run to profile) and print their kernel times")
    ap.add_argument("--vs-fp64", action="store_true",
                    help="after the timed steps, evaluate the whole problem in FP64 (outside the timed "
                         "region, over slices of about 1500 triples) and report its time, the energy "
                         "difference and the speedup")
    ap.add_argument("--vs-fp32", action="store_true",
                    help="with --vs-fp64: also evaluate the whole problem in FP32 the same way")
    ap.add_argument("--blas-reference", action="store_true",
                    help="only time torch.matmul / torch.bmm in bf16 (hipBLASLt) on large square and on "
                         "contraction-shaped batched products, as a reference rate for the MFMA peak, and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device to device five times (reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.blas_reference:
        blas_reference()
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 4 * n, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the triple list would shard over GPUs with one 8-byte reduction; not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1609_08094_amd import ccsdt, synth

    if args.config == "batch":
        return bench_batch(args, torch, ccsdt, synth)
    if args.config in synth.MP2_CONFIGS:
        return bench_mp2(args, torch, ccsdt, synth)
    cfg = synth.CONFIGS[args.config]
    o, v = cfg["o"], cfg["v"]
    log(f"bench: generating {args.config} o={o} v={v} seed={args.seed}")
    t0 = time.perf_counter()
    df = args.input == "df"
    dev = synth.make_problem_device(o, v, seed=args.seed, device="cuda", with_vvvo=not df, with_df=df)
    energy = ctx_energy_df if df else ctx_energy
    if args.input == "host":
        log("bench: moving vvvo to pinned host memory")
        h = torch.empty(dev["vvvo"].shape, dtype=torch.float64, pin_memory=True)
        h.copy_(dev["vvvo"])
        dev["vvvo"] = h
        torch.cuda.empty_cache()
    torch.cuda.synchronize()
    log(f"bench: inputs ready in {time.perf_counter() - t0:.1f}s")

    F = ccsdt.flops(o, v)
    ctx = ccsdt.Context()
    ctx.profile(True)
    stream = torch.cuda.current_stream()
    if args.partial_triples:
        trips = [(0, 1, 2 + n) for n in range(args.partial_triples)]
        run = ctx.triple_energies_df if df else ctx.triple_energies
        run(dev, trips, args.precision, stream)
        ctx.profile_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = run(dev, trips, args.precision, stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        prof = {name: ctx.profile_get(name) for name in ccsdt.KERNEL_CLASSES}
        fl = len(trips) * triple_flops(o, v, 6)
        n, ms = prof["contract"]
        print(json.dumps({"partial_triples": trips, "precision": args.precision, "config": args.config,
                          "wall_ms": wall, "kernels_ms": {k: t for k, (c, t) in prof.items()},
                          "contract_mfma_tflops": MFMA_FACTOR[args.precision] * fl / (ms * 1e-3) / 1e12,
                          "e": [x[0] for x in e]}), flush=True)
        ctx.close()
        return
    log("bench: prime pass (allocation, kernel load)")
    triples = ctx.triple_energies_df if df else ctx.triple_energies
    triples(dev, [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)], args.precision, stream)
    for w in range(args.warmup):
        log(f"bench: warmup {w}")
        energy(ctx, dev, args.precision, stream)
    ctx.profile_reset()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} step(s)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        E, E4, E5 = energy(ctx, dev, args.precision, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    gflops = F / (ms * 1e-3) / 1e9
    log(f"bench: E={E!r} ms/step={ms:.1f} GFLOP/s={gflops:.1f}")

    prof = {name: ctx.profile_get(name) for name in ccsdt.KERNEL_CLASSES}
    na, ms_a = prof["contract"]
    avg_a = ms_a / max(na, 1)
    flops_a_per_launch = F * args.steps / max(na, 1)
    mf = MFMA_FACTOR[args.precision]
    achieved = mf * flops_a_per_launch / (avg_a * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    kernels = {k: {"launches": n // max(args.steps, 1), "ms_per_step": t / args.steps} for k, (n, t) in prof.items()}
    # energy kernel (HBM-bound): algorithmic bytes per triple = W_A + W_B read
    # once (2 v^3 elements of W) plus the three v x v FP64 integral slices
    ne, ms_e = prof["energy"]
    ntrip = o * (o + 1) * (o + 2) // 6 - o
    e_bytes = args.steps * ntrip * (2.0 * v ** 3 * (8 if args.precision == "fp64" else 4) + 3.0 * v * v * 8)
    e_gbs = e_bytes / (ms_e * 1e-3) / 1e9 if ms_e > 0 else 0.0
    energy_roofline = {"bound": "hbm", "achieved": e_gbs, "peak": 8000.0, "unit": "GB/s", "frac": e_gbs / 8000.0,
                       "kernel": "energy", "avg_launch_ms": ms_e / max(ne, 1),
                       "bytes_per_triple": e_bytes / max(args.steps * ntrip, 1)}
    # traffic (bytes per launch) was measured for the default plan of C3 BF16x3
    traffic = None
    if args.config == "C3" and args.precision == "bf16x3" and not df and ctx.plan_get(args.precision, v) == 6 \
            and not os.environ.get("CCSDT_TILE"):
        traffic = measured_traffic("contract_lds_kernel<PrecB3,64,64,128,2,true>|C3")

    def sliced(prec):
        """Whole-problem energy in another precision over slices of the triple
        list (each call packs the operands once), summed exactly; (E, ms, n)."""
        import math
        allt = [(i, j, k) for i in range(o) for j in range(i, o) for k in range(j, o) if not (i == j == k)]
        nsl = max(1, -(-len(allt) // 1500))
        per = -(-len(allt) // nsl)
        parts, msum = [], 0.0
        for n in range(nsl):
            sl = allt[n * per:(n + 1) * per]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            parts += triples(dev, sl, prec, stream)
            torch.cuda.synchronize()
            msum += (time.perf_counter() - t0) * 1e3
            log(f"bench: {prec} comparison, slice {n + 1}/{nsl} ({len(sl)} triples) done")
        return math.fsum(x[0] for x in parts), msum, nsl

    vs64 = None
    if args.vs_fp64 and args.precision != "fp64":
        E64, ms64, nsl = sliced("fp64")
        vs64 = {"fp64_ms_per_step": ms64, "fp64_slices": nsl, "E_fp64": E64, "dE": E - E64,
                "rel_dE": abs(E - E64) / abs(E64), "speedup_vs_fp64": ms64 / ms,
                "within_1e-6": abs(E - E64) <= 1e-6 * max(1.0, abs(E64))}
        if args.vs_fp32 and args.precision != "fp32":
            E32, ms32, nsl32 = sliced("fp32")
            vs64["fp32"] = {"ms_per_step": ms32, "slices": nsl32, "E": E32, "dE": E32 - E64,
                            "rel_dE": abs(E32 - E64) / abs(E64), "speedup_vs_fp64": ms64 / ms32,
                            "within_1e-6": abs(E32 - E64) <= 1e-6 * max(1.0, abs(E64))}

    sample = [tuple(int(x) for x in s.split(",")) for s in args.sample.split(";") if s]
    parity = None
    cpu = None
    if sample:
        log(f"bench: sampled parity on {sample}")
        gpu_s = triples(dev, sample, args.precision, stream)
        gpu_64 = triples(dev, sample, "fp64", stream)
        parity = {"triples": [list(t) for t in sample],
                  "e_gpu": [g[0] for g in gpu_s], "e_gpu_fp64": [g[0] for g in gpu_64]}
        if not args.no_cpu_baseline:
            log("bench: CPU oracle on the sample")
            res, dt, fl, threads = cpu_baseline(dev, sample)
            parity["e_oracle"] = [r[0] for r in res]
            parity["max_rel_gpu_fp64_vs_oracle"] = max(abs(a[0] - b[0]) / abs(b[0]) for a, b in zip(gpu_64, res))
            parity["max_rel_gpu_vs_oracle"] = max(abs(a[0] - b[0]) / abs(b[0]) for a, b in zip(gpu_s, res))
            cpu = {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
                   "sample": f"{len(sample)} restricted triple(s) {sample} of {args.config} "
                             f"(o={o}, v={v}), {fl:.3e} algorithmic flops in {dt:.1f}s"}
        else:
            parity["max_rel_gpu_vs_gpu_fp64"] = max(abs(a[0] - b[0]) / abs(b[0]) for a, b in zip(gpu_s, gpu_64))

    line = {
        "metric": "(T) GFLOP/s & MFMA util; FP32/BF16-mixed vs FP64 at |dE(T)|<=1e-6 Eh",
        "value": gflops, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic (density-fitted integrals, MP2 doubles; seeded)",
        "config": {"workload": f"closed-shell (T) {args.config}: o={o} v={v} naux={3 * (o + v)} "
                               f"seed={args.seed}, {args.precision}"
                               + (", density-fitted (vv|vo) assembled on the GPU" if df else "")
                               + (", (vv|vo) streamed from pinned host memory" if args.input == "host" else ""),
                   "input": args.input,
                   "nocc": o, "nvirt": v, "precision": args.precision, "algorithmic_flops": F},
        "energy": {"E": E, "E4": E4, "E5": E5},
        "mfma_util": achieved / peak,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "contraction", "avg_launch_ms": avg_a, "launches_per_step": na // args.steps},
        "energy_roofline": energy_roofline,
        "kernels": kernels,
        "parity_sample": parity,
        "cpu_baseline": cpu,
    }
    if vs64 is not None:
        line["vs_fp64"] = vs64
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_mp2(args, torch, ccsdt, synth):
    """RI-MP2 energy: one step = pack, every pair product and pair energy, and
    the final sum.  roofline: the pair-product kernel, 2 v^2 naux flops per
    pair (x3 MFMA flops for BF16X3)."""
    cfg = synth.MP2_CONFIGS[args.config]
    o, v, naux = cfg["o"], cfg["v"], cfg["naux"]
    log(f"bench: generating RI-MP2 {args.config} o={o} v={v} naux={naux}")
    t0 = time.perf_counter()
    dev = synth.make_mp2_problem(o, v, naux, seed=args.seed, device="cuda")
    torch.cuda.synchronize()
    log(f"bench: inputs ready in {time.perf_counter() - t0:.1f}s")
    F = ccsdt.rimp2_flops(o, v, naux)
    ctx = ccsdt.Context()
    ctx.profile(True)
    stream = torch.cuda.current_stream()
    # prime: a full chunk of pairs sizes every workspace buffer and loads the kernels
    prime = [(i, j) for i in range(o) for j in range(i, o)][:256]
    ctx.rimp2_pair_energies(dev, prime, args.precision, stream)
    for w in range(args.warmup):
        ctx.rimp2_energy(dev, args.precision, stream)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        E = ctx.rimp2_energy(dev, args.precision, stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    prof = {name: ctx.profile_get(name) for name in ccsdt.KERNEL_CLASSES}
    ng, msg = prof["mp2_gemm"]
    avg = msg / max(ng, 1)
    mfma_factor = {"fp64": 1.0, "fp32": 1.0, "bf16x3": 4.0}[args.precision]   # RI-MP2 keeps lo*lo
    achieved = mfma_factor * (F * args.steps / max(ng, 1)) / (avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    sample = [(0, 1), (o // 2, o - 1)]
    g_s = ctx.rimp2_pair_energies(dev, sample, args.precision, stream)
    g_64 = ctx.rimp2_pair_energies(dev, sample, "fp64", stream)
    parity = {"pairs": [list(t) for t in sample], "e_gpu": g_s, "e_gpu_fp64": g_64}
    cpu = None
    if not args.no_cpu_baseline:
        import numpy as np
        import oracle
        eo, ev = dev["eps_o"].cpu().numpy(), dev["eps_v"].cpu().numpy()
        rows = {i: dev["c_ov"][i].cpu().numpy() for t in sample for i in t}
        c_host = _RowStore(rows)
        t0 = time.perf_counter()
        res = [oracle.rimp2_pair_energy(i, j, eo, ev, c_host) for i, j in sample]
        dt = time.perf_counter() - t0
        parity["e_oracle"] = res
        parity["max_rel_gpu_vs_oracle"] = max(abs(a - b) / abs(b) for a, b in zip(g_s, res))
        parity["max_rel_gpu_fp64_vs_oracle"] = max(abs(a - b) / abs(b) for a, b in zip(g_64, res))
        fl = len(sample) * 2.0 * v * v * naux
        cpu = {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": _threads(), "kind": "oracle",
               "sample": f"{len(sample)} pair energies {sample} of RI-MP2 {args.config}, {fl:.3e} flops "
                         f"(pair products counted once) in {dt:.1f}s"}
    kernels = {k: {"launches": n // max(args.steps, 1), "ms_per_step": t / args.steps} for k, (n, t) in prof.items()}
    # energy kernel (HBM-bound): algorithmic bytes per triple = W_A + W_B read
    # once (2 v^3 elements of W) plus the three v x v FP64 integral slices
    ne, ms_e = prof["energy"]
    ntrip = o * (o + 1) * (o + 2) // 6 - o
    e_bytes = args.steps * ntrip * (2.0 * v ** 3 * (8 if args.precision == "fp64" else 4) + 3.0 * v * v * 8)
    e_gbs = e_bytes / (ms_e * 1e-3) / 1e9 if ms_e > 0 else 0.0
    energy_roofline = {"bound": "hbm", "achieved": e_gbs, "peak": 8000.0, "unit": "GB/s", "frac": e_gbs / 8000.0,
                       "kernel": "energy", "avg_launch_ms": ms_e / max(ne, 1),
                       "bytes_per_triple": e_bytes / max(args.steps * ntrip, 1)}
    line = {
        "metric": "RI-MP2 GFLOP/s & MFMA util (pair products o(o+1)/2 * 2 v^2 naux)",
        "value": F / (ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (fitting coefficients N(0, 0.1^2); seeded)",
        "config": {"workload": f"RI-MP2 {args.config}: o={o} v={v} naux={naux} seed={args.seed}, {args.precision}",
                   "algorithmic_flops": F},
        "energy": {"E_MP2": E},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": "mp2_gemm", "avg_launch_ms": avg,
                     "launches_per_step": ng // args.steps},
        "kernels": kernels, "parity_sample": parity, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


class _RowStore:
    """c_ov stand-in for the oracle: serves the rows c_ov[i] of the sampled i."""

    def __init__(self, rows):
        self.rows = rows

    def __getitem__(self, i):
        return self.rows[i]


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count()


def bench_batch(args, torch, ccsdt, synth):
    """64 independent problems per step, replayed from one captured graph;
    tiles autotuned per v bucket first.  Reports problems/s beside GFLOP/s and
    the per-problem |dE| of the mixed precision against the FP64 GPU path."""
    shapes = synth.batch_shapes(seed=args.seed)
    log(f"bench: generating {len(shapes)} batch members")
    devs = [synth.make_problem_device(int(o), int(v), seed=args.seed + n, device="cuda")
            for n, (o, v) in enumerate(shapes)]
    torch.cuda.synchronize()
    F = sum(ccsdt.flops(int(o), int(v)) for o, v in shapes)
    ctx = ccsdt.Context()
    stream = torch.cuda.current_stream()
    tuned = {}
    for n, (o, v) in enumerate(shapes):
        b = (int(v) - 1).bit_length()
        if b not in tuned:
            tuned[b] = ctx.autotune(devs[n], args.precision, stream)
            log(f"bench: autotune v bucket 2^{b}: cfg {tuned[b]}")
    log("bench: capture")
    ctx.energy_batched(devs, args.precision, stream)
    for w in range(args.warmup):
        ctx.energy_batched(devs, args.precision, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.energy_batched(devs, args.precision, stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    captures, replays = ctx.graph_stats()
    ref = ctx.energy_batched(devs, "fp64", stream)
    dE = [abs(a[0] - b[0]) for a, b in zip(res, ref)]
    line = {
        "metric": "(T) GFLOP/s & MFMA util; FP32/BF16-mixed vs FP64 at |dE(T)|<=1e-6 Eh",
        "value": F / (ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (density-fitted integrals, MP2 doubles; seeded per member)",
        "config": {"workload": f"batched (T): {len(shapes)} problems, o~U{{4..16}}, v~U{{40..160}}, "
                               f"seed={args.seed}, {args.precision}", "algorithmic_flops": F},
        "problems_per_s": len(shapes) / (ms * 1e-3),
        "graph": {"captures": captures, "replays": replays},
        "tiles": {f"v<=2^{b}": c for b, c in sorted(tuned.items())},
        "max_abs_dE_vs_fp64": max(dE), "max_rel_dE_vs_fp64": max(d / abs(b[0]) for d, b in zip(dE, ref)),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
