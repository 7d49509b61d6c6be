"""Benchmark of the closed-shell (T) energy on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C3] [--precision bf16x3]
                    [--budget SECONDS]

One step = one complete E(T) evaluation (pack, both contraction passes, the
energy kernel and every reduction) over synthetic inputs already resident in
HBM.  Prints one JSON line.  The metric is algorithmic GFLOP/s, with
F = (o^3 - o)(2 v^4 + 2 o v^3) the distinct contraction flops under i<=j<=k.

Wall-clock budget: a full step of the default workload (o=40, v=600, BF16x3)
takes close to a minute, so --steps and --warmup are upper bounds.  The run
(from process start: imports, input generation, the CPU baseline, warmup,
timed steps and the sampled parity) is held to --budget seconds: at most one
long warmup step, then whole steps while another one still fits.  Steps are
never cut short; `steps` in the line is the number actually timed and
`steps_requested` the number asked for.  The JSON line is always printed.

roofline: the dominant kernel is the contraction (both passes, all six
permutation terms of W).  `achieved` counts its algorithmic flops, m (2 v^4 +
2 o v^3) per triple, over the average launch duration, against the MFMA peak
of the instruction the kernel issues (for BF16X3 the dense bf16 peak); for
BF16X3 every useful multiply-add issues three bf16 products, so `frac` is at
most 1/3 and `frac_issue` (three times it) is the MFMA issue rate.  Durations
come from HIP events the library records around every launch on the launch
stream.

cpu_baseline: the CPU oracle (test infrastructure) on a small fixed sample of
triples of the same workload, timed on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
MFMA_FACTOR = {"fp64": 1.0, "fp32": 1.0, "bf16x3": 3.0}
DEFAULT_BUDGET_S = 480.0
POST_RESERVE_S = 20.0        # sampled parity on the GPU and the JSON line, after the timed steps


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- the budget
class StepBudget:
    """Wall-clock budget of one run, counted from process start.

    Pure host arithmetic (unit-tested without a GPU): decides whether one more
    warmup or timed step fits, from the time left and an estimate of one step.
    """

    def __init__(self, budget_s: float, t0: float = T_START, clock=time.perf_counter):
        self.budget = float(budget_s)
        self.t0 = t0
        self.clock = clock

    def left(self) -> float:
        return self.t0 + self.budget - self.clock()

    def want_warmup(self, done: int, requested: int, est_step_s: float, warm_s: float,
                    reserve_s: float = 0.0) -> bool:
        """Another warmup step runs while fewer than `requested` ran, it and
        one timed step still fit, and (after the first) warmup has used less
        than a tenth of the budget: long steps get one warmup, short ones all."""
        if done >= requested:
            return False
        if self.left() - reserve_s < 2.0 * est_step_s:
            return False
        return done == 0 or warm_s + est_step_s <= 0.1 * self.budget

    def want_step(self, done: int, requested: int, est_step_s: float, reserve_s: float = 0.0) -> bool:
        """The first timed step always runs; later ones while one more fits."""
        if done >= requested:
            return False
        return done == 0 or self.left() - reserve_s >= est_step_s


def run_timed(step, budget: StepBudget, requested: int, est_step_s: float, reserve_s: float, sync):
    """Time whole steps (`step` is synchronous) while the budget allows.
    Returns (steps done, total seconds, last result)."""
    sync()
    t0 = time.perf_counter()
    n, res, est = 0, None, est_step_s
    while budget.want_step(n, requested, est, reserve_s):
        res = step()
        n += 1
        est = max(est_step_s if n == 1 else 0.0, (time.perf_counter() - t0) / n)
        log(f"bench: timed step {n} done ({time.perf_counter() - t0:.1f}s so far, {budget.left():.0f}s left)")
    sync()
    return n, time.perf_counter() - t0, res


def run_warmup(step, budget: StepBudget, requested: int, est_step_s: float, reserve_s: float):
    """Untimed whole steps while the budget allows; returns (count, seconds,
    measured seconds of one step or the estimate if none ran)."""
    n, spent, est = 0, 0.0, est_step_s
    while budget.want_warmup(n, requested, est, spent, reserve_s):
        t0 = time.perf_counter()
        step()
        dt = time.perf_counter() - t0
        spent += dt
        n += 1
        est = spent / n
        log(f"bench: warmup {n} done in {dt:.1f}s ({budget.left():.0f}s left)")
    return n, spent, est


# ------------------------------------------------------------- host details
def host_info() -> dict:
    """Cores, affinity, CPU model and BLAS of this host."""
    info = {"cpu_count": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):  # pragma: no cover
        info["affinity"] = None
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    info["cpu_model"] = model
    try:
        from threadpoolctl import threadpool_info
        blas = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        info["blas"] = [{"vendor": d.get("internal_api"), "version": d.get("version"),
                         "threads": d.get("num_threads")} for d in blas]
        info["threads"] = max([d.get("num_threads", 1) for d in blas] or [1])
    except Exception:  # pragma: no cover
        info["blas"] = None
        info["threads"] = os.cpu_count()
    return info


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


def multiplicity(i, j, k):
    if i == j == k:
        return 0
    return 3 if (i == j or j == k or i == k) else 6


def whole_problem_weight(o):
    """Distinct and two-equal triple counts of the restricted list."""
    two = o * (o - 1)
    distinct = o * (o - 1) * (o - 2) // 6
    return distinct, two


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


def cpu_baseline(dev, sample, cpu_budget_s):
    """The oracle on the sampled triples, one by one, stopping once the next
    one would overrun `cpu_budget_s` (the first always runs).  Returns
    (per-triple results, triples run, seconds, algorithmic flops)."""
    import numpy as np
    import oracle
    host = {f: dev[f].cpu().numpy() for f in ("eps_o", "eps_v", "t1", "t2", "ovoo", "ovov")}
    o, v = dev["nocc"], dev["nvirt"]
    res, ran, dt = [], [], 0.0
    for t in sample:
        if ran and dt * (len(ran) + 1) / len(ran) > cpu_budget_s:
            break
        if "vvvo" in dev:
            store = _SliceStore({p: np.ascontiguousarray(dev["vvvo"][..., p].cpu().numpy()) for p in set(t)})
            t0 = time.perf_counter()
        else:
            # density-fitted input: the oracle assembles the needed (vv|vo)
            # slices itself (timed as part of the baseline)
            bvv, bvo = dev["bvv"].cpu().numpy(), dev["bvo"].cpu().numpy()
            t0 = time.perf_counter()
            store = _SliceStore({p: oracle.vvvo_from_df(bvv, np.ascontiguousarray(bvo[:, p:p + 1, :]))[..., 0]
                                 for p in set(t)})
        res.append(oracle.triple_restricted(*t, host["eps_o"], host["eps_v"], host["t1"], host["t2"],
                                            store, host["ovoo"], host["ovov"]))
        dt += time.perf_counter() - t0
        ran.append(t)
        log(f"bench: oracle triple {t} done ({dt:.1f}s)")
    fl = sum(triple_flops(o, v, multiplicity(*t)) for t in ran)
    return res, ran, dt, fl


def probe_step_seconds(ctx, triples_fn, dev, prec, stream, ccsdt):
    """Estimate one whole step from the kernel times of four distinct triples
    (after a first pass that loads the kernels and sizes the workspace)."""
    o, v = dev["nocc"], dev["nvirt"]
    probe = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)] if o >= 4 else [(0, 0, 1)] if o >= 2 else []
    if not probe:
        return 0.0
    triples_fn(dev, probe, prec, stream)
    ctx.profile_reset()
    triples_fn(dev, probe, prec, stream)
    prof = {name: ctx.profile_get(name)[1] for name in ccsdt.KERNEL_CLASSES}
    ctx.profile_reset()
    per = (prof["contract"] + prof["energy"] + prof["reduce"]) / len(probe) * 1e-3
    fixed = (prof["pack"] + prof["assemble"]) * 1e-3
    distinct, two = whole_problem_weight(o)
    if o < 4:
        return 1.05 * (fixed + per * two)
    return 1.05 * (fixed + per * (distinct + 0.5 * two))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1,
                    help="timed whole steps (an upper bound: steps stop once another would overrun --budget)")
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed whole steps before the timed ones (an upper bound, see --budget); an untimed "
                         "prime pass over four triples always runs first: it allocates every workspace buffer "
                         "at full size and loads the kernels")
    ap.add_argument("--budget", type=float, default=float(os.environ.get("CCSDT_BENCH_BUDGET", DEFAULT_BUDGET_S)),
                    help="wall-clock seconds for the whole run from process start (default %(default)s)")
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
    ap.add_argument("--phys", action="store_true",
                    help="physically scaled variant: B multiplied by the workload's factor in "
                         "synth.PHYSICAL_B_SCALE so that |E(T)| is of physical size (0.1-1 Eh), where the "
                         "mixed-precision bar is the literal 1e-6 Eh")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sample", default="0,1,2;3,3,17",
                    help="triples for the CPU baseline and the sampled parity, as i,j,k[;i,j,k] "
                         "(indices past nocc - 1 are clipped)")
    ap.add_argument("--cpu-budget", type=float, default=70.0,
                    help="seconds of oracle work for the CPU baseline (the first sampled triple always runs)")
    ap.add_argument("--partial-triples", type=int, default=0, metavar="N",
                    help="profiling aid: instead of a step, evaluate the N distinct triples (0, 1, 2..N+1) "
                         "twice (kernel loading, then the run to profile) and print their kernel times")
    ap.add_argument("--vs-fp64", action="store_true",
                    help="after the timed steps, evaluate the whole problem in FP64 (outside the timed "
                         "region, over slices of about 1500 triples) and report its time, the energy "
                         "difference and the speedup (not held to --budget)")
    ap.add_argument("--vs-fp32", action="store_true",
                    help="with --vs-fp64: also evaluate the whole problem in FP32 the same way")
    ap.add_argument("--blas-reference", action="store_true",
                    help="only time torch.matmul / torch.bmm in bf16 (hipBLASLt) on large square and on "
                         "contraction-shaped batched products, as a reference rate for the MFMA peak, and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device to device five times (reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the triple list would shard over GPUs with one 24-byte reduction; not built)",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
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

    budget = StepBudget(args.budget)
    import torch
    from paper_1609_08094_amd import ccsdt, synth
    log(f"bench: torch and the library loaded at {time.perf_counter() - T_START:.1f}s")

    if args.config == "batch":
        return bench_batch(args, budget, torch, ccsdt, synth)
    if args.config in synth.MP2_CONFIGS:
        return bench_mp2(args, budget, torch, ccsdt, synth)
    cfg = synth.CONFIGS[args.config]
    o, v = cfg["o"], cfg["v"]
    b_scale = synth.PHYSICAL_B_SCALE[args.config] if args.phys else 1.0
    log(f"bench: generating {args.config} o={o} v={v} seed={args.seed} b_scale={b_scale}")
    t0 = time.perf_counter()
    df = args.input == "df"
    dev = synth.make_problem_device(o, v, seed=args.seed, device="cuda", with_vvvo=not df, with_df=df,
                                    b_scale=b_scale)
    energy = ctx_energy_df if df else ctx_energy
    if args.input == "host":
        log("bench: moving vvvo to pinned host memory")
        h = torch.empty(dev["vvvo"].shape, dtype=torch.float64, pin_memory=True)
        h.copy_(dev["vvvo"])
        dev["vvvo"] = h
        torch.cuda.empty_cache()
    torch.cuda.synchronize()
    log(f"bench: inputs ready in {time.perf_counter() - t0:.1f}s ({budget.left():.0f}s of the budget left)")

    F = ccsdt.flops(o, v)
    ctx = ccsdt.Context()
    ctx.profile(True)
    stream = torch.cuda.current_stream()
    triples = ctx.triple_energies_df if df else ctx.triple_energies
    if args.partial_triples:
        trips = [(0, 1, 2 + n) for n in range(args.partial_triples)]
        triples(dev, trips, args.precision, stream)
        ctx.profile_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = triples(dev, trips, args.precision, stream)
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

    log("bench: prime pass (allocation, kernel load) and step estimate")
    est = probe_step_seconds(ctx, triples, dev, args.precision, stream, ccsdt)
    log(f"bench: estimated step {est:.2f}s ({budget.left():.0f}s left)")

    sample = []
    for s in args.sample.split(";"):
        if s:
            t = tuple(sorted(min(int(x), o - 1) for x in s.split(",")))
            if multiplicity(*t) and t not in sample:
                sample.append(t)
    # the oracle before the timed steps, so that only the timed loop absorbs
    # what is left of the budget
    cpu, oracle_res, cpu_ran = None, [], []
    if sample and not args.no_cpu_baseline:
        log(f"bench: CPU oracle on the sample {sample}")
        # the oracle may use what the budget has left beyond one warmup and
        # one timed step (the first sampled triple always runs)
        cpu_budget = min(args.cpu_budget, max(0.0, budget.left() - 2.0 * est - POST_RESERVE_S))
        oracle_res, cpu_ran, dt, fl = cpu_baseline(dev, sample, cpu_budget)
        hi = host_info()
        distinct, two = whole_problem_weight(o)
        per_t = dt / len(cpu_ran)
        cpu = {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": hi["threads"], "kind": "oracle",
               "sample": f"{len(cpu_ran)} restricted triple(s) {cpu_ran} of {args.config} (o={o}, v={v}), "
                         f"{fl:.3e} algorithmic flops in {dt:.1f}s; the oracle forms all six X pieces of every "
                         "triple, so a two-equal triple costs it as much as a distinct one",
               "seconds": dt,
               "whole_problem_s_extrapolated": per_t * (distinct + two),
               "extrapolation": f"{per_t:.2f}s per triple x {distinct + two} triples (extrapolated, not run)",
               "host": hi}

    def step():
        return energy(ctx, dev, args.precision, stream)

    warm_n, warm_s, est = run_warmup(step, budget, args.warmup, est, POST_RESERVE_S)
    ctx.profile_reset()
    log(f"bench: timing up to {args.steps} step(s) ({budget.left():.0f}s left)")
    nsteps, secs, (E, E4, E5) = run_timed(step, budget, args.steps, est, POST_RESERVE_S, torch.cuda.synchronize)
    ms = secs * 1e3 / nsteps
    gflops = F / (ms * 1e-3) / 1e9
    log(f"bench: E={E!r} ms/step={ms:.1f} GFLOP/s={gflops:.1f} over {nsteps} step(s)")

    prof = {name: ctx.profile_get(name) for name in ccsdt.KERNEL_CLASSES}
    na, ms_a = prof["contract"]
    avg_a = ms_a / max(na, 1)
    flops_a_per_launch = F * nsteps / max(na, 1)
    mf = MFMA_FACTOR[args.precision]
    achieved = flops_a_per_launch / (avg_a * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    kernels = {k: {"launches": n // nsteps, "ms_per_step": t / nsteps} for k, (n, t) in prof.items()}
    # energy kernel (HBM-bound): algorithmic bytes per triple = W_A + W_B read
    # once (2 v^3 elements of W) plus the three v x v FP64 integral slices
    ne, ms_e = prof["energy"]
    ntrip = o * (o + 1) * (o + 2) // 6 - o
    e_bytes = nsteps * ntrip * (2.0 * v ** 3 * (8 if args.precision == "fp64" else 4) + 3.0 * v * v * 8)
    e_gbs = e_bytes / (ms_e * 1e-3) / 1e9 if ms_e > 0 else 0.0
    energy_roofline = {"bound": "hbm", "achieved": e_gbs, "peak": 8000.0, "unit": "GB/s", "frac": e_gbs / 8000.0,
                       "kernel": "energy", "avg_launch_ms": ms_e / max(ne, 1),
                       "bytes_per_triple": e_bytes / max(nsteps * ntrip, 1)}
    # traffic (bytes per launch) was measured for the default plan of C3 BF16x3
    traffic = None
    if args.config == "C3" and args.precision == "bf16x3" and not df and ctx.plan_get(args.precision, v) == 6 \
            and not os.environ.get("CCSDT_TILE"):
        traffic = measured_traffic("contract_lds_kernel<PrecB3,64,64,128,2,true>|C3")

    parity = None
    if sample:
        log(f"bench: sampled parity on {sample}")
        gpu_s = triples(dev, sample, args.precision, stream)
        gpu_64 = triples(dev, sample, "fp64", stream)
        parity = {"triples": [list(t) for t in sample],
                  "e_gpu": [g[0] for g in gpu_s], "e_gpu_fp64": [g[0] for g in gpu_64],
                  "max_rel_gpu_vs_gpu_fp64": max(abs(a[0] - b[0]) / abs(b[0]) for a, b in zip(gpu_s, gpu_64))}
        if oracle_res:
            n = len(oracle_res)
            parity["oracle_triples"] = [list(t) for t in cpu_ran]
            parity["e_oracle"] = [r[0] for r in oracle_res]
            parity["max_rel_gpu_fp64_vs_oracle"] = max(abs(a[0] - b[0]) / abs(b[0])
                                                       for a, b in zip(gpu_64[:n], oracle_res))
            parity["max_rel_gpu_vs_oracle"] = max(abs(a[0] - b[0]) / abs(b[0]) for a, b in zip(gpu_s[:n], oracle_res))

    vs64 = None
    if args.vs_fp64 and args.precision != "fp64":
        vs64 = compare_precisions(args, dev, triples, stream, o, E, ms, torch)

    line = {
        "metric": "(T) GFLOP/s & MFMA util; FP32/BF16-mixed vs FP64 at |dE(T)|<=1e-6 Eh",
        "value": gflops, "unit": "GFLOP/s", "n_gpus": 1, "steps": nsteps, "steps_requested": args.steps,
        "warmup": warm_n, "warmup_requested": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic (density-fitted integrals, MP2 doubles; seeded)",
        "config": {"workload": f"closed-shell (T) {args.config}: o={o} v={v} naux={3 * (o + v)} "
                               f"seed={args.seed}, {args.precision}"
                               + (", density-fitted (vv|vo) assembled on the GPU" if df else "")
                               + (", (vv|vo) streamed from pinned host memory" if args.input == "host" else "")
                               + (f", physically scaled (B x {b_scale})" if args.phys else ""),
                   "input": args.input,
                   "nocc": o, "nvirt": v, "precision": args.precision, "algorithmic_flops": F},
        "budget": {"seconds": args.budget, "used_s": time.perf_counter() - T_START,
                   "timed_s": secs, "warmup_s": warm_s, "budget_limited": nsteps < args.steps},
        "energy": {"E": E, "E4": E4, "E5": E5},
        "mfma_util": mf * achieved / peak,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "frac_issue": mf * achieved / peak,
                     "mfma_flops_per_useful_flop": mf, "traffic": traffic,
                     "kernel": "contraction", "avg_launch_ms": avg_a, "launches_per_step": na // nsteps},
        "energy_roofline": energy_roofline,
        "kernels": kernels,
        "parity_sample": parity,
        "cpu_baseline": cpu,
    }
    if vs64 is not None:
        line["vs_fp64"] = vs64
    print(json.dumps(line), flush=True)
    ctx.close()


def compare_precisions(args, dev, triples, stream, o, E, ms, torch):
    """Whole-problem energy in FP64 (and FP32) over slices of the triple
    list (each call packs the operands once), summed exactly, outside the
    timed region."""

    def sliced(prec):
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

    E64, ms64, nsl = sliced("fp64")
    vs64 = {"fp64_ms_per_step": ms64, "fp64_slices": nsl, "E_fp64": E64, "dE": E - E64,
            "rel_dE": abs(E - E64) / abs(E64), "speedup_vs_fp64": ms64 / ms,
            "within_1e-6": abs(E - E64) <= 1e-6 * max(1.0, abs(E64))}
    if args.vs_fp32 and args.precision != "fp32":
        E32, ms32, nsl32 = sliced("fp32")
        vs64["fp32"] = {"ms_per_step": ms32, "slices": nsl32, "E": E32, "dE": E32 - E64,
                        "rel_dE": abs(E32 - E64) / abs(E64), "speedup_vs_fp64": ms64 / ms32,
                        "within_1e-6": abs(E32 - E64) <= 1e-6 * max(1.0, abs(E64))}
    return vs64


def bench_mp2(args, budget, torch, ccsdt, synth):
    """RI-MP2 energy: one step = pack, every pair product and pair energy, and
    the final sum.  roofline: the pair-product kernel, 2 v^2 naux flops per
    pair (x4 MFMA flops for the BF16 split, which keeps lo*lo here)."""
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
    t0 = time.perf_counter()
    ctx.rimp2_pair_energies(dev, prime, args.precision, stream)
    torch.cuda.synchronize()
    est = (time.perf_counter() - t0) * (o * (o + 1) // 2) / len(prime)

    def step():
        return ctx.rimp2_energy(dev, args.precision, stream)

    warm_n, warm_s, est = run_warmup(step, budget, args.warmup, est, POST_RESERVE_S)
    ctx.profile_reset()
    nsteps, secs, E = run_timed(step, budget, args.steps, est, POST_RESERVE_S, torch.cuda.synchronize)
    ms = secs * 1e3 / nsteps
    prof = {name: ctx.profile_get(name) for name in ccsdt.KERNEL_CLASSES}
    ng, msg = prof["mp2_gemm"]
    avg = msg / max(ng, 1)
    mfma_factor = {"fp64": 1.0, "fp32": 1.0, "bf16x3": 4.0}[args.precision]   # RI-MP2 keeps lo*lo
    achieved = (F * nsteps / max(ng, 1)) / (avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    sample = [(0, 1), (o // 2, o - 1)]
    g_s = ctx.rimp2_pair_energies(dev, sample, args.precision, stream)
    g_64 = ctx.rimp2_pair_energies(dev, sample, "fp64", stream)
    parity = {"pairs": [list(t) for t in sample], "e_gpu": g_s, "e_gpu_fp64": g_64}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        eo, ev = dev["eps_o"].cpu().numpy(), dev["eps_v"].cpu().numpy()
        rows = {i: dev["c_ov"][i].cpu().numpy() for t in sample for i in t}
        t0 = time.perf_counter()
        res = [oracle.rimp2_pair_energy(i, j, eo, ev, rows) for i, j in sample]
        dt = time.perf_counter() - t0
        parity["e_oracle"] = res
        parity["max_rel_gpu_vs_oracle"] = max(abs(a - b) / abs(b) for a, b in zip(g_s, res))
        parity["max_rel_gpu_fp64_vs_oracle"] = max(abs(a - b) / abs(b) for a, b in zip(g_64, res))
        fl = len(sample) * 2.0 * v * v * naux
        hi = host_info()
        cpu = {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": hi["threads"], "kind": "oracle",
               "sample": f"{len(sample)} pair energies {sample} of RI-MP2 {args.config}, {fl:.3e} flops "
                         f"(pair products counted once) in {dt:.1f}s", "seconds": dt, "host": hi}
    kernels = {k: {"launches": n // nsteps, "ms_per_step": t / nsteps} for k, (n, t) in prof.items()}
    line = {
        "metric": "RI-MP2 GFLOP/s & MFMA util (pair products o(o+1)/2 * 2 v^2 naux)",
        "value": F / (ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": nsteps,
        "steps_requested": args.steps, "warmup": warm_n, "warmup_requested": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (fitting coefficients N(0, 0.1^2); seeded)",
        "config": {"workload": f"RI-MP2 {args.config}: o={o} v={v} naux={naux} seed={args.seed}, {args.precision}",
                   "algorithmic_flops": F},
        "budget": {"seconds": args.budget, "used_s": time.perf_counter() - T_START, "timed_s": secs,
                   "warmup_s": warm_s, "budget_limited": nsteps < args.steps},
        "energy": {"E_MP2": E},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "frac_issue": mfma_factor * achieved / peak,
                     "mfma_flops_per_useful_flop": mfma_factor, "traffic": None, "kernel": "mp2_gemm",
                     "avg_launch_ms": avg, "launches_per_step": ng // nsteps},
        "kernels": kernels, "parity_sample": parity, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_batch(args, budget, torch, ccsdt, synth):
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
    t0 = time.perf_counter()
    ctx.energy_batched(devs, args.precision, stream)
    est = time.perf_counter() - t0

    def step():
        return ctx.energy_batched(devs, args.precision, stream)

    warm_n, warm_s, est = run_warmup(step, budget, args.warmup, est, POST_RESERVE_S)
    nsteps, secs, res = run_timed(step, budget, args.steps, est, POST_RESERVE_S, torch.cuda.synchronize)
    ms = secs * 1e3 / nsteps
    captures, replays = ctx.graph_stats()
    ref = ctx.energy_batched(devs, "fp64", stream)
    dE = [abs(a[0] - b[0]) for a, b in zip(res, ref)]
    line = {
        "metric": "(T) GFLOP/s & MFMA util; FP32/BF16-mixed vs FP64 at |dE(T)|<=1e-6 Eh",
        "value": F / (ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": nsteps,
        "steps_requested": args.steps, "warmup": warm_n, "warmup_requested": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (density-fitted integrals, MP2 doubles; seeded per member)",
        "config": {"workload": f"batched (T): {len(shapes)} problems, o~U{{4..16}}, v~U{{40..160}}, "
                               f"seed={args.seed}, {args.precision}", "algorithmic_flops": F},
        "budget": {"seconds": args.budget, "used_s": time.perf_counter() - T_START, "timed_s": secs,
                   "warmup_s": warm_s, "budget_limited": nsteps < args.steps},
        "problems_per_s": len(shapes) / (ms * 1e-3),
        "graph": {"captures": captures, "replays": replays},
        "tiles": {f"v<=2^{b}": c for b, c in sorted(tuned.items())},
        "max_abs_dE_vs_fp64": max(dE), "max_rel_dE_vs_fp64": max(d / abs(b[0]) for d, b in zip(dE, ref)),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
