"""Batched submissions, captured graphs and tile plans, through the C ABI.

Graph replays are checked against the eager path of the same library
(identical kernels and summation order, so FP64 and FP32 agree bit for bit)
and, for small members, against the CPU oracle.  Between replays the inputs
are modified in place and other (eager) library work runs, as a graph user
would do.
"""
import numpy as np
import pytest

import oracle
from paper_1609_08094_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ccsdt_mod():
    _need_gpu()
    from paper_1609_08094_amd import ccsdt
    ccsdt.load_library()
    return ccsdt


def say(msg):
    print(msg, flush=True)


def _args(p):
    return (p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["vvvo"], p["ovoo"], p["ovov"])


def _eager(ctx, devs, prec, monkeypatch):
    monkeypatch.setenv("CCSDT_GRAPH", "0")
    try:
        return ctx.energy_batched(devs, prec)
    finally:
        monkeypatch.delenv("CCSDT_GRAPH")


# uneven members on both sides of the v = 64 tile-plan boundary
SHAPES = [(4, 40), (7, 70), (3, 23), (5, 97), (6, 50), (4, 130)]


@pytest.fixture(scope="module")
def batch():
    probs = [synth.make_problem(o, v, seed=900 + n) for n, (o, v) in enumerate(SHAPES)]
    return probs, [synth.to_device(p) for p in probs]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_graph_replays_match_eager(ccsdt_mod, batch, prec, monkeypatch):
    probs, devs = batch
    ctx = ccsdt_mod.Context()
    say(f"graph capture {prec}")
    g = ctx.energy_batched(devs, prec)
    assert ctx.graph_stats() == (1, 1)
    e = _eager(ctx, devs, prec, monkeypatch)
    assert g == e
    saved = [d["t1"].clone() for d in devs]
    for r, scale in enumerate([-1.0, 2.5, 0.0]):
        for d in devs:
            d["t1"].mul_(scale)
        torch.cuda.synchronize()
        say(f"graph replay {r} {prec} (t1 scaled by {scale})")
        g = ctx.energy_batched(devs, prec)
        e = _eager(ctx, devs, prec, monkeypatch)
        assert g == e
        for d, s in zip(devs, saved):
            d["t1"].copy_(s)
    assert ctx.graph_stats() == (1, 4)
    if prec == "fp64":
        for p, x in zip(probs[:3], ctx.energy_batched(devs, prec)):
            ref = oracle.triples_energy(*_args(p))
            assert abs(x[0] - ref[0]) <= 1e-10 * abs(ref[1])
    ctx.close()


def test_graph_rebuilt_after_workspace_growth(ccsdt_mod, batch, monkeypatch):
    probs, devs = batch
    ctx = ccsdt_mod.Context()
    say("graph, then a larger eager problem, then graph again")
    a = ctx.energy_batched(devs[:3], "fp64")
    big = synth.to_device(synth.make_problem(9, 150, seed=950))
    ctx.energy(big, "fp64")
    b = ctx.energy_batched(devs[:3], "fp64")
    assert a == b
    assert ctx.graph_stats() == (2, 2)
    # a different problem list is a new capture too
    c = ctx.energy_batched(devs[1:4], "fp64")
    assert c[:2] == b[1:3]
    assert ctx.graph_stats() == (3, 3)
    ctx.close()


def test_batched_denominator_errors_name_the_problem(ccsdt_mod, batch):
    probs, devs = batch
    ctx = ccsdt_mod.Context()
    bad = list(devs[:4])
    bad[2] = dict(bad[2], eps_o=bad[2]["eps_o"] + 10.0)
    say("batched EDENOM")
    with pytest.raises(ccsdt_mod.CcsdtError) as e:
        ctx.energy_batched(bad, "fp32")
    assert e.value.status == -5 and "problem 2" in str(e.value)
    nan = list(devs[:4])
    eo = nan[1]["eps_o"].clone()
    eo[0] = float("nan")
    nan[1] = dict(nan[1], eps_o=eo)
    say("batched non-finite eps")
    with pytest.raises(ccsdt_mod.CcsdtError) as e:
        ctx.energy_batched(nan, "fp32")
    assert e.value.status == -1 and "problem 1" in str(e.value)
    say("batched after errors")
    good = ctx.energy_batched(devs[:4], "fp64")
    for d, g in zip(devs[:4], good):
        assert g == ctx.energy(d, "fp64")
    ctx.close()


def test_batch_of_64_uneven_problems(ccsdt_mod):
    """The 64-member batch recipe (o ~ U{4..16}, v ~ U{40..160}), FP32 and
    BF16X3 against FP64 for every member, FP64 against single-problem calls,
    and the four cheapest members (generated on the host, same recipe) in all
    three precisions against the oracle."""
    ctx = ccsdt_mod.Context()
    shapes = synth.batch_shapes(seed=0)
    cost = [int(o) ** 3 * int(v) ** 4 for o, v in shapes]
    small = sorted(range(len(shapes)), key=lambda n: cost[n])[:4]
    devs, host = [], {}
    for n, (o, v) in enumerate(shapes):
        if n in small:
            host[n] = synth.make_problem(int(o), int(v), seed=n)
            devs.append(synth.to_device(host[n]))
        else:
            devs.append(synth.make_problem_device(int(o), int(v), seed=n, device="cuda"))
    torch.cuda.synchronize()
    say("batch of 64: fp64")
    e64 = ctx.energy_batched(devs, "fp64")
    for n in (0, 17, 63):
        assert e64[n] == ctx.energy(devs[n], "fp64")
    em = {}
    for prec in ("fp32", "bf16x3"):
        say(f"batch of 64: {prec}")
        em[prec] = ctx.energy_batched(devs, prec)
        for a, b in zip(em[prec], e64):
            assert abs(a[0] - b[0]) <= 1e-6 * max(1.0, abs(b[0]))
    for n in small:
        o, v = shapes[n]
        say(f"batch member {n} (o={o}, v={v}) against the oracle")
        ref = oracle.triples_energy(*_args(host[n]))
        assert abs(e64[n][0] - ref[0]) <= 1e-10 * abs(ref[1])
        for prec in ("fp32", "bf16x3"):
            assert abs(em[prec][n][0] - ref[0]) <= 1e-6 * max(1.0, abs(ref[0])), (n, prec, em[prec][n], ref)
    ctx.close()


def test_autotune_and_plans(ccsdt_mod):
    ctx = ccsdt_mod.Context()
    p = synth.make_problem(4, 130, seed=960)
    d = synth.to_device(p)
    ref = oracle.triples_energy(*_args(p))
    assert ctx.plan_get("bf16x3", 130) == 6
    say("autotune bf16x3 o=4 v=130")
    cfg = ctx.autotune(d, "bf16x3")
    assert 0 <= cfg < ccsdt_mod.NTILE_CFG
    assert ctx.plan_get("bf16x3", 130) == cfg
    assert ctx.plan_get("bf16x3", 129) == cfg      # same bucket (128, 256]
    assert ctx.plan_get("bf16x3", 128) == 6        # other bucket untouched
    assert ctx.plan_get("fp64", 130) == 6          # other precision untouched
    E = ctx.energy(d, "bf16x3")[0]
    assert abs(E - ref[0]) <= 1e-6 * max(1.0, abs(ref[0]))
    n, _ = ctx.profile_get("contract")
    assert n == 0                                   # tuning launches are not profiled
    for c in range(ccsdt_mod.NTILE_CFG):
        ctx.plan_set("fp64", 130, c)
        say(f"plan_set fp64 cfg={c}")
        E = ctx.energy(d, "fp64")[0]
        assert abs(E - ref[0]) <= 1e-10 * abs(ref[1])
    ctx.plan_set("fp64", 130, -1)
    assert ctx.plan_get("fp64", 130) == 6
    with pytest.raises(ccsdt_mod.CcsdtError):
        ctx.plan_set("fp64", 130, ccsdt_mod.NTILE_CFG)
    ctx.close()


@pytest.mark.parametrize("cfg", [16, 22, 24])
def test_graph_replays_with_persistent_and_paced_tiles(ccsdt_mod, batch, cfg, monkeypatch):
    """Captured graphs of the persistent (16), 32x32-block (22) and paced (24,
    which clears its counters with a kernel before each launch) contraction
    configurations, replayed with modified inputs, against the eager path."""
    probs, devs = batch
    monkeypatch.setenv("CCSDT_TILE", str(cfg))
    ctx = ccsdt_mod.Context()
    say(f"graph with tile configuration {cfg}")
    g0 = ctx.energy_batched(devs, "bf16x3")
    saved = [d["t1"].clone() for d in devs]
    for d in devs:
        d["t1"].mul_(-1.0)
    torch.cuda.synchronize()
    g1 = ctx.energy_batched(devs, "bf16x3")
    e1 = _eager(ctx, devs, "bf16x3", monkeypatch)
    for d, s in zip(devs, saved):
        d["t1"].copy_(s)
    torch.cuda.synchronize()
    g2 = ctx.energy_batched(devs, "bf16x3")
    assert g1 == e1 and g2 == g0
    assert ctx.graph_stats() == (1, 3)
    ctx.close()
