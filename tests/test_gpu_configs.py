"""Parity of whole problems and sampled triples at the two mid-size
workloads, against the oracle, through the C ABI.

* o=20, v=200 (FP64 workload), seeds 0, 1 and 2, plus the physically scaled
  variant of seed 0: whole-problem E, E[4], E[5] and every per-triple
  partial against stored oracle values (tests/golden/c1_*.json, written by
  tests/golden/make_golden.py from the oracle alone).  FP64 at 1e-10
  relative; FP32 and BF16X3 at 1e-6 max(1, |E|) (the synthetic inputs), and
  at the literal 1e-6 Eh for the physically scaled variant.
* o=30, v=400 (FP32-mixed workload): sampled triples, distinct and
  two-equal, in all three precisions against the oracle evaluated triple by
  triple on the host.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1609_08094_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


def mixed_tol(e_ref):
    return 1e-6 * max(1.0, abs(e_ref))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08094_amd import ccsdt
    ccsdt.load_library()
    c = ccsdt.Context()
    yield c
    c.close()


def _golden(name):
    path = os.path.join(HERE, "golden", name)
    if not os.path.exists(path):
        pytest.fail(f"missing stored oracle values {name} (python tests/golden/make_golden.py c1)")
    with open(path) as f:
        return json.load(f)


# ------------------------------------------------------------- o=20, v=200
@pytest.mark.parametrize("name", ["c1_seed0.json", "c1_seed1.json", "c1_seed2.json", "c1_phys_seed0.json"])
def test_c1_whole_problem_against_oracle(ctx, name):
    g = _golden(name)
    o, v = g["o"], g["v"]
    say(f"C1 {name}: generating o={o} v={v} seed={g['seed']} b_scale={g['b_scale']} on the host")
    p = synth.make_problem(o, v, seed=g["seed"], b_scale=g["b_scale"])
    d = synth.to_device(p)
    phys = g["b_scale"] != 1.0
    say("  fp64")
    E, E4, E5 = ctx.energy(d, "fp64")
    say(f"  fp64 E={E!r} ref={g['E']!r} rel={abs(E - g['E']) / abs(g['E']):.2e}")
    assert abs(E - g["E"]) <= 1e-10 * abs(g["E"])
    assert abs(E4 - g["E4"]) <= 1e-10 * abs(g["E4"])
    assert abs(E5 - g["E5"]) <= 1e-10 * abs(g["E4"])
    for prec in ("fp32", "bf16x3"):
        say(f"  {prec}")
        Em, E4m, E5m = ctx.energy(d, prec)
        say(f"  {prec} dE={Em - g['E']:.3e} rel={abs(Em - g['E']) / abs(g['E']):.2e} dE5={E5m - g['E5']:.3e}")
        if phys:
            assert abs(Em - g["E"]) <= 1e-6
            assert abs(E5m - g["E5"]) <= 1e-6
        else:
            assert abs(Em - g["E"]) <= mixed_tol(g["E"])
            assert abs(E5m - g["E5"]) <= mixed_tol(g["E"])


@pytest.mark.parametrize("name", ["c1_seed0.json", "c1_seed1.json"])
def test_c1_every_triple_against_oracle(ctx, name):
    """Every restricted triple's (e, e4, e5) in FP64 against the stored
    oracle partials; the mixed paths per triple at 1e-6 max(1, |e|)."""
    g = _golden(name)
    o, v = g["o"], g["v"]
    p = synth.make_problem(o, v, seed=g["seed"], b_scale=g["b_scale"])
    d = synth.to_device(p)
    trips = [tuple(int(x) for x in k.split(",")) for k in g["triples"]]
    say(f"C1 {name}: {len(trips)} triples, fp64")
    got = ctx.triple_energies(d, trips, "fp64")
    worst = 0.0
    for t, row in zip(trips, got):
        ref = g["triples"]["%d,%d,%d" % t]
        for a, b in zip(row, ref):
            worst = max(worst, abs(a - b) / abs(ref[1]))
            assert abs(a - b) <= 1e-10 * abs(ref[1]), (t, row, ref)
    say(f"  fp64 worst per-triple |de|/|e4| = {worst:.2e}")
    for prec in ("fp32", "bf16x3"):
        say(f"C1 {name}: {len(trips)} triples, {prec}")
        got = ctx.triple_energies(d, trips, prec)
        worst = 0.0
        for t, row in zip(trips, got):
            ref = g["triples"]["%d,%d,%d" % t]
            worst = max(worst, abs(row[0] - ref[0]) / max(1.0, abs(ref[0])))
            assert abs(row[0] - ref[0]) <= mixed_tol(ref[0]), (prec, t, row, ref)
        say(f"  {prec} worst per-triple |de|/max(1,|e|) = {worst:.2e}")


# ------------------------------------------------------------- o=30, v=400
C2_TRIPS = [(0, 1, 2), (4, 4, 17), (7, 19, 29), (28, 29, 29), (11, 12, 13), (0, 0, 29)]


@pytest.fixture(scope="module")
def c2(ctx):
    cfg = synth.CONFIGS["C2"]
    say("generating C2 inputs (o=30, v=400, seed 0) on the GPU")
    d = synth.make_problem_device(cfg["o"], cfg["v"], seed=0, device="cuda")
    torch.cuda.synchronize()
    res = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        say(f"C2 sampled triples {C2_TRIPS} {prec}")
        res[prec] = ctx.triple_energies(d, C2_TRIPS, prec)
    host = {f: d[f].cpu().numpy() for f in ("eps_o", "eps_v", "t1", "t2", "ovoo", "ovov")}
    yield d, res, host
    del d
    torch.cuda.empty_cache()


class _Slices:
    """vvvo[..., q] for the occupied indices of one triple, on the host."""

    def __init__(self, vvvo, qs):
        self.s = {q: np.ascontiguousarray(vvvo[..., q].cpu().numpy()) for q in qs}

    def __getitem__(self, key):
        return self.s[key[-1]]


@pytest.mark.parametrize("n", range(len(C2_TRIPS)))
def test_c2_triple_against_oracle(c2, n):
    d, res, host = c2
    t = C2_TRIPS[n]
    say(f"oracle C2 triple {t} (host)")
    ref = oracle.triple_restricted(*t, host["eps_o"], host["eps_v"], host["t1"], host["t2"],
                                   _Slices(d["vvvo"], sorted(set(t))), host["ovoo"], host["ovov"])
    got = res["fp64"][n]
    assert abs(got[0] - ref[0]) <= 1e-10 * abs(ref[1]), (t, got, ref)
    assert abs(got[2] - ref[2]) <= 1e-10 * abs(ref[1]), (t, got, ref)
    for prec in ("fp32", "bf16x3"):
        g = res[prec][n]
        say(f"  {t} {prec}: de/|e| = {abs(g[0] - ref[0]) / abs(ref[0]):.3e}")
        assert abs(g[0] - ref[0]) <= mixed_tol(ref[0]), (prec, t, g, ref)
        assert abs(g[2] - ref[2]) <= mixed_tol(ref[0]), (prec, t, g, ref)
