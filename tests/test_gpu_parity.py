"""Parity of the HIP path against the CPU oracle, through the C ABI.

Bars (stated by the target of this work):
* FP64 path: |dE| <= 1e-10 |E_ref|.
* Mixed paths (FP32, BF16x3): |dE| <= 1e-6 Eh * max(1, |E_ref| / 1 Eh), i.e. the
  absolute 1 uEh bar at physical magnitudes and a 1e-6 relative bar for the
  synthetic inputs, whose |E| is far above physical values.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import triples as T
from paper_1609_08094_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

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


@pytest.fixture(scope="module")
def ctx(ccsdt_mod):
    c = ccsdt_mod.Context()
    yield c
    c.close()


def _args(p):
    return (p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["vvvo"], p["ovoo"], p["ovov"])


def mixed_tol(e_ref):
    return 1e-6 * max(1.0, abs(e_ref))


# Unit roundoff of one contraction term: FP32 accumulation of Kp products
# (2^-24 each), and for BF16X3 the two-term split x = hi + lo + d with
# |d| <= 2^-16 |x| plus the dropped lo*lo product: <= 3 * 2^-16 per product.
U_TERM = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 3 * 2.0 ** -16}


def w_bound(p, t, prec):
    """Elementwise bound on |W_gpu - W| from the abs-valued contraction."""
    import numpy as np
    absW = T.w_tensor(*t, np.abs(p["t2"]), np.abs(p["vvvo"]), -np.abs(p["ovoo"]))
    K = p["nocc"] + p["nvirt"]
    u = U_TERM[prec] + K * 2.0 ** -24 if prec != "fp64" else K * U_TERM["fp64"]
    return 2.0 * u * absW


def say(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ C0 full
@pytest.fixture(scope="module")
def c0():
    with open(os.path.join(HERE, "golden", "c0_seed0.json")) as f:
        g = json.load(f)
    p = synth.make_problem(6, 30, seed=0)
    return p, g


def test_c0_fp64_matches_oracle(ctx, c0):
    p, g = c0
    say("C0 fp64 o=6 v=30 seed=0")
    E, E4, E5 = ctx.energy(synth.to_device(p), "fp64")
    assert abs(E - g["E"]) <= 1e-10 * abs(g["E"])
    assert abs(E4 - g["E4"]) <= 1e-10 * abs(g["E4"])
    assert abs(E5 - g["E5"]) <= 1e-10 * abs(g["E4"])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_c0_mixed_matches_oracle(ctx, c0, prec):
    p, g = c0
    say(f"C0 {prec} o=6 v=30 seed=0")
    E, E4, E5 = ctx.energy(synth.to_device(p), prec)
    say(f"  E={E!r} ref={g['E']!r} dE={E - g['E']:.3e} dE5={E5 - g['E5']:.3e}")
    assert abs(E - g["E"]) <= mixed_tol(g["E"])
    assert abs(E4 - g["E4"]) <= mixed_tol(g["E4"])
    assert abs(E5 - g["E5"]) <= mixed_tol(g["E"])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_c0_physically_scaled(ctx, prec):
    """C0 with B scaled so that |E(T)| is of physical size (0.34 Eh): FP64 at
    1e-10 relative, the mixed paths at the literal 1e-6 Eh."""
    with open(os.path.join(HERE, "golden", "c0_phys_seed0.json")) as f:
        g = json.load(f)
    p = synth.make_problem(6, 30, seed=0, b_scale=g["b_scale"])
    say(f"C0 physically scaled (b_scale={g['b_scale']}) {prec}")
    E, E4, E5 = ctx.energy(synth.to_device(p), prec)
    say(f"  E={E!r} ref={g['E']!r} dE={E - g['E']:.3e}")
    if prec == "fp64":
        assert abs(E - g["E"]) <= 1e-10 * abs(g["E"])
        assert abs(E5 - g["E5"]) <= 1e-10 * abs(g["E"])
    else:
        assert abs(E - g["E"]) <= 1e-6
        assert abs(E5 - g["E5"]) <= 1e-6


def test_c0_per_triple_energies(ctx, c0):
    p, g = c0
    trips = [tuple(int(x) for x in k.split(",")) for k in g["triples"]]
    say("C0 fp64 per-triple energies")
    got = ctx.triple_energies(synth.to_device(p), trips, "fp64")
    for t, row in zip(trips, got):
        ref = g["triples"]["%d,%d,%d" % t]
        for a, b in zip(row, ref):
            assert abs(a - b) <= 1e-11 * abs(ref[1])


def test_c0_w_matches_oracle(ctx, c0):
    p, _ = c0
    d = synth.to_device(p)
    for t in [(0, 1, 2), (0, 0, 5), (2, 4, 4), (1, 3, 5)]:
        say(f"C0 debug W {t}")
        W = ctx.debug_w(d, *t, precision="fp64")
        ref = T.w_tensor(*t, p["t2"], p["vvvo"], p["ovoo"])
        assert np.abs(W - ref).max() <= 1e-12 * np.abs(ref).max()
        for prec in ("fp32", "bf16x3"):
            Wm = ctx.debug_w(d, *t, precision=prec)
            assert np.all(np.abs(Wm - ref) <= w_bound(p, t, prec))


# ---------------------------------------------------------- odd and tiny shapes
SHAPES = [(1, 7), (2, 1), (2, 7), (3, 17), (5, 33), (3, 65), (2, 129), (4, 48)]


@pytest.mark.parametrize("o,v", SHAPES)
def test_odd_shapes_fp64(ctx, o, v):
    p = synth.make_problem(o, v, seed=o * 100 + v)
    say(f"shape fp64 o={o} v={v}")
    ref = oracle.triples_energy(*_args(p))
    E, E4, E5 = ctx.energy(synth.to_device(p), "fp64")
    scale = max(abs(ref[1]), 1e-300)
    if o == 1 or v == 1:
        assert abs(E) <= 1e-13 * max(1.0, scale)
        return
    assert abs(E - ref[0]) <= 1e-10 * scale
    assert abs(E4 - ref[1]) <= 1e-10 * scale
    assert abs(E5 - ref[2]) <= 1e-10 * scale


@pytest.mark.parametrize("o,v", [(3, 17), (5, 33), (2, 129)])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_odd_shapes_mixed(ctx, o, v, prec):
    """Both mixed paths meet the mixed bar at every size, on E and on each of
    E[4] and E[5] (E[5] within the absolute budget of E: it is a cancelling
    sum whose error comes from W alone, since Z is formed from the FP64
    integrals)."""
    p = synth.make_problem(o, v, seed=o * 100 + v)
    say(f"shape {prec} o={o} v={v}")
    ref = oracle.triples_energy(*_args(p))
    E, E4, E5 = ctx.energy(synth.to_device(p), prec)
    say(f"  dE/|E| = {abs(E - ref[0]) / abs(ref[0]):.3e} dE5/|E5| = {abs(E5 - ref[2]) / abs(ref[2]):.3e}")
    assert abs(E - ref[0]) <= mixed_tol(ref[0])
    assert abs(E4 - ref[1]) <= mixed_tol(ref[1])
    assert abs(E5 - ref[2]) <= mixed_tol(ref[0])
    d = synth.to_device(p)
    t = (0, 1, min(2, o - 1))
    Wm = ctx.debug_w(d, *t, precision=prec)
    ref_w = T.w_tensor(*t, p["t2"], p["vvvo"], p["ovoo"])
    assert np.all(np.abs(Wm - ref_w) <= w_bound(p, t, prec))


# ------------------------------------------------------------- tile configs
@pytest.fixture(scope="module")
def tile_cases():
    cases = []
    for (o, v) in [(3, 45), (4, 130)]:
        p = synth.make_problem(o, v, seed=700 + v)
        cases.append((p, oracle.triples_energy(*_args(p))))
    return cases


@pytest.mark.parametrize("cfg", list(range(27)))
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_every_tile_config(ctx, tile_cases, cfg, prec, monkeypatch):
    monkeypatch.setenv("CCSDT_TILE", str(cfg))
    for p, ref in tile_cases:
        say(f"tile cfg={cfg} {prec} o={p['nocc']} v={p['nvirt']}")
        E, E4, E5 = ctx.energy(synth.to_device(p), prec)
        if prec == "fp64":
            assert abs(E - ref[0]) <= 1e-10 * abs(ref[1])
        else:
            assert abs(E - ref[0]) <= mixed_tol(ref[0])


@pytest.fixture(scope="module")
def hbm_case():
    """A problem whose packed operands (4.6 GB in FP64) live in HBM far beyond
    the caches, so that staging latencies are those of the large workloads."""
    d = synth.make_problem_device(16, 320, seed=720, device="cuda")
    torch.cuda.synchronize()
    trips = [(0, 1, 2), (3, 7, 15), (5, 9, 12), (2, 2, 11), (4, 8, 8)]
    return d, trips


def test_tile_configs_agree_at_hbm_scale(ctx, hbm_case, monkeypatch):
    """Every tile configuration against the register-direct one (no LDS
    staging), per triple, at a size where operands stream from HBM; one
    triple of the reference also against the oracle."""
    d, trips = hbm_case
    monkeypatch.setenv("CCSDT_TILE", "0")
    say("hbm scale reference cfg 0 fp64")
    ref = ctx.triple_energies(d, trips, "fp64")
    host = {f: d[f].cpu().numpy() for f in ("eps_o", "eps_v", "t1", "t2", "ovoo", "ovov")}
    i, j, k = trips[0]

    class Slices:  # serves vvvo[..., q] for the triple's occupied indices only
        def __init__(self):
            self.s = {q: np.ascontiguousarray(d["vvvo"][..., q].cpu().numpy()) for q in (i, j, k)}

        def __getitem__(self, key):
            return self.s[key[-1]]

    vv = Slices()
    o_ref = T.triple_restricted(i, j, k, host["eps_o"], host["eps_v"], host["t1"], host["t2"], vv,
                                host["ovoo"], host["ovov"])
    assert abs(ref[0][0] - o_ref[0]) <= 1e-10 * abs(o_ref[1])
    for cfg in range(1, 27):
        monkeypatch.setenv("CCSDT_TILE", str(cfg))
        for prec in ("fp64", "fp32", "bf16x3"):
            say(f"hbm scale cfg {cfg} {prec}")
            got = ctx.triple_energies(d, trips, prec)
            for g, r in zip(got, ref):
                tol = 1e-12 if prec == "fp64" else 1e-6
                assert abs(g[0] - r[0]) <= tol * abs(r[1]), (cfg, prec, g, r)


# ------------------------------------------------------------------- invariants
def test_relabeling_invariance_gpu(ctx):
    from tests.test_oracle_pins import relabel
    p = synth.make_problem(5, 40, seed=31)
    rng = np.random.default_rng(1)
    q = relabel(p, rng.permutation(5), rng.permutation(40))
    say("relabel o=5 v=40")
    a = ctx.energy(synth.to_device(p), "fp64")
    b = ctx.energy(synth.to_device(q), "fp64")
    for x, y in zip(a, b):
        assert abs(x - y) <= 1e-12 * abs(a[1])


def test_w_pair_symmetry_gpu(ctx):
    """W^abc_iik = W^bac_iik and W^abc_ijj = W^acb_ijj (joint pair symmetry)."""
    p = synth.make_problem(4, 37, seed=32)
    d = synth.to_device(p)
    say("W symmetry o=4 v=37")
    W = ctx.debug_w(d, 1, 1, 3, precision="fp64")
    assert np.abs(W - W.transpose(1, 0, 2)).max() <= 1e-12 * np.abs(W).max()
    W = ctx.debug_w(d, 0, 2, 2, precision="fp64")
    assert np.abs(W - W.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(W).max()


def test_t1_sign_split_gpu(ctx):
    p = synth.make_problem(4, 30, seed=33)
    d = synth.to_device(p)
    say("t1 sign split o=4 v=30")
    Ep, E4, E5 = ctx.energy(d, "fp64")
    d2 = dict(d, t1=-d["t1"])
    Em = ctx.energy(d2, "fp64")[0]
    assert abs((Ep - Em) - 2 * E5) <= 1e-12 * abs(E4)
    assert abs((Ep + Em) - 2 * E4) <= 1e-12 * abs(E4)


def test_zero_integrals_gpu(ctx):
    p = synth.make_problem(4, 20, seed=34)
    for f in ("vvvo", "ovoo", "ovov"):
        p[f] = np.zeros_like(p[f])
    say("zero integrals o=4 v=20")
    for prec in ("fp64", "fp32", "bf16x3"):
        assert ctx.energy(synth.to_device(p), prec) == (0.0, 0.0, 0.0)


def test_fp64_bitwise_deterministic(ctx):
    p = synth.make_problem(6, 50, seed=35)
    d = synth.to_device(p)
    say("determinism o=6 v=50")
    a = ctx.energy(d, "fp64")
    b = ctx.energy(d, "fp64")
    assert a == b


# ------------------------------------------------------------------ batched
def test_batched_matches_single(ctx):
    shapes = [(4, 40), (7, 55), (5, 61), (9, 40), (6, 100)]
    probs = [synth.make_problem(o, v, seed=50 + n) for n, (o, v) in enumerate(shapes)]
    devs = [synth.to_device(p) for p in probs]
    say("batched fp64 5 problems")
    got = ctx.energy_batched(devs, "fp64")
    for p, g in zip(probs, got):
        ref = oracle.triples_energy(*_args(p))
        assert abs(g[0] - ref[0]) <= 1e-10 * abs(ref[1])
    say("batched fp32 5 problems")
    got32 = ctx.energy_batched(devs, "fp32")
    for g64, g32 in zip(got, got32):
        assert abs(g32[0] - g64[0]) <= mixed_tol(g64[0])


# ------------------------------------------------------------------ errors
def test_error_paths(ctx, ccsdt_mod):
    p = synth.make_problem(3, 10, seed=36)
    d = synth.to_device(p)
    say("error paths")
    with pytest.raises(ccsdt_mod.CcsdtError) as e:
        ctx.energy(d, 7)
    assert e.value.status == -4
    bad = dict(d, eps_o=d["eps_o"] + 10.0)
    with pytest.raises(ccsdt_mod.CcsdtError) as e:
        ctx.energy(bad, "fp64")
    assert e.value.status == -5
    lib = ccsdt_mod.load_library()
    import ctypes
    s = ccsdt_mod.make_problem_struct(d)
    s.vvvo = ctypes.c_void_p(p["vvvo"].ctypes.data)    # host pointer
    out = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
    rc = lib.ccsdt_energy(ctx._h, ctypes.byref(s), 0, None, out)
    assert rc == -1 and list(out) == [1.0, 2.0, 3.0]
    s = ccsdt_mod.make_problem_struct(d)
    s.nocc = 0
    assert lib.ccsdt_energy(ctx._h, ctypes.byref(s), 0, None, out) == -1
    with pytest.raises(ccsdt_mod.CcsdtError):
        ctx.triple_energies(d, [(2, 1, 0)])


def test_memory_cap_gives_enomem(ccsdt_mod, monkeypatch):
    monkeypatch.setenv("CCSDT_MAX_DEVICE_BYTES", "1024")
    c = ccsdt_mod.Context()
    p = synth.make_problem(3, 20, seed=37)
    say("memory cap")
    with pytest.raises(ccsdt_mod.CcsdtError) as e:
        c.energy(synth.to_device(p), "fp64")
    assert e.value.status == -2
    c.close()


def test_edge_cases(ctx, ccsdt_mod):
    """Size limits, an empty triple list, triples with i = j = k only, and
    repeated triples."""
    import ctypes
    p = synth.make_problem(4, 20, seed=38)
    d = synth.to_device(p)
    lib = ccsdt_mod.load_library()
    out = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
    for field, value in (("nvirt", 2049), ("nocc", 1025)):
        s = ccsdt_mod.make_problem_struct(d)
        setattr(s, field, value)
        say(f"limit {field}={value}")
        assert lib.ccsdt_energy(ctx._h, ctypes.byref(s), 0, None, out) == -1
        assert list(out) == [1.0, 2.0, 3.0]
    say("empty triple list")
    with pytest.raises(ccsdt_mod.CcsdtError) as e:
        ctx.triple_energies(d, [], "fp64")
    assert e.value.status == -1
    say("triples with i = j = k only")
    assert ctx.triple_energies(d, [(0, 0, 0), (3, 3, 3)], "fp32") == [(0.0, 0.0, 0.0)] * 2
    say("repeated and zero triples mixed")
    trips = [(0, 1, 2), (1, 1, 1), (0, 1, 2), (2, 3, 3), (0, 1, 2)]
    r = ctx.triple_energies(d, trips, "fp64")
    assert r[0] == r[2] == r[4] and r[1] == (0.0, 0.0, 0.0)
    ref = oracle.triples_energy(*_args(p), triples=[(0, 1, 2), (2, 3, 3)])
    assert abs(r[0][0] + r[3][0] - ref[0]) <= 1e-10 * abs(ref[1])


def test_one_shot_entry_point(ctx, ccsdt_mod):
    """ccsdt_triples_energy (its own context per call) equals the context call
    bit for bit, and the oracle in FP64."""
    p = synth.make_problem(5, 37, seed=39)
    d = synth.to_device(p)
    ref = oracle.triples_energy(*_args(p))
    for prec in ("fp64", "fp32", "bf16x3"):
        say(f"one-shot {prec}")
        e = ccsdt_mod.triples_energy(d, prec)
        assert e == ctx.energy(d, prec)[0]
        assert e == ccsdt_mod.triples_energy(d, prec)
    assert abs(ccsdt_mod.triples_energy(d, "fp64") - ref[0]) <= 1e-10 * abs(ref[1])


def test_calls_on_a_side_stream(ctx, ccsdt_mod):
    """Work enqueued on a caller's non-default stream (default priority): the
    single-problem, batched (captured graph) and RI-MP2 calls give the same
    results as on the current stream, and the inputs written on that stream
    just before the call are the ones read."""
    p = synth.make_problem(4, 41, seed=40)
    d = synth.to_device(p)
    s = torch.cuda.Stream()
    ref = ctx.energy(d, "fp32")
    say("side stream: single problem")
    with torch.cuda.stream(s):
        t1 = d["t1"].clone()
        d2 = dict(d, t1=t1)                      # written on s, read on s
        got = ctx.energy(d2, "fp32", stream=s)
    s.synchronize()
    assert got == ref
    say("side stream: batched graph")
    devs = [synth.to_device(synth.make_problem(3, 20 + 9 * n, seed=41 + n)) for n in range(3)]
    b0 = ctx.energy_batched(devs, "fp64")
    b1 = ctx.energy_batched(devs, "fp64", stream=s)
    s.synchronize()
    assert b0 == b1
    say("side stream: RI-MP2")
    m = synth.make_mp2_problem(3, 30, 40, seed=42)
    dm = dict(nocc=3, nvirt=30, naux=40, eps_o=torch.from_numpy(m["eps_o"]).cuda(),
              eps_v=torch.from_numpy(m["eps_v"]).cuda(), c_ov=torch.from_numpy(m["c_ov"]).cuda())
    assert ctx.rimp2_energy(dm, "fp64", stream=s) == ctx.rimp2_energy(dm, "fp64")


def _random_shapes(n=8, seed=2024):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(1, 8)), int(rng.integers(1, 91))) for _ in range(n)]


@pytest.mark.parametrize("o,v", _random_shapes())
def test_random_shapes_all_precisions(ctx, o, v):
    """Shapes drawn from a fixed seed (o in 1..7, v in 1..90): FP64 against
    the oracle at 1e-10, FP32 and BF16X3 at the mixed bar."""
    p = synth.make_problem(o, v, seed=5000 + 100 * o + v)
    say(f"random shape o={o} v={v}")
    ref = oracle.triples_energy(*_args(p))
    d = synth.to_device(p)
    E = ctx.energy(d, "fp64")
    assert abs(E[0] - ref[0]) <= 1e-10 * max(abs(ref[1]), 1e-300)
    for prec in ("fp32", "bf16x3"):
        Em = ctx.energy(d, prec)[0]
        say(f"  {prec} dE = {Em - ref[0]:.3e} (E = {ref[0]:.6e})")
        assert abs(Em - ref[0]) <= mixed_tol(ref[0]), (prec, Em, ref)


# ------------------------------------------------------------ runtime hooks
def test_shuffled_work_order_is_bitwise_neutral(ccsdt_mod, monkeypatch):
    """Any order of the work list (CCSDT_SHUFFLE seeds a shuffle of the
    triples inside each tile plan, so chunks hold other triples) gives the
    same energies bit for bit: every triple is computed on its own and the
    sums run in a fixed order."""
    probs = [synth.make_problem(6, 70, seed=42), synth.make_problem(5, 41, seed=43)]
    devs = [synth.to_device(p) for p in probs]
    c0 = ccsdt_mod.Context()
    ref = {prec: c0.energy(devs[0], prec) for prec in ("fp64", "fp32", "bf16x3")}
    ref_b = c0.energy_batched(devs, "fp32")
    ref_t = c0.triple_energies(devs[0], [(0, 1, 2), (2, 2, 5), (1, 3, 4)], "fp64")
    c0.close()
    for seed in ("1", "987654321"):
        monkeypatch.setenv("CCSDT_SHUFFLE", seed)
        c1 = ccsdt_mod.Context()
        say(f"shuffled work list, seed {seed}")
        for prec, r in ref.items():
            assert c1.energy(devs[0], prec) == r, prec
        assert c1.energy_batched(devs, "fp32") == ref_b
        assert c1.triple_energies(devs[0], [(0, 1, 2), (2, 2, 5), (1, 3, 4)], "fp64") == ref_t
        c1.close()


def test_injected_launch_failures(ccsdt_mod, monkeypatch):
    """CCSDT_FAIL_AT=<kernel class> makes the next launch of that class
    return CCSDT_EHIP (nothing is launched on the GPU); the call reports it,
    leaves its outputs alone, and a context made without the hook works."""
    import ctypes
    p = synth.make_problem(4, 30, seed=44)
    d = synth.to_device(p)
    for cls in ("pack", "contract", "energy", "reduce"):
        monkeypatch.setenv("CCSDT_FAIL_AT", cls)
        c = ccsdt_mod.Context()
        say(f"injected failure at {cls}")
        lib = ccsdt_mod.load_library()
        s = ccsdt_mod.make_problem_struct(d)
        out = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
        rc = lib.ccsdt_energy(c._h, ctypes.byref(s), 0, None, out)
        assert rc == -3 and cls in lib.ccsdt_last_error().decode()
        assert list(out) == [1.0, 2.0, 3.0]
        with pytest.raises(ccsdt_mod.CcsdtError) as e:
            c.energy_batched([d, d], "fp32")
        assert e.value.status == -3
        c.close()
    monkeypatch.delenv("CCSDT_FAIL_AT")
    torch.cuda.synchronize()
    c = ccsdt_mod.Context()
    ref = oracle.triples_energy(*_args(p))
    assert abs(c.energy(d, "fp64")[0] - ref[0]) <= 1e-10 * abs(ref[1])
    c.close()
