"""The allocation-free entry point (ccsdt_energy_noalloc) through the C ABI,
against the context entry point (ccsdt_energy) on the same inputs: FP64 at
1e-10 relative, FP32 and BF16X3 at 1e-6 max(1, |E|), on two calls in a row,
the second with a smaller problem, so that the second call runs on the
contents the first one left in the shared workspace.  Also the size limit
(rejected on the host before any device work) and the device-side
denominator check (NaN results)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1609_08094_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08094_amd import ccsdt
    ccsdt.load_library()
    return ccsdt


def _noalloc(mod, d, prec):
    out = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    mod.energy_noalloc(d, prec, out=out)
    torch.cuda.synchronize()
    return tuple(float(x) for x in out.cpu())


def _close(a, b, prec):
    tol = 1e-10 * abs(b[1]) if prec == "fp64" else 1e-6 * max(1.0, abs(b[0]))
    return all(abs(x - y) <= tol for x, y in zip(a, b))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_context_call_twice(mod, prec):
    # first a problem that spans several tiles and, with the workspace it
    # needs, many chunks of the W area (one triple per chunk in FP64), then a
    # smaller one (fewer triples, smaller v, the other tile plan)
    shapes = [(9, 130, 71), (5, 45, 72)]
    ctx = mod.Context()
    try:
        for o, v, seed in shapes:
            p = synth.make_problem(o, v, seed=seed)
            d = synth.to_device(p)
            say(f"noalloc {prec} o={o} v={v}")
            got = _noalloc(mod, d, prec)
            ref = ctx.energy(d, prec)
            say(f"  noalloc {got[0]!r} context {ref[0]!r}")
            assert _close(got, ref, prec), (o, v, prec, got, ref)
            if prec == "fp64":
                o_ref = oracle.triples_energy(p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["vvvo"], p["ovoo"],
                                              p["ovov"])
                assert abs(got[0] - o_ref[0]) <= 1e-10 * abs(o_ref[1])
    finally:
        ctx.close()


def test_noalloc_degenerate_and_rejected(mod):
    lib = mod.load_library()
    # o = 1: no triple at all, E = 0 exactly
    d = synth.to_device(synth.make_problem(1, 20, seed=73))
    say("noalloc o=1")
    assert _noalloc(mod, d, "fp64") == (0.0, 0.0, 0.0)
    # a denominator that is not negative: NaN on the device
    d = synth.to_device(synth.make_problem(4, 20, seed=74))
    bad = dict(d, eps_o=d["eps_o"] + 10.0)
    say("noalloc positive gap check")
    got = _noalloc(mod, bad, "fp32")
    assert all(np.isnan(x) for x in got)
    say("noalloc after the failed check")
    ctx = mod.Context()
    ref = ctx.energy(d, "fp32")
    ctx.close()
    assert _close(_noalloc(mod, d, "fp32"), ref, "fp32")
    # too large for the static workspace: rejected before any device work
    big = synth.to_device(synth.make_problem(4, 20, seed=75))
    s = mod.make_problem_struct(big)
    s.nvirt = 2000     # sizes only: the host rejects it from nocc and nvirt
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    say("noalloc size limit")
    rc = lib.ccsdt_energy_noalloc(ctypes.byref(s), 0, None, ctypes.c_void_p(out.data_ptr()))
    assert rc == -1 and "workspace" in lib.ccsdt_last_error().decode()
    torch.cuda.synchronize()
    assert out.abs().sum().item() == 0.0
