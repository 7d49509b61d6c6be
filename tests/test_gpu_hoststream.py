"""vvvo in page-locked host memory, streamed through the device staging
buffers (the paper's host-staged integral tiles, Sec. 3), against the same
problem with vvvo on the device and against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1609_08094_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ccsdt_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08094_amd import ccsdt
    ccsdt.load_library()
    return ccsdt


def say(msg):
    print(msg, flush=True)


def pinned(t):
    h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    h.copy_(t)
    return h


def host_problem(d):
    p = dict(d)
    p["vvvo"] = pinned(d["vvvo"].cpu())
    return p


def _call(ccsdt_mod, ctx, p, prec):
    return ctx.energy(p, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_host_vvvo_matches_device_vvvo(ccsdt_mod, prec, monkeypatch):
    p = synth.make_problem(5, 70, seed=600)
    d = synth.to_device(p)
    h = host_problem(d)
    # staging for three rows y per buffer: 24 chunks, the last one ragged
    monkeypatch.setenv("CCSDT_STAGE_BYTES", str(2 * 3 * 70 * 70 * 5 * 8))
    ctx = ccsdt_mod.Context()
    say(f"host-streamed vvvo {prec}")
    a = ctx.energy(d, prec)
    b = _call(ccsdt_mod, ctx, h, prec)
    assert a == b
    if prec == "fp64":
        ref = oracle.triples_energy(p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["vvvo"], p["ovoo"], p["ovov"])
        assert abs(b[0] - ref[0]) <= 1e-10 * abs(ref[1])
    ctx.close()


def test_host_vvvo_single_chunk_and_repeat(ccsdt_mod):
    p = synth.make_problem(4, 45, seed=601)
    d = synth.to_device(p)
    h = host_problem(d)
    ctx = ccsdt_mod.Context()
    say("host-streamed vvvo, default staging, twice")
    a = ctx.energy(d, "fp64")
    b = _call(ccsdt_mod, ctx, h, "fp64")
    c = _call(ccsdt_mod, ctx, h, "fp64")
    assert a == b == c
    ctx.close()


def test_pageable_host_vvvo_is_rejected(ccsdt_mod):
    p = synth.make_problem(3, 10, seed=602)
    d = synth.to_device(p)
    bad = dict(d)
    bad["vvvo"] = torch.from_numpy(p["vvvo"])          # pageable host memory
    ctx = ccsdt_mod.Context()
    say("pageable vvvo")
    with pytest.raises(ValueError):                     # the binding refuses it
        ctx.energy(bad, "fp64")
    import ctypes
    st = ccsdt_mod.make_problem_struct(d)
    st.vvvo = ctypes.c_void_p(p["vvvo"].ctypes.data)    # the C ABI refuses it too
    out = (ctypes.c_double * 3)()
    assert ccsdt_mod.load_library().ccsdt_energy(ctx._h, ctypes.byref(st), 0, None, out) == -1
    assert "pinned" in ccsdt_mod.load_library().ccsdt_last_error().decode()
    ctx.close()


def test_batched_mix_of_host_and_device_vvvo(ccsdt_mod):
    """A batch whose members hold vvvo on the device or in pinned host memory
    runs eagerly (no captured graph) and gives each member's single-problem
    energy bit for bit."""
    probs = [synth.make_problem(o, v, seed=610 + n) for n, (o, v) in enumerate([(3, 33), (4, 50), (5, 21)])]
    devs = [synth.to_device(p) for p in probs]
    mixed = [devs[0], host_problem(devs[1]), devs[2]]
    ctx = ccsdt_mod.Context()
    say("batch with one host-resident vvvo")
    got = ctx.energy_batched(mixed, "fp32")
    assert ctx.graph_stats() == (0, 0)
    for d, g in zip(devs, got):
        assert g == ctx.energy(d, "fp32")
    ctx.close()


def test_host_vvvo_per_triple_energies(ccsdt_mod):
    p = synth.make_problem(5, 40, seed=615)
    d = synth.to_device(p)
    h = host_problem(d)
    trips = [(0, 1, 2), (1, 1, 4), (2, 3, 3), (0, 0, 0), (1, 2, 4)]
    ctx = ccsdt_mod.Context()
    say("per-triple energies with host-resident vvvo")
    assert ctx.triple_energies(h, trips, "bf16x3") == ctx.triple_energies(d, trips, "bf16x3")
    ctx.close()
