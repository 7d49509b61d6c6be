"""C-ABI library: loads, exports every declared symbol, host-only entry points.

No GPU compute is issued here: only calls that return before touching a
device (argument errors, the flop formula, the error string).
"""
import ctypes
import os
import re

import pytest

from paper_1609_08094_amd import ccsdt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccsdt.h")


def _lib():
    if not os.path.exists(ccsdt.LIB_PATH):
        from paper_1609_08094_amd import build
        build.build()
    return ccsdt.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccsdt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("ccsdt_triples_energy", "ccsdt_energy", "ccsdt_energy_batched", "ccsdt_triple_energies",
              "ccsdt_debug_w", "ccsdt_context_create", "ccsdt_context_destroy", "ccsdt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(ccsdt.EXPORTS) | {"ccsdt_flops"}


def test_flops_formula():
    lib = _lib()
    for o, v in [(6, 30), (20, 200), (40, 600)]:
        assert lib.ccsdt_flops(o, v) == pytest.approx((o ** 3 - o) * (2 * v ** 4 + 2 * o * v ** 3), rel=1e-15)


def test_null_arguments_are_rejected_without_a_device():
    lib = _lib()
    assert lib.ccsdt_context_create(None) == -1
    assert "null" in lib.ccsdt_last_error().decode()
    assert lib.ccsdt_context_destroy(None) == -1
    out = (ctypes.c_double * 3)()
    assert lib.ccsdt_energy(None, None, 0, None, out) == -1
    assert lib.ccsdt_triples_energy(6, 30, *([None] * 7), 0, None, None) == -1
    assert lib.ccsdt_profile_get(None, 0, None, None) == -1


def test_plan_and_graph_entry_points_reject_null_context():
    lib = _lib()
    cfg = ctypes.c_int()
    assert lib.ccsdt_autotune(None, None, 0, None, ctypes.byref(cfg)) == -1
    assert lib.ccsdt_plan_get(None, 0, 100, ctypes.byref(cfg)) == -1
    assert lib.ccsdt_plan_set(None, 0, 100, 0) == -1
    c, r = ctypes.c_int64(), ctypes.c_int64()
    assert lib.ccsdt_graph_stats(None, ctypes.byref(c), ctypes.byref(r)) == -1
    assert "null" in lib.ccsdt_last_error().decode()


def _cpu_problem(o=3, v=5):
    import torch
    return dict(nocc=o, nvirt=v, eps_o=torch.zeros(o, dtype=torch.float64),
                eps_v=torch.zeros(v, dtype=torch.float64), t1=torch.zeros(o, v, dtype=torch.float64),
                t2=torch.zeros(o, o, v, v, dtype=torch.float64), vvvo=torch.zeros(v, v, v, o, dtype=torch.float64),
                ovoo=torch.zeros(o, v, o, o, dtype=torch.float64), ovov=torch.zeros(o, v, o, v, dtype=torch.float64))


@pytest.mark.parametrize("field", ["eps_o", "eps_v", "t1", "t2", "vvvo", "ovoo", "ovov"])
def test_binding_rejects_a_block_of_the_wrong_size(field):
    """A block whose element count disagrees with (nocc, nvirt) is refused by
    the binding before any pointer reaches the library (the library cannot
    see sizes and would read past the end)."""
    import torch
    p = _cpu_problem()
    p[field] = torch.zeros(p[field].numel() - 1, dtype=torch.float64)
    with pytest.raises(ValueError, match=field):
        ccsdt.make_problem_struct(p)


def test_binding_rejects_wrong_sizes_for_df_and_mp2():
    import torch
    p = _cpu_problem()
    p.update(naux=4, bvv=torch.zeros(5 * 5 * 4, dtype=torch.float64), bvo=torch.zeros(5 * 3 * 3, dtype=torch.float64))
    with pytest.raises(ValueError, match="bvo"):
        ccsdt.make_problem_df_struct(p)
    m = dict(nocc=3, nvirt=5, naux=4, eps_o=torch.zeros(3, dtype=torch.float64),
             eps_v=torch.zeros(5, dtype=torch.float64), c_ov=torch.zeros(3 * 5 * 5, dtype=torch.float64))
    with pytest.raises(ValueError, match="c_ov"):
        ccsdt.make_mp2_struct(m)


def test_binding_size_check_passes_correct_blocks_to_the_device_check():
    # correctly sized CPU tensors get past the size check and stop at the
    # device check
    with pytest.raises(ValueError, match="HIP device"):
        ccsdt.make_problem_struct(_cpu_problem())
