"""Thin ctypes binding over libccsdt.so (C ABI in include/ccsdt.h).

Argument marshalling only: every step of the (T) computation runs in the
library's HIP kernels.  Inputs are contiguous float64 torch tensors on the HIP
device; results come back as Python floats.  If the library is missing the
binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libccsdt.so")

FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
STATUS = {0: "CCSDT_OK", -1: "CCSDT_EINVAL", -2: "CCSDT_ENOMEM", -3: "CCSDT_EHIP",
          -4: "CCSDT_EUNSUPPORTED", -5: "CCSDT_EDENOM"}
KERNEL_CLASSES = {"pack": 0, "contract": 1, "energy": 2, "reduce": 3, "assemble": 4, "mp2_gemm": 5,
                  "mp2_energy": 6}
FIELDS = ("eps_o", "eps_v", "t1", "t2", "vvvo", "ovoo", "ovov")
EXPORTS = ("ccsdt_context_create", "ccsdt_context_destroy", "ccsdt_energy", "ccsdt_triples_energy",
           "ccsdt_triple_energies", "ccsdt_debug_w", "ccsdt_energy_batched", "ccsdt_profile_enable",
           "ccsdt_profile_get", "ccsdt_profile_reset", "ccsdt_flops", "ccsdt_last_error", "ccsdt_autotune",
           "ccsdt_plan_get", "ccsdt_plan_set", "ccsdt_graph_stats", "ccsdt_energy_df",
           "ccsdt_triple_energies_df", "ccsdt_rimp2_energy", "ccsdt_rimp2_pair_energies", "ccsdt_rimp2_flops",
           "ccsdt_energy_noalloc")
NOALLOC_SCRATCH_BYTES = 256 << 20
DF_FIELDS = ("eps_o", "eps_v", "t1", "t2", "bvv", "bvo", "ovoo", "ovov")
NTILE_CFG = 27


class CcsdtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int), ("nvirt", ctypes.c_int)] + \
               [(f, ctypes.c_void_p) for f in FIELDS]


class ProblemDF(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int), ("nvirt", ctypes.c_int), ("naux", ctypes.c_int)] + \
               [(f, ctypes.c_void_p) for f in DF_FIELDS]


class MP2Problem(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int), ("nvirt", ctypes.c_int), ("naux", ctypes.c_int),
                ("eps_o", ctypes.c_void_p), ("eps_v", ctypes.c_void_p), ("c_ov", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libccsdt.so and declare its signatures (raises if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1609_08094_amd.build`")
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER(Problem)
    lib.ccsdt_context_create.argtypes = [ctypes.POINTER(vp)]
    lib.ccsdt_context_destroy.argtypes = [vp]
    lib.ccsdt_energy.argtypes = [vp, P, ip, vp, dp]
    lib.ccsdt_triples_energy.argtypes = [ip, ip] + [vp] * 7 + [ip, vp, dp]
    lib.ccsdt_energy_noalloc.argtypes = [P, ip, vp, vp]
    lib.ccsdt_triple_energies.argtypes = [vp, P, ip, ip, ctypes.POINTER(ctypes.c_int), vp, dp]
    lib.ccsdt_debug_w.argtypes = [vp, P, ip, ip, ip, ip, vp, dp]
    lib.ccsdt_energy_batched.argtypes = [vp, ip, P, ip, vp, dp]
    lib.ccsdt_profile_enable.argtypes = [vp, ip]
    lib.ccsdt_profile_get.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int64), dp]
    lib.ccsdt_profile_reset.argtypes = [vp]
    PD = ctypes.POINTER(ProblemDF)
    lib.ccsdt_energy_df.argtypes = [vp, PD, ip, vp, dp]
    lib.ccsdt_triple_energies_df.argtypes = [vp, PD, ip, ip, ctypes.POINTER(ctypes.c_int), vp, dp]
    PM = ctypes.POINTER(MP2Problem)
    lib.ccsdt_rimp2_energy.argtypes = [vp, PM, ip, vp, dp]
    lib.ccsdt_rimp2_pair_energies.argtypes = [vp, PM, ip, ip, ctypes.POINTER(ctypes.c_int), vp, dp]
    lib.ccsdt_rimp2_flops.argtypes = [ip, ip, ip]
    lib.ccsdt_rimp2_flops.restype = ctypes.c_double
    lib.ccsdt_autotune.argtypes = [vp, P, ip, vp, ctypes.POINTER(ip)]
    lib.ccsdt_plan_get.argtypes = [vp, ip, ip, ctypes.POINTER(ip)]
    lib.ccsdt_plan_set.argtypes = [vp, ip, ip, ip]
    lib.ccsdt_graph_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.ccsdt_flops.argtypes = [ip, ip]
    lib.ccsdt_flops.restype = ctypes.c_double
    lib.ccsdt_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("ccsdt_flops", "ccsdt_last_error", "ccsdt_rimp2_flops"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise CcsdtError(rc, load_library().ccsdt_last_error().decode())


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# Element count of every input block as a function of (o, v, naux), from the
# layouts of include/ccsdt.h.  The library receives bare pointers and cannot
# check sizes itself; a block shorter than its layout would be read out of
# bounds, so the binding refuses it.
_NUMEL = {
    "eps_o": lambda o, v, q: o,
    "eps_v": lambda o, v, q: v,
    "t1": lambda o, v, q: o * v,
    "t2": lambda o, v, q: o * o * v * v,
    "vvvo": lambda o, v, q: v * v * v * o,
    "ovoo": lambda o, v, q: o * v * o * o,
    "ovov": lambda o, v, q: o * v * o * v,
    "bvv": lambda o, v, q: v * v * q,
    "bvo": lambda o, v, q: v * o * q,
    "c_ov": lambda o, v, q: o * v * q,
}


def _dev_ptrs(prob: dict, fields, host_ok=()) -> list:
    import torch
    o, v = int(prob["nocc"]), int(prob["nvirt"])
    q = int(prob.get("naux", 0))
    for f in fields:
        t = prob[f]
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{f} must be a contiguous float64 tensor")
        want = _NUMEL[f](o, v, q)
        if t.numel() != want:
            raise ValueError(f"{f} has {t.numel()} elements; nocc={o}, nvirt={v}"
                             + (f", naux={q}" if f in ("bvv", "bvo", "c_ov") else "") + f" need {want}")
    vals = []
    for f in fields:
        t = prob[f]
        if not t.is_cuda and not (f in host_ok and t.is_pinned()):
            raise ValueError(f"{f} must be on the HIP device" + (" or in pinned host memory" if f in host_ok else ""))
        vals.append(ctypes.c_void_p(t.data_ptr()))
    return vals


def make_problem_struct(prob: dict) -> Problem:
    """Problem struct from a dict of contiguous float64 tensors on the device
    (vvvo may also be a pinned host tensor, which the library streams)."""
    return Problem(int(prob["nocc"]), int(prob["nvirt"]), *_dev_ptrs(prob, FIELDS, host_ok=("vvvo",)))


def make_problem_df_struct(prob: dict) -> ProblemDF:
    """ProblemDF struct (factors bvv[a][b][Q], bvo[c][i][Q]) from device tensors."""
    return ProblemDF(int(prob["nocc"]), int(prob["nvirt"]), int(prob["naux"]), *_dev_ptrs(prob, DF_FIELDS))


def flops(nocc: int, nvirt: int) -> float:
    return load_library().ccsdt_flops(nocc, nvirt)


def rimp2_flops(nocc: int, nvirt: int, naux: int) -> float:
    return load_library().ccsdt_rimp2_flops(nocc, nvirt, naux)


def make_mp2_struct(prob: dict) -> MP2Problem:
    """MP2Problem struct (c_ov[i][a][Q]) from device tensors."""
    vals = _dev_ptrs(prob, ("eps_o", "eps_v", "c_ov"))
    return MP2Problem(int(prob["nocc"]), int(prob["nvirt"]), int(prob["naux"]), *vals)


class Context:
    """Owns a ccsdt_context (device workspace and plan caches)."""

    def __init__(self):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.ccsdt_context_create(ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().ccsdt_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- energies -----------------------------------------------------------
    def energy(self, prob: dict, precision="fp64", stream=None):
        """(E, E4, E5) of one problem."""
        p = make_problem_struct(prob)
        out = (ctypes.c_double * 3)()
        _check(load_library().ccsdt_energy(self._h, ctypes.byref(p), _prec(precision), _stream(stream), out))
        return out[0], out[1], out[2]

    def energy_df(self, prob: dict, precision="fp64", stream=None):
        """(E, E4, E5) of a density-fitted problem (factors instead of vvvo)."""
        p = make_problem_df_struct(prob)
        out = (ctypes.c_double * 3)()
        _check(load_library().ccsdt_energy_df(self._h, ctypes.byref(p), _prec(precision), _stream(stream), out))
        return out[0], out[1], out[2]

    def triple_energies_df(self, prob: dict, triples, precision="fp64", stream=None):
        """[(e, e4, e5)] per restricted triple of a density-fitted problem."""
        flat = [int(x) for t in triples for x in t]
        ijk = (ctypes.c_int * len(flat))(*flat)
        out = (ctypes.c_double * (3 * len(triples)))()
        p = make_problem_df_struct(prob)
        _check(load_library().ccsdt_triple_energies_df(self._h, ctypes.byref(p), _prec(precision), len(triples),
                                                        ijk, _stream(stream), out))
        return [(out[3 * n], out[3 * n + 1], out[3 * n + 2]) for n in range(len(triples))]

    def rimp2_energy(self, prob: dict, precision="fp32", stream=None) -> float:
        """RI-MP2 correlation energy of {nocc, nvirt, naux, eps_o, eps_v, c_ov}."""
        p = make_mp2_struct(prob)
        e = ctypes.c_double()
        _check(load_library().ccsdt_rimp2_energy(self._h, ctypes.byref(p), _prec(precision), _stream(stream),
                                                  ctypes.byref(e)))
        return e.value

    def rimp2_pair_energies(self, prob: dict, pairs, precision="fp32", stream=None):
        """[e_ij] for pairs (i, j), i <= j."""
        flat = [int(x) for t in pairs for x in t]
        ij = (ctypes.c_int * len(flat))(*flat)
        out = (ctypes.c_double * len(pairs))()
        p = make_mp2_struct(prob)
        _check(load_library().ccsdt_rimp2_pair_energies(self._h, ctypes.byref(p), _prec(precision), len(pairs), ij,
                                                         _stream(stream), out))
        return list(out)

    def energy_batched(self, probs: list, precision="fp32", stream=None):
        """[(E, E4, E5)] for many problems in one submission."""
        arr = (Problem * len(probs))(*[make_problem_struct(p) for p in probs])
        out = (ctypes.c_double * (3 * len(probs)))()
        _check(load_library().ccsdt_energy_batched(self._h, len(probs), arr, _prec(precision),
                                                    _stream(stream), out))
        return [(out[3 * n], out[3 * n + 1], out[3 * n + 2]) for n in range(len(probs))]

    def triple_energies(self, prob: dict, triples, precision="fp64", stream=None):
        """[(e, e4, e5)] per restricted triple (i<=j<=k), multiplicity included."""
        flat = [int(x) for t in triples for x in t]
        ijk = (ctypes.c_int * len(flat))(*flat)
        out = (ctypes.c_double * (3 * len(triples)))()
        p = make_problem_struct(prob)
        _check(load_library().ccsdt_triple_energies(self._h, ctypes.byref(p), _prec(precision), len(triples),
                                                     ijk, _stream(stream), out))
        return [(out[3 * n], out[3 * n + 1], out[3 * n + 2]) for n in range(len(triples))]

    def debug_w(self, prob: dict, i: int, j: int, k: int, precision="fp64", stream=None):
        """W[a,b,c] of one triple as a float64 numpy array."""
        import numpy as np
        v = int(prob["nvirt"])
        w = np.empty((v, v, v), dtype=np.float64)
        p = make_problem_struct(prob)
        _check(load_library().ccsdt_debug_w(self._h, ctypes.byref(p), _prec(precision), i, j, k,
                                             _stream(stream), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return w

    # -- plans and graphs ------------------------------------------------------
    def autotune(self, prob: dict, precision="fp64", stream=None) -> int:
        """Time every tile configuration on a few triples; keep the fastest."""
        p = make_problem_struct(prob)
        cfg = ctypes.c_int()
        _check(load_library().ccsdt_autotune(self._h, ctypes.byref(p), _prec(precision), _stream(stream),
                                              ctypes.byref(cfg)))
        return cfg.value

    def plan_get(self, precision, nvirt: int) -> int:
        cfg = ctypes.c_int()
        _check(load_library().ccsdt_plan_get(self._h, _prec(precision), int(nvirt), ctypes.byref(cfg)))
        return cfg.value

    def plan_set(self, precision, nvirt: int, cfg: int):
        _check(load_library().ccsdt_plan_set(self._h, _prec(precision), int(nvirt), int(cfg)))

    def graph_stats(self) -> tuple[int, int]:
        c, r = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().ccsdt_graph_stats(self._h, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    # -- profiling ----------------------------------------------------------
    def profile(self, on: bool = True):
        _check(load_library().ccsdt_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self):
        _check(load_library().ccsdt_profile_reset(self._h))

    def profile_get(self, cls) -> tuple[int, float]:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        c = KERNEL_CLASSES[cls] if isinstance(cls, str) else int(cls)
        _check(load_library().ccsdt_profile_get(self._h, c, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


def triples_energy(prob: dict, precision="fp64", stream=None) -> float:
    """One-shot E(T) through ccsdt_triples_energy."""
    lib = load_library()
    vals = make_problem_struct(prob)
    e = ctypes.c_double()
    _check(lib.ccsdt_triples_energy(vals.nocc, vals.nvirt, *[getattr(vals, f) for f in FIELDS],
                                    _prec(precision), _stream(stream), ctypes.byref(e)))
    return e.value


def energy_noalloc(prob: dict, precision="fp64", out=None, stream=None):
    """Enqueue E(T) through ccsdt_energy_noalloc (no device allocation, no
    synchronization); `out` is a float64 device tensor of 3 elements (made
    here if None) that holds (E, E4, E5) once the stream has run the work.
    Returns `out`."""
    import torch
    p = make_problem_struct(prob)
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=prob["eps_o"].device)
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
            and out.is_contiguous() and out.numel() >= 3):
        raise ValueError("out must be a contiguous float64 device tensor of at least 3 elements")
    _check(load_library().ccsdt_energy_noalloc(ctypes.byref(p), _prec(precision), _stream(stream),
                                               ctypes.c_void_p(out.data_ptr())))
    return out
