"""Closed-shell CCSD(T) perturbative-triples energy on MI355X (gfx950).

The compute path lives in the HIP library ``libccsdt.so`` (C ABI declared in
``include/ccsdt.h``); ``paper_1609_08094_amd.ccsdt`` is the thin ctypes
binding and ``paper_1609_08094_amd.synth`` the seeded input generator.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["ccsdt", "synth"]
