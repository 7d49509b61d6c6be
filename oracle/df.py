"""Density-fitted (vv|vo) block for the (T) oracle (test infrastructure).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the library never does.

Paper Sec. 2.1, eq. eri_sym_decomp: a four-index integral is the sum over
the auxiliary index of a product of two three-index factors,
    (ab|ci) = sum_Q B^Q_ab B^Q_ci .
The factors are taken with the auxiliary index fastest, bvv[a][b][Q] and
bvo[c][i][Q].  The energy of a density-fitted problem is the (T) energy of
triples.py evaluated on the assembled block.
"""
from __future__ import annotations

import numpy as np

from .triples import triples_energy, triple_restricted


def vvvo_from_df(bvv: np.ndarray, bvo: np.ndarray) -> np.ndarray:
    """vvvo[a][b][c][i] = sum_Q bvv[a][b][Q] bvo[c][i][Q] (one matrix product)."""
    v, v2, naux = bvv.shape
    v3, o, naux2 = bvo.shape
    assert v == v2 == v3 and naux == naux2
    return (bvv.reshape(v * v, naux) @ bvo.reshape(v * o, naux).T).reshape(v, v, v, o)


def triples_energy_df(eps_o, eps_v, t1, t2, bvv, bvo, ovoo, ovov, mode: str = "restricted"):
    """(E, E4, E5) of a density-fitted problem."""
    return triples_energy(eps_o, eps_v, t1, t2, vvvo_from_df(bvv, bvo), ovoo, ovov, mode=mode)


def triple_restricted_df(i, j, k, eps_o, eps_v, t1, t2, bvv, bvo, ovoo, ovov):
    """Per-triple (e, e4, e5) of a density-fitted problem."""
    return triple_restricted(i, j, k, eps_o, eps_v, t1, t2, vvvo_from_df(bvv, bvo), ovoo, ovov)
