"""CPU oracle for the closed-shell RI-MP2 correlation energy.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the library never does, and the
two share no code.

Paper Sec. 2.1:
* eq. mp2_energy: E_MP2 = - sum_ab sum_ij g_aibj (2 g_aibj - g_ajbi) / eps^ab_ij,
* eq. e_orb_diff: eps^ab_ij = eps_a + eps_b - (eps_i + eps_j)  (> 0),
* eq. eri_sym_decomp: g_aibj = sum_gamma C^gamma_ai C^gamma_bj, with the
  fitting coefficients C of eq. fitting_coef given as input.
Layout: c_ov[i][a][gamma] = C^gamma_ai (o x v x naux, gamma fastest), real
orbitals, so g_aibj = (ai|bj) = (ia|jb).

Two forms:
* ``rimp2_energy``: the definition, one matrix product for all g and the sum
  over every ordered (i, j);
* ``rimp2_pair_energy``: e_ij for one ordered pair (the quantity the GPU
  kernel forms per pair); e_ji = e_ij by swapping a and b, so
  E = sum_i e_ii + 2 sum_{i<j} e_ij.

Pins (tests/test_oracle_rimp2.py): the textbook spin-orbital MP2 sum over a
full ERI tensor (independent route), a one-orbital closed form, homogeneity
and shift invariance, relabelling invariance.
"""
from __future__ import annotations

import numpy as np


def g_ovov(c_ov: np.ndarray) -> np.ndarray:
    """g[i,a,j,b] = sum_gamma C^gamma_ai C^gamma_bj = (ia|jb)."""
    o, v, naux = c_ov.shape
    m = c_ov.reshape(o * v, naux)
    return (m @ m.T).reshape(o, v, o, v)


def rimp2_energy(eps_o: np.ndarray, eps_v: np.ndarray, c_ov: np.ndarray) -> float:
    """E_MP2 of eq. mp2_energy with the integrals of eq. eri_sym_decomp."""
    g = g_ovov(c_ov)                                       # g_aibj at [i,a,j,b]
    g_ex = g.transpose(2, 1, 0, 3)                         # g_ajbi at [i,a,j,b]
    den = (eps_v[None, :, None, None] + eps_v[None, None, None, :]
           - eps_o[:, None, None, None] - eps_o[None, None, :, None])
    return float(-np.sum(g * (2.0 * g - g_ex) / den))


def rimp2_pair_energy(i: int, j: int, eps_o, eps_v, c_ov) -> float:
    """e_ij = - sum_ab g_aibj (2 g_aibj - g_ajbi) / eps^ab_ij for one ordered pair."""
    gij = c_ov[i] @ c_ov[j].T                              # [a,b] = g_aibj
    gji = c_ov[j] @ c_ov[i].T                              # [a,b] = g_ajbi
    den = eps_v[:, None] + eps_v[None, :] - eps_o[i] - eps_o[j]
    return float(-np.sum(gij * (2.0 * gij - gji) / den))


def rimp2_energy_pairs(eps_o, eps_v, c_ov) -> float:
    """E_MP2 as sum_i e_ii + 2 sum_{i<j} e_ij (restricted pair loop)."""
    o = eps_o.shape[0]
    e = 0.0
    for i in range(o):
        for j in range(i, o):
            e += (1.0 if i == j else 2.0) * rimp2_pair_energy(i, j, eps_o, eps_v, c_ov)
    return e


def spin_orbital_mp2(eri: np.ndarray, eps_o: np.ndarray, eps_v: np.ndarray) -> float:
    """Textbook spin-orbital MP2, E = 1/4 sum_ijab |<ij||ab>|^2 / (f_i + f_j - f_a - f_b),
    from the full spatial ERI tensor eri[p,q,r,s] = (pq|rs) (occupied first);
    spin orbital 2P + s, <pq|rs> = (PR|QS) d(sp,sr) d(sq,ss)."""
    o, v = eps_o.shape[0], eps_v.shape[0]
    n = o + v
    so = np.arange(2 * n) // 2
    sp = np.arange(2 * n) % 2
    same = (sp[:, None] == sp[None, :]).astype(float)
    g = eri[np.ix_(so, so, so, so)]
    phys = g.transpose(0, 2, 1, 3) * same[:, None, :, None] * same[None, :, None, :]
    asym = phys - phys.transpose(0, 1, 3, 2)
    no = 2 * o
    f = np.concatenate([np.repeat(eps_o, 2), np.repeat(eps_v, 2)])
    oo, vv = slice(0, no), slice(no, 2 * n)
    a = asym[oo, oo, vv, vv]
    den = f[oo][:, None, None, None] + f[oo][None, :, None, None] - f[vv][None, None, :, None] - f[vv][None, None, None, :]
    return float(0.25 * np.sum(a * a / den))
