"""CPU oracle for the closed-shell CCSD(T) triples energy E(T) = E[4] + E[5].

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The library's product path must
never call it.  It shares no code with the HIP path.

Plain float64 numpy, written from Sec. 2.2 of the paper (Eriksen,
arXiv:1609.08094):

* eq. piecuch_4th_and_5th_order: E[4] = sum t~ t eps, E[5] = sum z~ t eps over
  all ordered occupied (i,j,k) and virtual (a,b,c);
* eq. analytical_triples_ampl: the connected triples amplitudes, built from a
  particle term (sum over a virtual d) and a hole term (sum over an occupied l),
  symmetrized by P^abc_ijk;
* eq. symm_operator: P sums the six simultaneous permutations of the index
  pairs (a,i), (b,j), (c,k);
* eq. piecuch_z_coefficients: the disconnected (t1) coefficients;
* eq. piecuch_tilde_quantity: x~ = 2 (2/3 x^abc - x^acb + 1/3 x^bca).

Readings where the text is ambiguous (each is pinned by a test):

* Sign of the denominator.  The text defines eps^abc_ijk "on par with" the
  positive virtual-minus-occupied difference of eq. e_orb_diff, which would
  make E[4] >= 0.  E[4] must be <= 0, so the energy is evaluated with
  D = e_i + e_j + e_k - e_a - e_b - e_c < 0.  With t = W / D, z = Z / D:
      E[4] = sum W~ W / D,     E[5] = sum Z~ W / D.
* Particle term.  The text writes sum_d t^ad_ij g_ckbd.  We use the
  (a,i) <-> (c,k) pair-swapped form sum_d (bd|ai) t^cd_kj, which P maps onto
  the same W because the swap is one of P's six permutations.
* Element reads (real orbitals, Mulliken notation): (bd|ai) = vvvo[b,d,a,i],
  (kc|jl) = ovoo[k,c,j,l], (jb|kc) = ovov[j,b,k,c], t^ab_ij = t2[i,j,a,b].
* Restricted summation (Sec. 3: restricted occupied loops; task count of eq.
  tasks_ccsdpt).  Summing the six orderings of a triple with i<j<k (three for
  a triple with two equal indices) and relabelling the virtual indices with
  the joint permutation symmetry of W, Z and D turns the tilde weights into
  their average over S3 conjugacy classes:
      e_ijk = m/3 sum_abc W_abc [4V_abc + V_bca + V_cab - 2V_acb - 2V_bac - 2V_cba] / D_abc
  with V = W + Z, m = 6 (all distinct), 3 (two equal); i=j=k gives exactly 0.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "x_piece", "w_tensor", "z_tensor", "d_tensor", "triple_literal",
    "triple_restricted", "triples_energy", "triple_list", "multiplicity",
]


def _perm(x: np.ndarray, src: str) -> np.ndarray:
    """Return Y[a,b,c] = x[<src>], e.g. src='bca' gives Y[a,b,c] = x[b,c,a]."""
    return np.einsum(src + "->abc", x)


def x_piece(i, j, k, t2, vvvo, ovoo):
    """Unsymmetrized connected piece (eq. analytical_triples_ampl, bracket):

        X^abc_ijk = sum_d (bd|ai) t^cd_kj - sum_l (kc|jl) t^ab_il

    Returned as an array X[a,b,c]."""
    # particle term: (bd|ai) = vvvo[b,d,a,i], t^cd_kj = t2[k,j,c,d]
    g = vvvo[:, :, :, i]                                   # [b,d,a]
    part = np.tensordot(g, t2[k, j], axes=([1], [1]))       # [b,a,c]
    part = _perm(part, "bac")                               # -> [a,b,c]
    # hole term: (kc|jl) = ovoo[k,c,j,l], t^ab_il = t2[i,l,a,b]
    h = ovoo[k, :, j, :]                                   # [c,l]
    hole = np.tensordot(t2[i], h, axes=([0], [1]))          # [a,b,c]
    return part - hole


def w_tensor(i, j, k, t2, vvvo, ovoo):
    """W^abc_ijk = P^abc_ijk X^abc_ijk (eq. symm_operator):
    X^abc_ijk + X^acb_ikj + X^bac_jik + X^bca_jki + X^cab_kij + X^cba_kji."""
    return (x_piece(i, j, k, t2, vvvo, ovoo)
            + _perm(x_piece(i, k, j, t2, vvvo, ovoo), "acb")
            + _perm(x_piece(j, i, k, t2, vvvo, ovoo), "bac")
            + _perm(x_piece(j, k, i, t2, vvvo, ovoo), "bca")
            + _perm(x_piece(k, i, j, t2, vvvo, ovoo), "cab")
            + _perm(x_piece(k, j, i, t2, vvvo, ovoo), "cba"))


def z_tensor(i, j, k, t1, ovov):
    """Numerator of eq. piecuch_z_coefficients:
    Z^abc_ijk = t^a_i (jb|kc) + t^b_j (ia|kc) + t^c_k (ia|jb)."""
    return (np.einsum("a,bc->abc", t1[i], ovov[j, :, k, :])
            + np.einsum("b,ac->abc", t1[j], ovov[i, :, k, :])
            + np.einsum("c,ab->abc", t1[k], ovov[i, :, j, :]))


def d_tensor(i, j, k, eps_o, eps_v):
    """D^abc_ijk = e_i + e_j + e_k - e_a - e_b - e_c (negative for a gapped
    canonical reference)."""
    ev = eps_v
    return (eps_o[i] + eps_o[j] + eps_o[k]
            - ev[:, None, None] - ev[None, :, None] - ev[None, None, :])


def _tilde(x):
    """eq. piecuch_tilde_quantity: 2 (2/3 x^abc - x^acb + 1/3 x^bca)."""
    return 2.0 * ((2.0 / 3.0) * x - _perm(x, "acb") + (1.0 / 3.0) * _perm(x, "bca"))


def triple_literal(i, j, k, eps_o, eps_v, t1, t2, vvvo, ovoo, ovov):
    """(E[4], E[5]) contribution of one ORDERED occupied triple, as printed
    (eq. piecuch_4th_and_5th_order), with the negative denominator D."""
    W = w_tensor(i, j, k, t2, vvvo, ovoo)
    Z = z_tensor(i, j, k, t1, ovov)
    D = d_tensor(i, j, k, eps_o, eps_v)
    e4 = math.fsum((_tilde(W) * W / D).ravel())
    e5 = math.fsum((_tilde(Z) * W / D).ravel())
    return e4, e5


def multiplicity(i, j, k) -> int:
    """Number of ordered triples an i<=j<=k triple stands for (0 for i=j=k,
    whose contribution vanishes identically)."""
    if i == j == k:
        return 0
    if i == j or j == k or i == k:
        return 3
    return 6


def triple_list(nocc: int):
    """Restricted occupied triples i<=j<=k with non-zero multiplicity."""
    return [(i, j, k) for i in range(nocc) for j in range(i, nocc) for k in range(j, nocc)
            if multiplicity(i, j, k)]


def _bracket(V):
    return (4.0 * V + _perm(V, "bca") + _perm(V, "cab")
            - 2.0 * _perm(V, "acb") - 2.0 * _perm(V, "bac") - 2.0 * _perm(V, "cba"))


def triple_restricted(i, j, k, eps_o, eps_v, t1, t2, vvvo, ovoo, ovov):
    """(e, e4, e5) of one restricted triple i<=j<=k including its multiplicity:
        e = m/3 sum_abc W [4V + V_bca + V_cab - 2V_acb - 2V_bac - 2V_cba] / D."""
    m = multiplicity(i, j, k)
    if m == 0:
        return 0.0, 0.0, 0.0
    W = w_tensor(i, j, k, t2, vvvo, ovoo)
    Z = z_tensor(i, j, k, t1, ovov)
    D = d_tensor(i, j, k, eps_o, eps_v)
    e4 = (m / 3.0) * math.fsum((W * _bracket(W) / D).ravel())
    e5 = (m / 3.0) * math.fsum((W * _bracket(Z) / D).ravel())
    return e4 + e5, e4, e5


def triples_energy(eps_o, eps_v, t1, t2, vvvo, ovoo, ovov, mode: str = "restricted",
                   triples=None):
    """E(T), E[4], E[5].

    mode='literal'    : all o^3 ordered triples, eq. piecuch_4th_and_5th_order as printed.
    mode='restricted' : i<=j<=k with multiplicities (or the given ``triples``).
    Per-triple partials are summed with math.fsum."""
    o = eps_o.shape[0]
    if mode == "literal":
        e4s, e5s = [], []
        for i in range(o):
            for j in range(o):
                for k in range(o):
                    a, b = triple_literal(i, j, k, eps_o, eps_v, t1, t2, vvvo, ovoo, ovov)
                    e4s.append(a)
                    e5s.append(b)
        e4, e5 = math.fsum(e4s), math.fsum(e5s)
        return e4 + e5, e4, e5
    if mode != "restricted":
        raise ValueError(mode)
    trip = triple_list(o) if triples is None else triples
    e4s, e5s = [], []
    for (i, j, k) in trip:
        _, a, b = triple_restricted(i, j, k, eps_o, eps_v, t1, t2, vvvo, ovoo, ovov)
        e4s.append(a)
        e5s.append(b)
    e4, e5 = math.fsum(e4s), math.fsum(e5s)
    return e4 + e5, e4, e5


def problem_energy(prob: dict, mode: str = "restricted"):
    """Convenience wrapper over a problem dict with the input arrays."""
    return triples_energy(prob["eps_o"], prob["eps_v"], prob["t1"], prob["t2"],
                          prob["vvvo"], prob["ovoo"], prob["ovov"], mode=mode)
