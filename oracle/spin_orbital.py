"""Spin-orbital brute-force (T) energy for tiny sizes.

TEST INFRASTRUCTURE: an independent check of the closed-shell oracle in
``oracle.triples``; never called by the library.

This is the textbook spin-orbital form of the (T) correction (as in Crawford
and Schaefer, Rev. Comput. Chem. 14 (2000), the CCSD(T) section), written out
with explicit six-index arrays; it shares no formula with the closed-shell
expressions of Sec. 2.2 of the paper, only the meaning of the inputs:

    D t(c)^abc_ijk = P(i/jk) P(a/bc) [ sum_e t^ae_jk <ei||bc> - sum_m t^bc_im <ma||jk> ]
    D t(d)^abc_ijk = P(i/jk) P(a/bc) t^a_i <jk||bc>
    P(i/jk) f(ijk) = f(ijk) - f(jik) - f(kji)
    E(T) = 1/36 sum_{ijkabc} t(c) D (t(c) + t(d)),  D = f_ii+f_jj+f_kk-f_aa-f_bb-f_cc
    E[4] = 1/36 sum t(c) D t(c),  E[5] = 1/36 sum t(c) D t(d)

Spin orbitals are (spatial P, spin s) with index 2P+s.  From the spatial
closed-shell quantities (real orbitals, Mulliken (pq|rs)):
    <pq|rs> = (PR|QS) d(sp,sr) d(sq,ss),   <pq||rs> = <pq|rs> - <pq|sr>
    t^a_i   = t^A_I d(sa,si)
    t^ab_ij = t^AB_IJ d(sa,si) d(sb,sj) - t^BA_IJ d(sb,si) d(sa,sj)
"""
from __future__ import annotations

import math

import numpy as np


def _spin_delta(n):
    s = np.arange(2 * n) % 2
    return (s[:, None] == s[None, :]).astype(float)


def spin_orbital_triples(eri, eps_o, eps_v, t1, t2):
    """E(T), E[4], E[5] from the full spatial ERI tensor eri[p,q,r,s] = (pq|rs)
    over n = o + v orbitals (occupied first), orbital energies, t1[I,A] and
    t2[I,J,A,B] = t^AB_IJ."""
    o = eps_o.shape[0]
    v = eps_v.shape[0]
    n = o + v
    # spin-orbital expansion: index 2P + s
    rep = lambda x: np.repeat(x, 2)
    so_of = np.arange(2 * n) // 2
    sp = np.arange(2 * n) % 2
    same = (sp[:, None] == sp[None, :]).astype(float)
    g = eri[np.ix_(so_of, so_of, so_of, so_of)]           # (PQ|RS) on spin indices
    # <pq|rs> = (pr|qs) d(sp,sr) d(sq,ss)
    phys = g.transpose(0, 2, 1, 3) * same[:, None, :, None] * same[None, :, None, :]
    asym = phys - phys.transpose(0, 1, 3, 2)               # <pq||rs>
    no, nv = 2 * o, 2 * v
    occ = slice(0, no)
    vir = slice(no, 2 * n)
    f = np.concatenate([rep(eps_o), rep(eps_v)])
    fo, fv = f[occ], f[vir]
    # amplitudes on spin orbitals
    so_o = np.arange(no) // 2
    so_v = np.arange(nv) // 2
    s_o = np.arange(no) % 2
    s_v = np.arange(nv) % 2
    d_ov = (s_o[:, None] == s_v[None, :]).astype(float)    # d(si, sa)
    T1 = t1[np.ix_(so_o, so_v)] * d_ov
    tt = t2[np.ix_(so_o, so_o, so_v, so_v)]                # t^AB_IJ on spin indices
    ttx = t2[np.ix_(so_o, so_o, so_v, so_v)].transpose(0, 1, 3, 2)  # t^BA_IJ at [i,j,a,b]
    dia = d_ov[:, None, :, None]                           # d(si,sa)
    djb = d_ov[None, :, None, :]                           # d(sj,sb)
    dib = d_ov[:, None, None, :]                           # d(si,sb)
    dja = d_ov[None, :, :, None]                           # d(sj,sa)
    T2 = tt * dia * djb - ttx * dib * dja
    # integral blocks
    vovv = asym[vir, occ, vir, vir]                        # <ei||bc> [e,i,b,c]
    ovoo = asym[occ, vir, occ, occ]                        # <ma||jk> [m,a,j,k]
    oovv = asym[occ, occ, vir, vir]                        # <jk||bc> [j,k,b,c]
    # unpermuted connected and disconnected pieces, index order ijkabc
    conn = (np.einsum("jkae,eibc->ijkabc", T2, vovv, optimize=True)
            - np.einsum("imbc,majk->ijkabc", T2, ovoo, optimize=True))
    disc = np.einsum("ia,jkbc->ijkabc", T1, oovv, optimize=True)

    def P_i_jk(x):
        return x - np.einsum("jikabc->ijkabc", x) - np.einsum("kjiabc->ijkabc", x)

    def P_a_bc(x):
        return x - np.einsum("ijkbac->ijkabc", x) - np.einsum("ijkcba->ijkabc", x)

    Dtc = P_i_jk(P_a_bc(conn))                             # D t(c)
    Dtd = P_i_jk(P_a_bc(disc))                             # D t(d)
    D = (fo[:, None, None, None, None, None] + fo[None, :, None, None, None, None]
         + fo[None, None, :, None, None, None] - fv[None, None, None, :, None, None]
         - fv[None, None, None, None, :, None] - fv[None, None, None, None, None, :])
    e4 = math.fsum((Dtc * Dtc / D).ravel()) / 36.0
    e5 = math.fsum((Dtc * Dtd / D).ravel()) / 36.0
    return e4 + e5, e4, e5, Dtc


def connected_antisymmetry_defect(Dtc) -> float:
    """max |t(c) + t(c) with i<->j| and |t(c) + t(c) with a<->b|: both vanish
    for a correctly antisymmetrized triples amplitude."""
    a = np.abs(Dtc + np.einsum("jikabc->ijkabc", Dtc)).max()
    b = np.abs(Dtc + np.einsum("ijkbac->ijkabc", Dtc)).max()
    return float(max(a, b))
