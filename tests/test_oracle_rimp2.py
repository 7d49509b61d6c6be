"""Pins of the RI-MP2 oracle (CPU only; paper Sec. 2.1, eqs. mp2_energy,
e_orb_diff, eri_sym_decomp)."""
import numpy as np
import pytest

import oracle
from paper_1609_08094_amd import synth


@pytest.mark.parametrize("o,v,seed", [(1, 1, 0), (2, 3, 1), (3, 4, 2), (2, 6, 3)])
def test_matches_spin_orbital_mp2(o, v, seed):
    p = synth.mp2_from_factors(o, v, seed=seed)
    ref = oracle.spin_orbital_mp2(p["eri"], p["eps_o"], p["eps_v"])
    got = oracle.rimp2_energy(p["eps_o"], p["eps_v"], p["c_ov"])
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-15)
    assert got <= 0.0


def test_one_orbital_closed_form():
    c = np.array([[[0.3, -0.2, 0.5]]])                  # o = v = 1, naux = 3
    eo, ev = np.array([-1.1]), np.array([0.7])
    g = float(c[0, 0] @ c[0, 0])
    assert oracle.rimp2_energy(eo, ev, c) == pytest.approx(-g * g / (2 * (0.7 + 1.1)), rel=1e-15)


def test_pair_form_equals_definition():
    p = synth.make_mp2_problem(5, 9, 14, seed=4)
    a = oracle.rimp2_energy(p["eps_o"], p["eps_v"], p["c_ov"])
    b = oracle.rimp2_energy_pairs(p["eps_o"], p["eps_v"], p["c_ov"])
    assert a == pytest.approx(b, rel=1e-13)


def test_homogeneity_and_shift():
    p = synth.make_mp2_problem(3, 7, 10, seed=5)
    e = oracle.rimp2_energy(p["eps_o"], p["eps_v"], p["c_ov"])
    assert oracle.rimp2_energy(p["eps_o"], p["eps_v"], 1.7 * p["c_ov"]) == pytest.approx(1.7 ** 4 * e, rel=1e-13)
    # the energy depends on orbital-energy differences only
    assert oracle.rimp2_energy(p["eps_o"] + 0.4, p["eps_v"] + 0.4, p["c_ov"]) == pytest.approx(e, rel=1e-13)
    # E is additive over independent auxiliary blocks only through g, so
    # dropping the exchange term must change it (the exchange is really used)
    g = oracle.g_ovov(p["c_ov"])
    den = (p["eps_v"][None, :, None, None] + p["eps_v"][None, None, None, :]
           - p["eps_o"][:, None, None, None] - p["eps_o"][None, None, :, None])
    assert abs(-np.sum(2 * g * g / den) - e) > 1e-6 * abs(e)


def test_relabeling_invariance():
    p = synth.make_mp2_problem(4, 8, 12, seed=6)
    rng = np.random.default_rng(0)
    po, pv = rng.permutation(4), rng.permutation(8)
    e = oracle.rimp2_energy(p["eps_o"], p["eps_v"], p["c_ov"])
    f = oracle.rimp2_energy(p["eps_o"][po], p["eps_v"][pv], p["c_ov"][po][:, pv])
    assert f == pytest.approx(e, rel=1e-13)


def test_planted_transpose_is_caught():
    """A plausible slip -- the exchange integral taken as g_aibj itself -- fails
    the spin-orbital pin."""
    p = synth.mp2_from_factors(2, 4, seed=7)
    g = oracle.g_ovov(p["c_ov"])
    den = (p["eps_v"][None, :, None, None] + p["eps_v"][None, None, None, :]
           - p["eps_o"][:, None, None, None] - p["eps_o"][None, None, :, None])
    wrong = float(-np.sum(g * (2 * g - g) / den))
    ref = oracle.spin_orbital_mp2(p["eri"], p["eps_o"], p["eps_v"])
    assert abs(wrong - ref) > 1e-6 * abs(ref)
