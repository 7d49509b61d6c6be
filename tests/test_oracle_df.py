"""Pins of the density-fitted (vv|vo) assembly of the oracle (CPU only).

Paper Sec. 2.1, eq. eri_sym_decomp.  The assembled block is checked against
closed forms of rank-one factors (which catch a transposed or swapped
operand), against the generator's full-ERI route (an einsum over all orbitals
followed by 8-fold symmetrization: different code), for additivity over
auxiliary blocks, and the resulting E(T) against the explicit-integral
oracle, itself pinned by the spin-orbital brute force.
"""
import numpy as np

import oracle
from paper_1609_08094_amd import synth


def test_rank_one_factors_give_the_outer_product():
    rng = np.random.default_rng(3)
    v, o = 5, 3
    u, w, x, y = (rng.normal(size=n) for n in (v, v, v, o))
    bvv = (u[:, None] * w[None, :])[:, :, None]          # B_ab = u_a w_b (not symmetric)
    bvo = (x[:, None] * y[None, :])[:, :, None]          # B_ci = x_c y_i
    g = oracle.vvvo_from_df(bvv, bvo)
    ref = u[:, None, None, None] * w[None, :, None, None] * x[None, None, :, None] * y[None, None, None, :]
    assert np.allclose(g, ref, rtol=1e-14, atol=0)
    assert not np.allclose(g, g.transpose(1, 0, 2, 3))   # the a,b order is really tested


def test_additive_over_auxiliary_blocks():
    rng = np.random.default_rng(4)
    v, o = 4, 2
    b1, b2 = rng.normal(size=(v, v, 3)), rng.normal(size=(v, v, 5))
    c1, c2 = rng.normal(size=(v, o, 3)), rng.normal(size=(v, o, 5))
    whole = oracle.vvvo_from_df(np.concatenate([b1, b2], 2), np.concatenate([c1, c2], 2))
    parts = oracle.vvvo_from_df(b1, c1) + oracle.vvvo_from_df(b2, c2)
    assert np.allclose(whole, parts, rtol=1e-13, atol=1e-15)


def test_matches_full_eri_route():
    p = synth.make_problem(3, 6, seed=5, with_eri=True, with_df=True)
    g = oracle.vvvo_from_df(p["bvv"], p["bvo"])
    assert np.abs(g - p["vvvo"]).max() <= 1e-15 * max(1.0, np.abs(p["vvvo"]).max()) * 10


def test_df_energy_matches_explicit_integrals():
    for (o, v, seed) in [(3, 6, 6), (4, 9, 7)]:
        p = synth.make_problem(o, v, seed=seed, with_eri=True, with_df=True)
        a = oracle.triples_energy(p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["vvvo"], p["ovoo"], p["ovov"])
        b = oracle.triples_energy_df(p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["bvv"], p["bvo"], p["ovoo"],
                                     p["ovov"])
        for x, y in zip(a, b):
            assert abs(x - y) <= 1e-12 * abs(a[1])


def test_df_energy_matches_spin_orbital_brute_force():
    p = synth.make_problem(2, 4, seed=8, with_eri=True, with_df=True)
    E, E4, E5, _ = oracle.spin_orbital_triples(p["eri"], p["eps_o"], p["eps_v"], p["t1"], p["t2"])
    got = oracle.triples_energy_df(p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["bvv"], p["bvo"], p["ovoo"],
                                   p["ovov"])
    assert abs(got[0] - E) <= 1e-10 * abs(E4) + 1e-14
    assert abs(got[1] - E4) <= 1e-10 * abs(E4) + 1e-14
