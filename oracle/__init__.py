"""CPU oracle for the closed-shell (T) energy (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the library never does, and the two share no code.
"""
from .triples import (triples_energy, triple_restricted, triple_literal, triple_list,
                      multiplicity, w_tensor, z_tensor, d_tensor, x_piece, problem_energy)
from .spin_orbital import spin_orbital_triples, connected_antisymmetry_defect
from .df import vvvo_from_df, triples_energy_df, triple_restricted_df
from .rimp2 import g_ovov, rimp2_energy, rimp2_pair_energy, rimp2_energy_pairs, spin_orbital_mp2
