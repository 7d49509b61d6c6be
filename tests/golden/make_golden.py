"""Writes the stored oracle values under tests/golden/.

Calls only the oracle (and the seeded input generator); nothing here comes
from the HIP path.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1609_08094_amd import synth  # noqa: E402


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    o, v, seed = 6, 30, 0
    p = synth.make_problem(o, v, seed=seed)
    E, E4, E5 = oracle.problem_energy(p, mode="literal")
    trip = {}
    for t in [(0, 1, 2), (0, 0, 5), (2, 4, 4), (1, 3, 5)]:
        e, e4, e5 = oracle.triple_restricted(*t, p["eps_o"], p["eps_v"], p["t1"], p["t2"],
                                             p["vvvo"], p["ovoo"], p["ovov"])
        trip["%d,%d,%d" % t] = [e, e4, e5]
    rec = dict(o=o, v=v, seed=seed, generator="synth.make_problem (numpy PCG64)",
               source="oracle literal mode (all ordered triples), math.fsum",
               E=E, E4=E4, E5=E5, triples=trip)
    with open(os.path.join(here, "c0_seed0.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
