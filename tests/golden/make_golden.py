"""Writes the stored oracle values under tests/golden/.

Calls only the oracle (and the seeded input generator); nothing here comes
from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py            # C0 (literal mode) and C0 physically scaled
    python tests/golden/make_golden.py c1 [-j N]  # C1 seeds 0-2 and C1 physically scaled (restricted mode)

The C1 values take the oracle about an hour and a half per problem on one
core; the triples are spread over N worker processes (one BLAS thread each),
and every per-triple partial is kept so that the GPU tests can compare
triple by triple.  Sums use math.fsum over the per-triple partials in the
order of oracle.triple_list.
"""
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))


def c0_records():
    import oracle
    from paper_1609_08094_amd import synth
    out = {}
    for name, scale in (("c0_seed0.json", 1.0), ("c0_phys_seed0.json", synth.PHYSICAL_B_SCALE["C0"])):
        o, v, seed = 6, 30, 0
        p = synth.make_problem(o, v, seed=seed, b_scale=scale)
        E, E4, E5 = oracle.problem_energy(p, mode="literal")
        trip = {}
        for t in [(0, 1, 2), (0, 0, 5), (2, 4, 4), (1, 3, 5)]:
            e, e4, e5 = oracle.triple_restricted(*t, p["eps_o"], p["eps_v"], p["t1"], p["t2"],
                                                 p["vvvo"], p["ovoo"], p["ovov"])
            trip["%d,%d,%d" % t] = [e, e4, e5]
        rec = dict(o=o, v=v, seed=seed, b_scale=scale, generator="synth.make_problem (numpy PCG64)",
                   source="oracle literal mode (all ordered triples), math.fsum",
                   E=E, E4=E4, E5=E5, triples=trip)
        out[name] = rec
    return out


_CACHE = {}


def _worker_triples(args):
    o, v, seed, scale, trips = args
    import oracle
    from paper_1609_08094_amd import synth
    key = (o, v, seed, scale)
    if key not in _CACHE:
        _CACHE.clear()
        _CACHE[key] = synth.make_problem(o, v, seed=seed, b_scale=scale)
    p = _CACHE[key]
    return [oracle.triple_restricted(*t, p["eps_o"], p["eps_v"], p["t1"], p["t2"], p["vvvo"], p["ovoo"], p["ovov"])
            for t in trips]


def c1_record(pool, o, v, seed, scale, nworkers):
    import oracle
    trips = oracle.triple_list(o)
    # interleaved chunks so that every worker sees a mix of cheap and costly triples
    chunks = [trips[w::nworkers * 4] for w in range(nworkers * 4)]
    t0 = time.perf_counter()
    parts = pool.map(_worker_triples, [(o, v, seed, scale, c) for c in chunks])
    res = {}
    for c, r in zip(chunks, parts):
        for t, x in zip(c, r):
            res[t] = x
    e4 = math.fsum(res[t][1] for t in trips)
    e5 = math.fsum(res[t][2] for t in trips)
    dt = time.perf_counter() - t0
    print(f"C1 seed={seed} b_scale={scale}: E4={e4!r} E5={e5!r} in {dt:.0f}s", flush=True)
    return dict(o=o, v=v, seed=seed, b_scale=scale, generator="synth.make_problem (numpy PCG64)",
                source="oracle restricted mode (i<=j<=k with multiplicities), math.fsum over the "
                       "per-triple partials in triple_list order",
                E=e4 + e5, E4=e4, E5=e5,
                triples={"%d,%d,%d" % t: list(res[t]) for t in trips})


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "c1":
        from paper_1609_08094_amd import synth
        nworkers = int(sys.argv[sys.argv.index("-j") + 1]) if "-j" in sys.argv else os.cpu_count() or 1
        for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[var] = "1"
        ctx = mp.get_context("spawn")
        jobs = [(0, 1.0, "c1_seed0.json"), (1, 1.0, "c1_seed1.json"), (2, 1.0, "c1_seed2.json"),
                (0, synth.PHYSICAL_B_SCALE["C1"], "c1_phys_seed0.json")]
        with ctx.Pool(nworkers) as pool:
            for seed, scale, name in jobs:
                path = os.path.join(HERE, name)
                if os.path.exists(path) and "--force" not in sys.argv:
                    print(f"{name} exists, kept", flush=True)
                    continue
                rec = c1_record(pool, 20, 200, seed, scale, nworkers)
                with open(path, "w") as f:
                    json.dump(rec, f, separators=(",", ":"))
        return
    for name, rec in c0_records().items():
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(rec, f, indent=1)
        print(name, json.dumps({k: rec[k] for k in ("E", "E4", "E5")}))


if __name__ == "__main__":
    main()
