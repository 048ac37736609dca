"""Writes batched_targets.json: per problem of the many-problem workload
(256 dense int16 QUBOs, n = floor(256 * 16^U), weights uniform in
[-1000, 1000], seed 0), the best energy the oracle's generational loop
(Sections III-IV) reaches with a fixed prefix budget -- instances 0..7,
3 rounds, s = 0.1, b = 1, tau 8, 2 pools x 16, generator key 50000 + p.
These are the time-to-target energies of the batched-versus-one-at-a-time
comparison.  Calls only the oracle; run from the repository root:

    python tests/golden/make_batched_targets.py
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

INSTANCES, ROUNDS, SEED0, CAPACITY, NPOOLS, TAU = 8, 3, 50000, 16, 2, 8


def target(p):
    import oracle
    from paper_2207_03069_amd import inputs
    sizes = inputs.batched_sizes(256, seed=0)
    n = int(sizes[p])
    W = inputs.dense_qubo(n, -1000, 1000, 0 * 100003 + p + 1)
    g = oracle.ga_params(T=max(1, round(0.1 * n)), Bn=n, tau=TAU, seed=SEED0 + p, capacity=CAPACITY, npools=NPOOLS)
    return int(oracle.solve(W, g, INSTANCES, ROUNDS)["best_e"])


def main():
    import oracle
    oracle.build(force=False)
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        targets = pool.map(target, range(256))
    out = {"description": "per problem of the many-problem workload (256 dense int16 QUBOs, n log-uniform in "
                          "[256, 4096), weights uniform in [-1000, 1000], seed 0): the best energy of the oracle's "
                          "generational loop with instances 0..7, 3 rounds, s = 0.1, b = 1, tau 8, 2 pools x 16, "
                          "generator key 50000 + problem index",
           "instances": INSTANCES, "rounds": ROUNDS, "seed0": SEED0, "capacity": CAPACITY, "npools": NPOOLS,
           "tau": TAU, "targets": targets}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_targets.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote %d targets" % len(targets))


if __name__ == "__main__":
    main()
