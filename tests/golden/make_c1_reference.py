"""Write tests/golden/c1_oracle_chains.json: independent oracle Markov chains
at the plain L=3 shape (N = 18, U/t = 3.8, beta t = 3, dtau = 0.1, M = 30,
n_stab = 10), the reference of the GPU independent-run test.

Calls only oracle/ (and the seeded input generators): 64 chains, fields
i.i.d. +-1 from seed 1000 + c, Metropolis uniforms from NumPy's generator
(RandomSource, seed 2000 + c), 100 warm-up sweeps, then 1500 sweeps with a
measurement at every recomputation; the per-chain means of the estimators
are stored.  Run from the repository root:

    python tests/golden/make_c1_reference.py
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle.dqmc import Chain, Model, RandomSource  # noqa: E402

N_CHAINS, WARMUP, SWEEPS = 64, 100, 1500
KEYS = ("D", "ekin", "e", "Szz_G", "Szz_dk", "m2")


def run_chain(c):
    d = workloads.plain_L3()[0]
    m = Model(d["L"], d["U"], d["beta"], d["dtau"], t=d["t"], n_stab=d["n_stab"])
    ch = Chain(m, workloads.random_fields(1000 + c, m.M, m.N))
    src = RandomSource(2000 + c)
    for _ in range(WARMUP):
        ch.sweep(src, measure=False)
    ch.samples = []
    for _ in range(SWEEPS):
        ch.sweep(src, measure=True)
    return {k: float(np.mean([s[k] for s in ch.samples])) for k in KEYS}


def main():
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        per = pool.map(run_chain, range(N_CHAINS))
    d = workloads.plain_L3()[0]
    out = {"what": "oracle independent chains, per-chain estimator means",
           "config": {k: d[k] for k in ("L", "U", "beta", "dtau", "n_stab", "t")},
           "chains": N_CHAINS, "warmup": WARMUP, "sweeps": SWEEPS,
           "per_chain": {k: [p[k] for p in per] for k in KEYS}}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle_chains.json"), "w") as f:
        json.dump(out, f, indent=1)
    for k in KEYS:
        x = np.array(out["per_chain"][k])
        print("%-7s %.6f +- %.6f" % (k, x.mean(), x.std(ddof=1) / np.sqrt(len(x))))


if __name__ == "__main__":
    main()
