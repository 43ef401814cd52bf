"""Writes the oracle's converged results for the named workloads to JSON fixtures.

Calls only the CPU oracle (oracle/) and the input generators; nothing here touches
the GPU library.  Usage: python tests/golden/make_golden.py single fcc2 [fcc5]
Each fixture records the parameters it was made with, the energies, the multiplier,
the constraint, the forces, u and phi at sampled nodes, and a hash of the oracle source
that wrote it (a test checks that it equals the hash of the current source, so a change
of the oracle's arithmetic forces the fixtures to be written again).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1405_6456_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def oracle_source_hash():
    """sha256 (first 16 hex digits) of the oracle's C++ source."""
    with open(os.path.join(ROOT, "oracle", "oracle.cpp"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def sample_nodes(grid, count=64, seed=99):
    u = synth.stream(seed, 3 * count).reshape(count, 3)
    return [[int(u[m, a] * grid.n[a]) for a in range(3)] for m in range(count)]


def make(name, method=0, threads=None):
    oracle.set_threads(threads or os.cpu_count())
    S = synth.config(name)
    prm = oracle.params(method=method)
    u0 = synth.initial_u(S.grid, S.N)
    t = time.time()
    r = oracle.solve(S, prm, u0)
    wall = time.time() - t
    nodes = sample_nodes(S.grid)
    out = {
        "workload": name,
        "method": method,
        "oracle_sha256_16": oracle_source_hash(),
        "params": {"fd_n": 6, "lambda": 0.2, "xc": "LDA_PZ", "gauss_s": 1.0, "r_cut": 7.0, "eta0": -0.2,
                   "mu0": 1.0, "kappa": 0.1, "tol_constraint": 1e-8, "tol_grad": 1e-6, "tol_poisson": 1e-10,
                   "bc": "multipole", "u0": "synth.initial_u seed 6456"},
        "oracle_wall_s": wall,
        "oracle_threads": oracle.get_threads(),
        "M": S.M,
        "N": S.N,
        "n": list(S.grid.n),
        "h": S.grid.h,
        "result": {k: (v if not isinstance(v, (np.floating, np.integer)) else v.item())
                   for k, v in r.items() if not isinstance(v, np.ndarray)},
        "forces": r["forces"].tolist(),
        "sample_nodes": nodes,
        "u_samples": [float(r["u"][k, j, i]) for i, j, k in nodes],
        "phi_samples": [float(r["phi"][k, j, i]) for i, j, k in nodes],
    }
    suffix = "" if method == 0 else {1: "_penalty", 2: "_lagrange"}[method]
    path = os.path.join(HERE, f"oracle_{name}{suffix}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: status {r['status']} E={r['E_total']:.12f} eta={r['eta']:.10f} wall {wall:.1f}s -> {path}")


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        name, _, m = arg.partition(":")
        make(name, int(m) if m else 0)
