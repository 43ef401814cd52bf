"""The committed oracle fixtures were written by the current oracle source, and their
stored results satisfy the properties the oracle's minimiser must have (CPU only)."""
import hashlib
import json
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def oracle_hash():
    with open(os.path.join(ROOT, "oracle", "oracle.cpp"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


@pytest.mark.parametrize("name", ["single", "fcc2"])
def test_fixture_written_by_current_oracle(name):
    with open(os.path.join(GOLDEN, f"oracle_{name}.json")) as f:
        gold = json.load(f)
    assert gold.get("oracle_sha256_16") == oracle_hash(), \
        "oracle.cpp changed since the fixture was written: run tests/golden/make_golden.py single fcc2"
    r = gold["result"]
    assert r["status"] == 0
    assert abs(r["C"]) / gold["N"] < 1e-8 and r["gnorm"] < 1e-6 and r["poisson_relres"] < 1e-10
    # the energy is the sum of its terms
    parts = r["E_TF"] + r["E_vW"] + r["E_xc"] + r["E_es"] + r["E_c"] + r["E_ext"]
    assert abs(parts - r["E_total"]) < 1e-12 * abs(r["E_total"])
    # the sampled fields are finite and u >= 0
    assert np.all(np.array(gold["u_samples"]) >= 0) and np.all(np.isfinite(gold["phi_samples"]))
    # the forces sum to zero up to the solve's accuracy (no external field)
    f = np.array(gold["forces"])
    assert np.abs(f.sum(axis=0)).max() < 1e-3
