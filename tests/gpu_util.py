"""Helpers shared by the GPU tests."""
import json
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1405_6456_amd as lib

    return lib.Context(0)


def golden(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"fixture {path} not generated")
    with open(path) as f:
        return json.load(f)
