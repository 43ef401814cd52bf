"""Failure handling driven from the host: invalid and non-finite inputs, and a solve
cancelled while it runs (every kernel still exits normally)."""
import threading
import time

import numpy as np
import pytest

from paper_1405_6456_amd import synth
from tests.gpu_util import ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    c = ctx()
    yield c
    c.close()


def test_nan_in_host_guess_is_refused(C):
    import paper_1405_6456_amd as lib

    S = synth.single_atom(L=16.0, n=21)
    u0 = synth.initial_u(S.grid, S.N)
    u0[10, 10, 10] = np.nan
    with pytest.raises(lib.AlofdftError) as err:
        C.solve(S, lib.default_params(), u0)
    assert err.value.status == lib.INVALID_ARGUMENT


def test_nan_in_device_guess_is_numerical(C):
    import torch

    import paper_1405_6456_amd as lib

    S = synth.single_atom(L=16.0, n=21)
    u0 = torch.from_numpy(synth.initial_u(S.grid, S.N)).cuda()
    u0[10, 10, 10] = float("nan")
    with pytest.raises(lib.AlofdftError) as err:
        C.solve_device(S, lib.default_params(), u0)
    assert err.value.status == lib.NUMERICAL


@pytest.mark.parametrize("N", [0.0, -3.0, float("nan")])
def test_bad_electron_count_is_refused(C, N):
    import paper_1405_6456_amd as lib

    S = synth.single_atom(L=16.0, n=21)
    S.N = N
    with pytest.raises(lib.AlofdftError) as err:
        C.solve(S, lib.default_params(), None)
    assert err.value.status == lib.INVALID_ARGUMENT


def test_grid_beyond_the_array_limit_is_refused(C):
    # a padded FP64 array of an 800^3 grid passes 4 GiB, past what the kernels' 32-bit
    # buffer offsets reach: refused before anything is allocated, and the context still works
    import paper_1405_6456_amd as lib

    S = synth.single_atom(L=16.0, n=21)
    S.grid = synth.Grid((800, 800, 800), 0.02, (0.0, 0.0, 0.0))
    with pytest.raises(lib.AlofdftError) as err:
        C.solve(S, lib.default_params(), None, want_fields=False)
    assert err.value.status == lib.INVALID_ARGUMENT
    assert "4 GiB" in str(err.value)
    S = synth.single_atom(L=16.0, n=21)
    out = C.solve(S, lib.default_params(), None, want_fields=False)
    assert out["status"] == lib.OK


def test_cancel_mid_solve_then_solve_again(C):
    import paper_1405_6456_amd as lib

    S = synth.config("fcc2")
    prm = lib.default_params()
    ref = C.solve(S, prm, None, want_fields=False)
    out = {}

    def run():
        try:
            out["r"] = C.solve(S, prm, None, want_fields=False)
        except lib.AlofdftError as e:
            out["err"] = e

    th = threading.Thread(target=run)
    th.start()
    time.sleep(0.25)
    C.cancel()
    th.join(60)
    assert not th.is_alive()
    assert "err" in out and out["err"].status == lib.CANCELLED
    # the context is usable afterwards and gives the same result as before
    again = C.solve(S, prm, None, want_fields=False)
    assert again["status"] == 0 and again["E_total"] == ref["E_total"]
