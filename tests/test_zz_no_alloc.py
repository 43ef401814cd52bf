"""The allocation-free Laplacian entry point (alofdft_apply_laplacian_noalloc), called
through the C ABI, gives what alofdft_apply_laplacian gives, on two calls in a row (the
second on a smaller grid, in the other precision), and refuses a grid beyond its scratch."""
import ctypes as C

import numpy as np
import pytest

from paper_1405_6456_amd import synth
from tests.gpu_util import ctx

pytestmark = pytest.mark.gpu


def _noalloc(c, x, h, fdn):
    import torch

    import paper_1405_6456_amd as lib

    dtype = {torch.float64: 0, torch.float32: 1}[x.dtype]
    y = torch.full_like(x, float("nan"))
    n = (C.c_int * 3)(x.shape[2], x.shape[1], x.shape[0])
    st = lib.lib().alofdft_apply_laplacian_noalloc(c.handle, n, h, fdn, dtype, C.c_void_p(x.data_ptr()),
                                                   C.c_void_p(y.data_ptr()))
    torch.cuda.synchronize()
    return st, y


def test_noalloc_matches_the_allocating_entry_point():
    import torch

    import paper_1405_6456_amd as lib

    c = ctx()
    try:
        cases = [((70, 45, 29), 0.37, 6, torch.float64), ((33, 21, 18), 0.5, 3, torch.float32)]
        for nn, h, fdn, dt in cases:
            g = synth.Grid(nn, h, (0.0, 0.0, 0.0))
            x = torch.from_numpy(synth.random_field(g, 40 + fdn)).to(device="cuda:0", dtype=dt)
            ref = c.apply_laplacian(x, h, fdn)
            st, y = _noalloc(c, x, h, fdn)
            assert st == lib.OK
            # the same kernels on the same padded layout: bit-identical
            assert torch.equal(y, ref), float((y - ref).abs().max())
        # a grid whose padded x and y exceed the scratch is refused, with the reason
        big = torch.zeros((160, 160, 160), dtype=torch.float64, device="cuda:0")
        st, _ = _noalloc(c, big, 0.5, 6)
        assert st == lib.INVALID_ARGUMENT
        assert b"scratch" in lib.lib().alofdft_last_error(c.handle)
        # and a call after the refusal still works
        g = synth.Grid((24, 24, 24), 0.5, (0.0, 0.0, 0.0))
        x = torch.from_numpy(synth.random_field(g, 9)).cuda()
        st, y = _noalloc(c, x, 0.5, 6)
        assert st == lib.OK and torch.equal(y, c.apply_laplacian(x, 0.5, 6))
    finally:
        c.close()
