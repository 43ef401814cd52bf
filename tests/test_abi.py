"""The C-ABI library loads and exports every function that include/alofdft.h declares
(no device calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alofdft.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(alofdft_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("alofdft_create", "alofdft_solve", "alofdft_solve_device", "alofdft_apply_laplacian",
              "alofdft_poisson", "alofdft_energy_gradient", "alofdft_forces", "alofdft_pseudocharge",
              "alofdft_relax"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1405_6456_amd as lib

    if not os.path.exists(lib.LIB_PATH):
        pytest.skip("library not built")
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(so, n)]
    assert not missing, missing


def test_host_only_calls():
    import paper_1405_6456_amd as lib

    if not os.path.exists(lib.LIB_PATH):
        pytest.skip("library not built")
    L = lib.lib()
    assert L.alofdft_strerror(0) == b"ok"
    assert L.alofdft_strerror(-1) == b"invalid argument"
    p = lib.default_params()
    assert p.fd_half_width == 6 and p.lambda_ == 0.2 and p.eta0 == -0.2 and p.mu0 == 1.0 and p.kappa == 0.1
    assert p.tol_constraint == 1e-8 and p.tol_grad == 1e-6 and p.tol_poisson == 1e-10
    assert L.alofdft_default_params(None) == lib.INVALID_ARGUMENT
    assert L.alofdft_set_tuning(None, 0, 1024, 4) == lib.INVALID_ARGUMENT
    assert L.alofdft_set_cg_schedule(None, 1) == lib.INVALID_ARGUMENT
    rp = lib.default_relax_params()
    assert rp.ftol == 1e-3 and rp.max_move == 0.3 and rp.probe == 0.05 and rp.max_steps == 50
    assert rp.max_secant == 3 and rp.secant_rel == 0.1
    assert L.alofdft_default_relax_params(None) == lib.INVALID_ARGUMENT
    assert L.alofdft_relax(None, None, None, None, None, None, None, None, None) == lib.INVALID_ARGUMENT


def test_binding_refuses_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1405_6456_amd as lib

    with pytest.raises(RuntimeError):
        lib.Context(0)
