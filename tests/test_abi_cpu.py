"""CPU checks of the boundary: the library builds, loads and exports every
entry point include/dbas_mppi.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dbas_mppi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mppi_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_2504_06437_amd import _lib as A
    assert sorted(A.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2504_06437_amd import _lib as A
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(A.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_config_defaults_and_struct_layout():
    """mppi_config_default runs on the host; the ctypes struct matches the C
    layout (every field lands where the library writes it)."""
    from paper_2504_06437_amd import _lib as A
    L = A.load()
    for model, P, lim in ((0, 7, 0.5 * 0.5 * 9.81), (1, 7, 4.0), (2, 8, 1.013)):
        c = A.Config()
        assert L.mppi_config_default(model, 1024, 30, ctypes.byref(c)) == A.OK
        assert c.abi_version == A.ABI_VERSION and c.K == 1024 and c.T == 30 and c.P == P
        assert abs(c.u_max[0] - lim) < 1e-6 and c.lam == 1.0 and abs(c.h_eps - 1e-4) < 1e-10
        assert c.tile_samples == 0 and c.export_noise == 0 and list(c.reserved) == [0] * 2
        assert c.adaptive_explore == 0 and abs(c.explore_mu - 0.4) < 1e-7
    assert L.mppi_config_default(7, 1, 1, ctypes.byref(A.Config())) == A.E_INVALID
    assert L.mppi_status_string(A.E_NUMERIC) == b"MPPI_E_NUMERIC"


def test_binding_config_from_workload_params():
    from paper_2504_06437_amd import workloads as W
    from paper_2504_06437_amd.controller import make_config
    c = make_config(W.base_params("car", 4096, 50))
    assert c.model == 2 and c.P == 8 and c.shape[0][0] == 2.0 and abs(c.shape[0][1] - 1.5) < 1e-7
    c = make_config(W.base_params("quad5", 64, 5))
    assert abs(c.sigma[0] ** 2 - 0.4) < 1e-6 and abs(c.sigma[1] ** 2 - 0.12) < 1e-6


def test_package_lazy_exports_resolve():
    """Every name the package lists resolves to the class in ``controller``
    (no library load is needed to resolve them)."""
    import paper_2504_06437_amd as pkg
    from paper_2504_06437_amd import controller
    for name in pkg.__all__:
        obj = getattr(pkg, name)
        if name != "workloads":
            assert obj is getattr(controller, name)
    with pytest.raises(AttributeError):
        getattr(pkg, "NoSuchThing")
