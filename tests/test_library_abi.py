"""The C-ABI library loads on the CPU host and exports every entry point the
header declares (no compute call is made: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nebem.h")
LIB = os.path.join(ROOT, "paper_2606_24154_amd", "libnebem.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nebem_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_path(lib):
    names = declared()
    for must in ("nebem_assemble", "nebem_solve", "nebem_eval", "nebem_spacecharge_step",
                 "nebem_session_create", "nebem_session_eval"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_match_header():
    import paper_2606_24154_amd as nb
    assert sorted(nb.EXPORTED) == declared()


def test_default_options_and_last_error(lib):
    import paper_2606_24154_amd as nb
    o = nb.options()
    assert o.precision == nb.FP64 and o.near_factor == 4.0 and o.ir_tol == 1e-10
    assert o.sc_resolve_every == 10 and o.sc_dt == 1e-12 and o.sc_mobility == 1e-4
    lib.nebem_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.nebem_last_error(), bytes)


def test_argument_errors_need_no_gpu(lib):
    """Validation errors return before any device work."""
    import paper_2606_24154_amd as nb
    assert nb.lib.nebem_eval(None, None, None, None, None, None, 0, None, None, None, None, None, None) == \
        nb.NEBEM_EINVAL
    assert nb.lib.nebem_solve(None, -1, None, 1, None, None, None, None, None) == nb.NEBEM_EINVAL
    bad = nb.options(precision=7)
    p = nb.Panels()
    p.n = 0
    assert nb.lib.nebem_assemble(ctypes.byref(p), None, None, None, None, ctypes.byref(bad), None, None) == \
        nb.NEBEM_EINVAL
    assert b"precision" in nb.lib.nebem_last_error()
    h = ctypes.c_void_p()
    assert nb.lib.nebem_session_create(ctypes.byref(p), None, None, None, ctypes.byref(h)) == nb.NEBEM_EINVAL


def test_line_charge_entry_points_validate_without_gpu(lib):
    """The point-to-line entry points refuse bad arguments before any
    device work: a NULL session, a voxel grid with an empty axis."""
    import paper_2606_24154_amd as nb
    n = ctypes.c_int64(5)
    assert nb.lib.nebem_spacecharge_step_lines(None, None, None, None, None, 0, 0, None, 0, None, None, None,
                                               ctypes.byref(n), None) == nb.NEBEM_EINVAL
    assert n.value == 0
    g = nb.grid_struct((0.0, 0.0, 0.0), (1e-6, 1e-6, 1e-6), (4, 0, 4))
    nl, out = ctypes.c_int64(), ctypes.c_int64()
    assert nb.lib.nebem_voxelize_charges(None, None, None, None, 0, ctypes.byref(g), 0, None, 0, ctypes.byref(nl),
                                         ctypes.byref(out), None) == nb.NEBEM_EINVAL
    # an unknown line placement
    g = nb.grid_struct((0.0, 0.0, 0.0), (1e-6, 1e-6, 1e-6), (4, 4, 4))
    assert nb.lib.nebem_voxelize_charges(None, None, None, None, 0, ctypes.byref(g), 2, None, 0, ctypes.byref(nl),
                                         ctypes.byref(out), None) == nb.NEBEM_EINVAL
    assert nb.lib.nebem_charge_field_lines(None, None, None, None, 0, ctypes.byref(g), 5, None, None, None,
                                           ctypes.byref(nl), None) == nb.NEBEM_EINVAL


def test_server_options_layout_and_validation(lib):
    """The binding's server-option structure matches the library's (the
    defaults read back through it), and bad options or a NULL output are
    refused before anything touches a device."""
    import paper_2606_24154_amd as nb
    o = nb.server_default_options()
    assert o.hbm_budget == 2 << 30 and o.batch_interactions == 1e10 and o.max_items == 65536
    assert o.large_interactions == 1e11 and o.max_large == 1
    assert ctypes.sizeof(nb.ServerOptions) == 40
    h = ctypes.c_void_p()
    assert nb.lib.nebem_server_create(None, 0, ctypes.byref(o), ctypes.byref(h)) == nb.NEBEM_EINVAL
    assert nb.lib.nebem_server_create(None, 1, ctypes.byref(o), None) == nb.NEBEM_EINVAL
    arr = (ctypes.c_void_p * 1)(None)
    for field, bad in (("max_large", -1), ("large_interactions", 0.0), ("hbm_budget", 100)):
        b = nb.server_default_options()
        setattr(b, field, bad)
        assert nb.lib.nebem_server_create(arr, 1, ctypes.byref(b), ctypes.byref(h)) == nb.NEBEM_EINVAL, field
        assert b"bad options" in nb.lib.nebem_last_error(), field
    assert nb.lib.nebem_server_create(arr, 1, ctypes.byref(o), ctypes.byref(h)) == nb.NEBEM_EINVAL
    assert b"NULL session" in nb.lib.nebem_last_error()
    assert nb.lib.nebem_server_wait(None, 1, None) == nb.NEBEM_EINVAL
