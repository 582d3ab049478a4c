"""The C-ABI library loads and exports every entry point include/ahr.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ahr.h")
LIB = os.path.join(ROOT, "paper_2511_10073_amd", "libahr.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ahr_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for need in ["ahr_graph_build", "ahr_graph_update_hints", "ahr_filter", "ahr_refine", "ahr_hpwl",
                 "ahr_graph_export", "ahr_graph_destroy", "ahr_last_error", "ahr_graph_workspace_size",
                 "ahr_graph_refine", "ahr_gift", "ahr_wa", "ahr_macro_charge"]:
        assert need in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (the HIP runtime torch ships is the one the library binds to)
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name
    lib.ahr_version.restype = ctypes.c_char_p
    assert lib.ahr_version().startswith(b"ahr")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
def test_invalid_arguments_fail_before_any_device_work():
    import paper_2511_10073_amd as A
    lib = A.load()
    h = ctypes.c_void_p()
    # NULL netlist
    assert lib.ahr_graph_build(None, None, None, 0, None, 0, None, ctypes.byref(h)) == A.EINVAL
    assert b"netlist" in lib.ahr_last_error()
    nl = A._Netlist(10, 0, 0, 0, 0, 0, 0, 0, 0, 0, (ctypes.c_float * 4)(0, 0, 1, 1))
    hp = A.hint_params()
    assert lib.ahr_graph_build(ctypes.byref(nl), ctypes.byref(hp), None, 0, None, 0, None, ctypes.byref(h)) == A.EINVAL
    nl2 = A._Netlist(10, 0, 0, 0, 8, 0, 8, 0, 8, 8, (ctypes.c_float * 4)(0, 0, 1, 1))
    bad = A.hint_params(nbx=0)
    assert lib.ahr_graph_build(ctypes.byref(nl2), ctypes.byref(bad), None, 0, None, 0, None, ctypes.byref(h)) == A.EINVAL
    big = A.hint_params(nbx=256, nby=256)
    assert lib.ahr_graph_build(ctypes.byref(nl2), ctypes.byref(big), None, 0, None, 0, None,
                               ctypes.byref(h)) == A.EUNSUPPORTED
    spec = A.filter_spec(ks=(65,), alphas=(1.0,))
    assert lib.ahr_filter(ctypes.c_void_p(8), ctypes.byref(spec), 8, 16, 2, None) == A.EINVAL
    spec = A.filter_spec(ks=(4,), alphas=(1.0,))
    assert lib.ahr_filter(None, ctypes.byref(spec), 8, 16, 2, None) == A.EINVAL
    assert lib.ahr_hpwl(None, 8, 2, 8, None) == A.EINVAL
    assert lib.ahr_hpwl(ctypes.byref(nl2), 8, 3, 8, None) == A.EINVAL
    assert lib.ahr_hpwl(ctypes.byref(nl2), None, 2, 8, None) == A.EINVAL
    assert lib.ahr_graph_refine(ctypes.c_void_p(8), ctypes.byref(spec), 8, 2, 1, 1.5, 16, None) == A.EINVAL
    assert lib.ahr_refine(ctypes.byref(nl2), ctypes.byref(hp), ctypes.byref(spec), 8, 2, 1, 1.5, 16, None, 0,
                          None) == A.EINVAL
    assert h.value is None
    # the gradient's rounding mode is 0 or 1
    assert lib.ahr_mlp_loss_grad(8, 8, 8, 4, 8, None, 2, None) == A.EINVAL
    assert b"rounding" in lib.ahr_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
def test_profile_read_fills_every_field():
    """With no stage recorded, reading the profile makes no device call and
    sets every field of the struct, including the last stage's."""
    import paper_2511_10073_amd as A
    lib = A.load()
    p = A._Profile()
    for name, ty in A._Profile._fields_:
        setattr(p, name, 7 if ty is ctypes.c_int64 else 7.0)
    assert lib.ahr_profile_enable(0) == A.OK
    assert lib.ahr_profile_read(ctypes.byref(p), 1) == A.OK
    for name, _ in A._Profile._fields_:
        assert getattr(p, name) == 0, name
    assert lib.ahr_profile_read(None, 1) == A.EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
def test_profile_levels():
    """Profiling accepts 0 (off), 1 (every stage) and 2 (hop launches only),
    and rejects other values."""
    import paper_2511_10073_amd as A
    lib = A.load()
    for on in (1, 2, 0):
        assert lib.ahr_profile_enable(on) == A.OK
    for on in (-1, 3):
        assert lib.ahr_profile_enable(on) == A.EINVAL
    assert lib.ahr_profile_enable(0) == A.OK


def no_gpu():
    import torch
    return torch.cuda.device_count() == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
def test_workspace_too_small_fails_before_device_work():
    """A workspace smaller than the arrays every graph of the netlist holds
    is refused with AHR_ENOMEM before any device call (the device pointers
    here are never touched), for the graph build and for ahr_refine."""
    import paper_2511_10073_amd as A
    lib = A.load()
    nl = A._Netlist(100000, 120000, 400000, 0, 8, 8, 8, 0, 8, 8, (ctypes.c_float * 4)(0, 0, 1, 1))
    hp = A.hint_params()
    h = ctypes.c_void_p()
    assert lib.ahr_graph_build(ctypes.byref(nl), ctypes.byref(hp), 8, 4, ctypes.c_void_p(4096), 1 << 20, None,
                               ctypes.byref(h)) == A.ENOMEM
    assert b"workspace too small" in lib.ahr_last_error()
    assert h.value is None
    spec = A.filter_spec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))
    assert lib.ahr_refine(ctypes.byref(nl), ctypes.byref(hp), ctypes.byref(spec), 8, 4, 3, 0.5, 1 << 40,
                          ctypes.c_void_p(4096), 1 << 20, None) == A.ENOMEM


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
@pytest.mark.skipif(not no_gpu(), reason="injects the failure by running without a device")
def test_failed_hip_call_gives_edevice_and_no_handle():
    """With no device, the first HIP call of a valid build fails: the call
    returns AHR_EDEVICE with the HIP error in the message and leaves the
    output handle unset (nothing is launched on fake pointers: the failing
    call is the device query that comes first)."""
    import paper_2511_10073_amd as A
    lib = A.load()
    nl = A._Netlist(10, 2, 4, 0, 8, 8, 8, 0, 8, 8, (ctypes.c_float * 4)(0, 0, 1, 1))
    hp = A.hint_params()
    h = ctypes.c_void_p()
    assert lib.ahr_graph_build(ctypes.byref(nl), ctypes.byref(hp), None, 0, None, 0, None, ctypes.byref(h)) == A.EDEVICE
    assert b"failed" in lib.ahr_last_error()
    assert h.value is None
    size = ctypes.c_size_t(7)
    assert lib.ahr_graph_workspace_size(ctypes.byref(nl), ctypes.byref(hp), 4, None, ctypes.byref(size)) == A.EDEVICE
    assert size.value == 7


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
def test_hop_tune_values():
    """The hop launch shape: AHR_HOP_AUTO by default, every documented value
    accepted and read back, anything else refused with the setting kept
    (host-only calls)."""
    import paper_2511_10073_amd as A
    lib = A.load()
    saved = A.filter_get_tune()
    try:
        A.filter_tune(A.HOP_AUTO, 0)
        for lanes in (1, 2, 4, 8, 16, 32, 64, A.HOP_ROW_BLOCK, A.HOP_AUTO):
            A.filter_tune(lanes, -1)
            assert A.filter_get_tune() == (lanes, 0)
        A.filter_tune(0, 1)                                   # 0 keeps the shape
        assert A.filter_get_tune() == (A.HOP_AUTO, 1)
        for bad in (3, 128, -2, 512, 2048):
            assert lib.ahr_filter_tune(bad, -1) == A.EINVAL
            assert b"AHR_HOP_AUTO" in lib.ahr_last_error()
            assert A.filter_get_tune() == (A.HOP_AUTO, 1)
    finally:
        A.filter_tune(*saved)


def test_hop_auto_constants_match_the_header():
    import paper_2511_10073_amd as A
    src = open(HEADER).read()
    for name in ("AHR_HOP_AUTO", "AHR_HOP_ROW_BLOCK", "AHR_LAYOUT_AUTO", "AHR_LAYOUT_NETLIST"):
        v = int(re.search(r"#define\s+%s\s+(\d+)" % name, src).group(1))
        assert getattr(A, name[4:]) == v, name
