"""CPU-side checks of the C ABI: the library loads, exports every entry point
include/selfjoin.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "selfjoin.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(selfjoin_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1809_09930_amd import selfjoin
    return selfjoin.load_library()


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("selfjoin_build_index", "selfjoin_run", "selfjoin_fetch_pairs"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1809_09930_amd import selfjoin
    names = declared_functions()
    assert set(names) == set(selfjoin.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name


def test_default_options(lib):
    from paper_1809_09930_amd import selfjoin
    o = selfjoin.default_options()
    assert o.struct_size == ctypes.sizeof(selfjoin.SjOptions)
    assert (o.k, o.k_min, o.k_max, o.reorder, o.shortc, o.precision) == (0, 4, 8, 1, 1, 0)
    assert (o.batch_pairs, o.min_batches, o.mem_budget) == (0, 0, 0)


@pytest.mark.parametrize("n,d,eps,null_out,msg", [
    (10, 0, 0.5, False, "d must be"),
    (10, 129, 0.5, False, "d must be"),
    (10, 4, float("nan"), False, "epsilon"),
    (10, 4, -1.0, False, "epsilon"),
    (10, 4, 0.0, False, "epsilon"),
    (10, 4, float("inf"), False, "epsilon"),
    (10, 4, 1e200, False, "overflows"),
    (2 ** 32, 4, 0.5, False, "below 2^32"),
    (10, 4, 0.5, True, "out is NULL"),
])
def test_build_rejects_bad_arguments_without_a_gpu(lib, n, d, eps, null_out, msg):
    from paper_1809_09930_amd import selfjoin
    h = ctypes.c_void_p()
    buf = (ctypes.c_float * 8)()
    rc = lib.selfjoin_build_index(ctypes.cast(buf, ctypes.c_void_p), n, d, eps, None, None,
                                  None if null_out else ctypes.byref(h))
    assert rc == selfjoin.SJ_ERR_INVALID_ARG
    assert msg in lib.selfjoin_last_error().decode()
    assert h.value is None


def test_null_handles_are_rejected(lib):
    from paper_1809_09930_amd import selfjoin
    total = ctypes.c_uint64(7)
    assert lib.selfjoin_run(None, None, ctypes.byref(total)) == selfjoin.SJ_ERR_INVALID_ARG
    assert total.value == 7
    info = selfjoin.SjInfo()
    info.struct_size = ctypes.sizeof(info)
    assert lib.selfjoin_get_info(None, ctypes.byref(info)) == selfjoin.SJ_ERR_INVALID_ARG
    nw = ctypes.c_uint64()
    assert lib.selfjoin_fetch_pairs(None, 0, 1, None, None, None, ctypes.byref(nw),
                                    None) == selfjoin.SJ_ERR_INVALID_ARG
    off = (ctypes.c_uint64 * 4)()
    assert lib.selfjoin_fetch_offsets(None, off, None) == selfjoin.SJ_ERR_INVALID_ARG
    lib.selfjoin_free(None)


def test_bad_option_struct_size(lib):
    from paper_1809_09930_amd import selfjoin
    o = selfjoin.default_options()
    o.struct_size = 3
    h = ctypes.c_void_p()
    buf = (ctypes.c_float * 8)()
    rc = lib.selfjoin_build_index(ctypes.cast(buf, ctypes.c_void_p), 2, 4, 0.5, ctypes.byref(o),
                                  None, ctypes.byref(h))
    assert rc == selfjoin.SJ_ERR_INVALID_ARG


@pytest.mark.parametrize("field,value,msg", [("fp32_form", 3, "fp32_form"),
                                             ("sortidu", 2, "sortidu"),
                                             ("precision", 7, "precision")])
def test_bad_option_values(lib, field, value, msg):
    from paper_1809_09930_amd import selfjoin
    o = selfjoin.default_options()
    setattr(o, field, value)
    h = ctypes.c_void_p()
    buf = (ctypes.c_float * 8)()
    rc = lib.selfjoin_build_index(ctypes.cast(buf, ctypes.c_void_p), 2, 4, 0.5, ctypes.byref(o),
                                  None, ctypes.byref(h))
    assert rc == selfjoin.SJ_ERR_INVALID_ARG
    assert msg in lib.selfjoin_last_error().decode()
    assert h.value is None


def test_short_option_struct_takes_defaults(lib):
    """A caller built against the header before fp32_form passes the shorter
    struct; the call validates like the defaults (it reaches the argument
    checks, which reject the NULL handle pointer here)."""
    from paper_1809_09930_amd import selfjoin
    o = selfjoin.default_options()
    o.struct_size = selfjoin.SjOptions.fp32_form.offset
    buf = (ctypes.c_float * 8)()
    rc = lib.selfjoin_build_index(ctypes.cast(buf, ctypes.c_void_p), 2, 4, 0.5, ctypes.byref(o),
                                  None, None)
    assert rc == selfjoin.SJ_ERR_INVALID_ARG
    assert "struct_size" not in lib.selfjoin_last_error().decode()


def test_build_query_rejects_null_arguments(lib):
    """Argument checks of the general join entry point run before any device
    call, so they hold without a GPU."""
    from paper_1809_09930_amd import selfjoin
    h = ctypes.c_void_p()
    buf = (ctypes.c_float * 8)()
    rc = lib.selfjoin_build_query(None, ctypes.cast(buf, ctypes.c_void_p), 2, None,
                                  ctypes.byref(h))
    assert rc == selfjoin.SJ_ERR_INVALID_ARG and h.value is None
    assert "NULL" in lib.selfjoin_last_error().decode()
    rc = lib.selfjoin_build_query(ctypes.cast(buf, ctypes.c_void_p),
                                  ctypes.cast(buf, ctypes.c_void_p), 2, None, None)
    assert rc == selfjoin.SJ_ERR_INVALID_ARG


def test_default_options_leave_sortidu_off(lib):
    from paper_1809_09930_amd import selfjoin
    o = selfjoin.default_options()
    assert (o.sortidu, o.fp32_form) == (0, selfjoin.SJ_FP32_AUTO)
