"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/slg.h declares. No compute is launched."""
import ctypes

import pytest

import paper_2201_11326_amd as slg


def test_library_loads_and_exports_header_symbols():
    L = slg.lib()
    names = slg.header_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert slg.version().startswith("slg")


def test_header_and_binding_agree_on_constants():
    text = open(slg.HEADER).read()
    assert f"#define SLG_MAX_S {slg.SLG_MAX_S}" in text
    assert f"#define SLG_VALIDATE {slg.SLG_VALIDATE}u" in text
    for name, code in [("SLG_OK", 0), ("SLG_ERR_INVALID_ARG", 1), ("SLG_ERR_INVALID_GRAPH", 2),
                       ("SLG_ERR_OUT_OF_MEMORY", 3), ("SLG_ERR_DEVICE", 4), ("SLG_ERR_OVERFLOW", 5),
                       ("SLG_ERR_CANCELLED", 6), ("SLG_ERR_TIMEOUT", 7)]:
        assert f"{name} = {code}" in text
        assert getattr(slg, name) == code


def test_null_arguments_are_rejected_on_the_host():
    L = slg.lib()
    assert L.slg_context_destroy(None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_graph_release(None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_plan_destroy(None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_result_free(None) == slg.SLG_ERR_INVALID_ARG
    e = ctypes.c_int64()
    assert L.slg_plan_info(None, 0, ctypes.byref(e), None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_last_error(None) == b"null context"
    assert L.slg_context_create(0, 0, None, None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_server_create(None, 4, 0, None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_server_destroy(None) == slg.SLG_ERR_INVALID_ARG
    t = ctypes.c_uint64()
    assert L.slg_server_submit(None, None, None, 1, ctypes.byref(t)) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_server_wait(None, 1, 0, None, None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_server_next(None, 0, None, None) == slg.SLG_ERR_INVALID_ARG
    assert L.slg_server_stats(None, None, 0, None) == slg.SLG_ERR_INVALID_ARG


def test_request_info_layout_matches_header():
    # uint64 ticket, enum status, int32 attempts, 2 doubles, int64, char[192]
    assert ctypes.sizeof(slg.RequestInfo) == 8 + 4 + 4 + 8 + 8 + 8 + 192
    assert slg.RequestInfo.queue_ms.offset == 16 and slg.RequestInfo.message.offset == 40


def test_context_create_without_gpu_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert slg.lib().slg_context_create(0, 0, None, ctypes.byref(h)) == slg.SLG_ERR_DEVICE
