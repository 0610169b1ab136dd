"""The C-ABI library loads and exports every function its header declares;
host-side argument handling that needs no GPU."""

import ctypes
import os
import re
import subprocess

import pytest

from paper_1610_08128_amd import rcm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rcm.h")
SERVER_HEADER = os.path.join(ROOT, "include", "rcm_server.h")
APPLY_HEADER = os.path.join(ROOT, "include", "rcm_apply.h")


def _declared_functions(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rcm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_documented_entry_points():
    assert _declared_functions() == sorted(rcm.EXPORTED)


def test_server_header_declares_the_documented_entry_points():
    from paper_1610_08128_amd import serve

    assert _declared_functions(SERVER_HEADER) == sorted(serve.SERVER_EXPORTED)


def test_library_exports_every_declared_symbol():
    L = rcm.lib()
    declared = (_declared_functions() + _declared_functions(SERVER_HEADER)
                + _declared_functions(APPLY_HEADER))
    for name in declared:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rcm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (rcm_[a-z_]+)", out))
    assert set(declared) <= exported


def test_apply_header_declares_the_documented_entry_points():
    from paper_1610_08128_amd import apply

    assert _declared_functions(APPLY_HEADER) == sorted(apply.APPLY_EXPORTED)
    assert apply.permute_workspace_bytes(0, 0) == 0
    assert 0 < apply.permute_workspace_bytes(1000, 7000) < apply.permute_workspace_bytes(
        1000, 7000, with_values=True)


def test_server_config_checks_need_no_gpu():
    from paper_1610_08128_amd import serve

    with pytest.raises(rcm.RcmError) as e:
        serve.Server(executors=9)
    assert e.value.status == rcm.ERR_INVALID_ARGUMENT
    with pytest.raises(rcm.RcmError) as e:
        serve.Server(max_batch=-1)
    assert e.value.status == rcm.ERR_INVALID_ARGUMENT
    with pytest.raises(rcm.RcmError) as e:
        serve.Server(pp_variant=3)
    assert e.value.status == rcm.ERR_INVALID_ARGUMENT
    # footprint grows with the request
    assert 0 == serve.request_bytes(0, 0)
    assert 0 < serve.request_bytes(100, 500) < serve.request_bytes(1000, 5000)


def test_status_strings():
    for code in range(8):
        s = rcm.status_string(code)
        assert isinstance(s, str) and s
    assert rcm.status_string(99) == "unknown status"


def test_workspace_bytes_is_host_arithmetic():
    assert rcm.workspace_bytes(0, 0) == 0
    a = rcm.workspace_bytes(1000, 5000)
    b = rcm.workspace_bytes(2000, 10000)
    assert 0 < a < b
    assert a % 256 == 0
    # a single graph's workspace does not depend on its entry count; a
    # batch's holds the globalised CSR, so it grows with the entries
    assert rcm.workspace_bytes(1000, 9000) == a
    c = rcm.batched_workspace_bytes(3, 1000, 5000)
    assert 0 < c < rcm.batched_workspace_bytes(3, 1000, 9000)
    assert c % 256 == 0


def test_invalid_arguments_need_no_gpu():
    # rejected before any device work: negative n, bad options
    status, st = rcm.order_raw(-1, 0, 0, 0)
    assert status == rcm.ERR_INVALID_ARGUMENT
    assert st["num_components"] == 0
    status, _ = rcm.order_raw(5, 0, 0, 0)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(pp_variant=2)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(block_threads=1024)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(small_threads=128)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(max_teams=65)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(async_search=-2)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(async_search=2)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(label_mode=3)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(label_team=257)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    bad = rcm.make_options(team_size=257)
    status, _ = rcm.order_raw(0, 0, 0, 0, options=bad)
    assert status == rcm.ERR_INVALID_ARGUMENT
    # n == 0 is a no-op
    status, st = rcm.order_raw(0, 0, 0, 0)
    assert status == rcm.OK and all(v == 0 for v in st.values())


def test_batched_argument_checks_need_no_gpu():
    L = rcm.lib()
    import numpy as np

    vo = np.array([0, 5, 3], np.int64)  # decreasing offsets
    no = np.array([0, 10, 20], np.int64)
    st = (rcm.Stats * 2)()
    status = L.rcm_order_batched(2, vo.ctypes.data_as(ctypes.c_void_p),
                                 no.ctypes.data_as(ctypes.c_void_p), None, None, None,
                                 ctypes.cast(st, ctypes.c_void_p), None, None, 0, None)
    assert status == rcm.ERR_INVALID_ARGUMENT
    status = L.rcm_order_batched(0, None, None, None, None, None, None, None, None, 0, None)
    assert status == rcm.OK
