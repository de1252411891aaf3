"""The C-ABI library loads, exports every symbol include/sssp.h declares, and
rejects bad arguments before touching a device. CPU only: no compute call."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2105_06145_amd import _native as N

HEADER = N.HEADER


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sssp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert {"sssp_graph_create", "sssp_graph_destroy", "sssp_solve", "sssp_status_string",
            "sssp_last_error", "sssp_default_params", "sssp_graph_info", "sssp_abi_version",
            "sssp_solve_noalloc", "sssp_server_start_budget"} <= set(names)
    lib = ctypes.CDLL(N.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    # The memory-ceiling microbenchmarks' library and header.
    names = declared_functions(N.CEIL_HEADER)
    assert names == ["sssp_ceiling_atomic_min64", "sssp_ceiling_gather16"]
    lib = ctypes.CDLL(N.CEIL_LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    # Compile a probe against the header with the host C compiler and compare
    # every field offset and struct size with the ctypes mirror.
    structs = [N.sssp_tuning, N.sssp_step_record, N.sssp_params, N.sssp_stats, N.sssp_server_load]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "%s"' % HEADER, "int main(void) {"]
    for S in structs:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (S.__name__, S.__name__))
        for f, _ in S._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (S.__name__, f, S.__name__, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", str(src), "-o", str(exe)])
    got = dict(ln.split() for ln in subprocess.check_output([str(exe)]).decode().splitlines())
    for S in structs:
        assert int(got[S.__name__]) == ctypes.sizeof(S), S.__name__
        for f, _ in S._fields_:
            assert int(got[f"{S.__name__}.{f}"]) == getattr(S, f).offset, (S.__name__, f)


def test_version_strings_defaults():
    assert N.sssp_abi_version() == 4
    assert N.sssp_status_string(N.SSSP_OK) == "ok"
    assert "argument" in N.sssp_status_string(N.SSSP_ERR_INVALID_ARGUMENT)
    assert N.sssp_status_string(99) == "unknown status"
    p = N.sssp_default_params()
    assert p.rule == N.SSSP_RULE_RHO and p.rho == 1 << 20 and p.delta == 1 << 13 and p.max_steps == 0
    assert not p.tuning and not p.trace and not p.extract_counts


def _create(n, m, off, tgt, w, flags=N.SSSP_INPUT_HOST, ow=None):
    off = np.ascontiguousarray(off)
    if ow is None:
        ow = N.SSSP_OFFSETS_I64 if off.dtype == np.int64 else N.SSSP_OFFSETS_I32
    tgt = np.ascontiguousarray(tgt, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    return N.sssp_graph_create(n, m, ow, ctypes.c_void_p(off.ctypes.data), ctypes.c_void_p(tgt.ctypes.data),
                               ctypes.c_void_p(w.ctypes.data), flags, None)


@pytest.mark.parametrize("case,code,needle", [
    ("n0", N.SSSP_ERR_INVALID_ARGUMENT, "n must"),
    ("nbig", N.SSSP_ERR_INVALID_ARGUMENT, "n must"),
    ("mneg", N.SSSP_ERR_INVALID_ARGUMENT, "m must"),
    ("flags", N.SSSP_ERR_INVALID_ARGUMENT, "exactly one"),
    ("off0", N.SSSP_ERR_INVALID_GRAPH, "offsets[0]"),
    ("decrease", N.SSSP_ERR_INVALID_GRAPH, "decrease at index 1"),
    ("offn", N.SSSP_ERR_INVALID_GRAPH, "offsets[n] != m"),
    ("target", N.SSSP_ERR_INVALID_GRAPH, "arc 2"),
    ("negtarget", N.SSSP_ERR_INVALID_GRAPH, "arc 0"),
    ("i32big", N.SSSP_ERR_INVALID_ARGUMENT, "int32 offsets"),
])
def test_graph_create_rejects(case, code, needle):
    off = np.array([0, 2, 3, 3], dtype=np.int64)
    tgt = np.array([1, 2, 0])
    w = np.array([1, 1, 1])
    n, m, flags, ow = 3, 3, N.SSSP_INPUT_HOST, None
    if case == "n0":
        n = 0
    elif case == "nbig":
        n = 1 << 31
    elif case == "mneg":
        m = -1
    elif case == "flags":
        flags = N.SSSP_INPUT_HOST | N.SSSP_INPUT_DEVICE
    elif case == "off0":
        off = np.array([1, 2, 3, 3], dtype=np.int64)
    elif case == "decrease":
        off = np.array([0, 2, 1, 3], dtype=np.int64)
    elif case == "offn":
        off = np.array([0, 2, 3, 4], dtype=np.int64)
        tgt = np.array([1, 2, 0, 0])
        w = np.array([1, 1, 1, 1])
    elif case == "target":
        tgt = np.array([1, 2, 3])
    elif case == "negtarget":
        tgt = np.array([-1, 2, 0])
    elif case == "i32big":
        m = 1 << 31
        ow = N.SSSP_OFFSETS_I32
    rc, h = _create(n, m, off, tgt, w, flags, ow)
    assert rc == code and h is None
    assert needle in N.sssp_last_error()


def test_null_arguments():
    lib = N.lib()
    h = ctypes.c_void_p()
    rc = lib.sssp_graph_create(3, 0, 1, None, None, None, N.SSSP_INPUT_HOST, None, ctypes.byref(h))
    assert rc == N.SSSP_ERR_INVALID_ARGUMENT
    rc = lib.sssp_graph_create(3, 0, 1, None, None, None, N.SSSP_INPUT_HOST, None, None)
    assert rc == N.SSSP_ERR_INVALID_ARGUMENT
    p = N.sssp_default_params()
    assert N.sssp_solve(None, None, 1, p, None, None, None) == N.SSSP_ERR_INVALID_ARGUMENT
    assert "NULL" in N.sssp_last_error()
    assert N.sssp_graph_destroy(None) == N.SSSP_OK
    assert N.sssp_graph_info(None)[0] == N.SSSP_ERR_INVALID_ARGUMENT


def test_serving_and_checksum_null_arguments():
    # Every check here returns before any device call.
    lib = N.lib()
    p = N.sssp_default_params()
    s = ctypes.c_void_p()
    assert lib.sssp_server_start(None, ctypes.byref(p), None, 1, 1, 0, 0, None, None) == N.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_server_start(None, ctypes.byref(p), None, 1, 1, 0, 0, None,
                                 ctypes.byref(s)) == N.SSSP_ERR_INVALID_ARGUMENT
    assert not s.value
    t = ctypes.c_uint64()
    assert lib.sssp_server_submit(None, 0, 0, ctypes.byref(t)) == N.SSSP_ERR_INVALID_ARGUMENT
    c = ctypes.c_uint32()
    assert lib.sssp_server_poll(None, None, None, 0, ctypes.byref(c)) == N.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_server_stop(None, None) == N.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_server_destroy(None) == N.SSSP_OK
    h = ctypes.c_uint64()
    assert lib.sssp_row_hash(None, 5, None, ctypes.byref(h)) == N.SSSP_ERR_INVALID_ARGUMENT
    assert "NULL" in N.sssp_last_error()
    assert lib.sssp_server_start_budget(None, ctypes.byref(p), 1 << 30, 0, 0, None,
                                        ctypes.byref(s)) == N.SSSP_ERR_INVALID_ARGUMENT
    assert not s.value
    assert lib.sssp_server_enqueue(None, 0, ctypes.byref(t)) == N.SSSP_ERR_INVALID_ARGUMENT
    r = ctypes.c_void_p()
    assert lib.sssp_server_result(None, 0, ctypes.byref(r)) == N.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_server_release(None, 0) == N.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_server_take(None, 0, None, None) == N.SSSP_ERR_INVALID_ARGUMENT
    ld = N.sssp_server_load()
    assert lib.sssp_server_counts(None, ctypes.byref(ld)) == N.SSSP_ERR_INVALID_ARGUMENT


def test_async_solve_null_arguments():
    # Every check here returns before any device call.
    p = N.sssp_default_params()
    assert N.sssp_solve_async(None, None, 1, p, None, None) == N.SSSP_ERR_INVALID_ARGUMENT
    assert "NULL" in N.sssp_last_error()
    assert N.sssp_solve_query(None)[0] == N.SSSP_ERR_INVALID_ARGUMENT
    assert N.sssp_solve_wait(None, None) == N.SSSP_ERR_INVALID_ARGUMENT
    assert N.sssp_solve_cancel(None) == N.SSSP_ERR_INVALID_ARGUMENT
    assert N.sssp_status_string(N.SSSP_ERR_CANCELLED) == "cancelled"


def test_graph_create_rejects_unknown_flag_bits():
    lib = N.lib()
    off = np.array([0, 1, 2], dtype=np.int64)
    tgt = np.array([1, 0], dtype=np.int32)
    w = np.array([3, 3], dtype=np.uint32)
    h = ctypes.c_void_p()
    ptrs = [ctypes.c_void_p(a.ctypes.data) for a in (off, tgt, w)]
    rc = lib.sssp_graph_create(2, 2, N.SSSP_OFFSETS_I64, *ptrs, N.SSSP_INPUT_HOST | 0x100, None, ctypes.byref(h))
    assert rc == N.SSSP_ERR_INVALID_ARGUMENT and "flag" in N.sssp_last_error()


def test_noalloc_solve_null_arguments_and_limit():
    # Every check here returns before any device call.
    p = N.sssp_default_params()
    assert N.sssp_solve_noalloc(None, None, 1, p, None, None, None) == N.SSSP_ERR_INVALID_ARGUMENT
    assert "NULL" in N.sssp_last_error()
    text = open(HEADER).read()
    m = re.search(r"#define SSSP_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == N.SSSP_NOALLOC_SCRATCH_BYTES


def test_borrow_needs_device_input():
    off = np.array([0, 1, 2], dtype=np.int64)
    tgt = np.array([1, 0], dtype=np.int32)
    w = np.array([3, 3], dtype=np.uint32)
    rc, h = _create(2, 2, off, tgt, w, N.SSSP_INPUT_HOST | N.SSSP_BORROW_DEVICE)
    assert rc == N.SSSP_ERR_INVALID_ARGUMENT and h is None
    assert "BORROW" in N.sssp_last_error()


def test_tuning_fields_by_name():
    import paper_2105_06145_amd as sp
    t = sp.make_tuning(hub_defer_degree=64, hub_defer_div=300, group_min=4, local_budget=8192)
    assert (t.hub_defer_degree, t.hub_defer_div, t.group_min, t.local_budget) == (64, 300, 4, 8192)
    assert t.teams == 0 and t.queue == 0  # the rest: library defaults
    with pytest.raises(ValueError, match="group_mn"):
        sp.make_tuning(group_mn=4)
