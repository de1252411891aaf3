"""ctypes binding of libsssp.so (include/sssp.h), same names as the C ABI.

Argument marshalling only: every step of the shortest-path computation runs
in the library's HIP kernels. If the library is missing this module raises;
there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_REPO = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libsssp.so")
SOURCES = [os.path.join(_HERE, "csrc", "stepping.hip"), os.path.join(_HERE, "csrc", "graph.hip")]
HEADER = os.path.join(_REPO, "include", "sssp.h")
CEIL_LIB_PATH = os.path.join(_HERE, "libsssp_ceilings.so")
CEIL_SOURCES = [os.path.join(_HERE, "csrc", "ceilings.hip")]
CEIL_HEADER = os.path.join(_REPO, "include", "sssp_ceilings.h")

HIPCC_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# Bytes of the static workspace array behind sssp_solve_noalloc
SSSP_NOALLOC_SCRATCH_BYTES = 64 << 20

# Status codes (sssp_status)
SSSP_OK = 0
SSSP_ERR_INVALID_ARGUMENT = 1
SSSP_ERR_INVALID_GRAPH = 2
SSSP_ERR_OUT_OF_MEMORY = 3
SSSP_ERR_NO_DEVICE = 4
SSSP_ERR_DEVICE = 5
SSSP_ERR_STEP_LIMIT = 6
SSSP_ERR_UNSUPPORTED = 7
SSSP_ERR_CANCELLED = 8

# Rules (sssp_rule)
SSSP_RULE_RHO = 0
SSSP_RULE_DELTA_STAR = 1
SSSP_RULE_BF = 2
SSSP_RULE_MIN = 3
SSSP_RULE_RHO_EXACT = 4

SSSP_OFFSETS_I32 = 0
SSSP_OFFSETS_I64 = 1

SSSP_INPUT_HOST = 0x1
SSSP_INPUT_DEVICE = 0x2
SSSP_TRUST_INPUT = 0x4
SSSP_KEEP_ORDER = 0x8
SSSP_UNDIRECTED = 0x10
SSSP_BORROW_DEVICE = 0x20
SSSP_SOLVE_SNAPSHOT_KEYS = 0x1
SSSP_SERVE_HASH = 0x1


class sssp_tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_uint32), ("hub_degree", ctypes.c_uint32),
                ("chunk_edges", ctypes.c_uint32), ("list_divisor", ctypes.c_uint32),
                ("sample_cap", ctypes.c_uint32), ("probe_cap", ctypes.c_uint32),
                ("no_filter", ctypes.c_uint32), ("teams", ctypes.c_uint32),
                ("local_budget", ctypes.c_uint32), ("super_sparse_degree", ctypes.c_uint32),
                ("pull", ctypes.c_uint32), ("group_max", ctypes.c_uint32), ("queue", ctypes.c_uint32),
                ("repeat_skip", ctypes.c_uint32), ("hub_defer_degree", ctypes.c_uint32),
                ("hub_defer_div", ctypes.c_uint32), ("group_min", ctypes.c_uint32)]


class sssp_step_record(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_uint64), ("q", ctypes.c_uint64), ("extracted", ctypes.c_uint64),
                ("edges", ctypes.c_uint64), ("successes", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("samples", ctypes.c_uint32), ("local", ctypes.c_uint64), ("extract_ns", ctypes.c_uint64),
                ("relax_ns", ctypes.c_uint64)]


class sssp_params(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("rho", ctypes.c_uint64),
                ("delta", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("max_steps", ctypes.c_uint64),
                ("tuning", ctypes.POINTER(sssp_tuning)), ("extract_counts", ctypes.c_void_p),
                ("trace", ctypes.c_void_p), ("trace_capacity", ctypes.c_uint64)]


class sssp_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("extracted", ctypes.c_uint64), ("edges_relaxed", ctypes.c_uint64),
                ("writemin_success", ctypes.c_uint64), ("dense_steps", ctypes.c_uint64),
                ("sampled_steps", ctypes.c_uint64), ("device_ms", ctypes.c_double),
                ("phase_ms", ctypes.c_double * 4), ("relax_wg_ms", ctypes.c_double * 2),
                ("teams", ctypes.c_uint64), ("queue_dense", ctypes.c_uint64), ("queue_list", ctypes.c_uint64),
                ("list_appends", ctypes.c_uint64), ("local_vertices", ctypes.c_uint64),
                ("repeat_skipped", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        d["relax_wg_ms"] = list(self.relax_wg_ms)
        return d


class sssp_server_load(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_uint64), ("row_bytes", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("teams", ctypes.c_uint64), ("waiting", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("held", ctypes.c_uint64), ("free_rows", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile libsssp.so and libsssp_ceilings.so for gfx950 with hipcc (in-tree)."""
    for path, srcs in ((LIB_PATH, SOURCES), (CEIL_LIB_PATH, CEIL_SOURCES)):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["hipcc", *HIPCC_FLAGS, *srcs, "-o", tmp])
            os.replace(tmp, path)
    return LIB_PATH


_ceil = None


def ceilings_lib():
    """Load libsssp_ceilings.so (the memory-ceiling microbenchmarks; raises
    if it has not been built)."""
    global _ceil
    if _ceil is None:
        if not os.path.exists(CEIL_LIB_PATH):
            raise RuntimeError(f"{CEIL_LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(CEIL_LIB_PATH)
        vp = ctypes.c_void_p
        L.sssp_ceiling_gather16.argtypes = [vp, ctypes.c_uint64, vp, vp, vp]
        L.sssp_ceiling_gather16.restype = ctypes.c_int
        L.sssp_ceiling_atomic_min64.argtypes = [vp, ctypes.c_uint64, vp, vp]
        L.sssp_ceiling_atomic_min64.restype = ctypes.c_int
        _ceil = L
    return _ceil


_lib = None


def lib():
    """Load libsssp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.sssp_default_params.argtypes = [ctypes.POINTER(sssp_params)]
        L.sssp_default_params.restype = None
        L.sssp_graph_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, vp, vp, vp, ctypes.c_uint32,
                                        vp, ctypes.POINTER(vp)]
        L.sssp_graph_create.restype = ctypes.c_int
        L.sssp_graph_destroy.argtypes = [vp]
        L.sssp_graph_destroy.restype = ctypes.c_int
        L.sssp_graph_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_uint64)]
        L.sssp_graph_info.restype = ctypes.c_int
        L.sssp_solve.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(sssp_params), vp, vp,
                                 ctypes.POINTER(sssp_stats)]
        L.sssp_solve.restype = ctypes.c_int
        L.sssp_solve_noalloc.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(sssp_params), vp, vp,
                                         ctypes.POINTER(sssp_stats)]
        L.sssp_solve_noalloc.restype = ctypes.c_int
        L.sssp_solve_async.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(sssp_params), vp, vp]
        L.sssp_solve_async.restype = ctypes.c_int
        L.sssp_solve_query.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.sssp_solve_query.restype = ctypes.c_int
        L.sssp_solve_wait.argtypes = [vp, ctypes.POINTER(sssp_stats)]
        L.sssp_solve_wait.restype = ctypes.c_int
        L.sssp_solve_cancel.argtypes = [vp]
        L.sssp_solve_cancel.restype = ctypes.c_int
        L.sssp_status_string.argtypes = [ctypes.c_int]
        L.sssp_status_string.restype = ctypes.c_char_p
        L.sssp_last_error.argtypes = []
        L.sssp_last_error.restype = ctypes.c_char_p
        L.sssp_abi_version.argtypes = []
        L.sssp_abi_version.restype = ctypes.c_int
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.sssp_row_hash.argtypes = [vp, ctypes.c_int64, vp, u64p]
        L.sssp_row_hash.restype = ctypes.c_int
        L.sssp_server_start.argtypes = [vp, ctypes.POINTER(sssp_params), vp, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
        L.sssp_server_start.restype = ctypes.c_int
        L.sssp_server_start_budget.argtypes = [vp, ctypes.POINTER(sssp_params), ctypes.c_uint64, ctypes.c_uint32,
                                               ctypes.c_uint32, vp, ctypes.POINTER(vp)]
        L.sssp_server_start_budget.restype = ctypes.c_int
        L.sssp_server_enqueue.argtypes = [vp, ctypes.c_int32, u64p]
        L.sssp_server_enqueue.restype = ctypes.c_int
        L.sssp_server_result.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
        L.sssp_server_result.restype = ctypes.c_int
        L.sssp_server_release.argtypes = [vp, ctypes.c_uint64]
        L.sssp_server_release.restype = ctypes.c_int
        L.sssp_server_take.argtypes = [vp, ctypes.c_uint64, vp, vp]
        L.sssp_server_take.restype = ctypes.c_int
        L.sssp_server_counts.argtypes = [vp, ctypes.POINTER(sssp_server_load)]
        L.sssp_server_counts.restype = ctypes.c_int
        L.sssp_server_submit.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32, u64p]
        L.sssp_server_submit.restype = ctypes.c_int
        L.sssp_server_poll.argtypes = [vp, u64p, u64p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        L.sssp_server_poll.restype = ctypes.c_int
        L.sssp_server_stop.argtypes = [vp, ctypes.POINTER(sssp_stats)]
        L.sssp_server_stop.restype = ctypes.c_int
        L.sssp_server_destroy.argtypes = [vp]
        L.sssp_server_destroy.restype = ctypes.c_int
        _lib = L
    return _lib


# Same-named thin wrappers over the C entry points.

def sssp_default_params() -> sssp_params:
    p = sssp_params()
    lib().sssp_default_params(ctypes.byref(p))
    return p


def sssp_graph_create(n, m, ow, offsets_ptr, targets_ptr, weights_ptr, flags, stream_ptr):
    """Returns (status, handle or None)."""
    h = ctypes.c_void_p()
    rc = lib().sssp_graph_create(int(n), int(m), int(ow), offsets_ptr, targets_ptr, weights_ptr, int(flags),
                                 stream_ptr, ctypes.byref(h))
    return rc, (h if rc == SSSP_OK else None)


def sssp_graph_destroy(handle) -> int:
    return lib().sssp_graph_destroy(handle)


def sssp_graph_info(handle):
    n = ctypes.c_int64()
    m = ctypes.c_int64()
    b = ctypes.c_uint64()
    rc = lib().sssp_graph_info(handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(b))
    return rc, n.value, m.value, b.value


def sssp_solve(handle, sources_ptr, n_src, params: sssp_params, dist_ptr, stream_ptr, stats: sssp_stats | None):
    return lib().sssp_solve(handle, sources_ptr, int(n_src), ctypes.byref(params) if params is not None else None,
                            dist_ptr, stream_ptr, ctypes.byref(stats) if stats is not None else None)


def sssp_solve_noalloc(handle, sources_ptr, n_src, params: sssp_params, dist_ptr, stream_ptr,
                       stats: sssp_stats | None):
    return lib().sssp_solve_noalloc(handle, sources_ptr, int(n_src),
                                    ctypes.byref(params) if params is not None else None, dist_ptr, stream_ptr,
                                    ctypes.byref(stats) if stats is not None else None)


def sssp_solve_async(handle, sources_ptr, n_src, params: sssp_params, dist_ptr, stream_ptr):
    return lib().sssp_solve_async(handle, sources_ptr, int(n_src),
                                  ctypes.byref(params) if params is not None else None, dist_ptr, stream_ptr)


def sssp_solve_query(handle):
    """Returns (status, done)."""
    d = ctypes.c_int()
    rc = lib().sssp_solve_query(handle, ctypes.byref(d))
    return rc, d.value


def sssp_solve_wait(handle, stats: sssp_stats | None):
    return lib().sssp_solve_wait(handle, ctypes.byref(stats) if stats is not None else None)


def sssp_solve_cancel(handle):
    return lib().sssp_solve_cancel(handle)


def sssp_row_hash(dist_ptr, n, stream_ptr):
    """Returns (status, checksum)."""
    h = ctypes.c_uint64()
    rc = lib().sssp_row_hash(dist_ptr, int(n), stream_ptr, ctypes.byref(h))
    return rc, h.value


def sssp_server_start(handle, params: sssp_params, dist_ptr, rows, ring_capacity, flags, idle_ms, stream_ptr):
    """Returns (status, server handle or None)."""
    s = ctypes.c_void_p()
    rc = lib().sssp_server_start(handle, ctypes.byref(params) if params is not None else None, dist_ptr, int(rows),
                                 int(ring_capacity), int(flags), int(idle_ms), stream_ptr, ctypes.byref(s))
    return rc, (s if rc == SSSP_OK else None)


def sssp_server_start_budget(handle, params: sssp_params, budget_bytes, flags, idle_ms, stream_ptr):
    """Returns (status, server handle or None)."""
    s = ctypes.c_void_p()
    rc = lib().sssp_server_start_budget(handle, ctypes.byref(params) if params is not None else None,
                                        int(budget_bytes), int(flags), int(idle_ms), stream_ptr, ctypes.byref(s))
    return rc, (s if rc == SSSP_OK else None)


def sssp_server_enqueue(server, source):
    """Returns (status, ticket)."""
    t = ctypes.c_uint64()
    rc = lib().sssp_server_enqueue(server, int(source), ctypes.byref(t))
    return rc, t.value


def sssp_server_result(server, ticket):
    """Returns (status, device address of the row or None)."""
    p = ctypes.c_void_p()
    rc = lib().sssp_server_result(server, int(ticket), ctypes.byref(p))
    return rc, (p.value if rc == SSSP_OK else None)


def sssp_server_release(server, ticket):
    return lib().sssp_server_release(server, int(ticket))


def sssp_server_take(server, ticket, dst_ptr, stream_ptr):
    return lib().sssp_server_take(server, int(ticket), dst_ptr, stream_ptr)


def sssp_server_counts(server):
    """Returns (status, sssp_server_load)."""
    ld = sssp_server_load()
    rc = lib().sssp_server_counts(server, ctypes.byref(ld))
    return rc, ld


def sssp_server_submit(server, source, row):
    """Returns (status, ticket)."""
    t = ctypes.c_uint64()
    rc = lib().sssp_server_submit(server, int(source), int(row), ctypes.byref(t))
    return rc, t.value


def sssp_server_poll(server, tickets, hashes, max_count):
    """tickets / hashes: ctypes uint64 arrays (hashes may be None). Returns (status, count)."""
    c = ctypes.c_uint32()
    rc = lib().sssp_server_poll(server, tickets, hashes, int(max_count), ctypes.byref(c))
    return rc, c.value


def sssp_server_stop(server, stats: sssp_stats | None):
    return lib().sssp_server_stop(server, ctypes.byref(stats) if stats is not None else None)


def sssp_server_destroy(server) -> int:
    return lib().sssp_server_destroy(server)


def sssp_status_string(s: int) -> str:
    return lib().sssp_status_string(int(s)).decode()


def sssp_last_error() -> str:
    return lib().sssp_last_error().decode()


def sssp_abi_version() -> int:
    return lib().sssp_abi_version()
