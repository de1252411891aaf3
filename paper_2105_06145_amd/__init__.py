"""MI355X (gfx950) stepping-algorithm SSSP.

Python face of libsssp.so (include/sssp.h): load a CSR graph onto the GPU,
pick a stepping rule (rho-stepping, Delta*-stepping, Bellman-Ford; Table 2 of
Dong, Gu, Sun and Zhang, SPAA 2021) and solve into a uint64 distance array.
PyTorch supplies device memory and the stream; every step of the loop runs in
the library's HIP kernels.

    import paper_2105_06145_amd as sp
    g = sp.Graph.from_csr(offsets, targets, weights)       # numpy, host
    dist, stats = sp.solve(g, [src], rule="rho", rho=1 << 20)
    d = sp.to_numpy_u64(dist)                              # uint64, UINT64_MAX = unreachable
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _native as N
from ._native import (SSSP_RULE_BF, SSSP_RULE_DELTA_STAR, SSSP_RULE_MIN, SSSP_RULE_RHO, SSSP_RULE_RHO_EXACT,
                      sssp_abi_version,
                      sssp_default_params, sssp_graph_create, sssp_graph_destroy, sssp_graph_info,
                      sssp_last_error, sssp_params, sssp_row_hash, sssp_server_destroy, sssp_server_poll,
                      sssp_server_start, sssp_server_stop, sssp_server_submit, sssp_solve, sssp_solve_async,
                      sssp_solve_noalloc, sssp_solve_cancel, sssp_server_start_budget, sssp_server_enqueue,
                      sssp_server_result, sssp_server_release, sssp_server_take, sssp_server_counts, sssp_solve_query, sssp_solve_wait, sssp_stats,
                      sssp_status_string, sssp_step_record, sssp_tuning)

__all__ = ["Graph", "solve", "solve_async", "PendingSolve", "Server", "row_hash", "SSSPError", "to_numpy_u64", "RULES", "INF", "sssp_graph_create",
           "sssp_graph_destroy", "sssp_graph_info", "sssp_solve", "sssp_status_string", "sssp_last_error",
           "sssp_abi_version", "sssp_default_params", "sssp_params", "sssp_stats", "sssp_tuning",
           "sssp_step_record", "sssp_row_hash", "sssp_server_start", "sssp_server_submit", "sssp_server_poll",
           "sssp_server_stop", "sssp_server_destroy", "sssp_solve_async", "sssp_solve_query", "sssp_solve_wait",
           "sssp_solve_cancel", "sssp_solve_noalloc", "BudgetServer", "sssp_server_start_budget",
           "sssp_server_enqueue", "sssp_server_result", "sssp_server_release", "sssp_server_take",
           "sssp_server_counts"]

INF = 0xFFFFFFFFFFFFFFFF
RULES = {"rho": SSSP_RULE_RHO, "rho_exact": SSSP_RULE_RHO_EXACT, "delta": SSSP_RULE_DELTA_STAR,
         "delta_star": SSSP_RULE_DELTA_STAR,
         "bf": SSSP_RULE_BF, "min": SSSP_RULE_MIN}


class SSSPError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {sssp_status_string(status)} ({sssp_last_error()})")


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _summary(deg, w, reorder: bool) -> dict:
    """Shape summary of a graph for parameter caching: sizes, the log2
    histogram of out-degrees and weight quantiles (numpy or torch inputs)."""
    if hasattr(deg, "cpu"):
        torch = _torch()
        lg = torch.log2(deg.clamp(min=1).double()).floor().long().clamp(max=40)
        hist = torch.bincount(lg, minlength=41).cpu().numpy()
        hist[0] -= int((deg == 0).sum().item())
        zero = int((deg == 0).sum().item())
        ws = w.long() & 0xFFFFFFFF
        if ws.numel() > (1 << 20):
            ws = ws[:: ws.numel() // (1 << 20)]
        q = torch.quantile(ws.double(), torch.tensor([0.1, 0.5, 0.9], dtype=torch.float64, device=ws.device)) \
            if ws.numel() else torch.zeros(3, dtype=torch.float64)
        quant = [int(x) for x in q.cpu().numpy()]
    else:
        zero = int((deg == 0).sum())
        hist = np.bincount(np.floor(np.log2(np.maximum(deg, 1))).astype(np.int64).clip(max=40), minlength=41)
        hist[0] -= zero
        ws = np.asarray(w, dtype=np.uint32)
        if ws.size > (1 << 20):
            ws = ws[:: ws.size // (1 << 20)]
        quant = [int(x) for x in np.quantile(ws.astype(np.float64), [0.1, 0.5, 0.9])] if ws.size else [0, 0, 0]
    hist = [int(x) for x in hist]
    while hist and hist[-1] == 0:
        hist.pop()
    return {"zero_degree": zero, "degree_log2_hist": hist, "weight_q10_50_90": quant, "reorder": bool(reorder)}


class Graph:
    """A CSR graph resident on the current GPU (owned by the library)."""

    def __init__(self, handle, n: int, m: int, summary: dict | None = None):
        self._h = handle
        self.n = n
        self.m = m
        self.summary = {"n": n, "m": m, **(summary or {})}

    @property
    def fingerprint(self) -> str:
        """Stable hash of the graph's shape summary (sizes, degree histogram,
        weight quantiles, vertex order): graphs that share it are tuned alike."""
        import hashlib
        import json
        return hashlib.sha1(json.dumps(self.summary, sort_keys=True).encode()).hexdigest()[:16]

    @classmethod
    def from_csr(cls, offsets, targets, weights, validate: bool = True, reorder: bool = True,
                 undirected: bool = False, borrow: bool = False, stream=None) -> "Graph":
        """offsets (n+1, int32 or int64), targets (m, int32), weights (m,
        uint32): numpy arrays (host) or torch CUDA tensors (device). The
        library copies them into its own layout (renumbered by decreasing
        degree unless reorder=False; results always use the caller's ids).
        undirected=True asserts symmetric arcs (checked unless validate=False)
        and allows bidirectional relaxation (tuning pull=1). borrow=True (torch
        CUDA inputs only) uses the targets and weights tensors in place
        (SSSP_BORROW_DEVICE; caller order kept): the Graph holds references to
        them until it is closed."""
        torch = _torch()
        flags = (0 if validate else N.SSSP_TRUST_INPUT) | (0 if reorder else N.SSSP_KEEP_ORDER) | \
            (N.SSSP_UNDIRECTED if undirected else 0)
        if isinstance(offsets, torch.Tensor):
            if not (offsets.is_cuda and targets.is_cuda and weights.is_cuda):
                raise ValueError("torch inputs must be CUDA tensors")
            ow = N.SSSP_OFFSETS_I64 if offsets.dtype == torch.int64 else N.SSSP_OFFSETS_I32
            if offsets.dtype not in (torch.int32, torch.int64) or targets.dtype != torch.int32 or \
                    weights.dtype not in (torch.int32, torch.uint32):
                raise ValueError("dtypes: offsets int32/int64, targets int32, weights uint32 (or int32 bits)")
            offsets, targets, weights = offsets.contiguous(), targets.contiguous(), weights.contiguous()
            summary = _summary(offsets[1:].long() - offsets[:-1].long(), weights, reorder)
            n = offsets.numel() - 1
            m = targets.numel()
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (offsets, targets, weights)]
            flags |= N.SSSP_INPUT_DEVICE | (N.SSSP_BORROW_DEVICE if borrow else 0)
            keep = (offsets, targets, weights)
        else:
            if borrow:
                raise ValueError("borrow=True needs torch CUDA tensors")
            off = np.ascontiguousarray(offsets)
            if off.dtype not in (np.int32, np.int64):
                off = off.astype(np.int64)
            ow = N.SSSP_OFFSETS_I64 if off.dtype == np.int64 else N.SSSP_OFFSETS_I32
            tgt = np.ascontiguousarray(targets, dtype=np.int32)
            w = np.ascontiguousarray(weights, dtype=np.uint32)
            summary = _summary(np.diff(off.astype(np.int64)), w, reorder)
            n = off.shape[0] - 1
            m = tgt.shape[0]
            ptrs = [ctypes.c_void_p(a.ctypes.data) for a in (off, tgt, w)]
            flags |= N.SSSP_INPUT_HOST
            keep = (off, tgt, w)
        rc, h = sssp_graph_create(n, m, ow, ptrs[0], ptrs[1], ptrs[2], flags, _stream_ptr(stream))
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_graph_create")
        G = cls(h, n, m, summary)
        G._borrowed = keep[1:] if borrow else None
        return G

    def device_bytes(self) -> int:
        rc, _, _, b = sssp_graph_info(self._h)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_graph_info")
        return b

    def close(self):
        if getattr(self, "_h", None) is not None:
            sssp_graph_destroy(self._h)
            self._h = None
        self._borrowed = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_tuning(**kw) -> sssp_tuning:
    """An sssp_tuning with the given fields set (the rest zero: library
    defaults). Unknown field names raise ValueError (a ctypes structure would
    otherwise take them as plain attributes and pass nothing on)."""
    names = {f for f, _ in sssp_tuning._fields_}
    t = sssp_tuning()
    for k, v in kw.items():
        if k not in names:
            raise ValueError(f"unknown tuning field {k!r}; known: {', '.join(sorted(names))}")
        setattr(t, k, int(v))
    return t


def _params(rule, rho, delta, seed, tuning, snapshot_keys=False):
    p = sssp_params()
    N.lib().sssp_default_params(ctypes.byref(p))
    p.rule = RULES[rule]
    p.rho = int(rho)
    p.delta = int(delta)
    p.seed = int(seed)
    p.flags = N.SSSP_SOLVE_SNAPSHOT_KEYS if snapshot_keys else 0
    tun = None
    if tuning is not None:
        tun = tuning if isinstance(tuning, sssp_tuning) else make_tuning(**tuning)
        p.tuning = ctypes.pointer(tun)
    return p, tun


def solve(g: Graph, sources, rule: str = "rho", rho: int = 1 << 20, delta: int = 1 << 13, seed: int = 1,
          max_steps: int = 0, tuning: dict | sssp_tuning | None = None, out=None, stream=None,
          trace: int = 0, extract_counts: bool = False, snapshot_keys: bool = False, noalloc: bool = False):
    """Solve from each source. Returns (dist, stats) where dist is a torch
    int64 CUDA tensor (n_src, n) holding uint64 bit patterns (-1 = unreachable)
    and stats is a dict; with trace > 0 stats["trace"] holds per-step records,
    with extract_counts=True stats["extract_counts"] a (n_src, n) int32 tensor.
    snapshot_keys=True relaxes with the keys vertices were extracted with, which
    makes extraction sets independent of WriteMin ordering. noalloc=True
    calls sssp_solve_noalloc (workspace in the library's static scratch
    array, no device allocation by the library)."""
    torch = _torch()
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    ns = int(src.shape[0])
    if out is None:
        out = torch.empty((ns, g.n), dtype=torch.int64, device="cuda")
    elif out.dtype != torch.int64 or out.numel() != ns * g.n or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 CUDA tensor with n_src * n elements")
    p, tun = _params(rule, rho, delta, seed, tuning, snapshot_keys)
    p.max_steps = int(max_steps)
    counts = None
    if extract_counts:
        counts = torch.zeros((ns, g.n), dtype=torch.int32, device="cuda")
        p.extract_counts = counts.data_ptr()
    tr = None
    if trace > 0:
        tr = torch.zeros((int(trace), ctypes.sizeof(sssp_step_record) // 8), dtype=torch.int64, device="cuda")
        p.trace = tr.data_ptr()
        p.trace_capacity = int(trace)
    st = sssp_stats()
    entry = sssp_solve_noalloc if noalloc else sssp_solve
    rc = entry(g._h, ctypes.c_void_p(src.ctypes.data), ns, p, ctypes.c_void_p(out.data_ptr()),
               _stream_ptr(stream), st)
    if rc != N.SSSP_OK:
        raise SSSPError(rc, entry.__name__)
    stats = st.as_dict()
    if counts is not None:
        stats["extract_counts"] = counts
    if tr is not None:
        raw = tr.cpu().numpy().view(np.uint64)
        recs = []
        for i in range(min(int(trace), int(stats["steps"]) if ns == 1 else int(trace))):
            r = raw[i]
            recs.append({"theta": int(r[0]), "q": int(r[1]), "extracted": int(r[2]), "edges": int(r[3]),
                         "successes": int(r[4]), "flags": int(r[5]) & 0xFFFFFFFF, "samples": int(r[5]) >> 32,
                         "local": int(r[6]), "extract_ns": int(r[7]), "relax_ns": int(r[8])})
        stats["trace"] = recs
    return out, stats


class PendingSolve:
    """An asynchronous solve (sssp_solve_async): `out` is complete once the
    stream reaches the end of the launch; wait() returns (out, stats) and ends
    it, cancel() asks it to stop early (wait() then raises SSSPError with
    status SSSP_ERR_CANCELLED unless it had already finished)."""

    def __init__(self, g: Graph, out, keep):
        self.g, self.out, self._keep, self._open = g, out, keep, True

    def done(self) -> bool:
        rc, d = sssp_solve_query(self.g._h)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_solve_query")
        return bool(d)

    def cancel(self):
        if self._open:
            rc = sssp_solve_cancel(self.g._h)
            if rc != N.SSSP_OK:
                raise SSSPError(rc, "sssp_solve_cancel")

    def wait(self):
        if not self._open:
            raise RuntimeError("already waited")
        st = sssp_stats()
        rc = sssp_solve_wait(self.g._h, st)
        self._open = False
        self._keep = None
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_solve_wait")
        return self.out, st.as_dict()


def solve_async(g: Graph, sources, rule: str = "rho", rho: int = 1 << 20, delta: int = 1 << 13, seed: int = 1,
                max_steps: int = 0, tuning: dict | sssp_tuning | None = None, out=None,
                stream=None) -> PendingSolve:
    """Enqueue a solve on `stream` (default: the current torch stream) and
    return at once; see PendingSolve."""
    torch = _torch()
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    ns = int(src.shape[0])
    if out is None:
        out = torch.empty((ns, g.n), dtype=torch.int64, device="cuda")
    elif out.dtype != torch.int64 or out.numel() != ns * g.n or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 CUDA tensor with n_src * n elements")
    p, tun = _params(rule, rho, delta, seed, tuning)
    p.max_steps = int(max_steps)
    rc = sssp_solve_async(g._h, ctypes.c_void_p(src.ctypes.data), ns, p, ctypes.c_void_p(out.data_ptr()),
                          _stream_ptr(stream))
    if rc != N.SSSP_OK:
        raise SSSPError(rc, "sssp_solve_async")
    return PendingSolve(g, out, (p, tun))


def row_hash(row, stream=None) -> int:
    """Order-independent checksum of one device distance row (sssp_row_hash)."""
    rc, h = sssp_row_hash(ctypes.c_void_p(row.data_ptr()), row.numel(), _stream_ptr(stream))
    if rc != N.SSSP_OK:
        raise SSSPError(rc, "sssp_row_hash")
    return h


class Server:
    """A persistent serving launch on one graph (sssp_server_*): requests are
    posted while it runs and finish one by one into rows of `rows`, a
    contiguous int64 CUDA tensor of shape (R, n) owned by the caller. The
    library runs the launch on a hardware queue of its own; `stream` (default:
    the current stream) only orders its start. While it runs, keep GPU work
    off the default (NULL) stream, which HIP makes wait for the server's
    blocking stream: use a side stream (torch.cuda.stream(torch.cuda.Stream()))."""

    def __init__(self, g: Graph, rows, rule: str = "rho", rho: int = 1 << 20, delta: int = 1 << 13, seed: int = 1,
                 tuning: dict | sssp_tuning | None = None, ring_capacity: int = 1024, hash_rows: bool = False,
                 idle_ms: int = 0, stream=None):
        if rows.dtype != _torch().int64 or rows.dim() != 2 or rows.shape[1] != g.n or not rows.is_contiguous():
            raise ValueError("rows must be a contiguous int64 CUDA tensor of shape (R, n)")
        self.g = g
        self.rows = rows
        self.stream = stream if stream is not None else _torch().cuda.current_stream()
        p, self._tun = _params(rule, rho, delta, seed, tuning)
        self._cap = int(ring_capacity)
        rc, self._s = sssp_server_start(g._h, p, ctypes.c_void_p(rows.data_ptr()), rows.shape[0], self._cap,
                                        N.SSSP_SERVE_HASH if hash_rows else 0, idle_ms,
                                        ctypes.c_void_p(self.stream.cuda_stream))
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_start")
        self._t = (ctypes.c_uint64 * self._cap)()
        self._h = (ctypes.c_uint64 * self._cap)()
        self.stats = None

    def submit(self, source: int, row: int) -> int:
        rc, t = sssp_server_submit(self._s, source, row)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_submit")
        return t

    def poll(self) -> list[tuple[int, int]]:
        """(ticket, row checksum) of the requests finished since the last poll."""
        rc, c = sssp_server_poll(self._s, self._t, self._h, self._cap)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_poll")
        return [(self._t[i], self._h[i]) for i in range(c)]

    def stop(self) -> dict:
        st = sssp_stats()
        rc = sssp_server_stop(self._s, st)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_stop")
        self.stats = st.as_dict()
        return self.stats

    def close(self):
        if getattr(self, "_s", None) is not None:
            sssp_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BudgetServer:
    """A serving launch that admits requests by a device-memory budget
    (sssp_server_start_budget): the launch's workspace and as many result
    rows as fit come out of `budget_bytes`; enqueue() always accepts a
    request, which waits until a row is free; a finished request (poll())
    holds its row until take() copies it out or release() gives it back.
    Keep GPU work off the default (NULL) stream while it runs (see Server)."""

    def __init__(self, g: Graph, budget_bytes: int, rule: str = "rho", rho: int = 1 << 20, delta: int = 1 << 13,
                 seed: int = 1, tuning: dict | sssp_tuning | None = None, hash_rows: bool = False, idle_ms: int = 0,
                 stream=None):
        self.g = g
        self.stream = stream if stream is not None else _torch().cuda.current_stream()
        p, self._tun = _params(rule, rho, delta, seed, tuning)
        rc, self._s = sssp_server_start_budget(g._h, p, int(budget_bytes), N.SSSP_SERVE_HASH if hash_rows else 0,
                                               idle_ms, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_start_budget")
        self.rows = self.counts()["rows"]
        self._t = (ctypes.c_uint64 * self.rows)()
        self._h = (ctypes.c_uint64 * self.rows)()
        self.stats = None

    def enqueue(self, source: int) -> int:
        rc, t = sssp_server_enqueue(self._s, source)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_enqueue")
        return t

    def poll(self) -> list[tuple[int, int]]:
        """(ticket, row checksum) of the requests finished since the last poll."""
        rc, c = sssp_server_poll(self._s, self._t, self._h, self.rows)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_poll")
        return [(self._t[i], self._h[i]) for i in range(c)]

    def take(self, ticket: int, out=None, stream=None):
        """Copy a finished request's distances into `out` (an int64 CUDA
        tensor of n elements, allocated if None) and release its row."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.g.n, dtype=torch.int64, device="cuda")
        elif out.dtype != torch.int64 or out.numel() != self.g.n or not out.is_contiguous():
            raise ValueError("out must be a contiguous int64 CUDA tensor with n elements")
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = sssp_server_take(self._s, ticket, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_take")
        return out

    def release(self, ticket: int):
        rc = sssp_server_release(self._s, ticket)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_release")

    def counts(self) -> dict:
        rc, ld = sssp_server_counts(self._s)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_counts")
        return ld.as_dict()

    def stop(self) -> dict:
        st = sssp_stats()
        rc = sssp_server_stop(self._s, st)
        if rc != N.SSSP_OK:
            raise SSSPError(rc, "sssp_server_stop")
        self.stats = st.as_dict()
        return self.stats

    def close(self):
        if getattr(self, "_s", None) is not None:
            sssp_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_numpy_u64(t) -> np.ndarray:
    """Copy a dist tensor to host as uint64."""
    return t.detach().cpu().numpy().view(np.uint64)
