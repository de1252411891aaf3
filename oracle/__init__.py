"""CPU oracle for single-source shortest paths (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never loads it, and the two share no
code: the oracle is plain C (``oracle.c``) built with gcc, wrapped here with
ctypes and numpy.

What it pins (Sec. 2 problem statement; Sec. 3.2 Alg. 1 and Table 2): the
exact distance array d(s, .), uint64, ``UINT64_MAX`` for unreachable vertices.
All stepping rules reach that same array, so the oracle is the definition
computed by textbook algorithms (binary-heap Dijkstra, Bellman-Ford,
Floyd-Warshall), a linear-time certificate, and the hop depth used by the
extraction bound of Lemma 5.1.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
INF = np.uint64(0xFFFFFFFFFFFFFFFF)

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_dijkstra.argtypes = [i64, p, p, p, ctypes.c_int32, p, i64, p, p]
        lib.oracle_dijkstra.restype = ctypes.c_int
        lib.oracle_bellman_ford.argtypes = [i64, p, p, p, ctypes.c_int32, p]
        lib.oracle_bellman_ford.restype = i64
        lib.oracle_floyd_warshall.argtypes = [i64, p, p, p, p]
        lib.oracle_floyd_warshall.restype = ctypes.c_int
        lib.oracle_certificate.argtypes = [i64, p, p, p, ctypes.c_int32, p, p]
        lib.oracle_certificate.restype = ctypes.c_int
        lib.oracle_hop_depth.argtypes = [i64, p, p, p, ctypes.c_int32, p, p]
        lib.oracle_hop_depth.restype = i64
        lib.oracle_now.argtypes = []
        lib.oracle_now.restype = ctypes.c_double
        _lib = lib
    return _lib


def _arrays(offsets, targets, weights):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    tgt = np.ascontiguousarray(targets, dtype=np.int32)
    w = np.ascontiguousarray(weights, dtype=np.uint32)
    n = off.shape[0] - 1
    if n <= 0 or off[0] != 0 or off[-1] != tgt.shape[0] or tgt.shape[0] != w.shape[0]:
        raise ValueError("malformed CSR")
    return n, off, tgt, w


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def dijkstra(offsets, targets, weights, source: int, max_settled: int = 0, stats: bool = False):
    """Binary-heap Dijkstra. Returns dist (uint64[n]); with stats=True also
    (settled vertices, arcs scanned)."""
    n, off, tgt, w = _arrays(offsets, targets, weights)
    if not 0 <= source < n:
        raise ValueError("source out of range")
    dist = np.empty(n, dtype=np.uint64)
    settled = ctypes.c_int64(0)
    scanned = ctypes.c_int64(0)
    rc = _load().oracle_dijkstra(n, _ptr(off), _ptr(tgt), _ptr(w), int(source), _ptr(dist), int(max_settled),
                                 ctypes.byref(settled), ctypes.byref(scanned))
    if rc != 0:
        raise RuntimeError("oracle_dijkstra failed")
    if stats:
        return dist, settled.value, scanned.value
    return dist


def bellman_ford(offsets, targets, weights, source: int):
    """Brute-force Bellman-Ford (tiny graphs). Returns dist (uint64[n])."""
    n, off, tgt, w = _arrays(offsets, targets, weights)
    dist = np.empty(n, dtype=np.uint64)
    r = _load().oracle_bellman_ford(n, _ptr(off), _ptr(tgt), _ptr(w), int(source), _ptr(dist))
    if r < 0:
        raise RuntimeError("oracle_bellman_ford failed")
    return dist


def floyd_warshall(offsets, targets, weights):
    """All-pairs distances (n x n, uint64) by Floyd-Warshall (tiny graphs)."""
    n, off, tgt, w = _arrays(offsets, targets, weights)
    D = np.empty((n, n), dtype=np.uint64)
    if _load().oracle_floyd_warshall(n, _ptr(off), _ptr(tgt), _ptr(w), _ptr(D)) != 0:
        raise RuntimeError("oracle_floyd_warshall failed")
    return D


def certificate(offsets, targets, weights, source: int, dist):
    """Returns (code, witness): code 0 = dist is the exact distance array;
    1 = dist[source] != 0; 2 = a tense arc into `witness`; 3 = `witness` has a
    finite distance but no tight path from the source."""
    n, off, tgt, w = _arrays(offsets, targets, weights)
    d = np.ascontiguousarray(dist, dtype=np.uint64)
    if d.shape[0] != n:
        raise ValueError("dist has the wrong length")
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_certificate(n, _ptr(off), _ptr(tgt), _ptr(w), int(source), _ptr(d), ctypes.byref(bad))
    if rc == 4:
        raise MemoryError("oracle_certificate")
    return rc, bad.value


def hop_depth(offsets, targets, weights, source: int, dist):
    """Returns (hop int32[n] with -1 for unreachable, k_n = max hop)."""
    n, off, tgt, w = _arrays(offsets, targets, weights)
    d = np.ascontiguousarray(dist, dtype=np.uint64)
    hop = np.empty(n, dtype=np.int32)
    k = _load().oracle_hop_depth(n, _ptr(off), _ptr(tgt), _ptr(w), int(source), _ptr(d), _ptr(hop))
    if k < 0:
        raise MemoryError("oracle_hop_depth")
    return hop, int(k)


def distinct_finite(dist) -> int:
    """Number of distinct finite values in a distance array: the exact step
    count of the theta = min rule when every weight is >= 1 (Table 2, Dijkstra
    row: equal keys are extracted together, and each extracted key is final)."""
    d = np.asarray(dist, dtype=np.uint64)
    return int(np.unique(d[d != INF]).shape[0])


def reachable_arcs(offsets, dist) -> int:
    """Sum of out-degrees of reachable vertices: the arcs relaxed when every
    reachable vertex is extracted exactly once."""
    off = np.asarray(offsets, dtype=np.int64)
    d = np.asarray(dist, dtype=np.uint64)
    deg = off[1:] - off[:-1]
    return int(deg[d != INF].sum())


def now() -> float:
    return _load().oracle_now()
