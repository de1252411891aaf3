"""Seeded synthetic graph generators (inputs only; no shortest-path arithmetic).

Both the CPU oracle and the GPU library consume what this module produces.
The generators are C++ (``graphgen.cpp``, built with g++ and OpenMP) driven by
SplitMix64 counter streams, so a graph is a deterministic function of its
parameters, whatever the thread count.

The workload recipes at the bottom stand in for the paper's datasets (Sec. 7,
"Graphs"): the scale-free graphs take uniform integer weights in [1, 2^18),
the road-like graphs take rounded Euclidean lengths.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")

_lib = None


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("targets", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        P = ctypes.POINTER(_Csr)
        lib.gg_free.argtypes = [P]
        lib.gg_grid2d.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint64, P]
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_int, P]
        lib.gg_road.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, P]
        lib.gg_knn.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                               ctypes.c_double, ctypes.c_uint64, P]
        lib.gg_components.argtypes = [P, p]
        lib.gg_components.restype = ctypes.c_int64
        lib.gg_largest_component.argtypes = [P, p]
        lib.gg_largest_component.restype = ctypes.c_int64
        lib.gg_pick_sources.argtypes = [ctypes.c_int64, p, ctypes.c_uint64, ctypes.c_int32, p]
        lib.gg_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, p]
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Directed graph in CSR form: offsets int64[n+1], targets int32[m],
    weights uint32[m]. Rows are sorted by target; the graphs made here are
    symmetric (both arcs of a pair carry the same weight)."""

    offsets: np.ndarray
    targets: np.ndarray
    weights: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.targets.shape[0])

    def degrees(self) -> np.ndarray:
        return self.offsets[1:] - self.offsets[:-1]

    def _struct(self) -> _Csr:
        s = _Csr()
        s.n, s.m = self.n, self.m
        s.offsets = self.offsets.ctypes.data
        s.targets = self.targets.ctypes.data
        s.weights = self.weights.ctypes.data
        return s


def from_arcs(n: int, src, dst, w, name: str = "") -> CSR:
    """CSR from an arc list (kept as given: no symmetrisation or dedupe);
    arcs are ordered by (source, position in the list)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int32)
    w = np.asarray(w, dtype=np.uint32)
    order = np.argsort(src, kind="stable")
    counts = np.bincount(src, minlength=n).astype(np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return CSR(off, np.ascontiguousarray(dst[order]), np.ascontiguousarray(w[order]), name)


def _take(s: _Csr, name: str) -> CSR:
    try:
        n, m = s.n, s.m
        off = np.ctypeslib.as_array(ctypes.cast(s.offsets, ctypes.POINTER(ctypes.c_int64)), (n + 1,)).copy()
        if m > 0:
            tgt = np.ctypeslib.as_array(ctypes.cast(s.targets, ctypes.POINTER(ctypes.c_int32)), (m,)).copy()
            w = np.ctypeslib.as_array(ctypes.cast(s.weights, ctypes.POINTER(ctypes.c_uint32)), (m,)).copy()
        else:
            tgt = np.zeros(0, dtype=np.int32)
            w = np.zeros(0, dtype=np.uint32)
    finally:
        _load().gg_free(ctypes.byref(s))
    return CSR(off, tgt, w, name)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"graphgen {what} failed (code {rc})")


def grid2d(width: int, height: int, wlo: int = 1, whi: int = 1 << 16, seed: int = 1) -> CSR:
    s = _Csr()
    _check(_load().gg_grid2d(width, height, wlo, whi, seed, ctypes.byref(s)), "grid2d")
    return _take(s, f"grid{width}x{height}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         wlo: int = 1, whi: int = 1 << 18, seed: int = 1, relabel: bool = True) -> CSR:
    s = _Csr()
    _check(_load().gg_rmat(scale, edge_factor, a, b, c, wlo, whi, seed, int(relabel), ctypes.byref(s)), "rmat")
    return _take(s, f"rmat{scale}ef{edge_factor}")


def road(width: int, height: int, jitter: float = 0.4, del_frac: float = 0.1, extra_frac: float = 0.01,
         reach: int = 3, wscale: float = 1000.0, seed: int = 1) -> CSR:
    s = _Csr()
    _check(_load().gg_road(width, height, jitter, del_frac, extra_frac, reach, wscale, seed, ctypes.byref(s)),
           "road")
    return _take(s, f"road{width}x{height}")


def knn(clusters: int, per_cluster: int, sigma: float = 0.01, k: int = 10, wscale: float = 1e6,
        seed: int = 1) -> CSR:
    s = _Csr()
    _check(_load().gg_knn(clusters, per_cluster, sigma, k, wscale, seed, ctypes.byref(s)), "knn")
    return _take(s, f"knn{clusters}x{per_cluster}k{k}")


def components(g: CSR):
    """(labels int32[n], count) of the connected components (symmetric graphs)."""
    lab = np.empty(g.n, dtype=np.int32)
    s = g._struct()
    k = _load().gg_components(ctypes.byref(s), lab.ctypes.data)
    return lab, int(k)


def largest_component(g: CSR) -> np.ndarray:
    """bool[n] membership of the largest connected component (symmetric graphs)."""
    mask = np.empty(g.n, dtype=np.uint8)
    s = g._struct()
    _load().gg_largest_component(ctypes.byref(s), mask.ctypes.data)
    return mask.astype(bool)


def pick_sources(n: int, count: int, seed: int, mask=None) -> np.ndarray:
    """`count` seeded uniform vertices (with replacement), within `mask` if given."""
    out = np.empty(count, dtype=np.int32)
    mp = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        mp = mk.ctypes.data
    _check(_load().gg_pick_sources(n, mp, seed, count, out.ctypes.data), "pick_sources")
    return out


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_splitmix64(seed, count, out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Workload recipes. Seeds: graph = 1000 * id + 1, sources = 1000 * id + 3.

@dataclass
class Workload:
    name: str
    graph: CSR
    sources: np.ndarray
    rule: str
    params: dict


def workload(name: str, **overrides) -> Workload:
    """Build one of the named synthetic workloads.

    grid256    : 256 x 256 4-neighbour grid, w ~ U[1, 2^16), source 0, rho = 4096.
    rmat<s>    : R-MAT (0.57, 0.19, 0.19, 0.05) at scale s, edge factor 16,
                 relabelled, symmetrised and deduplicated, w ~ U[1, 2^18);
                 sources uniform in the largest component; rho-stepping.
    road<W>    : W x W jittered grid (+-0.4), 10% of grid edges deleted, 1%
                 extra edges within 3 cells, w = round(1000 * length); source
                 uniform in the largest component; Delta*-stepping / PQ-BF.
    knn<P>     : Gaussian mixture (1000 clusters, sigma 0.01) of P points per
                 cluster, 10-NN, union-symmetrised, w = round(1e6 * dist).
    """
    nsrc = int(overrides.pop("sources", 1))
    if name == "grid256" or name.startswith("grid"):
        side = 256 if name == "grid256" else int(name[4:])
        g = grid2d(side, side, 1, 1 << 16, seed=overrides.pop("seed", 1001))
        src = np.zeros(nsrc, dtype=np.int32)
        return Workload(name, g, src, "rho", {"rho": 4096})
    if name.startswith("rmat"):
        scale = int(name[4:])
        seed = overrides.pop("seed", 2001)
        g = rmat(scale, overrides.pop("edge_factor", 16), seed=seed)
        lcc = largest_component(g)
        src = pick_sources(g.n, nsrc, seed + 2, lcc)
        return Workload(name, g, src, "rho", {"rho": 1 << 20})
    if name.startswith("road"):
        side = int(name[4:])
        seed = overrides.pop("seed", 3001)
        g = road(side, side, seed=seed)
        lcc = largest_component(g)
        src = pick_sources(g.n, nsrc, seed + 2, lcc)
        return Workload(name, g, src, "delta", {"delta": 1 << 15})
    if name.startswith("knn"):
        per = int(name[3:])
        seed = overrides.pop("seed", 4001)
        g = knn(1000, per, 0.01, 10, 1e6, seed=seed)
        src = pick_sources(g.n, nsrc, seed + 2, None)
        return Workload(name, g, src, "rho", {"rho": 1 << 14})
    raise ValueError(f"unknown workload {name}")
