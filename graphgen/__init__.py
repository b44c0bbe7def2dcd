"""Seeded synthetic input graphs: R-MAT and 2D random geometric graphs.

Input preparation only: nothing here computes any step of the partitioning
method.  Graphs come back as symmetric CSR numpy arrays (int64 row offsets,
int32 neighbour ids, rows ascending, no self-loops or duplicates) with unit
weights, which both the oracle and the device library consume.

The workload recipes below fix the shapes of the synthetic inputs that stand
in for the paper's web, social and citation networks (Table 1), which are not
available here.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import weakref
from dataclasses import dataclass
from fractions import Fraction
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
        )
    return _LIB


class _Csr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("rp", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_rmat.argtypes = [
            ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_Csr),
        ]
        lib.gg_rgg.restype = ctypes.c_int
        lib.gg_rgg.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(_Csr)]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [ctypes.c_void_p]
        lib.gg_set_progress.restype = None
        lib.gg_set_progress.argtypes = [ctypes.c_int]
        lib.gg_draw_u64.restype = ctypes.c_uint64
        lib.gg_draw_u64.argtypes = [ctypes.c_uint64] * 4
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric CSR graph with integer weights (host arrays)."""

    row_ptr: np.ndarray            # int64[n+1]
    col: np.ndarray                # int32[m]
    ew: Optional[np.ndarray] = None  # int32[m]; None = unit edge weights
    nw: Optional[np.ndarray] = None  # int32 or int64[n]; None = unit node weights
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def node_weights(self) -> np.ndarray:
        if self.nw is None:
            return np.ones(self.n, dtype=np.int64)
        return self.nw.astype(np.int64)

    def edge_weights(self) -> np.ndarray:
        if self.ew is None:
            return np.ones(self.m, dtype=np.int32)
        return self.ew


def _take(out: _Csr) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    n, m = out.n, out.m
    rp = np.ctypeslib.as_array(out.rp, shape=(n + 1,))
    col = np.ctypeslib.as_array(out.col, shape=(max(m, 1),))[:m]
    rp_addr = ctypes.cast(out.rp, ctypes.c_void_p).value
    col_addr = ctypes.cast(out.col, ctypes.c_void_p).value
    weakref.finalize(rp, lib.gg_free, rp_addr)
    weakref.finalize(col, lib.gg_free, col_addr)
    return rp, col


def rmat_thresholds(a: str = "0.57", b: str = "0.19", c: str = "0.19") -> tuple[int, int, int]:
    """Quadrant thresholds floor(p * 2^32) of the cumulative probabilities."""
    fa, fb, fc = Fraction(a), Fraction(b), Fraction(c)
    t = [math.floor(x * (1 << 32)) for x in (fa, fa + fb, fa + fb + fc)]
    return t[0], t[1], t[2]


def rmat(scale: int, edge_factor: int, seed: int = 1, n: Optional[int] = None,
         abc: tuple[str, str, str] = ("0.57", "0.19", "0.19")) -> Graph:
    """R-MAT graph: edge_factor * n samples over a 2^scale grid, symmetrized,
    self-loops and duplicates removed.  With n < 2^scale, samples with an
    endpoint >= n are redrawn."""
    nn = (1 << scale) if n is None else int(n)
    ns = edge_factor * nn
    ta, tab, tabc = rmat_thresholds(*abc)
    out = _Csr()
    rc = _load().gg_rmat(scale, nn, ns, seed, ta, tab, tabc, ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"gg_rmat failed ({rc})")
    rp, col = _take(out)
    return Graph(rp, col, name=f"rmat-s{scale}-ef{edge_factor}-n{nn}-seed{seed}")


def rgg(n: int, avg_degree: float, seed: int = 1) -> Graph:
    """2D random geometric graph with radius sqrt(avg_degree / (pi n))."""
    out = _Csr()
    rc = _load().gg_rgg(int(n), float(avg_degree), seed, ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"gg_rgg failed ({rc})")
    rp, col = _take(out)
    return Graph(rp, col, name=f"rgg-n{n}-d{avg_degree}-seed{seed}")


def set_progress(on: bool) -> None:
    """Print a line to stderr after every phase of a generation."""
    _load().gg_set_progress(1 if on else 0)


def draw_u64(seed: int, tag: int, i: int, j: int) -> int:
    return int(_load().gg_draw_u64(seed, tag, i, j))


# ----------------------------------------------------------------------------
# Workload recipes (shapes of the synthetic stand-ins).
# ----------------------------------------------------------------------------

_MASK = (1 << 64) - 1


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


class Stream:
    """Counter-based SplitMix64 stream for workload parameters (Python side)."""

    def __init__(self, seed: int, tag: int):
        self.key = _mix((_mix((seed * 0x9E3779B97F4A7C15 + tag) & _MASK)) & _MASK)
        self.j = 0

    def u64(self) -> int:
        self.j += 1
        return _mix((self.key + self.j * 0x9E3779B97F4A7C15) & _MASK)

    def uniform(self) -> float:
        return (self.u64() >> 11) * (1.0 / (1 << 53))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + self.u64() % (hi - lo + 1)


@dataclass
class JobSpec:
    kind: str          # "rmat" | "rgg"
    n: int
    k: int
    seed: int
    edge_factor: int = 0
    avg_degree: float = 0.0

    def make(self) -> Graph:
        if self.kind == "rmat":
            scale = max(1, math.ceil(math.log2(self.n)))
            return rmat(scale, self.edge_factor, seed=self.seed, n=self.n)
        return rgg(self.n, self.avg_degree, seed=self.seed)


def batch_specs(count: int = 512, seed: int = 3, lg_lo: int = 8, lg_hi: int = 16) -> list[JobSpec]:
    """Mixed batch: n = floor(2^(lg_lo + (lg_hi-lg_lo) u)), half R-MAT (edge
    factor uniform in 4..32), half RGG (average degree uniform in [6, 12]),
    k uniform in {2, 4, 8, 16}."""
    st = Stream(seed, 0x4241544348)  # "BATCH"
    out = []
    for i in range(count):
        u = st.uniform()
        n = int(math.floor(2.0 ** (lg_lo + (lg_hi - lg_lo) * u)))
        k = [2, 4, 8, 16][st.randint(0, 3)]
        if i % 2 == 0:
            out.append(JobSpec("rmat", n, k, seed + 1 + i, edge_factor=st.randint(4, 32)))
        else:
            out.append(JobSpec("rgg", n, k, seed + 1 + i, avg_degree=6.0 + 6.0 * st.uniform()))
    return out


def serve_specs(count: int = 10000, seed: int = 4, lg_lo: int = 10, lg_hi: int = 20) -> list[JobSpec]:
    """Served stream: n log-uniform in [2^lg_lo, 2^lg_hi], R-MAT (edge factor
    16) and RGG (average degree 8) alternating, k a power of two in 2..64."""
    st = Stream(seed, 0x5345525645)  # "SERVE"
    out = []
    for i in range(count):
        u = st.uniform()
        n = int(math.floor(2.0 ** (lg_lo + (lg_hi - lg_lo) * u)))
        k = 1 << st.randint(1, 6)
        if i % 2 == 0:
            out.append(JobSpec("rmat", n, k, seed + 1 + i, edge_factor=16))
        else:
            out.append(JobSpec("rgg", n, k, seed + 1 + i, avg_degree=8.0))
    return out


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    st = Stream(seed, 0x504F4953)  # "POIS"
    t = 0.0
    out = np.empty(count, dtype=np.float64)
    for i in range(count):
        t += -math.log(1.0 - st.uniform()) / rate_per_s
        out[i] = t
    return out


def config1_graph() -> Graph:
    """R-MAT scale 14, edge factor 8, seed 1."""
    return rmat(14, 8, seed=1)


def config2_graphs() -> list[Graph]:
    """R-MAT scale 22 (edge factor 16) and RGG with n = 2^22, degree 10."""
    return [rmat(22, 16, seed=1), rgg(1 << 22, 10.0, seed=1)]
