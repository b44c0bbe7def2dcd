"""ctypes wrapper of the plain CPU oracle (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module.  The product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "sclap_oracle.c"), os.path.join(_HERE, "sclap_extensions.c"),
         os.path.join(_HERE, "seq_sclap.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

MAXLEV = 64
MAXR = 64
MAXCYC = 16

OK, EINVAL, ENOMEM, EOVERFLOW = 0, -1, -2, -3


def _stale() -> bool:
    if not os.path.exists(_LIB):
        return True
    t = os.path.getmtime(_LIB)
    return any(os.path.getmtime(f) > t for f in _SRCS + [os.path.join(_HERE, "sclap_oracle.h")])


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (single-threaded, no OpenMP); with
    force=False only when the library is missing or older than a source."""
    if force or _stale():
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", _LIB] + _SRCS)
    return _LIB


class _G(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64),
        ("rp", ctypes.c_void_p), ("col", ctypes.c_void_p),
        ("ew", ctypes.c_void_p), ("nw", ctypes.c_void_p),
    ]


class _Owned(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64),
        ("rp", ctypes.POINTER(ctypes.c_int64)), ("col", ctypes.POINTER(ctypes.c_int32)),
        ("ew", ctypes.POINTER(ctypes.c_int32)), ("nw", ctypes.POINTER(ctypes.c_int64)),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("n_level", ctypes.c_int64 * MAXLEV), ("m_level", ctypes.c_int64 * MAXLEV),
        ("rounds_c", ctypes.c_int32 * MAXLEV), ("rounds_r", ctypes.c_int32 * MAXLEV),
        ("moved_c", (ctypes.c_int64 * MAXR) * MAXLEV), ("moved_r", (ctypes.c_int64 * MAXR) * MAXLEV),
        ("visits_c", ctypes.c_int64 * MAXLEV), ("visits_r", ctypes.c_int64 * MAXLEV),
        ("lmax", ctypes.c_int64), ("W", ctypes.c_int64), ("U", ctypes.c_int64),
        ("threshold", ctypes.c_int64), ("n_isolated", ctypes.c_int64),
        ("ip_cut", ctypes.c_int64), ("cut", ctypes.c_int64), ("max_block", ctypes.c_int64),
    ]

    def to_dict(self) -> dict:
        L = self.levels
        d = {
            "levels": L,
            "n_level": [self.n_level[i] for i in range(L)],
            "m_level": [self.m_level[i] for i in range(L)],
            "rounds_c": [self.rounds_c[i] for i in range(L)],
            "rounds_r": [self.rounds_r[i] for i in range(L)],
            "moved_c": [[self.moved_c[i][r] for r in range(self.rounds_c[i])] for i in range(L)],
            "moved_r": [[self.moved_r[i][r] for r in range(self.rounds_r[i])] for i in range(L)],
            "visits_c": [self.visits_c[i] for i in range(L)],
            "visits_r": [self.visits_r[i] for i in range(L)],
        }
        for f in ("lmax", "W", "U", "threshold", "n_isolated", "ip_cut", "cut", "max_block"):
            d[f] = getattr(self, f)
        return d


class MLX(ctypes.Structure):
    """Options of the Section 4 extensions (all zero: the plain scheme)."""
    _fields_ = [
        ("vcycles", ctypes.c_int32), ("subrounds", ctypes.c_int32), ("ensemble", ctypes.c_int32),
        ("pad", ctypes.c_int32), ("delta_num", ctypes.c_int64), ("delta_den", ctypes.c_int64),
    ]


class Cycles(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int32), ("best", ctypes.c_int32),
        ("cut", ctypes.c_int64 * MAXCYC), ("max_block", ctypes.c_int64 * MAXCYC),
        ("visits", ctypes.c_int64 * MAXCYC), ("levels", ctypes.c_int32 * MAXCYC),
        ("lmax", (ctypes.c_int64 * MAXLEV) * MAXCYC),
    ]

    def to_dict(self) -> dict:
        c = self.cycles
        return {"cycles": c, "best": self.best, "cut": [self.cut[i] for i in range(c)],
                "max_block": [self.max_block[i] for i in range(c)], "visits": [self.visits[i] for i in range(c)],
                "levels": [self.levels[i] for i in range(c)],
                "lmax": [[self.lmax[i][j] for j in range(self.levels[i])] for i in range(c)]}


_lib = None
_i64p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.orc_bounds.restype = ctypes.c_int
        lib.orc_bounds.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_int64),
                                   P(ctypes.c_int64)]
        lib.orc_rate.restype = None
        lib.orc_rate.argtypes = [P(_G), _i64p, _i64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, _i64p]
        lib.orc_admit_apply.restype = ctypes.c_int64
        lib.orc_admit_apply.argtypes = [P(_G), _i64p, _i64p, _i64p, ctypes.c_int64, ctypes.c_int64, _i64p]
        lib.orc_cluster.restype = ctypes.c_int32
        lib.orc_cluster.argtypes = [P(_G), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    _i64p, _i64p, P(ctypes.c_int64)]
        lib.orc_contract.restype = ctypes.c_int
        lib.orc_contract.argtypes = [P(_G), _i64p, ctypes.c_int32, _i64p, P(_Owned)]
        lib.orc_owned_free.restype = None
        lib.orc_owned_free.argtypes = [P(_Owned)]
        lib.orc_initial_partition.restype = None
        lib.orc_initial_partition.argtypes = [P(_G), ctypes.c_int32, ctypes.c_int32, _i64p]
        lib.orc_cut.restype = ctypes.c_int64
        lib.orc_cut.argtypes = [P(_G), _i64p, ctypes.c_int32, _i64p]
        lib.orc_refine.restype = ctypes.c_int32
        lib.orc_refine.argtypes = [P(_G), ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   _i64p, _i64p, P(ctypes.c_int64)]
        lib.orc_place_isolated.restype = None
        lib.orc_place_isolated.argtypes = [_i64p, ctypes.c_int64, _i64p, ctypes.c_int32, _i64p, _i64p]
        lib.orc_partition.restype = ctypes.c_int
        lib.orc_partition.argtypes = [P(_G), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                      _i64p, P(Stats)]
        lib.orc_rate_ext.restype = ctypes.c_int64
        lib.orc_rate_ext.argtypes = [P(_G), _i64p, _i64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_int32, _i64p, _i64p, _i64p, _i64p]
        lib.orc_cluster_ext.restype = ctypes.c_int32
        lib.orc_cluster_ext.argtypes = [P(_G), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        _i64p, ctypes.c_int32, _i64p, _i64p, _i64p, P(ctypes.c_int64)]
        lib.orc_member_labels.restype = None
        lib.orc_member_labels.argtypes = [ctypes.c_int64, ctypes.c_int32, _i64p]
        lib.orc_overlay.restype = ctypes.c_int64
        lib.orc_overlay.argtypes = [ctypes.c_int64, _i64p, _i64p]
        lib.orc_ensemble.restype = ctypes.c_int32
        lib.orc_ensemble.argtypes = [P(_G), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, _i64p, ctypes.c_int32, _i64p, _i64p, P(ctypes.c_int64)]
        lib.orc_level_lmax.restype = ctypes.c_int64
        lib.orc_level_lmax.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int64]
        lib.orc_partition_ext.restype = ctypes.c_int
        lib.orc_partition_ext.argtypes = [P(_G), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                          P(MLX), _i64p, P(Stats), P(Cycles)]
        lib.seq_partition.restype = ctypes.c_int
        lib.seq_partition.argtypes = [P(_G), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _i64p, P(Stats)]
        lib.seq_cluster.restype = ctypes.c_int32
        lib.seq_cluster.argtypes = [P(_G), ctypes.c_int64, ctypes.c_int32, _i64p]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class OGraph:
    """Keeps contiguous typed copies alive for the C side."""

    def __init__(self, row_ptr, col, ew=None, nw=None):
        self.rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.ew = None if ew is None else np.ascontiguousarray(ew, dtype=np.int32)
        self.nw = None if nw is None else np.ascontiguousarray(nw, dtype=np.int64)
        self.n = self.rp.shape[0] - 1
        self.m = self.col.shape[0]
        self.s = _G(self.n, self.m, _ptr(self.rp), _ptr(self.col), _ptr(self.ew), _ptr(self.nw))

    @classmethod
    def of(cls, g) -> "OGraph":
        return g if isinstance(g, OGraph) else cls(g.row_ptr, g.col, g.ew, g.nw)

    def node_w(self) -> np.ndarray:
        return np.ones(self.n, np.int64) if self.nw is None else self.nw


def bounds(total_w: int, max_w: int, k: int, eps_num: int, eps_den: int, f: int) -> tuple[int, int, int]:
    lmax, W, U = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = _load().orc_bounds(total_w, max_w, k, eps_num, eps_den, f, ctypes.byref(lmax), ctypes.byref(W),
                            ctypes.byref(U))
    if rc:
        raise ValueError(f"orc_bounds: {rc}")
    return lmax.value, W.value, U.value


def rate(g, lab, Wt, cap: int, rnd: int, dir_rule: int = 1, refine: int = 0) -> np.ndarray:
    g = OGraph.of(g)
    lab = np.ascontiguousarray(lab, np.int32)
    Wt = np.ascontiguousarray(Wt, np.int64)
    desire = np.empty(g.n, np.int32)
    _load().orc_rate(ctypes.byref(g.s), _ptr(lab), _ptr(Wt), Wt.shape[0], cap, rnd, dir_rule, refine,
                     _ptr(desire))
    return desire


def admit_apply(g, desire, lab, Wt, cap: int):
    """Returns (new labels, new label weights, admitted flags, moved)."""
    g = OGraph.of(g)
    lab = np.array(lab, np.int32)
    Wt = np.array(Wt, np.int64)
    desire = np.ascontiguousarray(desire, np.int32)
    adm = np.zeros(g.n, np.uint8)
    moved = _load().orc_admit_apply(ctypes.byref(g.s), _ptr(desire), _ptr(lab), _ptr(Wt), Wt.shape[0], cap,
                                    _ptr(adm))
    return lab, Wt, adm.astype(bool), int(moved)


@dataclass
class ClusterResult:
    labels: np.ndarray
    rounds: int
    moved: list
    visits: int


def cluster(g, U: int, max_rounds: int = 10, stop_rule: int = 0, dir_rule: int = 1) -> ClusterResult:
    g = OGraph.of(g)
    lab = np.empty(g.n, np.int32)
    moved = np.zeros(max(max_rounds, 1), np.int64)
    visits = ctypes.c_int64()
    r = _load().orc_cluster(ctypes.byref(g.s), U, max_rounds, stop_rule, dir_rule, _ptr(lab), _ptr(moved),
                            ctypes.byref(visits))
    return ClusterResult(lab, int(r), [int(x) for x in moved[:r]], int(visits.value))


@dataclass
class Contracted:
    coarse_of: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    ew: np.ndarray
    nw: np.ndarray

    @property
    def n(self):
        return self.row_ptr.shape[0] - 1


def contract(g, labels, drop_isolated: int = 0) -> Contracted:
    g = OGraph.of(g)
    lab = np.ascontiguousarray(labels, np.int32)
    if g.n and (lab.min() < 0 or lab.max() >= g.n):
        raise ValueError("labels must lie in [0, n)")
    cof = np.empty(g.n, np.int32)
    out = _Owned()
    lib = _load()
    rc = lib.orc_contract(ctypes.byref(g.s), _ptr(lab), drop_isolated, _ptr(cof), ctypes.byref(out))
    try:
        if rc:
            raise OverflowError(f"orc_contract: {rc}")
        n, m = out.n, out.m
        rp = np.ctypeslib.as_array(out.rp, shape=(n + 1,)).copy()
        col = np.ctypeslib.as_array(out.col, shape=(max(m, 1),))[:m].copy()
        ew = np.ctypeslib.as_array(out.ew, shape=(max(m, 1),))[:m].copy()
        nw = np.ctypeslib.as_array(out.nw, shape=(max(n, 1),))[:n].copy()
    finally:
        lib.orc_owned_free(ctypes.byref(out))
    return Contracted(cof, rp, col, ew, nw)


def initial_partition(g, k: int, skip_isolated: int = 0) -> np.ndarray:
    g = OGraph.of(g)
    part = np.empty(g.n, np.int32)
    _load().orc_initial_partition(ctypes.byref(g.s), k, skip_isolated, _ptr(part))
    return part


def cut(g, part, k: int) -> tuple[int, np.ndarray]:
    g = OGraph.of(g)
    part = np.ascontiguousarray(part, np.int32)
    bw = np.zeros(max(k, 1), np.int64)
    c = _load().orc_cut(ctypes.byref(g.s), _ptr(part), k, _ptr(bw))
    return int(c), bw[:k]


def refine(g, part, k: int, lmax: int, max_rounds: int = 10, dir_rule: int = 1):
    """Returns (part, rounds, moved list, visits)."""
    g = OGraph.of(g)
    part = np.array(part, np.int32)
    moved = np.zeros(max(max_rounds, 1), np.int64)
    visits = ctypes.c_int64()
    r = _load().orc_refine(ctypes.byref(g.s), k, lmax, max_rounds, dir_rule, _ptr(part), _ptr(moved),
                           ctypes.byref(visits))
    if r < 0:
        raise AssertionError("orc_refine: a node outside the rated set wanted to move")
    return part, int(r), [int(x) for x in moved[:r]], int(visits.value)


def place_isolated(nw, isolated, k: int, B) -> np.ndarray:
    isolated = np.ascontiguousarray(isolated, np.uint8)
    n = isolated.shape[0]
    nw = None if nw is None else np.ascontiguousarray(nw, np.int64)
    B = np.ascontiguousarray(B, np.int64)
    part = np.full(n, -1, np.int32)
    _load().orc_place_isolated(_ptr(nw), n, _ptr(isolated), k, _ptr(B), _ptr(part))
    return part


def partition(g, k: int, eps: tuple[int, int] = (3, 100), f: int = 14, lp_rounds: int = 10,
              ref_rounds: int = 10, threshold: int = 0, dir_rule: int = 1) -> tuple[np.ndarray, dict]:
    g = OGraph.of(g)
    part = np.empty(g.n, np.int32)
    st = Stats()
    rc = _load().orc_partition(ctypes.byref(g.s), k, eps[0], eps[1], f, lp_rounds, ref_rounds, threshold,
                               dir_rule, _ptr(part), ctypes.byref(st))
    if rc:
        raise RuntimeError(f"orc_partition: {rc}")
    return part, st.to_dict()


def rate_ext(g, lab, Wt, cap: int, rnd: int, dir_rule: int = 1, vblk=None, lblk=None, active=None):
    """Clustering rating with the respect filter and an active mask; returns
    (desire, visits); visits is -1 if a cluster lies outside its block."""
    g = OGraph.of(g)
    lab = np.ascontiguousarray(lab, np.int32)
    Wt = np.ascontiguousarray(Wt, np.int64)
    vblk = None if vblk is None else np.ascontiguousarray(vblk, np.int32)
    lblk = None if lblk is None else np.ascontiguousarray(lblk, np.int32)
    active = None if active is None else np.ascontiguousarray(active, np.uint8)
    desire = np.empty(g.n, np.int32)
    vis = _load().orc_rate_ext(ctypes.byref(g.s), _ptr(lab), _ptr(Wt), Wt.shape[0], cap, rnd, dir_rule,
                               _ptr(vblk), _ptr(lblk), _ptr(active), _ptr(desire))
    return desire, int(vis)


def cluster_ext(g, U: int, max_rounds: int = 10, stop_rule: int = 0, dir_rule: int = 1, vblk=None,
                subrounds: int = 0, lab0=None) -> ClusterResult:
    g = OGraph.of(g)
    vblk = None if vblk is None else np.ascontiguousarray(vblk, np.int32)
    lab0 = None if lab0 is None else np.ascontiguousarray(lab0, np.int32)
    lab = np.empty(g.n, np.int32)
    moved = np.zeros(max(max_rounds, 1), np.int64)
    visits = ctypes.c_int64()
    r = _load().orc_cluster_ext(ctypes.byref(g.s), U, max_rounds, stop_rule, dir_rule, _ptr(vblk), subrounds,
                                _ptr(lab0), _ptr(lab), _ptr(moved), ctypes.byref(visits))
    if r < 0:
        raise AssertionError("orc_cluster_ext: a cluster left its block")
    return ClusterResult(lab, int(r), [int(x) for x in moved[:r]], int(visits.value))


def member_labels(n: int, e: int) -> np.ndarray:
    lab0 = np.empty(n, np.int32)
    _load().orc_member_labels(n, e, _ptr(lab0))
    return lab0


def overlay(O, C) -> tuple[np.ndarray, int]:
    O = np.array(O, np.int32)
    C = np.ascontiguousarray(C, np.int32)
    c = _load().orc_overlay(O.shape[0], _ptr(O), _ptr(C))
    return O, int(c)


def ensemble(g, U: int, members: int, max_rounds: int = 10, stop_rule: int = 1, dir_rule: int = 1, vblk=None,
             subrounds: int = 0) -> ClusterResult:
    g = OGraph.of(g)
    vblk = None if vblk is None else np.ascontiguousarray(vblk, np.int32)
    lab = np.empty(g.n, np.int32)
    moved = np.zeros(max(max_rounds, 1), np.int64)
    visits = ctypes.c_int64()
    r = _load().orc_ensemble(ctypes.byref(g.s), U, max_rounds, stop_rule, dir_rule, members, _ptr(vblk),
                             subrounds, _ptr(lab), _ptr(moved), ctypes.byref(visits))
    if r < 0:
        raise AssertionError("orc_ensemble: a cluster left its block")
    return ClusterResult(lab, int(r), [int(x) for x in moved[:r]], int(visits.value))


def level_lmax(C: int, k: int, eps: tuple[int, int], delta: tuple[int, int], q: int, i: int, lmax: int) -> int:
    """L_max on level i of q levels with extra imbalance delta (Section 4)."""
    return int(_load().orc_level_lmax(C, k, eps[0], eps[1], delta[0], delta[1], q, i, lmax))


def partition_ext(g, k: int, eps: tuple[int, int] = (3, 100), f: int = 14, lp_rounds: int = 10,
                  ref_rounds: int = 10, threshold: int = 0, dir_rule: int = 1, vcycles: int = 1,
                  subrounds: int = 0, ensemble: int = 1, delta: tuple[int, int] = (0, 1)):
    """Multilevel partition with the Section 4 extensions; returns (part,
    stats of the last cycle with the returned partition's cut, per-cycle
    results)."""
    g = OGraph.of(g)
    part = np.empty(g.n, np.int32)
    st = Stats()
    cy = Cycles()
    x = MLX(vcycles, subrounds, ensemble, 0, delta[0], delta[1])
    rc = _load().orc_partition_ext(ctypes.byref(g.s), k, eps[0], eps[1], f, lp_rounds, ref_rounds, threshold,
                                   dir_rule, ctypes.byref(x), _ptr(part), ctypes.byref(st), ctypes.byref(cy))
    if rc:
        raise RuntimeError(f"orc_partition_ext: {rc}")
    return part, st.to_dict(), cy.to_dict()


def seq_partition(g, k: int, eps: tuple[int, int] = (3, 100), f: int = 14, lp_rounds: int = 10,
                  ref_rounds: int = 10, threshold: int = 0) -> tuple[np.ndarray, dict]:
    """The paper's sequential SCLaP (quality reference, not the oracle)."""
    g = OGraph.of(g)
    part = np.empty(g.n, np.int32)
    st = Stats()
    rc = _load().seq_partition(ctypes.byref(g.s), k, eps[0], eps[1], f, lp_rounds, ref_rounds, threshold,
                               _ptr(part), ctypes.byref(st))
    if rc:
        raise RuntimeError(f"seq_partition: {rc}")
    return part, st.to_dict()


def seq_cluster(g, U: int, max_rounds: int = 10) -> np.ndarray:
    g = OGraph.of(g)
    lab = np.empty(g.n, np.int32)
    _load().seq_cluster(ctypes.byref(g.s), U, max_rounds, _ptr(lab))
    return lab
