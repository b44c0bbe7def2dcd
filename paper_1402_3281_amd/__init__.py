"""Python binding of the gfx950 SCLaP library (libsclap.so).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory and streams.  The library must have been
built (paper_1402_3281_amd/build.py); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsclap.so")

MAX_LEVELS = 64
MAX_ROUNDS = 64
MAX_CYCLES = 16
PATH_COUNTERS = ("rounds", "multi_job_rounds", "device_wide_bin_scans", "device_wide_contended", "hub_rounds")

OK, EINVAL, ENOTSYM, EOVERFLOW, ENOMEM, EHIP, EBUDGET, ENOTFOUND, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7, -8


class SclapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sclap error {code}: {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("ew", ctypes.c_void_p),
        ("nw", ctypes.c_void_p), ("nw_bytes", ctypes.c_int32), ("rows_sorted", ctypes.c_int32),
    ]


class LpParams(ctypes.Structure):
    _fields_ = [("max_rounds", ctypes.c_int32), ("stop_rule", ctypes.c_int32),
                ("direction_rule", ctypes.c_int32), ("subrounds", ctypes.c_int32)]


class RoundStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32), ("visits", ctypes.c_int64),
                ("moved", ctypes.c_int64 * MAX_ROUNDS), ("ms", ctypes.c_double)]

    def to_dict(self) -> dict:
        return {"rounds": self.rounds, "visits": self.visits,
                "moved": [self.moved[i] for i in range(self.rounds)], "ms": self.ms}


class MlParams(ctypes.Structure):
    _fields_ = [("f", ctypes.c_int32), ("lp_rounds", ctypes.c_int32), ("refine_rounds", ctypes.c_int32),
                ("direction_rule", ctypes.c_int32), ("threshold", ctypes.c_int64),
                ("vcycles", ctypes.c_int32), ("subrounds", ctypes.c_int32), ("ensemble", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("delta_num", ctypes.c_int64), ("delta_den", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("n_level", ctypes.c_int64 * MAX_LEVELS), ("m_level", ctypes.c_int64 * MAX_LEVELS),
        ("rounds_c", ctypes.c_int32 * MAX_LEVELS), ("rounds_r", ctypes.c_int32 * MAX_LEVELS),
        ("moved_c", (ctypes.c_int64 * MAX_ROUNDS) * MAX_LEVELS),
        ("moved_r", (ctypes.c_int64 * MAX_ROUNDS) * MAX_LEVELS),
        ("visits_c", ctypes.c_int64 * MAX_LEVELS), ("visits_r", ctypes.c_int64 * MAX_LEVELS),
        ("lmax", ctypes.c_int64), ("W", ctypes.c_int64), ("U", ctypes.c_int64), ("threshold", ctypes.c_int64),
        ("n_isolated", ctypes.c_int64), ("ip_cut", ctypes.c_int64), ("cut", ctypes.c_int64),
        ("max_block", ctypes.c_int64),
        ("ms_cluster", ctypes.c_double), ("ms_contract", ctypes.c_double), ("ms_initial", ctypes.c_double),
        ("ms_refine", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("cycles", ctypes.c_int32), ("best_cycle", ctypes.c_int32),
        ("cycle_cut", ctypes.c_int64 * MAX_CYCLES), ("cycle_max_block", ctypes.c_int64 * MAX_CYCLES),
        ("cycle_visits", ctypes.c_int64 * MAX_CYCLES), ("cycle_levels", ctypes.c_int32 * MAX_CYCLES),
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
        d["ms"] = {"cluster": self.ms_cluster, "contract": self.ms_contract, "initial": self.ms_initial,
                   "refine": self.ms_refine, "total": self.ms_total}
        c = self.cycles
        d["cycles"] = {"cycles": c, "best": self.best_cycle, "cut": [self.cycle_cut[i] for i in range(c)],
                       "max_block": [self.cycle_max_block[i] for i in range(c)],
                       "visits": [self.cycle_visits[i] for i in range(c)],
                       "levels": [self.cycle_levels[i] for i in range(c)]}
        return d


class Job(ctypes.Structure):
    _fields_ = [("graph", Csr), ("k", ctypes.c_int32), ("reserved", ctypes.c_int32), ("eps_num", ctypes.c_int64),
                ("eps_den", ctypes.c_int64), ("params", MlParams), ("part_out", ctypes.c_void_p)]


class JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_int32), ("cut", ctypes.c_int64),
                ("max_block", ctypes.c_int64), ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double)]


# Every exported symbol with its argument types (mirrors include/sclap.h).
_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32, _i64, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
SIGNATURES = {
    "sclap_create": (ctypes.c_int, [_P(_vp), ctypes.c_int]),
    "sclap_destroy": (ctypes.c_int, [_vp]),
    "sclap_last_error": (ctypes.c_char_p, [_vp]),
    "sclap_trim": (ctypes.c_int, [_vp]),
    "sclap_validate": (ctypes.c_int, [_vp, _P(Csr), _vp]),
    "sclap_bounds": (ctypes.c_int, [_i64, _i64, _i32, _i64, _i64, _i32, _P(_i64), _P(_i64), _P(_i64)]),
    "sclap_cluster": (ctypes.c_int, [_vp, _P(Csr), _i64, _P(LpParams), _vp, _P(_i64), _P(RoundStats), _vp]),
    "sclap_cluster_ext": (ctypes.c_int, [_vp, _P(Csr), _i64, _P(LpParams), _vp, _i32, _vp, _P(_i64),
                                         _P(RoundStats), _vp]),
    "sclap_overlay": (ctypes.c_int, [_vp, _i64, _vp, _vp, _P(_i64), _vp]),
    "sclap_contract": (ctypes.c_int, [_vp, _P(Csr), _vp, _i32, _vp, _P(_vp), _vp]),
    "sclap_graph_view": (ctypes.c_int, [_vp, _P(Csr)]),
    "sclap_graph_free": (ctypes.c_int, [_vp]),
    "sclap_graph_copy": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "sclap_initial_partition": (ctypes.c_int, [_vp, _P(Csr), _i32, _i32, _vp, _vp]),
    "sclap_refine": (ctypes.c_int, [_vp, _P(Csr), _i32, _i64, _P(LpParams), _vp, _P(RoundStats), _vp]),
    "sclap_cut": (ctypes.c_int, [_vp, _P(Csr), _vp, _i32, _P(_i64), _vp, _vp]),
    "sclap_cut_noalloc": (ctypes.c_int, [_P(Csr), _vp, _i32, _vp, _vp, _vp]),
    "sclap_partition": (ctypes.c_int, [_vp, _P(Csr), _i32, _i64, _i64, _P(MlParams), _vp, _P(Stats), _vp]),
    "sclap_partition_batch": (ctypes.c_int, [_vp, _i32, _P(Csr), _vp, _i64, _i64, _P(MlParams), _vp, _P(Stats),
                                             _vp]),
    "sclap_server_create": (ctypes.c_int, [_vp, _i64, _i32, _P(_vp)]),
    "sclap_server_submit": (ctypes.c_int, [_vp, _P(Job), _P(_u64)]),
    "sclap_server_poll": (ctypes.c_int, [_vp, _u64, _P(JobResult)]),
    "sclap_server_wait": (ctypes.c_int, [_vp, _u64, _P(JobResult)]),
    "sclap_submit": (ctypes.c_int, [_vp, _P(Job), _P(_u64)]),
    "sclap_poll": (ctypes.c_int, [_vp, _u64, _P(JobResult)]),
    "sclap_wait": (ctypes.c_int, [_vp, _u64, _P(JobResult)]),
    "sclap_server_footprint": (ctypes.c_int, [_P(Csr), _i32, _P(MlParams), _P(_i64), _P(_i64)]),
    "sclap_server_stats": (ctypes.c_int, [_vp, _P(ctypes.c_double), _P(ctypes.c_double), _P(ctypes.c_double),
                                          _P(_i64), _P(_i64), _P(_i64)]),
    "sclap_server_destroy": (ctypes.c_int, [_vp]),
    "sclap_server_hold": (ctypes.c_int, [_vp, _i32]),
    "sclap_profile_enable": (ctypes.c_int, [_vp, _i32]),
    "sclap_path_counters": (ctypes.c_int, [_vp, _i32, _P(_i64)]),
    "sclap_set_bin_bounds": (ctypes.c_int, [_vp, _P(_i32)]),
    "sclap_get_bin_bounds": (ctypes.c_int, [_vp, _P(_i32)]),
    "sclap_autotune": (ctypes.c_int, [_vp, _P(Csr), _i64, _i32, _P(_i32), _P(ctypes.c_double),
                                      _P(ctypes.c_double), _vp]),
    "sclap_server_path_counters": (ctypes.c_int, [_vp, _i32, _P(_i64)]),
    "sclap_profile_read": (ctypes.c_int, [_vp, _P(ctypes.c_double), _P(_i64), _P(_i64), _P(_i64),
                                          _P(ctypes.c_double), _P(_i64)]),
    "sclap_profile_kernels": (ctypes.c_int, [_vp, _i32, _P(ctypes.c_double), _P(ctypes.c_double), _P(_i64),
                                             _P(_i64), _P(_i64)]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsclap.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_1402_3281_amd/build.py (hipcc, gfx950)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int) -> None:
    if rc != OK:
        msg = load_library().sclap_last_error(None)
        raise SclapError(rc, msg.decode() if msg else "")


def _stream(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """Library context on one device (scratch memory, tuning state)."""

    def __init__(self, device: int = 0):
        self.device = device
        self.lib = load_library()
        h = ctypes.c_void_p()
        _check(self.lib.sclap_create(ctypes.byref(h), device))
        self.h = h

    def close(self) -> None:
        if self.h:
            self.lib.sclap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def trim(self) -> None:
        """Return the device blocks the context keeps cached to HIP."""
        _check(self.lib.sclap_trim(self.h))

    def bin_bounds(self) -> list:
        """Largest degrees of the rating bins 3..6 of clustering rounds."""
        hi = (ctypes.c_int32 * 4)()
        _check(self.lib.sclap_get_bin_bounds(self.h, hi))
        return list(hi)

    def set_bin_bounds(self, hi) -> None:
        arr = (ctypes.c_int32 * 4)(*hi)
        _check(self.lib.sclap_set_bin_bounds(self.h, arr))

    def autotune(self, g: "DeviceGraph", U: int, rounds: int = 3, stream=None) -> dict:
        """Time clustering rounds of g under candidate bin bounds and keep the
        fastest; returns the bounds and the times (ms)."""
        hi = (ctypes.c_int32 * 4)()
        bms, dms = ctypes.c_double(), ctypes.c_double()
        c = g.csr()
        _check(self.lib.sclap_autotune(self.h, ctypes.byref(c), U, rounds, hi, ctypes.byref(bms), ctypes.byref(dms),
                                       _stream(stream)))
        return {"bounds": list(hi), "ms": bms.value, "default_ms": dms.value}

    def path_counters(self) -> dict:
        """Paths the LP rounds of this context took since its creation."""
        out = (ctypes.c_int64 * 5)()
        _check(self.lib.sclap_path_counters(self.h, 5, out))
        return dict(zip(PATH_COUNTERS, list(out)))

    def profile(self, on: bool = True) -> None:
        _check(self.lib.sclap_profile_enable(self.h, 1 if on else 0))

    def profile_read(self) -> dict:
        ms, rnd_ms = ctypes.c_double(), ctypes.c_double()
        la, vis, nodes, rounds = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(self.lib.sclap_profile_read(self.h, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(vis),
                                           ctypes.byref(nodes), ctypes.byref(rnd_ms), ctypes.byref(rounds)))
        out = {"rate_ms": ms.value, "rate_launches": la.value, "visits": vis.value, "nodes": nodes.value,
               "round_ms": rnd_ms.value, "rounds": rounds.value}
        K = 6  # five rating groups and the refinement marking kernels
        kms, kb = (ctypes.c_double * K)(), (ctypes.c_double * K)()
        kv, kn = (ctypes.c_int64 * K)(), (ctypes.c_int64 * K)()
        kl, kr = (ctypes.c_int64 * K)(), ctypes.c_int64()
        _check(self.lib.sclap_profile_kernels(self.h, K, kms, kb, kv, kn, kl, ctypes.byref(kr)))
        out["kernels"] = [{"bin": i, "ms": kms[i], "bytes": kb[i], "visits": kv[i], "nodes": kn[i],
                           "launches": kl[i]} for i in range(K)]
        out["kernel_launches"] = kr.value
        return out


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class DeviceGraph:
    """CSR graph in device memory (torch tensors)."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, ew: Optional[torch.Tensor] = None,
                 nw: Optional[torch.Tensor] = None, rows_sorted: bool = False, owner=None):
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32
        assert ew is None or ew.dtype == torch.int32
        assert nw is None or nw.dtype in (torch.int32, torch.int64)
        self.row_ptr, self.col, self.ew, self.nw = row_ptr, col, ew, nw
        self.rows_sorted = rows_sorted
        self._owner = owner

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    @classmethod
    def from_host(cls, g, device="cuda", rows_sorted: Optional[bool] = None) -> "DeviceGraph":
        """From an object with numpy row_ptr/col and optional ew/nw."""
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, np.int64)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(g.col, np.int32)).to(device)
        ew = None if g.ew is None else torch.from_numpy(np.ascontiguousarray(g.ew, np.int32)).to(device)
        nw = None
        if g.nw is not None:
            a = np.ascontiguousarray(g.nw)
            nw = torch.from_numpy(a.astype(np.int64) if a.dtype != np.int32 else a).to(device)
        if rows_sorted is None:
            rows_sorted = False
        return cls(rp, col, ew, nw, rows_sorted)

    def csr(self) -> Csr:
        nwb = 0 if self.nw is None else self.nw.element_size()
        return Csr(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.ew), _ptr(self.nw), nwb,
                   1 if self.rows_sorted else 0)


class CoarseGraph:
    """Library-owned contracted graph; freed on close()/garbage collection."""

    def __init__(self, handle: ctypes.c_void_p):
        self.h = handle
        self.lib = load_library()
        v = Csr()
        _check(self.lib.sclap_graph_view(self.h, ctypes.byref(v)))
        self.view = v

    @property
    def n(self) -> int:
        return self.view.n

    @property
    def m(self) -> int:
        return self.view.m

    def csr(self) -> Csr:
        return self.view

    def to_device(self, stream=None) -> DeviceGraph:
        """Copy into torch tensors owned by the caller."""
        n, m = self.view.n, self.view.m
        rp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        ew = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        nw = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        _check(self.lib.sclap_graph_copy(self.h, _ptr(rp), _ptr(col), _ptr(ew), _ptr(nw), _stream(stream)))
        return DeviceGraph(rp, col[:m], ew[:m], nw[:n], rows_sorted=True)

    def to_host(self) -> dict:
        d = self.to_device()
        torch.cuda.synchronize()
        return {"row_ptr": d.row_ptr.cpu().numpy(), "col": d.col.cpu().numpy(), "ew": d.ew.cpu().numpy(),
                "nw": d.nw.cpu().numpy()}

    def close(self) -> None:
        if self.h:
            self.lib.sclap_graph_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Calls
# ---------------------------------------------------------------------------

def bounds(total_w: int, max_w: int, k: int, eps: tuple[int, int] = (3, 100), f: int = 14) -> tuple[int, int, int]:
    lmax, W, U = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().sclap_bounds(total_w, max_w, k, eps[0], eps[1], f, ctypes.byref(lmax), ctypes.byref(W),
                                       ctypes.byref(U)))
    return lmax.value, W.value, U.value


def server_footprint(n: int, m: int, k: int, weighted_edges: bool = False, nw_bytes: int = 0,
                     params: Optional[MlParams] = None) -> tuple[int, int]:
    """(input bytes, footprint bytes) a server charges for a job on a graph
    of n nodes and m stored entries (host math only)."""
    c = Csr()
    c.n, c.m = n, m
    c.ew = 1 if weighted_edges else None   # only the presence of the arrays matters
    c.nw = 1 if nw_bytes else None
    c.nw_bytes = nw_bytes
    inp, fp = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().sclap_server_footprint(ctypes.byref(c), k, None if params is None else ctypes.byref(params),
                                                 ctypes.byref(inp), ctypes.byref(fp)))
    return inp.value, fp.value


def validate(ctx: Context, g: DeviceGraph, stream=None) -> int:
    """Returns OK, ENOTSYM or EINVAL (no exception)."""
    c = g.csr()
    return ctx.lib.sclap_validate(ctx.h, ctypes.byref(c), _stream(stream))


def cluster(ctx: Context, g: DeviceGraph, U: int, max_rounds: int = 10, stop_rule: int = 0,
            direction_rule: int = 1, stream=None, labels_out: Optional[torch.Tensor] = None, subrounds: int = 0,
            blocks: Optional[torch.Tensor] = None, member: int = 0):
    """Size-constrained label propagation; returns (labels, n_clusters, round
    stats).  blocks / member / subrounds select the Section 4 extensions
    (sclap_cluster_ext); without them sclap_cluster runs."""
    labels = labels_out if labels_out is not None else torch.empty(max(g.n, 1), dtype=torch.int32,
                                                                     device=g.row_ptr.device)
    p = LpParams(max_rounds, stop_rule, direction_rule, subrounds)
    nc = ctypes.c_int64()
    rs = RoundStats()
    c = g.csr()
    if blocks is None and member == 0 and subrounds <= 1:
        _check(ctx.lib.sclap_cluster(ctx.h, ctypes.byref(c), U, ctypes.byref(p), _ptr(labels), ctypes.byref(nc),
                                     ctypes.byref(rs), _stream(stream)))
    else:
        _check(ctx.lib.sclap_cluster_ext(ctx.h, ctypes.byref(c), U, ctypes.byref(p), _ptr(blocks), member,
                                         _ptr(labels), ctypes.byref(nc), ctypes.byref(rs), _stream(stream)))
    return labels[:g.n], nc.value, rs.to_dict()


def overlay(ctx: Context, overlay_inout: torch.Tensor, labels: torch.Tensor, stream=None) -> int:
    """Overlay of two clusterings in place on overlay_inout (numbered by first
    occurrence); returns the cluster count."""
    nc = ctypes.c_int64()
    _check(ctx.lib.sclap_overlay(ctx.h, int(overlay_inout.shape[0]), _ptr(overlay_inout), _ptr(labels),
                                 ctypes.byref(nc), _stream(stream)))
    return nc.value


def contract(ctx: Context, g: DeviceGraph, labels: torch.Tensor, drop_isolated: bool = False, stream=None):
    """Cluster contraction; returns (coarse_of tensor, CoarseGraph)."""
    cof = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.row_ptr.device)
    h = ctypes.c_void_p()
    c = g.csr()
    _check(ctx.lib.sclap_contract(ctx.h, ctypes.byref(c), _ptr(labels), 1 if drop_isolated else 0, _ptr(cof),
                                  ctypes.byref(h), _stream(stream)))
    return cof[:g.n], CoarseGraph(h)


def initial_partition(ctx: Context, g, k: int, skip_isolated: bool = False, stream=None) -> torch.Tensor:
    part = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    c = g.csr()
    _check(ctx.lib.sclap_initial_partition(ctx.h, ctypes.byref(c), k, 1 if skip_isolated else 0, _ptr(part),
                                           _stream(stream)))
    return part[:g.n]


def refine(ctx: Context, g, part: torch.Tensor, k: int, lmax: int, max_rounds: int = 10, direction_rule: int = 1,
           stream=None):
    """LP local search in place on `part`; returns (part, round stats)."""
    p = LpParams(max_rounds, 0, direction_rule, 0)
    rs = RoundStats()
    c = g.csr()
    _check(ctx.lib.sclap_refine(ctx.h, ctypes.byref(c), k, lmax, ctypes.byref(p), _ptr(part), ctypes.byref(rs),
                                _stream(stream)))
    return part, rs.to_dict()


def cut(ctx: Context, g, part: torch.Tensor, k: int, stream=None) -> tuple[int, list]:
    cv = ctypes.c_int64()
    bw = (ctypes.c_int64 * k)()
    c = g.csr()
    _check(ctx.lib.sclap_cut(ctx.h, ctypes.byref(c), _ptr(part), k, ctypes.byref(cv), bw, _stream(stream)))
    return cv.value, list(bw)


def cut_noalloc(g, part: torch.Tensor, k: int, cut_out: torch.Tensor, block_w_out: Optional[torch.Tensor] = None,
                stream=None) -> None:
    """Cut (and block weights) into caller-owned device tensors (cut_out: 1
    int64, block_w_out: k int64), without any allocation by the library."""
    c = g.csr()
    _check(load_library().sclap_cut_noalloc(ctypes.byref(c), _ptr(part), k, _ptr(cut_out), _ptr(block_w_out),
                                            _stream(stream)))


def ml_params(f: int = 14, lp_rounds: int = 10, refine_rounds: int = 10, direction_rule: int = 1,
              threshold: int = 0, vcycles: int = 0, subrounds: int = 0, ensemble: int = 0,
              delta: tuple[int, int] = (0, 1)) -> MlParams:
    return MlParams(f, lp_rounds, refine_rounds, direction_rule, threshold, vcycles, subrounds, ensemble, 0,
                    delta[0], delta[1])


def partition(ctx: Context, g: DeviceGraph, k: int, eps: tuple[int, int] = (3, 100), f: int = 14,
              lp_rounds: int = 10, refine_rounds: int = 10, direction_rule: int = 1, threshold: int = 0,
              stream=None, part_out: Optional[torch.Tensor] = None, vcycles: int = 0, subrounds: int = 0,
              ensemble: int = 0, delta: tuple[int, int] = (0, 1)):
    """Multilevel partition; returns (part tensor, stats dict).  vcycles,
    subrounds, ensemble and delta select the Section 4 extensions."""
    part = part_out if part_out is not None else torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    p = ml_params(f, lp_rounds, refine_rounds, direction_rule, threshold, vcycles, subrounds, ensemble, delta)
    st = Stats()
    c = g.csr()
    _check(ctx.lib.sclap_partition(ctx.h, ctypes.byref(c), k, eps[0], eps[1], ctypes.byref(p), _ptr(part),
                                   ctypes.byref(st), _stream(stream)))
    return part[:g.n], st.to_dict()


def partition_batch(ctx: Context, graphs: Sequence[DeviceGraph], ks: Sequence[int], eps: tuple[int, int] = (3, 100),
                    f: int = 14, lp_rounds: int = 10, refine_rounds: int = 10, direction_rule: int = 1,
                    threshold: int = 0, stream=None, parts_out: Optional[list] = None, vcycles: int = 0,
                    subrounds: int = 0, ensemble: int = 0, delta: tuple[int, int] = (0, 1)):
    """Partition many graphs in fused launches; returns (parts, stats list)."""
    G = len(graphs)
    csrs = (Csr * max(G, 1))(*[g.csr() for g in graphs])
    karr = (ctypes.c_int32 * max(G, 1))(*ks)
    parts = parts_out if parts_out is not None else [
        torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") for g in graphs]
    pptr = (ctypes.c_void_p * max(G, 1))(*[p.data_ptr() for p in parts])
    sts = (Stats * max(G, 1))()
    p = ml_params(f, lp_rounds, refine_rounds, direction_rule, threshold, vcycles, subrounds, ensemble, delta)
    _check(ctx.lib.sclap_partition_batch(ctx.h, G, csrs, karr, eps[0], eps[1], ctypes.byref(p), pptr, sts,
                                         _stream(stream)))
    return [parts[i][:graphs[i].n] for i in range(G)], [sts[i].to_dict() for i in range(G)]


class Server:
    """Served partition jobs with continuous batching under an HBM budget."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_active: int = 64):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(ctx.lib.sclap_server_create(ctx.h, hbm_budget_bytes, max_active, ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, g: DeviceGraph, k: int, part_out: torch.Tensor, eps: tuple[int, int] = (3, 100),
               f: int = 14, lp_rounds: int = 10, refine_rounds: int = 10, direction_rule: int = 1,
               threshold: int = 0, vcycles: int = 0, subrounds: int = 0, ensemble: int = 0,
               delta: tuple[int, int] = (0, 1)) -> int:
        job = Job(g.csr(), k, 0, eps[0], eps[1],
                  ml_params(f, lp_rounds, refine_rounds, direction_rule, threshold, vcycles, subrounds, ensemble,
                            delta), _ptr(part_out))
        # the server copies the graph on a stream of its own
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        _check(self.ctx.lib.sclap_submit(self.h, ctypes.byref(job), ctypes.byref(t)))
        self._keep[t.value] = part_out
        return t.value

    def poll(self, ticket: int) -> Optional[dict]:
        r = JobResult()
        rc = self.ctx.lib.sclap_poll(self.h, ticket, ctypes.byref(r))
        if rc == EAGAIN:
            return None
        _check(rc)
        return self._res(ticket, r)

    def wait(self, ticket: int) -> dict:
        r = JobResult()
        _check(self.ctx.lib.sclap_wait(self.h, ticket, ctypes.byref(r)))
        return self._res(ticket, r)

    def _res(self, ticket: int, r: JobResult) -> dict:
        self._keep.pop(ticket, None)
        return {"status": r.status, "cut": r.cut, "max_block": r.max_block, "latency_ms": r.latency_ms,
                "queue_ms": r.queue_ms}

    def stats(self) -> dict:
        p50, p99, jps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        done, peak, pa = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(self.ctx.lib.sclap_server_stats(self.h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(jps),
                                               ctypes.byref(done), ctypes.byref(peak), ctypes.byref(pa)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "jobs_per_s": jps.value, "completed": done.value,
                "peak_bytes": peak.value, "peak_active": pa.value}

    def hold(self, on: bool = True) -> None:
        """Hold (or release) admission of queued jobs."""
        _check(self.ctx.lib.sclap_server_hold(self.h, 1 if on else 0))

    def path_counters(self) -> dict:
        """Paths the LP rounds of the server's context took since its creation."""
        out = (ctypes.c_int64 * 5)()
        _check(self.ctx.lib.sclap_server_path_counters(self.h, 5, out))
        return dict(zip(PATH_COUNTERS, list(out)))

    def close(self) -> None:
        if self.h:
            self.ctx.lib.sclap_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
