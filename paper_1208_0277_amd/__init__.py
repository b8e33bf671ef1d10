"""sccg — exact PixelBox pair areas and set Jaccard on MI355X (gfx950).

Thin ctypes binding of the C ABI declared in ``include/sccg.h``.  Every step
of the computation runs in the HIP kernels of ``libsccg.so``; this module only
marshals arguments.  PyTorch provides device memory and the stream.  There is
no fallback: if the library is missing, or no GPU is visible, calls raise.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsccg.so")

SCCG_OK = 0
SCCG_E_ARG = -1
SCCG_E_RANGE = -2
SCCG_E_POLY = -3
SCCG_E_HIP = -4
SCCG_E_NOMEM = -5
SCCG_E_DEVICE = -6
SCCG_E_STATE = -7

SCCG_PLAIN = 0
SCCG_BATCHED = 1

SCCG_F_NO_LPT = 0x1
SCCG_F_NO_KNOWN_INSIDE = 0x2
SCCG_F_NO_SPLIT_QUEUE = 0x4
SCCG_F_NO_GRAPH = 0x8
SCCG_F_PIXEL_ONLY = 0x10
SCCG_F_NO_SEP = 0x20
SCCG_F_NO_UNION_TILE = 0x40

SCCG_REL_INTERSECTS = 0x1
SCCG_REL_CONTAINS = 0x2
SCCG_REL_WITHIN = 0x4
SCCG_REL_EQUALS = 0x8
SCCG_REL_TOUCHES = 0x10

SCCG_J_NONZERO_ONLY = 0
SCCG_J_INCLUDE_ZERO = 1

#: C-ABI entry points the library must export (checked by the CPU tests).
EXPORTS = ("sccg_create", "sccg_destroy", "sccg_set_params", "sccg_get_params", "sccg_reserve",
           "sccg_area_pairs", "sccg_jaccard_sets", "sccg_validate_polys", "sccg_sync", "sccg_set_stats",
           "sccg_get_stats", "sccg_set_timing", "sccg_get_timing", "sccg_last_error", "sccg_version",
           "sccg_graph_launches", "sccg_valu_peak", "sccg_area_pairs_noalloc", "sccg_get_wave_times",
           "sccg_join_sets", "sccg_relate_pairs", "sccg_host_area_pairs", "sccg_server_create", "sccg_server_submit", "sccg_server_poll", "sccg_server_get_stats",
           "sccg_server_clock", "sccg_server_last_error", "sccg_server_destroy")

SERVER_STAT_KEYS = ("jobs_submitted", "jobs_done", "launches", "pairs_done", "peak_resident_vertices",
                    "peak_resident_slots", "peak_resident_pairs", "admission_waits", "max_jobs_per_launch",
                    "jobs_rejected", "jobs_migrated", "pairs_migrated")

STAT_KEYS = ("leaf_pixel_tests", "leaf_boxes", "split_boxes", "queued_boxes", "kept_boxes", "small_pairs",
             "large_pairs", "empty_pairs", "leaf_edge_updates", "classify_edge_visits", "leaf_staging_edges",
             "covered_pixels", "ring_scan_vertices", "union_tile_vertices", "leaf_vertex_updates")


class SccgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sccg error {code}: {msg}")
        self.code = code


class sccg_polys(ctypes.Structure):
    _fields_ = [("n_polys", ctypes.c_int64), ("offsets", ctypes.c_void_p), ("xy", ctypes.c_void_p)]


class sccg_params(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("box_threshold", ctypes.c_int32), ("split_gx", ctypes.c_int32),
                ("split_gy", ctypes.c_int32), ("queue_chunk", ctypes.c_int32), ("lds_vertex_cap", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("grid", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("waves_per_wg", ctypes.c_int32), ("min_queue_cells", ctypes.c_int32),
                ("n_queues", ctypes.c_int32), ("heavy_verts", ctypes.c_int32), ("min_classify_cells", ctypes.c_int32),
                ("sweep_pair_box", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class sccg_server_config(ctypes.Structure):
    _fields_ = [("vertex_cap", ctypes.c_int64), ("slot_cap", ctypes.c_int64), ("pair_cap", ctypes.c_int64),
                ("max_step_pairs", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("jaccard_flags", ctypes.c_uint32), ("cpu_threads", ctypes.c_int32), ("cpu_trigger", ctypes.c_int32),
                ("cpu_max_pairs", ctypes.c_int64)]


class sccg_job_result(ctypes.Structure):
    _fields_ = [("job_id", ctypes.c_uint64), ("status", ctypes.c_int32), ("jobs_in_launch", ctypes.c_int32),
                ("n_pairs", ctypes.c_int64), ("sum_i", ctypes.c_int64), ("sum_u", ctypes.c_int64),
                ("n_contrib", ctypes.c_int64), ("j", ctypes.c_double), ("jprime", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def _init_torch_gpu() -> None:
    """PyTorch ships its own HIP runtime and the library links the system's:
    both end up in one process, and a runtime that starts after the other has
    taken the device sees no GPU.  PyTorch's (which allocates the tensors the
    calls take) is therefore started first, when it can see a GPU at all."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load_library(path: str = LIB_PATH):
    """Load libsccg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"device library not built: {path} (run __graft_entry__.build())")
    _init_torch_gpu()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    u32 = ctypes.c_uint32
    sig = {
        "sccg_create": ([ctypes.POINTER(P), ctypes.c_int, P, ctypes.POINTER(sccg_params)], ctypes.c_int),
        "sccg_destroy": ([P], ctypes.c_int),
        "sccg_set_params": ([P, ctypes.POINTER(sccg_params)], ctypes.c_int),
        "sccg_get_params": ([P, ctypes.POINTER(sccg_params)], ctypes.c_int),
        "sccg_reserve": ([P, i64, i64, i64], ctypes.c_int),
        "sccg_area_pairs": ([P, ctypes.POINTER(sccg_polys), ctypes.POINTER(sccg_polys), i64, P, P, P, P, u32],
                            ctypes.c_int),
        "sccg_area_pairs_noalloc": ([P, ctypes.POINTER(sccg_polys), ctypes.POINTER(sccg_polys), i64, P, P, P, P],
                                    ctypes.c_int),
        "sccg_jaccard_sets": ([P, i64, P, P, P, u32, P, P, P, P, P], ctypes.c_int),
        "sccg_validate_polys": ([P, ctypes.POINTER(sccg_polys), P], ctypes.c_int),
        "sccg_sync": ([P], ctypes.c_int),
        "sccg_set_stats": ([P, ctypes.c_int], ctypes.c_int),
        "sccg_get_stats": ([P, P, ctypes.c_int], ctypes.c_int),
        "sccg_get_wave_times": ([P, ctypes.c_int, P, i64], ctypes.c_int64),
        "sccg_set_timing": ([P, ctypes.c_int], ctypes.c_int),
        "sccg_get_timing": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "sccg_last_error": ([P], ctypes.c_char_p),
        "sccg_version": ([], ctypes.c_char_p),
        "sccg_graph_launches": ([P], ctypes.c_int64),
        "sccg_valu_peak": ([P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                           ctypes.c_int),
        "sccg_join_sets": ([P, ctypes.POINTER(sccg_polys), ctypes.POINTER(sccg_polys), i64, P, P, ctypes.c_int32,
                            i64, P, P, P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "sccg_relate_pairs": ([P, ctypes.POINTER(sccg_polys), ctypes.POINTER(sccg_polys), i64, P, P, P, P],
                              ctypes.c_int),
        "sccg_host_area_pairs": ([ctypes.POINTER(sccg_polys), ctypes.POINTER(sccg_polys), i64, P, P, P, P,
                                  ctypes.c_int], ctypes.c_int),
        "sccg_server_create": ([ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(sccg_server_config),
                                ctypes.POINTER(sccg_params)], ctypes.c_int),
        "sccg_server_submit": ([P, ctypes.POINTER(sccg_polys), ctypes.POINTER(sccg_polys), i64, P, P, P, P,
                                ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "sccg_server_poll": ([P, ctypes.POINTER(sccg_job_result), ctypes.c_int, i64], ctypes.c_int),
        "sccg_server_get_stats": ([P, P, ctypes.c_int], ctypes.c_int),
        "sccg_server_clock": ([P], ctypes.c_double),
        "sccg_server_last_error": ([P], ctypes.c_char_p),
        "sccg_server_destroy": ([P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


@dataclass
class DevicePolys:
    """CSR rings resident on the device: offsets int64 [n+1], xy int32 [V, 2]."""
    offsets: "object"
    xy: "object"

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0]) - 1

    def c(self) -> sccg_polys:
        return sccg_polys(self.n, _ptr(self.offsets), _ptr(self.xy) if self.xy.numel() else None)

    @staticmethod
    def from_host(off: np.ndarray, xy: np.ndarray, device="cuda") -> "DevicePolys":
        import torch
        o = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).to(device)
        x = torch.from_numpy(np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)).to(device)
        return DevicePolys(o, x)


def _check_dev(t, dtype, name):
    import torch
    if t is None:
        raise ValueError(f"{name} is None")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """One sccg context on a device and stream (the current torch stream by default)."""

    def __init__(self, device: int = 0, stream=None, **params):
        import torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the sccg path runs only on the device")
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        p = sccg_params(**params) if params else None
        h = ctypes.c_void_p()
        rc = self.lib.sccg_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                                  ctypes.byref(p) if p is not None else None)
        if rc != SCCG_OK:
            raise SccgError(rc, "sccg_create failed")
        self.h = h

    def _rc(self, rc):
        if rc != SCCG_OK:
            msg = self.lib.sccg_last_error(self.h)
            raise SccgError(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.sccg_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ params
    def set_params(self, **params):
        self._rc(self.lib.sccg_set_params(self.h, ctypes.byref(sccg_params(**params))))

    def get_params(self) -> dict:
        p = sccg_params()
        self._rc(self.lib.sccg_get_params(self.h, ctypes.byref(p)))
        return p.as_dict()

    def reserve(self, max_polys_a: int, max_polys_b: int, max_pairs: int):
        self._rc(self.lib.sccg_reserve(self.h, max_polys_a, max_polys_b, max_pairs))

    def set_stats(self, enable: bool, stamps: bool = False):
        """Work counters (enable) and per-wave stamps (stamps) of later calls."""
        self._rc(self.lib.sccg_set_stats(self.h, (1 if enable else 0) | (2 if stamps else 0)))

    def get_stats(self) -> dict:
        out = np.zeros(16, np.int64)
        n = self.lib.sccg_get_stats(self.h, out.ctypes.data, 16)
        if n < 0:
            self._rc(n)
        return dict(zip(STAT_KEYS, (int(v) for v in out[:n])))

    def wave_times(self, kernel: int):
        """(start, end) counter stamps (100 MHz) of every wave of a batched
        kernel (0 union sweep, 1 medium sweep, 2 persistent) in the last call
        made with stamps on (set_stats(2)): an int64 array of shape (waves, 2)."""
        n = self.lib.sccg_get_wave_times(self.h, kernel, None, 0)
        if n < 0:
            self._rc(int(n))
        out = np.zeros((max(int(n), 0), 2), np.int64)
        if n > 0:
            m = self.lib.sccg_get_wave_times(self.h, kernel, out.ctypes.data, int(n))
            if m < 0:
                self._rc(int(m))
        return out

    def valu_peak(self, iters: int = 20000):
        """(sustained integer VALU lane-operations per second, kernel ms)."""
        rate, ms = ctypes.c_double(), ctypes.c_double()
        self._rc(self.lib.sccg_valu_peak(self.h, iters, ctypes.byref(rate), ctypes.byref(ms)))
        return float(rate.value), float(ms.value)

    def graph_launches(self) -> int:
        """BATCHED calls of this context that replayed its captured HIP graph."""
        return int(self.lib.sccg_graph_launches(self.h))

    def set_timing(self, enable: bool):
        self._rc(self.lib.sccg_set_timing(self.h, 1 if enable else 0))

    def get_timing(self):
        """(milliseconds summed over timed launches, number of launches)."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._rc(self.lib.sccg_get_timing(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    # ---------------------------------------------------------- compute
    def area_pairs(self, A: DevicePolys, B: DevicePolys, pair_a, pair_b, out_inter=None, out_union=None,
                   mode: int = SCCG_BATCHED):
        """Queue sccg_area_pairs; returns (inter, union) int64 device tensors."""
        import torch
        _check_dev(pair_a, torch.int32, "pair_a")
        _check_dev(pair_b, torch.int32, "pair_b")
        n = int(pair_a.shape[0])
        if int(pair_b.shape[0]) != n:
            raise ValueError("pair_a and pair_b differ in length")
        if out_inter is None:
            out_inter = torch.empty(n, dtype=torch.int64, device=pair_a.device)
        if out_union is None:
            out_union = torch.empty(n, dtype=torch.int64, device=pair_a.device)
        _check_dev(out_inter, torch.int64, "out_inter")
        _check_dev(out_union, torch.int64, "out_union")
        ca, cb = A.c(), B.c()
        self._rc(self.lib.sccg_area_pairs(self.h, ctypes.byref(ca), ctypes.byref(cb), n, _ptr(pair_a),
                                          _ptr(pair_b), _ptr(out_inter), _ptr(out_union), mode))
        return out_inter, out_union

    def area_pairs_noalloc(self, A: DevicePolys, B: DevicePolys, pair_a, pair_b, out_inter, out_union):
        """Queue sccg_area_pairs_noalloc (BATCHED counts, no device allocation
        in the library; the caller passes both outputs)."""
        import torch
        _check_dev(pair_a, torch.int32, "pair_a")
        _check_dev(pair_b, torch.int32, "pair_b")
        _check_dev(out_inter, torch.int64, "out_inter")
        _check_dev(out_union, torch.int64, "out_union")
        n = int(pair_a.shape[0])
        if int(pair_b.shape[0]) != n or int(out_inter.shape[0]) < n or int(out_union.shape[0]) < n:
            raise ValueError("pair arrays differ in length or an output is shorter")
        ca, cb = A.c(), B.c()
        self._rc(self.lib.sccg_area_pairs_noalloc(self.h, ctypes.byref(ca), ctypes.byref(cb), n, _ptr(pair_a),
                                                  _ptr(pair_b), _ptr(out_inter), _ptr(out_union)))
        return out_inter, out_union

    def jaccard_sets(self, set_pair_off, inter, uni, flags: int = SCCG_J_NONZERO_ONLY, jprime: bool = True):
        """Queue sccg_jaccard_sets; returns (sum_i, sum_u, n_contrib, J, J') device tensors."""
        import torch
        _check_dev(set_pair_off, torch.int64, "set_pair_off")
        _check_dev(inter, torch.int64, "inter")
        _check_dev(uni, torch.int64, "uni")
        ns = int(set_pair_off.shape[0]) - 1
        dev = inter.device
        si = torch.empty(ns, dtype=torch.int64, device=dev)
        su = torch.empty(ns, dtype=torch.int64, device=dev)
        nn = torch.empty(ns, dtype=torch.int64, device=dev)
        j = torch.empty(ns, dtype=torch.float64, device=dev)
        jp = torch.empty(ns, dtype=torch.float64, device=dev) if jprime else None
        self._rc(self.lib.sccg_jaccard_sets(self.h, ns, _ptr(set_pair_off), _ptr(inter), _ptr(uni), flags, _ptr(si),
                                            _ptr(su), _ptr(nn), _ptr(j), _ptr(jp)))
        return si, su, nn, j, jp

    def join_sets(self, A: DevicePolys, B: DevicePolys, a_set_off, b_set_off, cell: int = 64, cap: int | None = None):
        """Queue sccg_join_sets: candidate pairs by MBR intersection per set.
        Returns (pair_a, pair_b, set_off) device tensors; retries once with a
        larger buffer when `cap` (default 4 x |B|) is too small."""
        import torch
        _check_dev(a_set_off, torch.int64, "a_set_off")
        _check_dev(b_set_off, torch.int64, "b_set_off")
        ns = int(a_set_off.shape[0]) - 1
        if int(b_set_off.shape[0]) - 1 != ns:
            raise ValueError("a_set_off and b_set_off differ in length")
        dev = a_set_off.device
        cap = 4 * max(B.n, 1) if cap is None else cap
        so = torch.empty(ns + 1, dtype=torch.int64, device=dev)
        cA, cB = A.c(), B.c()
        for _ in range(2):
            pa = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            pb = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            total = ctypes.c_int64(0)
            self._rc(self.lib.sccg_join_sets(self.h, ctypes.byref(cA), ctypes.byref(cB), ns, _ptr(a_set_off),
                                             _ptr(b_set_off), cell, cap, _ptr(pa), _ptr(pb), _ptr(so),
                                             ctypes.byref(total)))
            if total.value <= cap:
                return pa[:total.value], pb[:total.value], so
            cap = total.value
        raise SccgError(SCCG_E_STATE, "join output did not fit after resizing")

    def relate_pairs(self, A: DevicePolys, B: DevicePolys, pair_a, pair_b, inter):
        """Queue sccg_relate_pairs; returns the uint32 relation bits per pair
        (as an int32 device tensor)."""
        import torch
        _check_dev(pair_a, torch.int32, "pair_a")
        _check_dev(pair_b, torch.int32, "pair_b")
        _check_dev(inter, torch.int64, "inter")
        n = int(pair_a.shape[0])
        out = torch.empty(n, dtype=torch.int32, device=pair_a.device)
        cA, cB = A.c(), B.c()
        self._rc(self.lib.sccg_relate_pairs(self.h, ctypes.byref(cA), ctypes.byref(cB), n, _ptr(pair_a), _ptr(pair_b),
                                            _ptr(inter), _ptr(out)))
        return out

    def validate_polys(self, P: DevicePolys):
        import torch
        out = torch.empty(1, dtype=torch.int64, device="cuda")
        cp = P.c()
        self._rc(self.lib.sccg_validate_polys(self.h, ctypes.byref(cp), _ptr(out)))
        return out

    def sync(self):
        """Wait for the stream; raise SccgError for errors the device latched."""
        return self._rc(self.lib.sccg_sync(self.h))

    def sync_code(self) -> int:
        """Wait for the stream and return the status code without raising."""
        return int(self.lib.sccg_sync(self.h))


def _host(a: np.ndarray, dtype, name: str) -> np.ndarray:
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags.c_contiguous:
        raise ValueError(f"{name} must be a C-contiguous numpy array of {np.dtype(dtype).name}")
    return a


class Server:
    """Continuous-batching server (sccg_server_*): jobs are host CSR pairs of
    polygon sets plus candidate pairs; results come back through poll().

    Arrays passed to submit() are borrowed until that job's result has been
    polled (the object keeps them alive until then).  Arrays that live in
    pinned memory (e.g. numpy views of ``torch.empty(..., pin_memory=True)``)
    are copied by DMA without staging."""

    def __init__(self, device: int = 0, params: dict | None = None, **config):
        self.lib = load_library()
        self.h = ctypes.c_void_p()
        cfg = sccg_server_config(**config)
        prm = sccg_params(**(params or {}))
        rc = self.lib.sccg_server_create(ctypes.byref(self.h), device, ctypes.byref(cfg), ctypes.byref(prm))
        if rc != SCCG_OK:
            self.h = ctypes.c_void_p()
            raise SccgError(rc, "sccg_server_create failed")
        self._live = {}
        import threading
        self._lock = threading.Lock()  # submit stores a job's arrays before poll may drop them

    def _rc(self, rc: int) -> int:
        if rc < 0:
            raise SccgError(rc, self.lib.sccg_server_last_error(self.h).decode())
        return rc

    def submit(self, a_off, a_xy, b_off, b_xy, pa, pb, out_inter=None, out_union=None) -> int:
        a_off = _host(a_off, np.int64, "a_off")
        b_off = _host(b_off, np.int64, "b_off")
        a_xy = _host(a_xy, np.int32, "a_xy")
        b_xy = _host(b_xy, np.int32, "b_xy")
        pa = _host(pa, np.int32, "pa")
        pb = _host(pb, np.int32, "pb")
        if len(pa) != len(pb):
            raise ValueError("pa and pb differ in length")
        for o, name in ((out_inter, "out_inter"), (out_union, "out_union")):
            if o is not None and (_host(o, np.int64, name).shape[0] < len(pa)):
                raise ValueError(f"{name} is shorter than the pair list")
        A = sccg_polys(len(a_off) - 1, a_off.ctypes.data, a_xy.ctypes.data if a_xy.size else None)
        B = sccg_polys(len(b_off) - 1, b_off.ctypes.data, b_xy.ctypes.data if b_xy.size else None)
        jid = ctypes.c_uint64()
        with self._lock:
            self._rc(self.lib.sccg_server_submit(
                self.h, ctypes.byref(A), ctypes.byref(B), len(pa), pa.ctypes.data if len(pa) else None,
                pb.ctypes.data if len(pb) else None, out_inter.ctypes.data if out_inter is not None else None,
                out_union.ctypes.data if out_union is not None else None, ctypes.byref(jid)))
            self._live[jid.value] = (a_off, a_xy, b_off, b_xy, pa, pb, out_inter, out_union)
        return jid.value

    def poll(self, max_results: int = 256, timeout: float | None = 0.0) -> list[dict]:
        """Finished jobs (dicts of sccg_job_result fields); waits up to
        `timeout` seconds for the first (None = without limit)."""
        buf = (sccg_job_result * max_results)()
        us = -1 if timeout is None else int(timeout * 1e6)
        n = self._rc(self.lib.sccg_server_poll(self.h, buf, max_results, us))
        out = []
        with self._lock:
            for k in range(n):
                d = buf[k].as_dict()
                self._live.pop(d["job_id"], None)
                out.append(d)
        return out

    def stats(self) -> dict:
        v = np.zeros(len(SERVER_STAT_KEYS), np.int64)
        n = self._rc(self.lib.sccg_server_get_stats(self.h, v.ctypes.data, len(v)))
        return {k: int(v[i]) for i, k in enumerate(SERVER_STAT_KEYS[:n])}

    def clock(self) -> float:
        return float(self.lib.sccg_server_clock(self.h))

    def close(self):
        if self.h:
            self.lib.sccg_server_destroy(self.h)
            self.h = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def host_area_pairs(a_off, a_xy, b_off, b_xy, pa, pb, threads: int = 1):
    """PixelBox on the host CPU (sccg_host_area_pairs): (inter, union) int64
    numpy arrays for host CSR rings and pair indices."""
    lib = load_library()
    a_off = _host(np.ascontiguousarray(a_off, np.int64), np.int64, "a_off")
    b_off = _host(np.ascontiguousarray(b_off, np.int64), np.int64, "b_off")
    a_xy = _host(np.ascontiguousarray(a_xy, np.int32).reshape(-1), np.int32, "a_xy")
    b_xy = _host(np.ascontiguousarray(b_xy, np.int32).reshape(-1), np.int32, "b_xy")
    pa = _host(np.ascontiguousarray(pa, np.int32), np.int32, "pa")
    pb = _host(np.ascontiguousarray(pb, np.int32), np.int32, "pb")
    n = len(pa)
    I = np.zeros(n, np.int64)
    U = np.zeros(n, np.int64)
    A = sccg_polys(len(a_off) - 1, a_off.ctypes.data, a_xy.ctypes.data if a_xy.size else None)
    B = sccg_polys(len(b_off) - 1, b_off.ctypes.data, b_xy.ctypes.data if b_xy.size else None)
    rc = lib.sccg_host_area_pairs(ctypes.byref(A), ctypes.byref(B), n, pa.ctypes.data if n else None,
                                  pb.ctypes.data if n else None, I.ctypes.data if n else None,
                                  U.ctypes.data if n else None, threads)
    if rc != SCCG_OK:
        raise SccgError(rc, "sccg_host_area_pairs failed")
    return I, U


def version() -> str:
    return load_library().sccg_version().decode()
