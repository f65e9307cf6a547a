"""Python binding of libbridges (argument marshalling only).

Every step of the path runs in the native library ``libbridges.so``: the
certificate kernels on the GPU (gfx950 HIP) and the final depth-first search
on the certificate in the library's host code.  PyTorch supplies device
memory and the current HIP stream.  There is no fallback: if the library is
missing and cannot be built, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_DIR, "libbridges.so")

BR_OK, BR_EINVAL, BR_ERANGE, BR_ENOMEM, BR_EHIP, BR_EBUSY, BR_ECAP, BR_EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7

EXPORTS = ["br_last_error", "br_create", "br_destroy", "br_cert_build", "br_cert_merge", "br_bridges_find",
           "br_certificate_bridges", "br_two_edge_components", "br_articulation_points",
           "br_bridges_find_batched", "br_batched_max_v", "br_set_profiling", "br_set_final_step", "br_get_profile",
           "br_server_create", "br_server_set_batching", "br_submit", "br_submit_device", "br_poll", "br_wait",
           "br_server_stats", "br_server_set_final_step", "br_server_destroy", "br_probe_read", "br_cert_build_static",
           "br_bridge_tree", "br_autotune", "br_lds_max_v"]


class BridgeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class _Profile(ctypes.Structure):
    _fields_ = [("ms_phase0", ctypes.c_double), ("ms_merge", ctypes.c_double), ("ms_cert", ctypes.c_double),
                ("ms_d2h", ctypes.c_double), ("ms_dfs", ctypes.c_double), ("ms_canon", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("cert_f1", ctypes.c_int64), ("cert_f2", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("launches", ctypes.c_int64), ("ms_bridge_dev", ctypes.c_double),
                ("plan_kind", ctypes.c_int64), ("alg_bytes", ctypes.c_int64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("edges_per_s", ctypes.c_double),
                ("peak_inflight", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("peak_device_bytes", ctypes.c_int64), ("batched_ticks", ctypes.c_int64),
                ("batched_requests", ctypes.c_int64)]


_lib = None


def load():
    """Load libbridges.so, building it first only if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(SO_PATH)
    vp, i64, i32, p64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    lib.br_last_error.restype = ctypes.c_char_p
    lib.br_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.br_destroy.argtypes = [vp]
    lib.br_cert_build.argtypes = [vp, vp, i64, i32, i32, vp, i64, vp, vp]
    lib.br_cert_merge.argtypes = [vp, vp, i64, vp, i64, i32, vp, i64, vp, vp]
    lib.br_cert_build_static.argtypes = [vp, vp, i64, i32, i32, vp, i64, vp, vp]
    lib.br_bridges_find.argtypes = [vp, vp, i64, i32, i32, vp, i64, p64, vp]
    lib.br_two_edge_components.argtypes = [vp, vp, i64, i32, i32, vp, p64, vp]
    lib.br_bridge_tree.argtypes = [vp, vp, i64, i32, i32, vp, vp, i64, p64, p64, vp]
    lib.br_autotune.argtypes = [vp, vp, i64, i32, i32, ctypes.c_char_p, i64, vp]
    lib.br_articulation_points.argtypes = [vp, vp, i64, i32, vp, i64, p64, vp]
    lib.br_certificate_bridges.argtypes = [vp, i64, vp, i64, i32, vp, i64, p64]
    lib.br_bridges_find_batched.argtypes = [vp, vp, vp, vp, i32, i32, vp, i64, vp, vp]
    lib.br_batched_max_v.restype = i32
    lib.br_lds_max_v.restype = i32
    lib.br_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.br_set_final_step.argtypes = [vp, ctypes.c_int]
    lib.br_get_profile.argtypes = [vp, ctypes.POINTER(_Profile)]
    lib.br_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64, i32]
    lib.br_submit.argtypes = [vp, vp, i64, i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.br_submit_device.argtypes = [vp, vp, i64, i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.br_poll.argtypes = [vp, ctypes.c_uint64, vp, i64, p64, ctypes.POINTER(ctypes.c_int)]
    lib.br_wait.argtypes = [vp, ctypes.c_uint64, vp, i64, p64]
    lib.br_server_stats.argtypes = [vp, ctypes.POINTER(_ServerStats), ctypes.c_int]
    lib.br_server_set_final_step.argtypes = [vp, ctypes.c_int]
    lib.br_server_set_batching.argtypes = [vp, i32, i64]
    lib.br_server_destroy.argtypes = [vp]
    lib.br_probe_read.argtypes = [vp, i64, vp, vp]
    _lib = lib
    return lib


def _check(rc):
    if rc != BR_OK:
        raise BridgeError(rc, load().br_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _edges_arg(t):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or t.dim() != 2 or t.shape[1] != 2:
        raise TypeError("edges must be a torch.int32 tensor of shape [E, 2]")
    if not t.is_cuda:
        raise TypeError("edges must be on the GPU")
    if not t.is_contiguous():
        raise TypeError("edges must be contiguous")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0), int(t.shape[0])


class Context:
    """One library context on a device (workspace, staging, host search buffers)."""

    def __init__(self, device: int = 0):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self.device = device
        self._batched_out = np.empty((0, 2), dtype=np.int32)   # reused output room of find_batched
        _check(self._lib.br_create(ctypes.byref(self._h), device))

    def close(self):
        if self._h:
            self._lib.br_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, level: int = 1):
        """0 off; 1 phase timings; 2 also the method's bytes (alg_bytes)."""
        _check(self._lib.br_set_profiling(self._h, int(level)))

    def set_final_step(self, mode: int):
        """1: bridge step on the GPU (the library's default); 0: Algorithm 1's
        search on the host over the copied certificate."""
        _check(self._lib.br_set_final_step(self._h, int(mode)))

    def profile(self) -> dict:
        p = _Profile()
        _check(self._lib.br_get_profile(self._h, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in _Profile._fields_}

    def autotune(self, edges, V: int, M: int = 1, stream=None) -> dict:
        """Measure and keep the fastest launch shapes for this input shape
        (see br_autotune); returns the choice."""
        import json
        ptr, E = _edges_arg(edges)
        buf = ctypes.create_string_buffer(1024)
        _check(self._lib.br_autotune(self._h, ptr, E, int(V), int(M), buf, len(buf), _stream(stream)))
        return json.loads(buf.value.decode())

    def find(self, edges, V: int, M: int = 1, stream=None) -> np.ndarray:
        """Canonical bridge set (int32 [B, 2], u < v, sorted) of the graph."""
        ptr, E = _edges_arg(edges)
        cap = max(int(V) - 1, 1)
        out = np.empty((cap, 2), dtype=np.int32)
        n = ctypes.c_int64(0)
        _check(self._lib.br_bridges_find(self._h, ptr, E, int(V), int(M), out.ctypes.data, cap, ctypes.byref(n),
                                         _stream(stream)))
        return out[:n.value].copy()

    def two_edge_components(self, edges, V: int, M: int = 1, stream=None):
        """(labels int32 [V] = smallest vertex of each 2-edge-connected class, number of classes)."""
        ptr, E = _edges_arg(edges)
        lab = np.empty(max(int(V), 1), dtype=np.int32)
        n = ctypes.c_int64(0)
        _check(self._lib.br_two_edge_components(self._h, ptr, E, int(V), int(M), lab.ctypes.data, ctypes.byref(n),
                                                _stream(stream)))
        return lab[:int(V)].copy(), n.value

    def bridge_tree(self, edges, V: int, M: int = 1, stream=None):
        """(labels int32 [V], tree edges int32 [B, 2]): the 2-edge-connected
        classes and the bridge tree between them (edges as (min, max) class
        labels, ascending)."""
        ptr, E = _edges_arg(edges)
        lab = np.empty(max(int(V), 1), dtype=np.int32)
        cap = max(int(V) - 1, 1)
        tree = np.empty((cap, 2), dtype=np.int32)
        nc, nt = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(self._lib.br_bridge_tree(self._h, ptr, E, int(V), int(M), lab.ctypes.data, tree.ctypes.data, cap,
                                        ctypes.byref(nc), ctypes.byref(nt), _stream(stream)))
        return lab[:int(V)].copy(), tree[:nt.value].copy()

    def articulation_points(self, edges, V: int, stream=None) -> np.ndarray:
        """Articulation points (int32 vertex ids ascending) through the scan-first certificate."""
        ptr, E = _edges_arg(edges)
        out = np.empty(max(int(V), 1), dtype=np.int32)
        n = ctypes.c_int64(0)
        _check(self._lib.br_articulation_points(self._h, ptr, E, int(V), out.ctypes.data, out.shape[0], ctypes.byref(n),
                                                _stream(stream)))
        return out[:n.value].copy()

    def _cert_result(self, out, counts, stream):
        import torch
        if stream is None:
            torch.cuda.current_stream().synchronize()
        elif hasattr(stream, "synchronize"):
            stream.synchronize()
        else:                                   # a raw hipStream_t handle
            torch.cuda.ExternalStream(int(stream)).synchronize()
        n1, n2, st = (int(x) for x in counts.cpu().tolist())
        if st != BR_OK:
            raise BridgeError(st, "certificate kernel reported status %d" % st)
        return out[:n1], out[n1:n1 + n2]

    def cert_build(self, edges, V: int, M: int = 1, stream=None):
        """Certificate (F, F') of the edge list over M chunks; device tensors."""
        import torch
        ptr, E = _edges_arg(edges)
        cap = max(min(E, 2 * (int(V) - 1)), 1)
        out = torch.empty((cap, 2), dtype=torch.int32, device=edges.device)
        counts = torch.zeros(3, dtype=torch.int64, device=edges.device)
        _check(self._lib.br_cert_build(self._h, ptr, E, int(V), int(M), ctypes.c_void_p(out.data_ptr()), cap,
                                       ctypes.c_void_p(counts.data_ptr()), _stream(stream)))
        return self._cert_result(out, counts, stream)

    def cert_build_static(self, edges, V: int, M: int = 1, out=None, counts=None, stream=None):
        """As cert_build, computed in the library's fixed device array (no
        device allocation inside the library); `out` (int32 [cap, 2]) and
        `counts` (int64 [3]) may be passed in so that nothing is allocated here
        either."""
        import torch
        ptr, E = _edges_arg(edges)
        cap = max(min(E, 2 * (int(V) - 1)), 1)
        if out is None:
            out = torch.empty((cap, 2), dtype=torch.int32, device=edges.device)
        if counts is None:
            counts = torch.zeros(3, dtype=torch.int64, device=edges.device)
        _check(self._lib.br_cert_build_static(self._h, ptr, E, int(V), int(M), ctypes.c_void_p(out.data_ptr()),
                                              int(out.shape[0]), ctypes.c_void_p(counts.data_ptr()), _stream(stream)))
        return self._cert_result(out, counts, stream)

    def cert_merge(self, a, b, V: int, stream=None):
        """Certificate of the union of two edge lists; device tensors (F, F')."""
        import torch
        pa, Ea = _edges_arg(a)
        pb, Eb = _edges_arg(b)
        cap = max(min(Ea + Eb, 2 * (int(V) - 1)), 1)
        out = torch.empty((cap, 2), dtype=torch.int32, device=a.device)
        counts = torch.zeros(3, dtype=torch.int64, device=a.device)
        _check(self._lib.br_cert_merge(self._h, pa, Ea, pb, Eb, int(V), ctypes.c_void_p(out.data_ptr()), cap,
                                       ctypes.c_void_p(counts.data_ptr()), _stream(stream)))
        return self._cert_result(out, counts, stream)

    def find_batched(self, edges, offsets, Vs, chunk_edges: int = 0, stream=None):
        """Bridges of G packed graphs; returns (pairs int32 [B,2], offsets int64 [G+1])."""
        ptr, _ = _edges_arg(edges)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        Vv = np.ascontiguousarray(Vs, dtype=np.int32)
        G = int(Vv.shape[0])
        if off.shape[0] != G + 1:
            raise ValueError("offsets must have G+1 entries")
        cap = max(int(np.maximum(Vv.astype(np.int64) - 1, 0).sum()), 1)
        if self._batched_out.shape[0] < cap:      # room for every possible bridge, kept between calls
            self._batched_out = np.empty((cap, 2), dtype=np.int32)
        out = self._batched_out
        boff = np.zeros(G + 1, dtype=np.int64)
        _check(self._lib.br_bridges_find_batched(self._h, ptr, off.ctypes.data, Vv.ctypes.data, G, int(chunk_edges),
                                                 out.ctypes.data, cap, boff.ctypes.data, _stream(stream)))
        return out[:boff[-1]].copy(), boff


class Server:
    """Continuous-batching bridge server on one device (see br_server_create)."""

    def __init__(self, device: int = 0, mem_budget: int = 64 << 30, max_slots: int = 8):
        self._lib = load()
        self._h = ctypes.c_void_p()
        _check(self._lib.br_server_create(ctypes.byref(self._h), device, int(mem_budget), int(max_slots)))

    def submit(self, edges, V: int) -> int:
        """Queue a query; `edges` is a host int32 [E, 2] array, or a contiguous
        int32 [E, 2] CUDA tensor that must stay alive until the ticket is done."""
        t = ctypes.c_uint64(0)
        if hasattr(edges, "is_cuda") and edges.is_cuda:
            import torch
            ptr, E = _edges_arg(edges)
            # the server reads the edges on its own streams: the stream that
            # produced them must be done first
            torch.cuda.current_stream(edges.device).synchronize()
            _check(self._lib.br_submit_device(self._h, ptr, E, int(V), ctypes.byref(t)))
        else:
            e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
            _check(self._lib.br_submit(self._h, e.ctypes.data if e.shape[0] else None, e.shape[0], int(V),
                                       ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, V: int):
        """(done, bridges or None)."""
        cap = max(int(V) - 1, 1)
        out = np.empty((cap, 2), dtype=np.int32)
        n, done = ctypes.c_int64(0), ctypes.c_int(0)
        _check(self._lib.br_poll(self._h, ticket, out.ctypes.data, cap, ctypes.byref(n), ctypes.byref(done)))
        return (True, out[:n.value].copy()) if done.value else (False, None)

    def wait(self, ticket: int, V: int) -> np.ndarray:
        cap = max(int(V) - 1, 1)
        out = np.empty((cap, 2), dtype=np.int32)
        n = ctypes.c_int64(0)
        _check(self._lib.br_wait(self._h, ticket, out.ctypes.data, cap, ctypes.byref(n)))
        return out[:n.value].copy()

    def set_final_step(self, mode: int):
        _check(self._lib.br_server_set_final_step(self._h, int(mode)))

    def set_batching(self, max_v: int, max_e: int = 1 << 21):
        """Requests submitted from now on with V <= max_v and E <= max_e may
        join the batch lane (one batched call per tick); max_v = 0 sends every
        request to a slot."""
        _check(self._lib.br_server_set_batching(self._h, int(max_v), int(max_e)))

    def stats(self, reset: bool = False) -> dict:
        st = _ServerStats()
        _check(self._lib.br_server_stats(self._h, ctypes.byref(st), int(reset)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if self._h:
            self._lib.br_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def find(edges, V: int, M: int = 1, stream=None) -> np.ndarray:
    """Bridges of (V, edges) through M-chunk certificates; canonical int32 [B, 2]."""
    return context(edges.device.index or 0).find(edges, V, M, stream)


def cert_build(edges, V: int, M: int = 1, stream=None):
    return context(edges.device.index or 0).cert_build(edges, V, M, stream)


def cert_merge(a, b, V: int, stream=None):
    return context(a.device.index or 0).cert_merge(a, b, V, stream)


def find_batched(edges, offsets, Vs, chunk_edges: int = 0, stream=None):
    return context(edges.device.index or 0).find_batched(edges, offsets, Vs, chunk_edges, stream)


def certificate_bridges(f1, f2, V: int) -> np.ndarray:
    """The final step alone (host): bridges of the certificate F u F' (numpy int32 [n, 2] each)."""
    a = np.ascontiguousarray(f1, dtype=np.int32).reshape(-1, 2)
    b = np.ascontiguousarray(f2, dtype=np.int32).reshape(-1, 2)
    cap = max(int(V) - 1, 1)
    out = np.empty((cap, 2), dtype=np.int32)
    n = ctypes.c_int64(0)
    _check(load().br_certificate_bridges(a.ctypes.data if a.shape[0] else None, a.shape[0],
                                         b.ctypes.data if b.shape[0] else None, b.shape[0], int(V),
                                         out.ctypes.data, cap, ctypes.byref(n)))
    return out[:n.value].copy()


def probe_read(buf, stream=None) -> None:
    """Read a device tensor once with 16-byte loads (a measurement utility,
    not a step of the method; time it with events on `stream`)."""
    import torch
    sink = torch.zeros(1, dtype=torch.int64, device=buf.device)
    _check(load().br_probe_read(ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                ctypes.c_void_p(sink.data_ptr()), _stream(stream)))
    return sink


def lds_max_v() -> int:
    """Largest V whose whole phase tree the library can run in one workgroup's LDS."""
    return int(load().br_lds_max_v())


def batched_max_v() -> int:
    return int(load().br_batched_max_v())
