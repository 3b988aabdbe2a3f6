"""ctypes binding of libgdist.so (include/gdist.h), argument marshalling only.

Every function keeps the C name.  Arrays may be numpy arrays (host) or torch
tensors; a CUDA/HIP torch tensor is passed to gdist_build as a device pointer.
A non-OK status raises :class:`GdistError` carrying the status and the
library's message.  The library must have been built (``build_lib.py``); there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdist.so")

GDIST_MIN, GDIST_MAX = 0, 1
GDIST_OK, GDIST_E_INVALID, GDIST_E_HANDLE, GDIST_E_OOM, GDIST_E_CAPACITY, GDIST_E_DEVICE, GDIST_E_BUSY = range(7)
STATUS_NAMES = ["OK", "E_INVALID", "E_HANDLE", "E_OOM", "E_CAPACITY", "E_DEVICE", "E_BUSY"]
GDIST_BUILD_DEVICE_PTR = 1
GDIST_BUILD_DEFORMABLE = 2
GDIST_F_TIED, GDIST_F_ZERO = 1, 2
GDIST_SERVER_DIRECT = 1


class GdistError(RuntimeError):
    def __init__(self, status: int, message: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"gdist {name}: {message}")
        self.status = status


class gdist_pose_t(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class gdist_result_t(C.Structure):
    _fields_ = [("distance", C.c_double), ("distance_fp32", C.c_double), ("err_bound", C.c_double),
                ("point_a", C.c_double * 3), ("point_b", C.c_double * 3),
                ("tri_a", C.c_uint32), ("tri_b", C.c_uint32), ("status", C.c_uint32),
                ("flags", C.c_uint32), ("n_candidates", C.c_uint32), ("n_ties", C.c_uint32)]

    def as_dict(self) -> dict:
        return {"distance": self.distance, "distance_fp32": self.distance_fp32,
                "err_bound": self.err_bound, "point_a": np.array(self.point_a[:]),
                "point_b": np.array(self.point_b[:]), "tri_a": int(self.tri_a),
                "tri_b": int(self.tri_b), "status": int(self.status), "flags": int(self.flags),
                "n_candidates": int(self.n_candidates), "n_ties": int(self.n_ties)}


class gdist_query_desc_t(C.Structure):
    _fields_ = [("a", C.c_uint64), ("b", C.c_uint64), ("pa", gdist_pose_t), ("pb", gdist_pose_t),
                ("mode", C.c_uint32), ("reserved", C.c_uint32)]


class gdist_mesh_info_t(C.Structure):
    _fields_ = [("n_tris", C.c_uint32), ("n_leaves", C.c_uint32), ("depth", C.c_uint32),
                ("reserved", C.c_uint32), ("device_bytes", C.c_uint64), ("root_box", C.c_float * 6)]


class gdist_stats_t(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "rounds", "entries_popped", "child_pairs", "entries_pushed", "leaf_pairs", "tri_pairs",
        "tri_full", "candidates", "front_peak", "bytes_refit", "bytes_traversal", "bytes_narrow", "retries")] + \
               [("ms_refit", C.c_double), ("ms_traversal", C.c_double), ("ms_total", C.c_double),
                ("ms_traverse_kernel", C.c_double), ("traverse_launches", C.c_uint64),
                ("child_boxes", C.c_uint64), ("leaf_tris", C.c_uint64), ("bytes_reeval", C.c_uint64),
                ("refit_trees", C.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class gdist_server_config_t(C.Structure):
    _fields_ = [("max_slots", C.c_uint32), ("rounds_per_step", C.c_uint32), ("front_capacity", C.c_uint64),
                ("cand_per_slot", C.c_uint32), ("max_tris", C.c_uint32), ("flags", C.c_uint32),
                ("stack_capacity", C.c_uint64)]


class gdist_completion_t(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("t_submit_ns", C.c_uint64), ("t_done_ns", C.c_uint64),
                ("result", gdist_result_t)]


class gdist_server_stats_t(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "admitted", "completed", "failed", "requeued",
                                          "steps", "rounds")] + \
               [(n, C.c_uint32) for n in ("active", "pending", "concurrency", "fallbacks")] + \
               [("device_ms", C.c_double), ("graph_steps", C.c_uint64), ("graph_mode", C.c_uint32),
                ("reserved", C.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    """Load libgdist.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2411_11244_amd/build_lib.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch
    # first makes this library bind to that one runtime; loading it second
    # would put two HIP runtimes in the process, and the later one finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    st, vp, u32, u64, fp, dp = C.c_int, C.c_void_p, C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p
    sig = {
        "gdist_create": [C.c_int, C.POINTER(vp)],
        "gdist_destroy": [vp],
        "gdist_set_option": [vp, C.c_char_p, C.c_double],
        "gdist_build": [vp, fp, u32, fp, u32, u32, C.POINTER(u64)],
        "gdist_release": [vp, u64],
        "gdist_update": [vp, u64, fp, u32, u32],
        "gdist_mesh_info": [vp, u64, C.POINTER(gdist_mesh_info_t)],
        "gdist_mesh_export": [vp, u64, fp, fp, fp],
        "gdist_query": [vp, u64, u64, C.POINTER(gdist_pose_t), C.POINTER(gdist_pose_t), C.c_int,
                        C.POINTER(gdist_result_t)],
        "gdist_query_noalloc": [vp, u64, u64, C.POINTER(gdist_pose_t), C.POINTER(gdist_pose_t), C.c_int,
                                C.POINTER(gdist_result_t)],
        "gdist_query_batch": [vp, u32, C.POINTER(gdist_query_desc_t), C.POINTER(gdist_result_t)],
        "gdist_query_one_to_many": [vp, u64, C.POINTER(gdist_pose_t), u32, C.POINTER(u64), C.POINTER(gdist_pose_t),
                                    C.c_int, C.POINTER(gdist_result_t)],
        "gdist_last_stats": [vp, C.POINTER(gdist_stats_t)],
        "gdist_eval_box_bounds": [vp, u32, fp, fp, fp],
        "gdist_eval_tri_tri": [vp, u32, fp, fp, u32, fp, dp],
        "gdist_query_batch_async": [vp, u32, C.POINTER(gdist_query_desc_t), C.POINTER(gdist_result_t), vp],
        "gdist_sync": [vp, vp],
        "gdist_set_allocator": [vp, ALLOC_FN, FREE_FN, vp],
        "gdist_server_start": [vp, C.POINTER(gdist_server_config_t), C.POINTER(vp)],
        "gdist_server_submit": [vp, C.POINTER(gdist_query_desc_t), u64],
        "gdist_server_stats": [vp, C.POINTER(gdist_server_stats_t)],
        "gdist_server_stop": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.gdist_server_poll.argtypes = [vp, C.POINTER(gdist_completion_t), u32]
    L.gdist_server_poll.restype = u32
    L.gdist_last_error.argtypes = []
    L.gdist_last_error.restype = C.c_char_p
    _lib = L
    return L


def exported_symbols() -> List[str]:
    return ["gdist_create", "gdist_destroy", "gdist_set_option", "gdist_build", "gdist_release",
            "gdist_mesh_info", "gdist_mesh_export", "gdist_query", "gdist_query_batch",
            "gdist_last_stats", "gdist_last_error", "gdist_eval_box_bounds", "gdist_eval_tri_tri",
            "gdist_server_start", "gdist_server_submit", "gdist_server_poll", "gdist_server_stats",
            "gdist_server_stop", "gdist_query_batch_async", "gdist_sync", "gdist_set_allocator",
            "gdist_update", "gdist_query_one_to_many", "gdist_query_noalloc"]


def gdist_last_error() -> str:
    return lib().gdist_last_error().decode()


def _check(status: int):
    if status != GDIST_OK:
        raise GdistError(status, gdist_last_error())


def _ptr(a) -> int:
    """Address of a C-contiguous numpy array or torch tensor."""
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def make_pose(R, t) -> gdist_pose_t:
    p = gdist_pose_t()
    R = np.asarray(R, np.float64).reshape(9)
    t = np.asarray(t, np.float64).reshape(3)
    p.R[:] = R.tolist()
    p.t[:] = t.tolist()
    return p


# ------------------------------------------------------------------ context
def gdist_create(device: int = 0) -> int:
    h = C.c_void_p()
    _check(lib().gdist_create(int(device), C.byref(h)))
    return h.value


def gdist_destroy(ctx: int) -> None:
    _check(lib().gdist_destroy(ctx))   # waits for queued asynchronous batches first
    _in_flight.pop(ctx, None)


def gdist_set_option(ctx: int, key: str, value: float) -> None:
    _check(lib().gdist_set_option(ctx, key.encode(), float(value)))


# ------------------------------------------------------------------- meshes
def gdist_build(ctx: int, verts, tris, flags: int = 0) -> int:
    """verts float32 [nv,3], tris uint32/int32 [nt,3] (numpy or torch)."""
    if _is_device(verts) or _is_device(tris):
        if not (_is_device(verts) and _is_device(tris)):
            raise ValueError("verts and tris must both be device tensors or both host arrays")
        import torch
        verts = verts.contiguous().to(torch.float32)
        tris = tris.contiguous().to(torch.int32)
        flags |= GDIST_BUILD_DEVICE_PTR
        nv, nt = int(verts.shape[0]), int(tris.shape[0])
    else:
        verts = np.ascontiguousarray(verts, dtype=np.float32)
        tris = np.ascontiguousarray(tris, dtype=np.uint32)
        if verts.ndim != 2 or verts.shape[1] != 3 or tris.ndim != 2 or tris.shape[1] != 3:
            raise ValueError("verts must be [nv,3] and tris [nt,3]")
        nv, nt = verts.shape[0], tris.shape[0]
    h = C.c_uint64()
    _check(lib().gdist_build(ctx, _ptr(verts), nv, _ptr(tris), nt, flags, C.byref(h)))
    return h.value


def gdist_release(ctx: int, mesh: int) -> None:
    _check(lib().gdist_release(ctx, mesh))


def gdist_update(ctx: int, mesh: int, verts) -> None:
    """New vertex positions (float32 [nv,3], numpy or a device tensor) for a
    mesh built with GDIST_BUILD_DEFORMABLE; its tree is refitted in place."""
    flags = 0
    if _is_device(verts):
        import torch
        verts = verts.contiguous().to(torch.float32)
        flags = GDIST_BUILD_DEVICE_PTR
        nv = int(verts.shape[0])
    else:
        verts = np.ascontiguousarray(verts, dtype=np.float32)
        if verts.ndim != 2 or verts.shape[1] != 3:
            raise ValueError("verts must be [nv,3]")
        nv = verts.shape[0]
    _check(lib().gdist_update(ctx, mesh, _ptr(verts), nv, flags))


def gdist_mesh_info(ctx: int, mesh: int) -> dict:
    info = gdist_mesh_info_t()
    _check(lib().gdist_mesh_info(ctx, mesh, C.byref(info)))
    return {"n_tris": info.n_tris, "n_leaves": info.n_leaves, "depth": info.depth,
            "device_bytes": info.device_bytes, "root_box": np.array(info.root_box[:], np.float32)}


def gdist_mesh_export(ctx: int, mesh: int) -> dict:
    info = gdist_mesh_info(ctx, mesh)
    L, n = info["n_leaves"], info["n_tris"]
    boxes = np.zeros((2 * L, 6), np.float32)
    tris = np.zeros((n, 9), np.float32)
    orig = np.zeros(n, np.uint32)
    _check(lib().gdist_mesh_export(ctx, mesh, boxes.ctypes.data, tris.ctypes.data, orig.ctypes.data))
    return {"boxes": boxes, "tris": tris, "orig": orig, **info}


# ------------------------------------------------------------------ queries
def gdist_query(ctx: int, a: int, b: int, pose_a, pose_b, mode: int = GDIST_MIN) -> dict:
    """pose_* = (R 3x3, t 3) in FP64 (or a gdist_pose_t)."""
    pa = pose_a if isinstance(pose_a, gdist_pose_t) else make_pose(*pose_a)
    pb = pose_b if isinstance(pose_b, gdist_pose_t) else make_pose(*pose_b)
    r = gdist_result_t()
    _check(lib().gdist_query(ctx, a, b, C.byref(pa), C.byref(pb), int(mode), C.byref(r)))
    return r.as_dict()


def gdist_query_noalloc(ctx: int, a: int, b: int, pose_a, pose_b, mode: int = GDIST_MIN) -> dict:
    """gdist_query through the entry point that allocates no device memory."""
    pa = pose_a if isinstance(pose_a, gdist_pose_t) else make_pose(*pose_a)
    pb = pose_b if isinstance(pose_b, gdist_pose_t) else make_pose(*pose_b)
    r = gdist_result_t()
    _check(lib().gdist_query_noalloc(ctx, a, b, C.byref(pa), C.byref(pb), int(mode), C.byref(r)))
    return r.as_dict()


def make_desc(a: int, b: int, pose_a, pose_b, mode: int = GDIST_MIN) -> gdist_query_desc_t:
    d = gdist_query_desc_t()
    d.a, d.b = a, b
    d.pa = make_pose(*pose_a)
    d.pb = make_pose(*pose_b)
    d.mode = int(mode)
    d.reserved = 0
    return d


def gdist_query_batch(ctx: int, descs: Sequence[gdist_query_desc_t], check: bool = True) -> List[dict]:
    n = len(descs)
    arr = (gdist_query_desc_t * n)(*descs)
    res = (gdist_result_t * n)()
    st = lib().gdist_query_batch(ctx, n, arr, res)
    if check:
        _check(st)
    return [res[i].as_dict() for i in range(n)]


def gdist_query_one_to_many(ctx: int, a: int, pose_a, bs: Sequence[int], poses_b, mode: int,
                            check: bool = True) -> List[dict]:
    """Mesh a at pose_a against bs[i] at poses_b[i] ((R, t) pairs), one batched call."""
    n = len(bs)
    hb = (C.c_uint64 * n)(*[int(h) for h in bs])
    pb = (gdist_pose_t * n)(*[make_pose(*p) for p in poses_b])
    res = (gdist_result_t * n)()
    pa = make_pose(*pose_a)
    st = lib().gdist_query_one_to_many(ctx, a, C.byref(pa), n, hb, pb, int(mode), res)
    if check:
        _check(st)
    return [res[i].as_dict() for i in range(n)]


class AsyncBatch:
    """Results of a gdist_query_batch_async call; read them after gdist_sync."""

    def __init__(self, descs):
        self.n = len(descs)
        self.descs = (gdist_query_desc_t * self.n)(*descs)
        self.res = (gdist_result_t * self.n)()

    def results(self) -> List[dict]:
        return [self.res[i].as_dict() for i in range(self.n)]


# Batches in flight per context: the library writes their result arrays after
# the submitting call returns, so they stay referenced until gdist_sync.
_in_flight: dict = {}


def gdist_query_batch_async(ctx: int, descs: Sequence[gdist_query_desc_t], stream=None) -> AsyncBatch:
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
    b = AsyncBatch(descs)
    h = getattr(stream, "cuda_stream", stream)
    _check(lib().gdist_query_batch_async(ctx, b.n, b.descs, b.res, h))
    _in_flight.setdefault(ctx, []).append(b)
    return b


def gdist_sync(ctx: int, stream=None) -> None:
    h = getattr(stream, "cuda_stream", stream)
    try:
        _check(lib().gdist_sync(ctx, h))
    finally:
        _in_flight.pop(ctx, None)


def gdist_set_allocator(ctx: int, alloc=None, free=None, user=None) -> tuple:
    """alloc(nbytes, user) -> device pointer (int), free(ptr, user) -> None; both
    None restores hipMalloc.  Returns the ctypes callbacks, which the caller must
    keep alive for as long as the context uses them."""
    if alloc is None and free is None:
        _check(lib().gdist_set_allocator(ctx, ALLOC_FN(), FREE_FN(), user))
        return ()
    a, f = ALLOC_FN(alloc), FREE_FN(free)
    _check(lib().gdist_set_allocator(ctx, a, f, user))
    return (a, f)


def gdist_last_stats(ctx: int) -> dict:
    s = gdist_stats_t()
    _check(lib().gdist_last_stats(ctx, C.byref(s)))
    return s.as_dict()


# -------------------------------------------------------------- self-checks
def gdist_eval_box_bounds(ctx: int, a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float32).reshape(-1, 6)
    b = np.ascontiguousarray(b, np.float32).reshape(-1, 6)
    out = np.zeros((a.shape[0], 4), np.float32)
    _check(lib().gdist_eval_box_bounds(ctx, a.shape[0], a.ctypes.data, b.ctypes.data, out.ctypes.data))
    return out


def gdist_eval_tri_tri(ctx: int, p, q, mode: int = 0):
    p = np.ascontiguousarray(p, np.float32).reshape(-1, 9)
    q = np.ascontiguousarray(q, np.float32).reshape(-1, 9)
    o32 = np.zeros(p.shape[0], np.float32)
    o64 = np.zeros(p.shape[0], np.float64)
    _check(lib().gdist_eval_tri_tri(ctx, p.shape[0], p.ctypes.data, q.ctypes.data, int(mode),
                                    o32.ctypes.data, o64.ctypes.data))
    return o32, o64


# ------------------------------------------------------------------ serving
def gdist_server_start(ctx: int, max_slots: int = 0, rounds_per_step: int = 0, front_capacity: int = 0,
                       cand_per_slot: int = 0, max_tris: int = 0, stack_capacity: int = 0,
                       flags: int = 0) -> int:
    cfg = gdist_server_config_t(max_slots, rounds_per_step, front_capacity, cand_per_slot, max_tris, flags,
                                stack_capacity)
    h = C.c_void_p()
    _check(lib().gdist_server_start(ctx, C.byref(cfg), C.byref(h)))
    return h.value


def gdist_server_submit(srv: int, desc: gdist_query_desc_t, tag: int) -> None:
    _check(lib().gdist_server_submit(srv, C.byref(desc), int(tag)))


def gdist_server_poll(srv: int, max_n: int = 256) -> List[dict]:
    """Finished queries: dicts with tag, t_submit_ns, t_done_ns and the result fields."""
    buf = (gdist_completion_t * max_n)()
    n = lib().gdist_server_poll(srv, buf, max_n)
    out = []
    for i in range(n):
        d = buf[i].result.as_dict()
        d.update(tag=int(buf[i].tag), t_submit_ns=int(buf[i].t_submit_ns), t_done_ns=int(buf[i].t_done_ns))
        out.append(d)
    return out


def gdist_server_stats(srv: int) -> dict:
    s = gdist_server_stats_t()
    _check(lib().gdist_server_stats(srv, C.byref(s)))
    return s.as_dict()


def gdist_server_stop(srv: int) -> None:
    _check(lib().gdist_server_stop(srv))


class Context:
    """Small RAII wrapper: ``with Context(0) as g: h = g.build(v, f)``."""

    def __init__(self, device: int = 0):
        self.ctx = gdist_create(device)
        self.meshes: dict = {}

    def build(self, verts, tris) -> int:
        return gdist_build(self.ctx, verts, tris)

    def query(self, a, b, pose_a, pose_b, mode=GDIST_MIN) -> dict:
        return gdist_query(self.ctx, a, b, pose_a, pose_b, mode)

    def query_batch(self, descs, check=True):
        return gdist_query_batch(self.ctx, descs, check)

    def stats(self) -> dict:
        return gdist_last_stats(self.ctx)

    def set(self, key, value):
        gdist_set_option(self.ctx, key, value)

    def close(self):
        if self.ctx:
            gdist_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
