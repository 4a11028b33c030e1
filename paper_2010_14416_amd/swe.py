"""Thin ctypes binding of libswe.so (include/swe.h), same function names.

Only argument marshalling happens here: numpy arrays are passed as host
memory, torch CUDA tensors (float64, contiguous) as device memory. Every step
of the method runs in the library's HIP kernels. The library must have been
built (``python -m paper_2010_14416_amd.build``); loading fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "swe.h")

SWE_OK = 0
SWE_EINVAL = -1
SWE_EMESH = -2
SWE_ESTATE = -3
SWE_EDEVICE = -4
SWE_ENOMEM = -5
SWE_ENOTREADY = -6
SWE_ENUMERIC = -7
STATUS_NAMES = {0: "SWE_OK", -1: "SWE_EINVAL", -2: "SWE_EMESH",
                -3: "SWE_ESTATE", -4: "SWE_EDEVICE", -5: "SWE_ENOMEM",
                -6: "SWE_ENOTREADY", -7: "SWE_ENUMERIC"}

SWE_BC_WALL = 0
SWE_BC_TRANSMISSIVE = 1
SWE_BC_INFLOW = 2
SWE_BC_FIXED_DEPTH = 3
SWE_BC_FIXED_STAGE = 4
SWE_MEM_HOST = 0
SWE_MEM_DEVICE = 1
SWE_MAX_TAG = 1024


class swe_params(C.Structure):
    _fields_ = [("g", C.c_double), ("cfl", C.c_double), ("h_dry", C.c_double),
                ("dt_max", C.c_double), ("check_every", C.c_int32),
                ("block_cells", C.c_int32), ("reorder", C.c_int32),
                ("block_threads", C.c_int32), ("load_schedule", C.c_int32),
                ("monitors", C.c_int32), ("store_all", C.c_int32),
                ("graph_steps", C.c_int32)]


class swe_mesh_stats(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_cells", C.c_int64),
                ("n_edges", C.c_int64), ("n_boundary_edges", C.c_int64),
                ("n_blocks", C.c_int64), ("n_block_edges", C.c_int64),
                ("block_cells", C.c_int32), ("max_block_edges", C.c_int32),
                ("min_inradius", C.c_double), ("total_area", C.c_double)]


class SweError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None
_p = C.c_void_p
_pd = C.POINTER(C.c_double)
_pi32 = C.POINTER(C.c_int32)
_pi64 = C.POINTER(C.c_int64)


def load():
    """Loads libswe.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: torch ships its own copy of the HIP and
    # HSA runtimes under the same soname (libamdhip64.so.7). Importing torch
    # first makes libswe.so bind to that copy instead of loading a second
    # runtime from /opt/rocm, which could not open the device again.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_2010_14416_amd.build` (the GPU path has no "
            "fallback)")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    L.swe_abi_version.restype = C.c_int
    L.swe_default_params.restype = st
    L.swe_default_params.argtypes = [C.POINTER(swe_params)]
    L.swe_create.restype = st
    L.swe_create.argtypes = [C.POINTER(_p), C.c_int]
    L.swe_destroy.argtypes = [_p]
    L.swe_last_error.restype = C.c_char_p
    L.swe_last_error.argtypes = [_p]
    L.swe_set_stream.restype = st
    L.swe_set_stream.argtypes = [_p, _p]
    L.swe_set_params.restype = st
    L.swe_set_params.argtypes = [_p, C.POINTER(swe_params)]
    L.swe_get_params.restype = st
    L.swe_get_params.argtypes = [_p, C.POINTER(swe_params)]
    L.swe_set_mesh.restype = st
    L.swe_set_mesh.argtypes = [_p, C.c_int64, _pd, C.c_int64, _pi32,
                               C.c_int64, _pi32, _pi32]
    L.swe_set_mesh_edges.restype = st
    L.swe_set_mesh_edges.argtypes = [_p, C.c_int64, _pd, C.c_int64, _pi32,
                                     C.c_int64, _pi32, _pi32, _pi32]
    L.swe_set_cell_groups.restype = st
    L.swe_set_cell_groups.argtypes = [_p, C.c_int64, C.POINTER(C.c_uint8)]
    L.swe_set_wet_cells.restype = st
    L.swe_set_wet_cells.argtypes = [_p, C.c_int64, C.POINTER(C.c_uint8),
                                    C.c_int32]
    L.swe_mesh_info.restype = st
    L.swe_mesh_info.argtypes = [_p, C.POINTER(swe_mesh_stats)]
    L.swe_mesh_digest.restype = st
    L.swe_mesh_digest.argtypes = [_p, C.POINTER(C.c_uint64)]
    L.swe_get_cell_order.restype = st
    L.swe_get_cell_order.argtypes = [_p, _pi32]
    L.swe_get_geometry.restype = st
    L.swe_get_geometry.argtypes = [_p, _pd, _pd]
    L.swe_set_bc.restype = st
    L.swe_set_bc.argtypes = [_p, C.c_int32, C.c_int, C.c_double]
    for name in ("swe_set_bathymetry", "swe_set_manning"):
        f = getattr(L, name)
        f.restype = st
        f.argtypes = [_p, _p, C.c_int]
    L.swe_set_state.restype = st
    L.swe_set_state.argtypes = [_p, _p, _p, _p, C.c_int]
    L.swe_get_state.restype = st
    L.swe_get_state.argtypes = [_p, _p, _p, _p, C.c_int]
    L.swe_set_time.restype = st
    L.swe_set_time.argtypes = [_p, C.c_double, C.c_int64]
    L.swe_get_time.restype = st
    L.swe_get_time.argtypes = [_p, _pd, _pd, _pi64]
    L.swe_advance.restype = st
    L.swe_advance.argtypes = [_p, C.c_int64, C.c_double, _pi64, _pd]
    L.swe_advance_dt.restype = st
    L.swe_advance_dt.argtypes = [_p, C.c_int64, _pd, _pd]
    L.swe_advance_dt_noalloc.restype = st
    L.swe_advance_dt_noalloc.argtypes = [_p, C.c_int64, _pd, _pd]
    L.swe_adjoint_gauges.restype = st
    L.swe_adjoint_gauges.argtypes = [_p, C.c_int64, C.c_int32, _pi32, _pd,
                                     C.c_int32, _pd, _pd, _pd]
    L.swe_get_diagnostics.restype = st
    L.swe_get_diagnostics.argtypes = [_p, _pd, _pd, _pi64]
    L.swe_reset_monitors.restype = st
    L.swe_reset_monitors.argtypes = [_p]
    L.swe_get_activity.restype = st
    L.swe_get_activity.argtypes = [_p, _pi64, _pi64]
    L.swe_discharge_async.restype = st
    L.swe_discharge_async.argtypes = [_p, _p]
    L.swe_discharge_wait.restype = st
    L.swe_discharge_wait.argtypes = [_p, C.c_int32, C.POINTER(C.c_int32)]
    L.swe_get_discharge.restype = st
    L.swe_get_discharge.argtypes = [_p, C.c_int32, _pd, _pd]
    L.swe_get_envelope.restype = st
    L.swe_get_envelope.argtypes = [_p, _p, _p, C.c_int]
    L.swe_ens_create.restype = st
    L.swe_ens_create.argtypes = [C.POINTER(_p), C.POINTER(_p), C.c_int32]
    L.swe_ens_destroy.argtypes = [_p]
    L.swe_ens_last_error.restype = C.c_char_p
    L.swe_ens_last_error.argtypes = [_p]
    L.swe_ens_set_stream.restype = st
    L.swe_ens_set_stream.argtypes = [_p, _p]
    L.swe_ens_workspace_bytes.restype = st
    L.swe_ens_workspace_bytes.argtypes = [_p, C.POINTER(C.c_size_t)]
    L.swe_ens_bind_workspace.restype = st
    L.swe_ens_bind_workspace.argtypes = [_p, _p, C.c_size_t]
    L.swe_ens_advance.restype = st
    L.swe_ens_advance.argtypes = [_p, C.c_int64, _pd]
    L.swe_ens_get_state.restype = st
    L.swe_ens_get_state.argtypes = [_p, C.c_int32, _p, _p, _p, C.c_int]
    L.swe_ens_get_time.restype = st
    L.swe_ens_get_time.argtypes = [_p, C.c_int32, _pd, _pd, _pi64]
    L.swe_ens_info.restype = st
    L.swe_ens_info.argtypes = [_p, _pi64, _pi64]
    L.swe_ens_get_activity.restype = st
    L.swe_ens_get_activity.argtypes = [_p, _pi64, _pi64]
    L.swe_workspace_bytes.restype = st
    L.swe_workspace_bytes.argtypes = [_p, C.POINTER(C.c_size_t)]
    L.swe_bind_workspace.restype = st
    L.swe_bind_workspace.argtypes = [_p, _p, C.c_size_t]
    _lib = L
    return L


def header_functions():
    """Names of the functions include/swe.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_[a-z_]+)\s*\(", text)))


def _check(ctx, status):
    if status != SWE_OK:
        msg = load().swe_last_error(ctx)
        raise SweError(status, msg.decode() if msg else "")


# -------------------------------------------------------------- marshalling

def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _cell_ptr(x, n, name):
    """(pointer, mem kind, keep-alive) of a per-cell float64 array."""
    if _is_torch(x):
        import torch
        if x.dtype != torch.float64 or x.numel() != n or \
                not x.is_contiguous():
            raise ValueError(f"{name}: need a contiguous float64 tensor of "
                             f"{n} elements")
        if x.is_cuda:
            return C.c_void_p(x.data_ptr()), SWE_MEM_DEVICE, x
        x = x.numpy()
    a = np.ascontiguousarray(x, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"{name}: need {n} values, got {a.size}")
    return C.c_void_p(a.ctypes.data), SWE_MEM_HOST, a


# -------------------------------------------------------- the C functions

def swe_abi_version():
    return load().swe_abi_version()


def swe_default_params():
    p = swe_params()
    _check(None, load().swe_default_params(C.byref(p)))
    return p


def swe_create(device=0):
    ctx = C.c_void_p()
    _check(None, load().swe_create(C.byref(ctx), int(device)))
    return ctx


def swe_destroy(ctx):
    load().swe_destroy(ctx)


def swe_last_error(ctx):
    m = load().swe_last_error(ctx)
    return m.decode() if m else ""


def swe_set_stream(ctx, stream):
    """stream: an int/pointer (hipStream_t) or a torch.cuda.Stream."""
    if hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(ctx, load().swe_set_stream(ctx, C.c_void_p(stream or 0)))


def swe_set_params(ctx, params):
    _check(ctx, load().swe_set_params(ctx, C.byref(params)))


def swe_get_params(ctx):
    p = swe_params()
    _check(ctx, load().swe_get_params(ctx, C.byref(p)))
    return p


def swe_set_mesh(ctx, xy, tri, bnd=None, bnd_tag=None):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    if bnd is None:
        bnd = np.zeros((0, 2), np.int32)
        bnd_tag = np.zeros(0, np.int32)
    bnd = np.ascontiguousarray(bnd, dtype=np.int32).reshape(-1, 2)
    bnd_tag = np.ascontiguousarray(bnd_tag, dtype=np.int32).reshape(-1)
    if bnd_tag.size != bnd.shape[0]:
        raise ValueError("bnd_tag must have one tag per boundary segment")
    _check(ctx, load().swe_set_mesh(
        ctx, xy.shape[0], xy.ctypes.data_as(_pd), tri.shape[0],
        tri.ctypes.data_as(_pi32), bnd.shape[0], bnd.ctypes.data_as(_pi32),
        bnd_tag.ctypes.data_as(_pi32)))


def swe_set_mesh_edges(ctx, xy, tri, edge_nodes, edge_cells, edge_tag=None):
    """Mesh with its edges given: edge_nodes (n, 2), edge_cells (n, 2) with
    -1 in one slot on the boundary, edge_tag (n,) or None (all 0)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    en = np.ascontiguousarray(edge_nodes, dtype=np.int32).reshape(-1, 2)
    ec = np.ascontiguousarray(edge_cells, dtype=np.int32).reshape(-1, 2)
    if ec.shape[0] != en.shape[0]:
        raise ValueError("edge_cells must have one row per edge")
    tag_p = None
    if edge_tag is not None:
        et = np.ascontiguousarray(edge_tag, dtype=np.int32).reshape(-1)
        if et.size != en.shape[0]:
            raise ValueError("edge_tag must have one tag per edge")
        tag_p = et.ctypes.data_as(_pi32)
    _check(ctx, load().swe_set_mesh_edges(
        ctx, xy.shape[0], xy.ctypes.data_as(_pd), tri.shape[0],
        tri.ctypes.data_as(_pi32), en.shape[0], en.ctypes.data_as(_pi32),
        ec.ctypes.data_as(_pi32), tag_p))


def swe_set_cell_groups(ctx, group):
    """Cell groups (uint8, user order) for the next swe_set_mesh; None
    clears them."""
    if group is None:
        _check(ctx, load().swe_set_cell_groups(ctx, 0, None))
        return
    g = np.ascontiguousarray(group, dtype=np.uint8).reshape(-1)
    _check(ctx, load().swe_set_cell_groups(
        ctx, g.size, g.ctypes.data_as(C.POINTER(C.c_uint8))))


def swe_set_wet_cells(ctx, wet, band=2):
    """Wet mask (user order) for the next swe_set_mesh: wet cells, dry
    cells within `band` edge-steps of them, other dry cells."""
    w = np.ascontiguousarray(wet, dtype=np.uint8).reshape(-1)
    _check(ctx, load().swe_set_wet_cells(
        ctx, w.size, w.ctypes.data_as(C.POINTER(C.c_uint8)), int(band)))


def swe_mesh_info(ctx):
    s = swe_mesh_stats()
    _check(ctx, load().swe_mesh_info(ctx, C.byref(s)))
    return {k: getattr(s, k) for k, _ in swe_mesh_stats._fields_}


def swe_mesh_digest(ctx):
    d = C.c_uint64()
    _check(ctx, load().swe_mesh_digest(ctx, C.byref(d)))
    return d.value


def swe_get_cell_order(ctx):
    n = swe_mesh_info(ctx)["n_cells"]
    out = np.empty(n, np.int32)
    _check(ctx, load().swe_get_cell_order(ctx, out.ctypes.data_as(_pi32)))
    return out


def swe_get_geometry(ctx):
    n = swe_mesh_info(ctx)["n_cells"]
    area, inr = np.empty(n), np.empty(n)
    _check(ctx, load().swe_get_geometry(ctx, area.ctypes.data_as(_pd),
                                        inr.ctypes.data_as(_pd)))
    return area, inr


def swe_set_bc(ctx, tag, kind, value=0.0):
    _check(ctx, load().swe_set_bc(ctx, int(tag), int(kind), float(value)))


def _n_cells(ctx):
    return swe_mesh_info(ctx)["n_cells"]


def swe_set_bathymetry(ctx, z):
    p, mem, keep = _cell_ptr(z, _n_cells(ctx), "z")
    _check(ctx, load().swe_set_bathymetry(ctx, p, mem))
    del keep


def swe_set_manning(ctx, n):
    p, mem, keep = _cell_ptr(n, _n_cells(ctx), "manning")
    _check(ctx, load().swe_set_manning(ctx, p, mem))
    del keep


def swe_set_state(ctx, h, hu, hv):
    nc = _n_cells(ctx)
    ph, mh, k1 = _cell_ptr(h, nc, "h")
    pu, mu, k2 = _cell_ptr(hu, nc, "hu")
    pv, mv, k3 = _cell_ptr(hv, nc, "hv")
    if not (mh == mu == mv):
        raise ValueError("h, hu, hv must all be host or all device arrays")
    _check(ctx, load().swe_set_state(ctx, ph, pu, pv, mh))
    del k1, k2, k3


def swe_get_state(ctx, out=None):
    """Returns (h, hu, hv) as numpy arrays, or fills `out` (three float64
    CUDA tensors or numpy arrays) and returns it."""
    nc = _n_cells(ctx)
    if out is None:
        out = (np.empty(nc), np.empty(nc), np.empty(nc))
    ptrs = [_cell_ptr(a, nc, "out") for a in out]
    mems = {m for _, m, _ in ptrs}
    if len(mems) != 1:
        raise ValueError("outputs must all be host or all device arrays")
    if mems == {SWE_MEM_HOST} and any(
            not isinstance(a, np.ndarray) for a in out):
        raise ValueError("host outputs must be numpy arrays")
    _check(ctx, load().swe_get_state(ctx, ptrs[0][0], ptrs[1][0], ptrs[2][0],
                                     mems.pop()))
    return out


def swe_set_time(ctx, t, step=0):
    _check(ctx, load().swe_set_time(ctx, float(t), int(step)))


def swe_get_time(ctx):
    t, dt, step = C.c_double(), C.c_double(), C.c_int64()
    _check(ctx, load().swe_get_time(ctx, C.byref(t), C.byref(dt),
                                    C.byref(step)))
    return t.value, dt.value, step.value


def swe_advance(ctx, max_steps, t_end=math.inf, want_time=False):
    """Returns (steps_done, t_now); t_now is None unless want_time or t_end
    is finite (reading it synchronises)."""
    done = C.c_int64()
    t = C.c_double()
    sync = want_time or math.isfinite(t_end)
    _check(ctx, load().swe_advance(ctx, int(max_steps), float(t_end),
                                   C.byref(done),
                                   C.byref(t) if sync else None))
    return done.value, (t.value if sync else None)


def swe_advance_dt(ctx, n, dt=None, record=False):
    """n steps with the given time steps (array of n) or, with dt None, the
    CFL time steps; returns the time steps taken if record."""
    d = None if dt is None else np.ascontiguousarray(dt, dtype=np.float64)
    if d is not None and d.size != n:
        raise ValueError("need one time step per step")
    out = np.empty(n) if record else None
    _check(ctx, load().swe_advance_dt(
        ctx, int(n), None if d is None else d.ctypes.data_as(_pd),
        None if out is None else out.ctypes.data_as(_pd)))
    return out


def swe_get_activity(ctx):
    """(blocks, cells) the next step computes (the rest are dormant)."""
    b, c = C.c_int64(), C.c_int64()
    _check(ctx, load().swe_get_activity(ctx, C.byref(b), C.byref(c)))
    return b.value, c.value


def swe_discharge_async(ctx, out):
    """Enqueues the copy of every tag's discharge rate and volume into out
    (2 * SWE_MAX_TAG float64: a numpy array, or a pinned torch tensor for a
    copy that overlaps the steps); out must stay alive until
    swe_discharge_wait returns True."""
    if _is_torch(out):
        if out.dtype.itemsize != 8 or out.numel() < 2 * SWE_MAX_TAG or \
                out.is_cuda or not out.is_contiguous():
            raise ValueError("need a contiguous host float64 tensor of "
                             f"{2 * SWE_MAX_TAG} values")
        ptr = out.data_ptr()
    else:
        if out.dtype != np.float64 or out.size < 2 * SWE_MAX_TAG or \
                not out.flags["C_CONTIGUOUS"]:
            raise ValueError(f"need a contiguous float64 array of "
                             f"{2 * SWE_MAX_TAG} values")
        ptr = out.ctypes.data
    _check(ctx, load().swe_discharge_async(ctx, ptr))


def swe_discharge_wait(ctx, block=True):
    """True once the pending asynchronous discharge copy has landed."""
    done = C.c_int32()
    _check(ctx, load().swe_discharge_wait(ctx, 1 if block else 0,
                                          C.byref(done)))
    return bool(done.value)


def swe_advance_dt_noalloc(ctx, n, dt=None, record=False):
    """swe_advance_dt that allocates no device memory (the context's
    workspace must exist already; at most SWE_NOALLOC_MAX_STEPS recorded
    time steps per call)."""
    d = None if dt is None else np.ascontiguousarray(dt, dtype=np.float64)
    if d is not None and d.size != n:
        raise ValueError("need one time step per step")
    out = np.empty(n) if record else None
    _check(ctx, load().swe_advance_dt_noalloc(
        ctx, int(n), None if d is None else d.ctypes.data_as(_pd),
        None if out is None else out.ctypes.data_as(_pd)))
    return out


def swe_adjoint_gauges(ctx, steps, gauges, h_target, checkpoint_every=0):
    """(loss, dL/dManning, dL/dz) of the gauge misfit after `steps` steps
    from the current state, with the run's time steps held fixed."""
    g = np.ascontiguousarray(gauges, dtype=np.int32)
    t = np.ascontiguousarray(h_target, dtype=np.float64)
    if g.size != t.size:
        raise ValueError("one target per gauge")
    n = _n_cells(ctx)
    gm, gz = np.empty(n), np.empty(n)
    loss = C.c_double()
    _check(ctx, load().swe_adjoint_gauges(
        ctx, int(steps), int(g.size), g.ctypes.data_as(_pi32),
        t.ctypes.data_as(_pd), int(checkpoint_every), C.byref(loss),
        gm.ctypes.data_as(_pd), gz.ctypes.data_as(_pd)))
    return loss.value, gm, gz


def swe_get_diagnostics(ctx):
    m, led, nw = C.c_double(), C.c_double(), C.c_int64()
    _check(ctx, load().swe_get_diagnostics(ctx, C.byref(m), C.byref(led),
                                           C.byref(nw)))
    return m.value, led.value, nw.value


def swe_reset_monitors(ctx):
    _check(ctx, load().swe_reset_monitors(ctx))


def swe_get_discharge(ctx, tag):
    """(rate [m^3/s] of the last step, volume [m^3] since the reset) leaving
    the domain through boundary tag `tag`."""
    r, v = C.c_double(), C.c_double()
    _check(ctx, load().swe_get_discharge(ctx, int(tag), C.byref(r),
                                         C.byref(v)))
    return r.value, v.value


def swe_get_envelope(ctx, out=None):
    """Returns (h_max, t_wet) as numpy arrays, or fills `out` (two float64
    CUDA tensors or numpy arrays) and returns it."""
    nc = _n_cells(ctx)
    if out is None:
        out = (np.empty(nc), np.empty(nc))
    ptrs = [_cell_ptr(a, nc, "out") for a in out]
    mems = {m for _, m, _ in ptrs}
    if len(mems) != 1:
        raise ValueError("outputs must all be host or all device arrays")
    _check(ctx, load().swe_get_envelope(ctx, ptrs[0][0], ptrs[1][0],
                                        mems.pop()))
    return out


def swe_workspace_bytes(ctx):
    b = C.c_size_t()
    _check(ctx, load().swe_workspace_bytes(ctx, C.byref(b)))
    return b.value


def swe_bind_workspace(ctx, ptr, nbytes):
    _check(ctx, load().swe_bind_workspace(ctx, C.c_void_p(ptr), int(nbytes)))


# ---------------------------------------------------------------- ensemble

def _echeck(ens, status):
    if status != SWE_OK:
        msg = load().swe_ens_last_error(ens)
        raise SweError(status, msg.decode() if msg else "")


def swe_ens_create(ctxs):
    arr = (C.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    ens = C.c_void_p()
    _echeck(None, load().swe_ens_create(C.byref(ens), arr, len(ctxs)))
    return ens


def swe_ens_destroy(ens):
    load().swe_ens_destroy(ens)


def swe_ens_set_stream(ens, stream):
    _echeck(ens, load().swe_ens_set_stream(ens, C.c_void_p(stream)))


def swe_ens_workspace_bytes(ens):
    b = C.c_size_t()
    _echeck(ens, load().swe_ens_workspace_bytes(ens, C.byref(b)))
    return b.value


def swe_ens_bind_workspace(ens, ptr, nbytes):
    _echeck(ens, load().swe_ens_bind_workspace(ens, C.c_void_p(ptr),
                                               int(nbytes)))


def swe_ens_advance(ens, steps, t_end=None):
    """t_end: None (all +inf) or one end time per member."""
    if t_end is None:
        _echeck(ens, load().swe_ens_advance(ens, int(steps), None))
        return
    t = np.ascontiguousarray(t_end, dtype=np.float64)
    _echeck(ens, load().swe_ens_advance(
        ens, int(steps), t.ctypes.data_as(_pd)))


def swe_ens_get_state(ens, member, n_cells):
    h, hu, hv = np.empty(n_cells), np.empty(n_cells), np.empty(n_cells)
    _echeck(ens, load().swe_ens_get_state(
        ens, int(member), h.ctypes.data, hu.ctypes.data, hv.ctypes.data,
        SWE_MEM_HOST))
    return h, hu, hv


def swe_ens_get_time(ens, member):
    t, dt, step = C.c_double(), C.c_double(), C.c_int64()
    _echeck(ens, load().swe_ens_get_time(ens, int(member), C.byref(t),
                                         C.byref(dt), C.byref(step)))
    return t.value, dt.value, step.value


def swe_ens_info(ens):
    n, b = C.c_int64(), C.c_int64()
    _echeck(ens, load().swe_ens_info(ens, C.byref(n), C.byref(b)))
    return dict(n_cells=n.value, n_blocks=b.value)


def swe_ens_get_activity(ens):
    """(blocks, cells) the ensemble's next step computes."""
    b, c = C.c_int64(), C.c_int64()
    _echeck(ens, load().swe_ens_get_activity(ens, C.byref(b), C.byref(c)))
    return b.value, c.value


# ------------------------------------------------------------ convenience

class Solver:
    """One context set up from a workloads.Case. With workspace="torch" the
    device memory is a torch uint8 tensor bound through swe_bind_workspace;
    with stream="torch" kernels run on torch's current stream. With
    group_wet (and reorder), the cells holding water in the case's state
    are ordered apart from the dry ones, and the dry cells within wet_band
    edge-steps of them apart from the rest (swe_set_wet_cells). The band
    lets the far dry blocks fall dormant, at the price of longer records
    in the seam blocks: it pays on large launches (throughput-bound) and not
    on small ones, whose step waits for their slowest block; wet_band=None
    takes 2 from a million cells on, else 0. With edges = (edge_nodes,
    edge_cells, edge_tag) the mesh is given with its edges
    (swe_set_mesh_edges) instead of boundary segments."""

    def __init__(self, case, device=0, workspace="torch", stream="torch",
                 block_cells=256, reorder=True, params=None, group_wet=True,
                 wet_band=None, edges=None):
        self.ctx = swe_create(device)
        self._ws = None
        self.device = device
        try:
            p = swe_default_params()
            p.g, p.cfl, p.h_dry = case.g, case.cfl, case.h_dry
            p.block_cells = int(block_cells)
            p.reorder = 1 if reorder else 0
            if params:
                for k, v in params.items():
                    setattr(p, k, v)
            swe_set_params(self.ctx, p)
            if group_wet and reorder:
                if wet_band is None:
                    wet_band = 2 if case.n_cells >= 1_000_000 else 0
                swe_set_wet_cells(self.ctx, case.h > p.h_dry, wet_band)
            if edges is None:
                swe_set_mesh(self.ctx, case.xy, case.tri, case.bnd,
                             case.bnd_tag)
            else:
                swe_set_mesh_edges(self.ctx, case.xy, case.tri, *edges)
            for tag, (kind, value) in case.bc.items():
                swe_set_bc(self.ctx, tag, kind, value)
            swe_set_bathymetry(self.ctx, case.z)
            swe_set_manning(self.ctx, case.manning)
            swe_set_state(self.ctx, case.h, case.hu, case.hv)
            if stream == "torch" or workspace == "torch":
                import torch
                dev = torch.device("cuda", device)
                if stream == "torch":
                    self.stream = torch.cuda.current_stream(dev)
                    swe_set_stream(self.ctx, self.stream.cuda_stream)
                if workspace == "torch":
                    nb = swe_workspace_bytes(self.ctx)
                    self._ws = torch.empty(nb + 256, dtype=torch.uint8,
                                           device=dev)
                    base = self._ws.data_ptr()
                    off = (-base) % 256
                    swe_bind_workspace(self.ctx, base + off, nb)
            elif stream is not None:
                swe_set_stream(self.ctx, stream)
        except Exception:
            self.close()
            raise

    def info(self):
        return swe_mesh_info(self.ctx)

    def advance(self, steps, t_end=math.inf, want_time=False):
        return swe_advance(self.ctx, steps, t_end, want_time)

    def state(self, out=None):
        return swe_get_state(self.ctx, out)

    def set_state(self, h, hu, hv):
        swe_set_state(self.ctx, h, hu, hv)

    def time(self):
        return swe_get_time(self.ctx)

    def diagnostics(self):
        return swe_get_diagnostics(self.ctx)

    def discharge(self, tag):
        return swe_get_discharge(self.ctx, tag)

    def envelope(self, out=None):
        return swe_get_envelope(self.ctx, out)

    def reset_monitors(self):
        swe_reset_monitors(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            swe_destroy(self.ctx)
            self.ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Members built from workloads.Case objects (each through a Solver with
    no device memory of its own), advanced together. Device memory is a
    torch uint8 tensor and kernels run on torch's current stream, unless
    workspace / stream are None."""

    def __init__(self, cases, device=0, block_cells=64, params=None,
                 workspace="torch", stream="torch", group_wet=True,
                 wet_band=2):
        # one launch for all members: throughput-bound, so the band pays
        # even on small members, and 64-cell blocks (finer dormant blocks
        # on coarse member meshes) beat 128- and 256-cell ones
        self.members = [Solver(c, device=device, workspace=None, stream=None,
                               block_cells=block_cells, params=params,
                               group_wet=group_wet, wet_band=wet_band)
                        for c in cases]
        self.n_cells = [c.n_cells for c in cases]
        self.ens = swe_ens_create([m.ctx for m in self.members])
        self._ws = None
        try:
            if stream == "torch" or workspace == "torch":
                import torch
                dev = torch.device("cuda", device)
                if stream == "torch":
                    self.stream = torch.cuda.current_stream(dev)
                    swe_ens_set_stream(self.ens, self.stream.cuda_stream)
                if workspace == "torch":
                    nb = swe_ens_workspace_bytes(self.ens)
                    self._ws = torch.empty(nb + 256, dtype=torch.uint8,
                                           device=dev)
                    base = self._ws.data_ptr()
                    swe_ens_bind_workspace(self.ens, base + (-base) % 256, nb)
        except Exception:
            self.close()
            raise
        # the members' host-side copies are no longer needed
        for m in self.members:
            m.close()
        self.members = []

    def advance(self, steps, t_end=None):
        swe_ens_advance(self.ens, steps, t_end)

    def state(self, member):
        return swe_ens_get_state(self.ens, member, self.n_cells[member])

    def time(self, member):
        return swe_ens_get_time(self.ens, member)

    def info(self):
        return swe_ens_info(self.ens)

    def activity(self):
        return swe_ens_get_activity(self.ens)


    def close(self):
        for m in getattr(self, "members", []):
            m.close()
        if getattr(self, "ens", None):
            swe_ens_destroy(self.ens)
            self.ens = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gauge_misfit(solver, manning, z, state, steps, gauges, h_target,
                 checkpoint_every=0):
    """The gauge misfit after `steps` steps from `state` (h, hu, hv) at time
    0, as a torch scalar differentiable with respect to the per-cell
    Manning field and bed (float64 tensors in user cell order, host or
    device): the forward run and the discrete adjoint run in
    swe_adjoint_gauges, with the run's time steps held fixed."""
    import torch

    class _GaugeMisfit(torch.autograd.Function):
        @staticmethod
        def forward(ctx, m, zz):
            swe_set_manning(solver.ctx, m.detach())
            swe_set_bathymetry(solver.ctx, zz.detach())
            swe_set_state(solver.ctx, *state)
            swe_set_time(solver.ctx, 0.0, 0)
            loss, gm, gz = swe_adjoint_gauges(solver.ctx, steps, gauges,
                                              h_target, checkpoint_every)
            ctx.save_for_backward(torch.from_numpy(gm).to(m.device),
                                  torch.from_numpy(gz).to(zz.device))
            return torch.tensor(loss, dtype=torch.float64)

        @staticmethod
        def backward(ctx, grad):
            gm, gz = ctx.saved_tensors
            g = grad.to(gm.device)
            return g * gm, g * gz

    return _GaugeMisfit.apply(manning, z)


def autotune_ensemble(cases, candidates=((64, 0, 0), (64, 2, 0), (64, 4, 0),
                                         (64, 2, 128), (128, 2, 0),
                                         (128, 2, 256), (256, 2, 0)),
                      sample=32, warmup=10, steps=20, seed=0, device=0,
                      params=None, warm_ms=100.0):
    """Launch shape of a batched ensemble chosen by timing: for each
    (block_cells, wet_band, block_threads) candidate (block_threads 0: one
    thread per cell), an Ensemble of a seeded sample of the members is built
    and `steps` steps are timed (HIP events on its stream) after `warmup`
    steps and at least `warm_ms` of untimed steps (a GPU just out of the
    host-side set-up runs the first tens of milliseconds of compute-heavy
    work slower).
    Every candidate gives the same results, bit for bit; only the time
    differs (block size: border edges evaluated twice against finer dormant
    blocks; band: dry cells near water grouped apart, so far dry blocks
    fall dormant; two threads per cell: shorter edge loops, fewer blocks per
    compute unit). Returns (best candidate, {candidate: ms per step})."""
    import torch
    rng = np.random.default_rng(seed)
    k = min(int(sample), len(cases))
    pick = np.sort(rng.choice(len(cases), size=k, replace=False))
    sub = [cases[i] for i in pick]
    times = {}
    for cand in candidates:
        bc, band, threads = (tuple(cand) + (0,))[:3]
        p = dict(params or {})
        p["block_threads"] = threads
        e = Ensemble(sub, device=device, block_cells=bc, params=p,
                     wet_band=band)
        try:
            e.advance(warmup)
            e.time(0)
            t0 = time.perf_counter()
            while (time.perf_counter() - t0) * 1e3 < warm_ms:
                e.advance(warmup)
                e.time(0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(e.stream)
            e.advance(steps)
            e1.record(e.stream)
            torch.cuda.synchronize()
            times[(bc, band, threads)] = e0.elapsed_time(e1) / steps
            e.time(0)   # raises on a numeric fault
        finally:
            e.close()
    best = min(times, key=times.get)
    return best, times
