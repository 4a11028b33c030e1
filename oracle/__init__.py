"""ctypes shim over the plain C FP64 oracle (``swe_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only importers. It shares no code with the GPU
library (``paper_2010_14416_amd``) and imports nothing from it; inputs come
from the ``workloads`` generators.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "swe_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

_d = C.c_double
_i = C.c_int
_i64 = C.c_int64
_pd = C.POINTER(C.c_double)
_pi32 = C.POINTER(C.c_int32)
_pi64 = C.POINTER(C.c_int64)
_p = C.c_void_p


# The tests that plant mistakes in a copy of the oracle point this at the
# planted copy; nothing else sets it.
_OVERRIDE = os.environ.get("SWE_ORACLE_LIB")


def compile_to(src: str, out: str) -> str:
    """gcc -O2 -ffp-contract=off -fopenmp: no fast-math and no contraction,
    so every operation rounds as written."""
    tmp = out + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
         "-std=c11", "-Wall", "-shared", "-fPIC", src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle in place (oracle/liboracle.so) if it is missing or
    older than its source."""
    if force or not os.path.exists(LIB) or \
            os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_to(SRC, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if _OVERRIDE:
            L = C.CDLL(_OVERRIDE)
        else:
            build()
            L = C.CDLL(LIB)
        L.ora_create.restype = _p
        L.ora_create.argtypes = [_i64, _pd, _i64, _pi32, _i64, _pi32, _pi32,
                                 C.c_char_p, _i]
        L.ora_destroy.argtypes = [_p]
        L.ora_set_bc.argtypes = [_p, _i, _i, _d]
        L.ora_set_params.argtypes = [_p, _d, _d, _d, _d]
        L.ora_set_fields.argtypes = [_p, _pd, _pd]
        L.ora_set_state.argtypes = [_p, _pd, _pd, _pd]
        L.ora_get_state.argtypes = [_p, _pd, _pd, _pd]
        L.ora_set_time.argtypes = [_p, _d, _i64]
        L.ora_get_time.argtypes = [_p, _pd, _pd, _pi64, _pd]
        L.ora_counts.argtypes = [_p, _pi64, _pi64, _pi64, _pi64]
        L.ora_geometry.argtypes = [_p, _pd, _pd, _pi32]
        L.ora_edges.argtypes = [_p, _pi32, _pi32, _pi32, _pd, _pd, _pd, _pi32,
                                C.POINTER(C.c_int8)]
        L.ora_min_rs.restype = _d
        L.ora_min_rs.argtypes = [_p]
        L.ora_mass.restype = _d
        L.ora_mass.argtypes = [_p]
        L.ora_run.argtypes = [_p, _i64, _d, _i, _pi64, _pd]
        L.ora_run_dt.argtypes = [_p, _i64, _pd, _i]
        L.ora_reset_monitors.argtypes = [_p]
        L.ora_discharge.argtypes = [_p, _i, _pd, _pd]
        L.ora_envelope.argtypes = [_p, _pd, _pd]
        L.ora_error.restype = C.c_char_p
        L.ora_error.argtypes = [_p]
        L.ora_star_depth.argtypes = [_d, _d, _d, _d, _d, _pd, _pd,
                                     C.POINTER(_i)]
        L.ora_wave_speeds.restype = _i
        L.ora_wave_speeds.argtypes = [_d, _d, _d, _d, _d, _i, _i, _pd, _pd,
                                      _pd]
        L.ora_wave_speeds_given_hs.argtypes = [_d, _d, _d, _d, _d, _d, _pd,
                                               _pd]
        L.ora_hllc.argtypes = [_d, _d, _d, _d, _d, _d, _d, _d, _pd]
        L.ora_interior_edge.argtypes = [_d, _d] + [_d] * 8 + [_d, _d, _d,
                                                            _pd, _pd]
        L.ora_boundary_edge.argtypes = [_d, _d, _i, _d, _d, _d, _d, _d, _d,
                                        _d, _d, _d, _pd]
        L.ora_cell_update.argtypes = [_d, _d, _d, _d, _d, _d, _d, _d, _pd,
                                      _pd, _pd]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# --------------------------------------------------------------------------
# single-edge / single-cell building blocks (for the pin tests)
# --------------------------------------------------------------------------

def hllc(hL, uL, vL, hR, uR, vR, g=9.81, h_dry=1e-6):
    G = (C.c_double * 3)()
    lib().ora_hllc(g, h_dry, hL, uL, vL, hR, uR, vR, G)
    return np.array(G[:])


def star_depth(hL, uL, hR, uR, g=9.81):
    h0, hs, br = C.c_double(), C.c_double(), C.c_int()
    lib().ora_star_depth(g, hL, uL, hR, uR, C.byref(h0), C.byref(hs),
                         C.byref(br))
    return h0.value, hs.value, br.value


def wave_speeds(hL, uL, hR, uR, g=9.81, h_dry=1e-6):
    SL, SR, Ss = C.c_double(), C.c_double(), C.c_double()
    wl, wr = int(hL > h_dry), int(hR > h_dry)
    if not wl:
        hL, uL = 0.0, 0.0
    if not wr:
        hR, uR = 0.0, 0.0
    ok = lib().ora_wave_speeds(g, hL, uL, hR, uR, wl, wr, C.byref(SL),
                               C.byref(SR), C.byref(Ss))
    if not ok:
        return None
    return SL.value, SR.value, Ss.value


def wave_speeds_given_hs(hL, uL, hR, uR, hs, g=9.81):
    SL, SR = C.c_double(), C.c_double()
    lib().ora_wave_speeds_given_hs(g, hL, uL, hR, uR, hs, C.byref(SL),
                                   C.byref(SR))
    return SL.value, SR.value


def interior_edge(Ui, zi, Uj, zj, n, L, g=9.81, h_dry=1e-6):
    cl = (C.c_double * 3)()
    cr = (C.c_double * 3)()
    lib().ora_interior_edge(g, h_dry, Ui[0], Ui[1], Ui[2], zi, Uj[0], Uj[1],
                            Uj[2], zj, n[0], n[1], L, cl, cr)
    return np.array(cl[:]), np.array(cr[:])


def boundary_edge(kind, value, q, Ui, zi, n, L, g=9.81, h_dry=1e-6):
    cl = (C.c_double * 3)()
    lib().ora_boundary_edge(g, h_dry, kind, value, q, Ui[0], Ui[1], Ui[2], zi,
                            n[0], n[1], L, cl)
    return np.array(cl[:])


def cell_update(dt, A, U, m, R, g=9.81, h_dry=1e-6):
    Rc = (C.c_double * 3)(*R)
    out = (C.c_double * 3)()
    clamp = C.c_double()
    lib().ora_cell_update(g, h_dry, dt, A, U[0], U[1], U[2], m, Rc, out,
                          C.byref(clamp))
    return np.array(out[:]), clamp.value


# --------------------------------------------------------------------------
# whole-mesh runs
# --------------------------------------------------------------------------

class OracleError(RuntimeError):
    pass


class Oracle:
    """The oracle's state for one Case: mesh, fields, boundary conditions,
    parameters, state and clock."""

    def __init__(self, case, threads: int = 0):
        L = lib()
        xy = np.ascontiguousarray(case.xy, dtype=np.float64)
        tri = np.ascontiguousarray(case.tri, dtype=np.int32)
        bnd = np.ascontiguousarray(case.bnd, dtype=np.int32).reshape(-1, 2)
        tag = np.ascontiguousarray(case.bnd_tag, dtype=np.int32)
        err = C.create_string_buffer(512)
        self._h = L.ora_create(xy.shape[0], _ptr(xy, C.c_double),
                               tri.shape[0], _ptr(tri, C.c_int32),
                               bnd.shape[0], _ptr(bnd, C.c_int32),
                               _ptr(tag, C.c_int32), err, 512)
        if not self._h:
            raise OracleError(err.value.decode())
        self.threads = threads
        self.n_cells = int(tri.shape[0])
        for t, (kind, value) in case.bc.items():
            if L.ora_set_bc(self._h, int(t), int(kind), float(value)) != 0:
                raise OracleError(f"bad boundary condition for tag {t}")
        self.set_params(case.g, case.cfl, case.h_dry, math.inf)
        z = np.ascontiguousarray(case.z, dtype=np.float64)
        m = np.ascontiguousarray(case.manning, dtype=np.float64)
        if L.ora_set_fields(self._h, _ptr(z, C.c_double),
                            _ptr(m, C.c_double)) != 0:
            raise OracleError("bad bathymetry or Manning field")
        self.set_state(case.h, case.hu, case.hv)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_destroy(h)
            self._h = None

    def set_params(self, g=9.81, cfl=0.9, h_dry=1e-6, dt_max=math.inf):
        if lib().ora_set_params(self._h, g, cfl, h_dry, dt_max) != 0:
            raise OracleError("bad parameters")

    def set_state(self, h, hu, hv):
        h = np.ascontiguousarray(h, dtype=np.float64)
        hu = np.ascontiguousarray(hu, dtype=np.float64)
        hv = np.ascontiguousarray(hv, dtype=np.float64)
        if lib().ora_set_state(self._h, _ptr(h, C.c_double),
                               _ptr(hu, C.c_double),
                               _ptr(hv, C.c_double)) != 0:
            raise OracleError("bad state")

    def state(self):
        n = self.n_cells
        h, hu, hv = np.empty(n), np.empty(n), np.empty(n)
        lib().ora_get_state(self._h, _ptr(h, C.c_double),
                            _ptr(hu, C.c_double), _ptr(hv, C.c_double))
        return h, hu, hv

    def run(self, max_steps: int, t_end: float = math.inf):
        done, t = C.c_int64(), C.c_double()
        rc = lib().ora_run(self._h, int(max_steps), float(t_end),
                           int(self.threads), C.byref(done), C.byref(t))
        if rc != 0:
            raise OracleError(lib().ora_error(self._h).decode())
        return done.value, t.value

    def run_dt(self, dt):
        """len(dt) steps, step k with time step dt[k]."""
        d = np.ascontiguousarray(dt, dtype=np.float64)
        if lib().ora_run_dt(self._h, d.size, _ptr(d, C.c_double),
                            int(self.threads)) != 0:
            raise OracleError(lib().ora_error(self._h).decode())

    def set_time(self, t: float, step: int = 0):
        lib().ora_set_time(self._h, t, step)

    def clock(self):
        t, dt, ledger = C.c_double(), C.c_double(), C.c_double()
        step = C.c_int64()
        lib().ora_get_time(self._h, C.byref(t), C.byref(dt), C.byref(step),
                           C.byref(ledger))
        return dict(t=t.value, last_dt=dt.value, step=step.value,
                    ledger=ledger.value)

    def reset_monitors(self):
        lib().ora_reset_monitors(self._h)

    def discharge(self, tag: int):
        """(rate of the last step, volume since the reset) leaving through
        boundary tag `tag`."""
        r, v = C.c_double(), C.c_double()
        lib().ora_discharge(self._h, int(tag), C.byref(r), C.byref(v))
        return r.value, v.value

    def envelope(self):
        n = self.n_cells
        hmax, twet = np.empty(n), np.empty(n)
        lib().ora_envelope(self._h, _ptr(hmax, C.c_double),
                           _ptr(twet, C.c_double))
        return hmax, twet

    def min_rs(self) -> float:
        return lib().ora_min_rs(self._h)

    def mass(self) -> float:
        return lib().ora_mass(self._h)

    def counts(self):
        a = [C.c_int64() for _ in range(4)]
        lib().ora_counts(self._h, *[C.byref(x) for x in a])
        return dict(n_nodes=a[0].value, n_cells=a[1].value,
                    n_edges=a[2].value, n_bnd_edges=a[3].value)

    def geometry(self):
        n = self.n_cells
        area, inr = np.empty(n), np.empty(n)
        tri = np.empty((n, 3), dtype=np.int32)
        lib().ora_geometry(self._h, _ptr(area, C.c_double),
                           _ptr(inr, C.c_double), _ptr(tri, C.c_int32))
        return area, inr, tri

    def edges(self):
        ne = self.counts()["n_edges"]
        n = self.n_cells
        left = np.empty(ne, np.int32)
        right = np.empty(ne, np.int32)
        tag = np.empty(ne, np.int32)
        nx, ny, ln = np.empty(ne), np.empty(ne), np.empty(ne)
        c_edge = np.empty((n, 3), np.int32)
        c_right = np.empty((n, 3), np.int8)
        lib().ora_edges(self._h, _ptr(left, C.c_int32),
                        _ptr(right, C.c_int32), _ptr(tag, C.c_int32),
                        _ptr(nx, C.c_double), _ptr(ny, C.c_double),
                        _ptr(ln, C.c_double), _ptr(c_edge, C.c_int32),
                        _ptr(c_right, C.c_int8))
        return dict(left=left, right=right, tag=tag, nx=nx, ny=ny, len=ln,
                    c_edge=c_edge, c_right=c_right)
