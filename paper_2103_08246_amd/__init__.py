"""Python binding of the MI355X immersed-boundary DNS library (libibdns.so).

Argument marshalling only: every stage of the time step runs in the HIP
kernels behind the C ABI declared in include/ibdns.h.  PyTorch provides the
device workspace and the stream.  Importing this package fails loudly if the
compiled library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibdns.so")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ESTATE, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
DIFFUSION_EXPLICIT, DIFFUSION_CN = 0, 1
LE_HINGED, LE_CLAMPED = 0, 1
TEST_VW_NEUMANN_X = 1
TEST_FLAG_WAIT_TIMEOUT = 2
STAGE_PREDICT, STAGE_FLUX, STAGE_IBM, STAGE_PROJECT, STAGE_FLAG, STAGE_ADVANCE = range(6)
(ARR_U, ARR_V, ARR_W, ARR_P, ARR_UT, ARR_VT, ARR_WT, ARR_HU, ARR_HV, ARR_HW, ARR_PHI,
 ARR_POINT_F, ARR_V_GHOST, ARR_W_GHOST) = range(14)

EXPORTED = ("ibdns_workspace_size", "ibdns_init_domain", "ibdns_set_geometry",
            "ibdns_get_grid_points", "ibdns_step",
            "ibdns_sync", "ibdns_get_fields", "ibdns_get_flag", "ibdns_destroy",
            "ibdns_strerror", "ibdns_run_stage", "ibdns_get_array", "ibdns_set_array",
            "ibdns_get_scalars", "ibdns_set_time", "ibdns_get_maps", "ibdns_enable_timing",
            "ibdns_kernel_times", "ibdns_batch_workspace_size", "ibdns_batch_create",
            "ibdns_batch_step", "ibdns_batch_use_graph", "ibdns_batch_autotune", "ibdns_autotune",
            "ibdns_batch_destroy", "ibdns_probe_workspace_size", "ibdns_set_probes",
            "ibdns_get_probe_stats", "ibdns_grid_forcing_workspace_size", "ibdns_set_grid_forcing",
            "ibdns_get_grid_forcing", "ibdns_flag_mls_workspace_size", "ibdns_set_flag_mls",
            "ibdns_get_flag_markers", "ibdns_set_tile", "ibdns_station_stats_size",
            "ibdns_get_station_stats", "ibdns_get_station_stats_noalloc")


class Domain(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("re", ctypes.c_double), ("u_in", ctypes.c_double), ("dt", ctypes.c_double),
                ("cfl", ctypes.c_double), ("noise_amp", ctypes.c_double),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("diffusion", ctypes.c_int32)]


class GridParams(ctypes.Structure):
    _fields_ = [("x_plane", ctypes.c_double), ("mesh", ctypes.c_double), ("bar", ctypes.c_double)]


class FlagParams(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int32), ("length", ctypes.c_double),
                ("x_le", ctypes.c_double), ("y_c", ctypes.c_double), ("z_c", ctypes.c_double),
                ("pitch", ctypes.c_double), ("mass_ratio", ctypes.c_double),
                ("bending", ctypes.c_double), ("stretch", ctypes.c_double),
                ("le_bc", ctypes.c_int32)]


class IbdnsError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


def _load():
    # torch ships its own HIP runtime (soname libamdhip64.so.7); importing it
    # first makes this library bind to that same runtime, so that device
    # pointers from torch allocations are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2103_08246_amd/build.py "
                          "(hipcc --offload-arch=gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    lib.ibdns_workspace_size.argtypes = [ctypes.POINTER(Domain), ctypes.POINTER(GridParams),
                                         ctypes.POINTER(FlagParams), ctypes.POINTER(ctypes.c_size_t)]
    lib.ibdns_init_domain.argtypes = [ctypes.POINTER(Domain), D, D, D, P, ctypes.c_size_t, P,
                                      ctypes.POINTER(P)]
    lib.ibdns_set_geometry.argtypes = [P, ctypes.POINTER(GridParams), ctypes.POINTER(FlagParams)]
    lib.ibdns_get_grid_points.argtypes = [P, ctypes.POINTER(ctypes.c_int64), D, D]
    lib.ibdns_step.argtypes = [P, ctypes.c_int32]
    lib.ibdns_sync.argtypes = [P]
    lib.ibdns_get_fields.argtypes = [P, D, D, D, D, D, ctypes.POINTER(ctypes.c_int64)]
    lib.ibdns_get_flag.argtypes = [P, D, D, D]
    lib.ibdns_destroy.argtypes = [P]
    lib.ibdns_strerror.argtypes = [ctypes.c_int]
    lib.ibdns_strerror.restype = ctypes.c_char_p
    lib.ibdns_run_stage.argtypes = [P, ctypes.c_int32]
    lib.ibdns_get_array.argtypes = [P, ctypes.c_int32, D]
    lib.ibdns_set_array.argtypes = [P, ctypes.c_int32, D]
    lib.ibdns_get_scalars.argtypes = [P, D]
    lib.ibdns_set_time.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32]
    lib.ibdns_get_maps.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.ibdns_enable_timing.argtypes = [P, ctypes.c_int32]
    lib.ibdns_kernel_times.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p), D,
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.ibdns_batch_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    lib.ibdns_batch_create.argtypes = [ctypes.POINTER(P), ctypes.c_int32, P, ctypes.c_size_t,
                                       ctypes.POINTER(P)]
    lib.ibdns_batch_step.argtypes = [P, ctypes.c_int32]
    lib.ibdns_batch_use_graph.argtypes = [P, ctypes.c_int32]
    lib.ibdns_batch_autotune.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.ibdns_autotune.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.ibdns_set_tile.argtypes = [P, ctypes.c_int32]
    lib.ibdns_batch_destroy.argtypes = [P]
    lib.ibdns_probe_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_size_t)]
    dd = ctypes.c_double
    lib.ibdns_set_probes.argtypes = [P, ctypes.c_int32, dd, dd, dd, dd, dd, ctypes.c_int32, P,
                                     ctypes.c_size_t]
    lib.ibdns_get_probe_stats.argtypes = [P, D]
    lib.ibdns_station_stats_size.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_size_t)]
    lib.ibdns_get_station_stats.argtypes = [P, P, ctypes.c_size_t, D]
    lib.ibdns_get_station_stats_noalloc.argtypes = [P, D]
    lib.ibdns_grid_forcing_workspace_size.argtypes = [ctypes.POINTER(Domain), ctypes.POINTER(GridParams),
                                                      ctypes.POINTER(ctypes.c_size_t)]
    lib.ibdns_set_grid_forcing.argtypes = [P, ctypes.POINTER(GridParams), P, ctypes.c_size_t]
    I64 = ctypes.POINTER(ctypes.c_int64)
    lib.ibdns_get_grid_forcing.argtypes = [P, ctypes.c_int32, I64, I64, I64, D]
    lib.ibdns_flag_mls_workspace_size.argtypes = [P, I64, ctypes.POINTER(ctypes.c_size_t)]
    lib.ibdns_set_flag_mls.argtypes = [P, P, ctypes.c_size_t]
    lib.ibdns_get_flag_markers.argtypes = [P, ctypes.POINTER(ctypes.c_int32), D, D, D, D]
    return lib


_lib = _load()


def lib():
    return _lib


def strerror(code: int) -> str:
    return _lib.ibdns_strerror(code).decode()


def _check(code, what):
    if code != OK:
        raise IbdnsError(code, what)
    return code


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_domain(nx, ny, nz, lx, ly, lz, re, u_in=1.0, dt=0.0, cfl=0.5, noise_amp=0.0,
                precision=FP64, flags=0, diffusion=DIFFUSION_EXPLICIT) -> Domain:
    return Domain(nx, ny, nz, lx, ly, lz, re, u_in, dt, cfl, noise_amp, precision, flags, diffusion)


def _ref(x):
    return ctypes.byref(x) if x is not None else None


def workspace_size(dom: Domain, grid: GridParams | None = None, flag: FlagParams | None = None) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.ibdns_workspace_size(ctypes.byref(dom), _ref(grid), _ref(flag), ctypes.byref(out)),
           "workspace_size")
    return out.value


def init_domain(dom: Domain, noise, ws_ptr: int, ws_bytes: int, stream_ptr: int):
    """noise: (zu, zv, zw) float64 arrays or None.  Returns the context handle."""
    ctx = ctypes.c_void_p()
    zu = zv = zw = None
    if noise is not None:
        zu, zv, zw = (np.ascontiguousarray(z, dtype=np.float64) for z in noise)
    _check(_lib.ibdns_init_domain(ctypes.byref(dom), _dptr(zu), _dptr(zv), _dptr(zw),
                                  ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(stream_ptr),
                                  ctypes.byref(ctx)), "init_domain")
    return ctx


def set_geometry(ctx, grid: GridParams | None = None, flag: FlagParams | None = None):
    _check(_lib.ibdns_set_geometry(ctx, _ref(grid), _ref(flag)), "set_geometry")


def get_grid_points(ctx):
    """(X (K, 3), dV (K,)) of the grid's solid points built by the library."""
    n = ctypes.c_int64(0)
    _check(_lib.ibdns_get_grid_points(ctx, ctypes.byref(n), None, None), "get_grid_points")
    X = np.empty((n.value, 3))
    dV = np.empty(n.value)
    if n.value:
        _check(_lib.ibdns_get_grid_points(ctx, ctypes.byref(n), _dptr(X), _dptr(dV)), "get_grid_points")
    return X, dV


def step(ctx, n: int = 1):
    _check(_lib.ibdns_step(ctx, n), "step")


def sync(ctx):
    return _check(_lib.ibdns_sync(ctx), "sync")


def run_stage(ctx, stage: int):
    _check(_lib.ibdns_run_stage(ctx, stage), "run_stage")


def destroy(ctx):
    _check(_lib.ibdns_destroy(ctx), "destroy")


def get_fields(ctx, nx, ny, nz, check=True):
    u = np.empty((nz, ny, nx + 1))
    v = np.empty((nz, ny, nx))
    w = np.empty((nz, ny, nx))
    p = np.empty((nz, ny, nx))
    t = ctypes.c_double()
    s = ctypes.c_int64()
    code = _lib.ibdns_get_fields(ctx, _dptr(u), _dptr(v), _dptr(w), _dptr(p), ctypes.byref(t),
                                 ctypes.byref(s))
    if check:
        _check(code, "get_fields")
    return u, v, w, p, t.value, s.value


def get_flag(ctx, ns, check=True):
    X = np.empty((ns, ns, 3))
    V = np.empty((ns, ns, 3))
    F = np.empty((ns, ns, 3))
    code = _lib.ibdns_get_flag(ctx, _dptr(X), _dptr(V), _dptr(F))
    if check:
        _check(code, "get_flag")
    return X, V, F


def get_array(ctx, which, shape):
    a = np.empty(shape)
    _check(_lib.ibdns_get_array(ctx, which, _dptr(a)), "get_array")
    return a


def set_array(ctx, which, arr):
    a = np.ascontiguousarray(arr, dtype=np.float64)
    _check(_lib.ibdns_set_array(ctx, which, _dptr(a)), "set_array")


def get_scalars(ctx, check=True):
    out = np.empty(6)
    code = _lib.ibdns_get_scalars(ctx, _dptr(out))
    if check:
        _check(code, "get_scalars")
    return dict(dt=out[0], dt_prev=out[1], t=out[2], speed=out[3], corr=out[4], nsub=int(out[5]))


def set_time(ctx, dt, dt_prev, first_step):
    _check(_lib.ibdns_set_time(ctx, dt, dt_prev, 1 if first_step else 0), "set_time")


def get_maps(ctx, comp, n_total):
    out = np.empty((n_total, 3), dtype=np.int32)
    _check(_lib.ibdns_get_maps(ctx, comp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "get_maps")
    return out


TIMING_OFF, TIMING_ALL, TIMING_PREDICT = 0, 1, 2


def enable_timing(ctx, mode=TIMING_ALL):
    """mode: TIMING_ALL (every kernel), TIMING_PREDICT (predictor only) or
    TIMING_OFF; True/False map to TIMING_ALL/TIMING_OFF."""
    if mode is True:
        mode = TIMING_ALL
    elif mode is False:
        mode = TIMING_OFF
    _check(_lib.ibdns_enable_timing(ctx, int(mode)), "enable_timing")


def kernel_times(ctx, nmax=64):
    names = (ctypes.c_char_p * nmax)()
    ms = np.zeros(nmax)
    cnt = np.zeros(nmax, dtype=np.int64)
    m = _lib.ibdns_kernel_times(ctx, nmax, names, _dptr(ms),
                                cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if m < 0:
        raise IbdnsError(m, "kernel_times")
    return {names[q].decode(): (ms[q], int(cnt[q])) for q in range(min(m, nmax))}


@dataclass
class Run:
    """A context plus the torch tensor that owns its workspace."""
    ctx: object
    ws: object
    nx: int
    ny: int
    nz: int
    ns: int = 0

    def step(self, n=1):
        step(self.ctx, n)

    def fields(self, check=True):
        return get_fields(self.ctx, self.nx, self.ny, self.nz, check)

    def flag(self, check=True):
        return get_flag(self.ctx, self.ns, check)

    def set_probes(self, n_x, x0, dx, yc, zc, dyz, n_lags, device="cuda:0"):
        """Place 9 n_x probes (record layout in include/ibdns.h); the workspace
        tensor is kept on this object."""
        import torch
        size = ctypes.c_size_t(0)
        _check(_lib.ibdns_probe_workspace_size(n_x, n_lags, ctypes.byref(size)),
               "probe_workspace_size")
        self.probe_ws = torch.empty(size.value, dtype=torch.uint8, device=device)
        _check(_lib.ibdns_set_probes(self.ctx, n_x, x0, dx, yc, zc, dyz, n_lags,
                                     ctypes.c_void_p(self.probe_ws.data_ptr()), size.value),
               "set_probes")
        self.probe_shape = (9 * n_x, 10 + 2 * n_lags)

    def probe_stats(self, check=True):
        # without probes the library answers ESTATE before writing anything
        out = np.empty(getattr(self, "probe_shape", (1, 1)))
        code = _lib.ibdns_get_probe_stats(self.ctx, _dptr(out))
        if check:
            _check(code, "get_probe_stats")
        return out

    def station_stats(self, device="cuda:0", check=True):
        """Per station: dict(k, anisotropy, f (L,), g (L,)) computed on the device
        (rule in include/ibdns.h); the staging tensor is allocated per call."""
        import torch
        ns_, L = ctypes.c_int32(0), ctypes.c_int32(0)
        size = ctypes.c_size_t(0)
        _check(_lib.ibdns_station_stats_size(self.ctx, ctypes.byref(ns_), ctypes.byref(L), ctypes.byref(size)),
               "station_stats_size")
        ws = torch.empty(max(size.value, 256), dtype=torch.uint8, device=device)
        out = np.empty((ns_.value, 2 + 2 * L.value))
        code = _lib.ibdns_get_station_stats(self.ctx, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _dptr(out))
        if check:
            _check(code, "get_station_stats")
        Lv = L.value
        return [dict(k=r[0], anisotropy=r[1], f=r[2:2 + Lv], g=r[2 + Lv:]) for r in out]

    def set_grid_forcing(self, dom: Domain, grid: GridParams, device="cuda:0"):
        """Eulerian forcing of the passive grid (rule in include/ibdns.h); the
        workspace tensor is kept on this object."""
        import torch
        size = ctypes.c_size_t(0)
        _check(_lib.ibdns_grid_forcing_workspace_size(ctypes.byref(dom), ctypes.byref(grid),
                                                      ctypes.byref(size)), "grid_forcing_workspace_size")
        self.grid_ws = torch.empty(max(size.value, 256), dtype=torch.uint8, device=device)
        _check(_lib.ibdns_set_grid_forcing(self.ctx, ctypes.byref(grid),
                                           ctypes.c_void_p(self.grid_ws.data_ptr()), self.grid_ws.numel()),
               "set_grid_forcing")

    def grid_forcing(self, comp):
        """(node, src, weight) of one component's forcing list, host-layout indices."""
        n = ctypes.c_int64(0)
        _check(_lib.ibdns_get_grid_forcing(self.ctx, comp, ctypes.byref(n), None, None, None),
               "get_grid_forcing")
        node = np.empty(n.value, dtype=np.int64)
        src = np.empty(n.value, dtype=np.int64)
        wgt = np.empty(n.value)
        I64 = ctypes.POINTER(ctypes.c_int64)
        _check(_lib.ibdns_get_grid_forcing(self.ctx, comp, ctypes.byref(n), node.ctypes.data_as(I64),
                                           src.ctypes.data_as(I64), _dptr(wgt)), "get_grid_forcing")
        return node, src, wgt

    def set_flag_mls(self, device="cuda:0"):
        """Couple the flag at the markers of its adaptive tiling by MLS (rule in
        include/ibdns.h); the workspace tensor is kept on this object."""
        import torch
        m = ctypes.c_int64(0)
        size = ctypes.c_size_t(0)
        _check(_lib.ibdns_flag_mls_workspace_size(self.ctx, ctypes.byref(m), ctypes.byref(size)),
               "flag_mls_workspace_size")
        self.mls_ws = torch.empty(max(size.value, 256), dtype=torch.uint8, device=device)
        _check(_lib.ibdns_set_flag_mls(self.ctx, ctypes.c_void_p(self.mls_ws.data_ptr()), self.mls_ws.numel()),
               "set_flag_mls")
        self.n_markers = m.value

    def flag_markers(self, check=True):
        """(tri (m, 3) int32, beta (m, 3), dV (m,), X (m, 3), F (m, 3)) of the MLS markers."""
        m = getattr(self, "n_markers", 0)
        tri = np.empty((max(m, 1), 3), dtype=np.int32)
        beta, X, F = (np.empty((max(m, 1), 3)) for _ in range(3))
        dV = np.empty(max(m, 1))
        code = _lib.ibdns_get_flag_markers(self.ctx, tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           _dptr(beta), _dptr(dV), _dptr(X), _dptr(F))
        if check:
            _check(code, "get_flag_markers")
        return tri[:m], beta[:m], dV[:m], X[:m], F[:m]

    def close(self):
        if self.ctx is not None:
            destroy(self.ctx)
            self.ctx = None


def create(dom: Domain, noise=None, grid=None, flag=None, device="cuda:0", stream=None,
           grid_forcing=None, flag_mls=False) -> Run:
    """Allocate the workspace with torch on ``device`` and build a context.
    grid: the passive grid as solid points; grid_forcing: the passive grid
    forced at the Eulerian nodes instead (then grid must be None); both
    GridParams or any object with x_plane, mesh, bar.  flag: FlagParams or any
    object with its fields.  flag_mls: couple the flag at its tiling markers
    by MLS instead of at its nodes by the delta."""
    import torch
    if grid is not None and not isinstance(grid, GridParams):
        grid = grid_from(grid)
    if grid_forcing is not None and not isinstance(grid_forcing, GridParams):
        grid_forcing = grid_from(grid_forcing)
    if flag is not None and not isinstance(flag, FlagParams):
        flag = flag_from(flag)
    ns = 0 if flag is None else flag.ns
    nbytes = workspace_size(dom, grid, flag)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    st = stream if stream is not None else torch.cuda.current_stream(device)
    ctx = init_domain(dom, noise, ws.data_ptr(), nbytes, st.cuda_stream)
    run = Run(ctx, ws, dom.nx, dom.ny, dom.nz, ns)
    try:
        if grid_forcing is not None:
            run.set_grid_forcing(dom, grid_forcing, device)
        if grid is not None or flag is not None:
            set_geometry(ctx, grid, flag)
        if flag_mls:
            run.set_flag_mls(device)
    except Exception:
        run.close()
        raise
    return run


def domain_from(w, precision=FP64, flags=0, diffusion=DIFFUSION_EXPLICIT) -> Domain:
    """Domain struct from any object with nx, ny, nz, lx, ly, lz, re, u_in, dt, cfl, noise_amp."""
    return make_domain(w.nx, w.ny, w.nz, w.lx, w.ly, w.lz, w.re, w.u_in, w.dt, w.cfl,
                       w.noise_amp, precision, flags, diffusion)


def flag_from(f) -> FlagParams | None:
    """FlagParams from any object with ns, length, x_le, y_c, z_c, pitch,
    mass_ratio, bending, stretch, le_bc (None passes through)."""
    if f is None:
        return None
    return FlagParams(f.ns, f.length, f.x_le, f.y_c, f.z_c, f.pitch, f.mass_ratio, f.bending,
                      f.stretch, f.le_bc)


def grid_from(g) -> GridParams | None:
    """GridParams from any object with x_plane, mesh, bar (None passes through)."""
    if g is None:
        return None
    return GridParams(g.x_plane, g.mesh, g.bar)


NUM_TILES = 14


def set_tile(ctx, variant: int):
    _check(_lib.ibdns_set_tile(ctx, variant), "set_tile")


def autotune(ctx) -> int:
    v = ctypes.c_int32(-1)
    _check(_lib.ibdns_autotune(ctx, ctypes.byref(v)), "autotune")
    return v.value


class Batch:
    """Independent runs advanced together (one launch per stage over all runs)."""

    def __init__(self, runs, device="cuda:0"):
        import torch
        self.runs = list(runs)
        n = len(self.runs)
        size = ctypes.c_size_t(0)
        _check(_lib.ibdns_batch_workspace_size(n, ctypes.byref(size)), "batch_workspace_size")
        self.ws = torch.empty(size.value, dtype=torch.uint8, device=device)
        arr = (ctypes.c_void_p * n)(*[r.ctx.value for r in self.runs])
        self.handle = ctypes.c_void_p()
        _check(_lib.ibdns_batch_create(arr, n, ctypes.c_void_p(self.ws.data_ptr()), size.value,
                                       ctypes.byref(self.handle)), "batch_create")

    def autotune(self) -> int:
        v = ctypes.c_int32(-1)
        _check(_lib.ibdns_batch_autotune(self.handle, ctypes.byref(v)), "batch_autotune")
        return v.value

    def use_graph(self, on=True):
        _check(_lib.ibdns_batch_use_graph(self.handle, 1 if on else 0), "batch_use_graph")

    def step(self, n=1):
        _check(_lib.ibdns_batch_step(self.handle, n), "batch_step")

    def close(self):
        if self.handle is not None and self.handle.value:
            _check(_lib.ibdns_batch_destroy(self.handle), "batch_destroy")
            self.handle = None
