"""MI355X-native HB-UGKS pseudo-step engine.

The work runs in the gfx950 HIP library ``libhbugks.so`` behind the C ABI of
``include/hb_ugks.h``; this module only marshals arguments through ctypes
(same entry-point names) and wraps a handle in :class:`Solver`.  There is no
CPU fallback: if the library is missing, loading fails loudly.

Host layouts: W[c][n][4], h/b[c][n][alpha], c = j*nx + i, alpha = iv*M + iu.
"""
import ctypes
import os

import numpy as np

from . import build as _build

HB_OK, HB_EINVAL, HB_ENOMEM, HB_ESTATE, HB_EDIVERGED, HB_EDEVICE, HB_ECAPACITY = 0, -1, -2, -3, -4, -5, -6
HB_FP64, HB_MIXED = 0, 1
HB_RULE_TRAPEZOID, HB_RULE_GAUSS_HERMITE = 0, 1
VARS = ("rho", "U", "V", "T", "Pxy", "qx", "qy")

_D = ctypes.POINTER(ctypes.c_double)


class hb_create_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("precision", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_size_t)]


class hb_geometry(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("H", ctypes.c_double), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("x_faces", _D), ("y_faces", _D)]


class hb_wall(ctypes.Structure):
    _fields_ = [("ut_mean", ctypes.c_double), ("ut_hat_re", ctypes.c_double), ("ut_hat_im", ctypes.c_double),
                ("T_mean", ctypes.c_double), ("T_hat_re", ctypes.c_double), ("T_hat_im", ctypes.c_double)]


class hb_vgrid(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("umax", ctypes.c_double), ("rule", ctypes.c_int), ("m_v", ctypes.c_int),
                ("vmax", ctypes.c_double)]


class hb_numerics(ctypes.Structure):
    _fields_ = [("cfl", ctypes.c_double), ("face_dt", ctypes.c_int), ("Pr", ctypes.c_double),
                ("omega_vss", ctypes.c_double), ("alpha_vss", ctypes.c_double), ("K_int", ctypes.c_int),
                ("dt_mode", ctypes.c_int), ("dt_fixed", ctypes.c_double), ("macro_flux_mode", ctypes.c_int),
                ("level_mass", ctypes.c_int)]


class hb_request(ctypes.Structure):
    _fields_ = [("geo", hb_geometry), ("Kn", ctypes.c_double), ("St", ctypes.c_double), ("n_harmonics", ctypes.c_int),
                ("walls", hb_wall * 4), ("vg", hb_vgrid), ("has_numerics", ctypes.c_int), ("num", hb_numerics),
                ("precision", ctypes.c_int), ("arrival_s", ctypes.c_double), ("var_mask", ctypes.c_uint),
                ("re", _D), ("im", _D), ("capacity", ctypes.c_size_t)]


class hb_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_long), ("residual", ctypes.c_double * 4),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("bytes", ctypes.c_size_t)]


EXPORTS = ("hb_vgrid_nodes", "hb_ugks_default_numerics", "hb_ugks_create", "hb_ugks_set_case", "hb_ugks_pseudo_step",
           "hb_ugks_td_step", "hb_ugks_td_period", "hb_ugks_time", "hb_ugks_wall_harmonic",
           "hb_ugks_residual", "hb_ugks_harmonics_out", "hb_ugks_harmonics_out_noalloc", "hb_ugks_state_out",
           "hb_ugks_state_in",
           "hb_ugks_sizes", "hb_ugks_device_bytes", "hb_ugks_enable_timing", "hb_ugks_kernel_times",
           "hb_ugks_destroy", "hb_ugks_strerror",
           "hb_batch_create", "hb_batch_case_bytes", "hb_batch_add", "hb_batch_remove", "hb_batch_set_active",
           "hb_batch_step", "hb_batch_residuals", "hb_batch_case", "hb_batch_tune", "hb_batch_shapes",
           "hb_batch_use_graph", "hb_batch_set_cache_bytes", "hb_batch_pool_info", "hb_batch_destroy",
           "hb_serve_run")

_LIB = None


def load_library(path=None):
    """Load libhbugks.so (never builds; raises if it is absent)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or _build.LIB
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(p)
    vp, ip, dp, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.hb_vgrid_nodes.argtypes = [ctypes.POINTER(hb_vgrid), _D, _D]
    L.hb_vgrid_nodes.restype = ctypes.c_int
    L.hb_ugks_default_numerics.argtypes = [ctypes.POINTER(hb_numerics)]
    L.hb_ugks_default_numerics.restype = None
    L.hb_ugks_create.argtypes = [ctypes.POINTER(hb_create_opts), ctypes.POINTER(vp)]
    L.hb_ugks_set_case.argtypes = [vp, ctypes.POINTER(hb_geometry), dp, dp, ip, ctypes.POINTER(hb_wall),
                                   ctypes.POINTER(hb_vgrid), ctypes.POINTER(hb_numerics)]
    L.hb_ugks_pseudo_step.argtypes = [vp, ip]
    L.hb_ugks_td_step.argtypes = [vp, ip]
    L.hb_ugks_td_period.argtypes = [vp, ip, _D]
    L.hb_ugks_time.argtypes = [vp, ctypes.POINTER(dp)]
    L.hb_ugks_wall_harmonic.argtypes = [vp, ip, ip, ip, _D]
    L.hb_ugks_residual.argtypes = [vp, _D, ctypes.POINTER(ctypes.c_long)]
    L.hb_ugks_harmonics_out.argtypes = [vp, ctypes.c_uint, _D, _D, sz]
    L.hb_ugks_harmonics_out_noalloc.argtypes = [vp, ctypes.c_uint, _D, _D, sz]
    L.hb_ugks_state_out.argtypes = [vp, _D, _D, _D, sz]
    L.hb_ugks_state_in.argtypes = [vp, _D, _D, _D]
    L.hb_ugks_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.hb_ugks_device_bytes.argtypes = [vp]
    L.hb_ugks_device_bytes.restype = sz
    L.hb_ugks_enable_timing.argtypes = [vp, ip]
    L.hb_ugks_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_long), _D, ip]
    L.hb_ugks_destroy.argtypes = [vp]
    L.hb_ugks_destroy.restype = None
    L.hb_ugks_strerror.argtypes = [ip]
    L.hb_ugks_strerror.restype = ctypes.c_char_p
    szp, lp = ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_long)
    L.hb_batch_create.argtypes = [ctypes.POINTER(hb_create_opts), sz, ip, ctypes.POINTER(vp)]
    L.hb_batch_case_bytes.argtypes = [vp, ip, ctypes.POINTER(hb_geometry), ip, ctypes.POINTER(hb_vgrid), szp]
    L.hb_batch_add.argtypes = [vp, ip, ctypes.POINTER(hb_geometry), dp, dp, ip, ctypes.POINTER(hb_wall),
                               ctypes.POINTER(hb_vgrid), ctypes.POINTER(hb_numerics), ctypes.POINTER(ip)]
    L.hb_batch_remove.argtypes = [vp, ip]
    L.hb_batch_set_active.argtypes = [vp, ip, ip]
    L.hb_batch_step.argtypes = [vp, ip]
    L.hb_batch_residuals.argtypes = [vp, _D, lp, ctypes.POINTER(ip), ctypes.POINTER(ip), ip]
    L.hb_batch_case.argtypes = [vp, ip, ctypes.POINTER(vp)]
    L.hb_batch_tune.argtypes = [vp, ip]
    L.hb_batch_shapes.argtypes = [vp, ctypes.POINTER(ip), ip]
    L.hb_batch_use_graph.argtypes = [vp, ip]
    L.hb_batch_set_cache_bytes.argtypes = [vp, sz]
    L.hb_batch_pool_info.argtypes = [vp, szp, szp, szp]
    L.hb_batch_destroy.argtypes = [vp]
    L.hb_batch_destroy.restype = None
    L.hb_serve_run.argtypes = [vp, ctypes.POINTER(hb_request), ip, dp, ip, ctypes.c_long, dp,
                               ctypes.POINTER(hb_result), ctypes.POINTER(dp)]
    L.hb_serve_run.restype = ctypes.c_int
    for name in ("hb_ugks_create", "hb_ugks_set_case", "hb_ugks_pseudo_step", "hb_ugks_td_step",
                 "hb_ugks_td_period", "hb_ugks_time", "hb_ugks_wall_harmonic", "hb_ugks_residual",
                 "hb_ugks_harmonics_out", "hb_ugks_harmonics_out_noalloc", "hb_ugks_state_out", "hb_ugks_state_in",
                 "hb_ugks_sizes",
                 "hb_ugks_enable_timing", "hb_ugks_kernel_times", "hb_batch_create", "hb_batch_case_bytes",
                 "hb_batch_add", "hb_batch_remove", "hb_batch_set_active", "hb_batch_step", "hb_batch_residuals",
                 "hb_batch_case", "hb_batch_tune", "hb_batch_shapes", "hb_batch_use_graph", "hb_batch_set_cache_bytes",
                 "hb_batch_pool_info"):
        getattr(L, name).restype = ctypes.c_int
    if path is None:
        _LIB = L
    return L


class HBError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = load_library().hb_ugks_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def _check(code, what):
    if code < 0:
        raise HBError(code, what)
    return code


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


# ------------------------------------------------------------- C-ABI mirrors
def hb_ugks_create(device=0, stream=None, precision=HB_FP64, hbm_budget_bytes=0):
    o = hb_create_opts(device, stream, precision, hbm_budget_bytes)
    h = ctypes.c_void_p()
    _check(load_library().hb_ugks_create(ctypes.byref(o), ctypes.byref(h)), "hb_ugks_create")
    return h


def default_numerics():
    n = hb_numerics()
    load_library().hb_ugks_default_numerics(ctypes.byref(n))
    return n


def _case_args(case):
    """(geometry, walls, vgrid, numerics, keep-alive arrays) of an hbcases.Case."""
    xf = None if case.x_faces is None else np.ascontiguousarray(case.x_faces, np.float64)
    yf = None if case.y_faces is None else np.ascontiguousarray(case.y_faces, np.float64)
    g = hb_geometry(case.L, case.H, case.nx, case.ny, _dp(xf), _dp(yf))
    walls = (hb_wall * 4)(*[hb_wall(*map(float, w)) for w in case.walls])
    vg = hb_vgrid(case.M, case.umax, case.vrule, getattr(case, "Mv", 0), getattr(case, "vmax", 0.0))
    nm = hb_numerics(case.cfl, case.face_dt, case.Pr, case.omega_vss, case.alpha_vss, case.K, case.dt_mode,
                     case.dt_fixed, case.macro_mode, getattr(case, "level_mass", 1))
    return g, walls, vg, nm, (xf, yf)


def hb_ugks_set_case(h, case):
    """case: an object with the fields of hbcases.Case."""
    g, walls, vg, nm, keep = _case_args(case)
    return _check(load_library().hb_ugks_set_case(h, ctypes.byref(g), case.Kn, case.St, case.NH, walls,
                                                   ctypes.byref(vg), ctypes.byref(nm)), "hb_ugks_set_case")


def hb_ugks_pseudo_step(h, nsteps):
    return _check(load_library().hb_ugks_pseudo_step(h, int(nsteps)), "hb_ugks_pseudo_step")


def hb_vgrid_nodes(m, umax=4.0, rule=HB_RULE_TRAPEZOID):
    """1-D nodes and weights of a velocity rule (host only)."""
    u = np.zeros(m)
    w = np.zeros(m)
    vg = hb_vgrid(int(m), float(umax), int(rule))
    _check(load_library().hb_vgrid_nodes(ctypes.byref(vg), _dp(u), _dp(w)), "hb_vgrid_nodes")
    return u, w


def hb_ugks_td_step(h, nsteps):
    return _check(load_library().hb_ugks_td_step(h, int(nsteps)), "hb_ugks_td_step")


def hb_ugks_td_period(h, nsteps):
    out = np.zeros(4)
    _check(load_library().hb_ugks_td_period(h, int(nsteps), _dp(out)), "hb_ugks_td_period")
    return out


def hb_ugks_time(h):
    t = ctypes.c_double()
    _check(load_library().hb_ugks_time(h, ctypes.byref(t)), "hb_ugks_time")
    return t.value


def hb_ugks_wall_harmonic(h, wall, var, k):
    out = np.zeros(2)
    _check(load_library().hb_ugks_wall_harmonic(h, int(wall), int(var), int(k), _dp(out)), "hb_ugks_wall_harmonic")
    return complex(out[0], out[1])


def hb_ugks_residual(h):
    out = np.zeros(4)
    k = ctypes.c_long()
    rc = load_library().hb_ugks_residual(h, _dp(out), ctypes.byref(k))
    return rc, out, k.value


def hb_ugks_sizes(h):
    s = (ctypes.c_int * 6)()
    _check(load_library().hb_ugks_sizes(h, s), "hb_ugks_sizes")
    return tuple(s)


def hb_ugks_harmonics_out(h, var_mask=0x7F):
    nx, ny, nc, M, nv, NT = hb_ugks_sizes(h)
    nsel = bin(var_mask & 0x7F).count("1")
    NH = (NT - 1) // 2
    re = np.zeros((nsel, NH + 1, nc))
    im = np.zeros((nsel, NH + 1, nc))
    _check(load_library().hb_ugks_harmonics_out(h, var_mask, _dp(re), _dp(im), re.size), "hb_ugks_harmonics_out")
    return re, im


def hb_ugks_harmonics_out_noalloc(h, var_mask=0x7F):
    """hb_ugks_harmonics_out through the library's static device scratch (no device allocation)."""
    nx, ny, nc, M, nv, NT = hb_ugks_sizes(h)
    nsel = bin(var_mask & 0x7F).count("1")
    NH = (NT - 1) // 2
    re = np.zeros((nsel, NH + 1, nc))
    im = np.zeros((nsel, NH + 1, nc))
    _check(load_library().hb_ugks_harmonics_out_noalloc(h, var_mask, _dp(re), _dp(im), re.size),
           "hb_ugks_harmonics_out_noalloc")
    return re, im


def hb_ugks_state_out(h):
    nx, ny, nc, M, nv, NT = hb_ugks_sizes(h)
    W = np.zeros((nc, NT, 4))
    hh = np.zeros((nc, NT, nv))
    bb = np.zeros((nc, NT, nv))
    _check(load_library().hb_ugks_state_out(h, _dp(W), _dp(hh), _dp(bb), hh.size), "hb_ugks_state_out")
    return W, hh, bb


def hb_ugks_state_in(h, W, hh, bb):
    nx, ny, nc, M, nv, NT = hb_ugks_sizes(h)
    W = None if W is None else np.ascontiguousarray(W, np.float64).reshape(-1)
    hh = None if hh is None else np.ascontiguousarray(hh, np.float64).reshape(-1)
    bb = None if bb is None else np.ascontiguousarray(bb, np.float64).reshape(-1)
    for a, n in ((W, nc * NT * 4), (hh, nc * NT * nv), (bb, nc * NT * nv)):
        if a is not None and a.size != n:
            raise ValueError("state array of the wrong size")
    return _check(load_library().hb_ugks_state_in(h, _dp(W), _dp(hh), _dp(bb)), "hb_ugks_state_in")


def hb_ugks_enable_timing(h, on=True):
    return _check(load_library().hb_ugks_enable_timing(h, int(on)), "hb_ugks_enable_timing")


def hb_ugks_kernel_times(h):
    cap = 16
    names = (ctypes.c_char_p * cap)()
    launches = (ctypes.c_long * cap)()
    ms = (ctypes.c_double * cap)()
    n = _check(load_library().hb_ugks_kernel_times(h, names, launches, ms, cap), "hb_ugks_kernel_times")
    return {names[k].decode(): (launches[k], ms[k]) for k in range(n)}


def hb_ugks_device_bytes(h):
    return load_library().hb_ugks_device_bytes(h)


def hb_ugks_destroy(h):
    load_library().hb_ugks_destroy(h)


class Solver:
    """One case on one GPU: create + set_case; methods mirror the C ABI."""

    def __init__(self, case, device=0, stream=None, precision=HB_FP64, hbm_budget_bytes=0):
        self.case = case
        self.h = hb_ugks_create(device, stream, precision, hbm_budget_bytes)
        try:
            hb_ugks_set_case(self.h, case)
        except Exception:
            hb_ugks_destroy(self.h)
            self.h = None
            raise
        self.sizes = hb_ugks_sizes(self.h)

    def close(self):
        if getattr(self, "h", None):
            hb_ugks_destroy(self.h)
            self.h = None

    __del__ = close

    def step(self, n=1):
        hb_ugks_pseudo_step(self.h, n)

    def td_step(self, n=1):
        hb_ugks_td_step(self.h, n)

    def td_period(self, nsteps):
        return hb_ugks_td_period(self.h, nsteps)

    def time(self):
        return hb_ugks_time(self.h)

    def wall_harmonic(self, wall, var, k=1):
        return hb_ugks_wall_harmonic(self.h, wall, var, k)

    def residual(self):
        rc, r, k = hb_ugks_residual(self.h)
        _check(rc, "hb_ugks_residual")
        return r

    def step_index(self):
        return hb_ugks_residual(self.h)[2]

    def state(self):
        return hb_ugks_state_out(self.h)

    def macro(self):
        """W[c][n][4] only (no distribution copy)."""
        nx, ny, nc, M, nv, NT = self.sizes
        W = np.zeros((nc, NT, 4))
        _check(load_library().hb_ugks_state_out(self.h, _dp(W), None, None, 0), "hb_ugks_state_out")
        return W

    def set_state(self, W, h, b):
        hb_ugks_state_in(self.h, W, h, b)

    def harmonics(self, var_mask=0x7F):
        return hb_ugks_harmonics_out(self.h, var_mask)

    def enable_timing(self, on=True):
        hb_ugks_enable_timing(self.h, on)

    def kernel_times(self):
        return hb_ugks_kernel_times(self.h)

    def device_bytes(self):
        return hb_ugks_device_bytes(self.h)


# ------------------------------------------------------------- batched form
def hb_batch_create(device=0, stream=None, pool_bytes=0, max_cases=64, hbm_budget_bytes=0):
    o = hb_create_opts(device, stream, HB_FP64, hbm_budget_bytes)
    b = ctypes.c_void_p()
    _check(load_library().hb_batch_create(ctypes.byref(o), pool_bytes, max_cases, ctypes.byref(b)),
           "hb_batch_create")
    return b


def hb_batch_case_bytes(b, case, precision=HB_FP64):
    g, walls, vg, nm, keep = _case_args(case)
    n = ctypes.c_size_t()
    _check(load_library().hb_batch_case_bytes(b, precision, ctypes.byref(g), case.NH, ctypes.byref(vg),
                                              ctypes.byref(n)), "hb_batch_case_bytes")
    return n.value


def hb_batch_add(b, case, precision=HB_FP64):
    """Returns the slot, or raises HBError (HB_ENOMEM: does not fit the pool now)."""
    g, walls, vg, nm, keep = _case_args(case)
    cid = ctypes.c_int()
    _check(load_library().hb_batch_add(b, precision, ctypes.byref(g), case.Kn, case.St, case.NH, walls,
                                       ctypes.byref(vg), ctypes.byref(nm), ctypes.byref(cid)), "hb_batch_add")
    return cid.value


def hb_batch_remove(b, cid):
    return _check(load_library().hb_batch_remove(b, int(cid)), "hb_batch_remove")


def hb_batch_set_active(b, cid, on):
    return _check(load_library().hb_batch_set_active(b, int(cid), int(on)), "hb_batch_set_active")


def hb_batch_step(b, nsteps):
    return _check(load_library().hb_batch_step(b, int(nsteps)), "hb_batch_step")


def hb_batch_residuals(b, capacity=4096):
    """{slot: (residual[4], steps, diverged)} of the active cases."""
    res = np.zeros((capacity, 4))
    steps = (ctypes.c_long * capacity)()
    div = (ctypes.c_int * capacity)()
    ids = (ctypes.c_int * capacity)()
    n = _check(load_library().hb_batch_residuals(b, _dp(res), steps, div, ids, capacity), "hb_batch_residuals")
    return {ids[k]: (res[k].copy(), steps[k], bool(div[k])) for k in range(n)}


def hb_batch_case(b, cid):
    h = ctypes.c_void_p()
    _check(load_library().hb_batch_case(b, int(cid), ctypes.byref(h)), "hb_batch_case")
    return h


def hb_batch_tune(b, reps=3):
    return _check(load_library().hb_batch_tune(b, int(reps)), "hb_batch_tune")


def hb_batch_shapes(b):
    out = (ctypes.c_int * 5 * 64)()
    n = _check(load_library().hb_batch_shapes(b, ctypes.cast(out, ctypes.POINTER(ctypes.c_int)), 5 * 64),
               "hb_batch_shapes")
    flat = ctypes.cast(out, ctypes.POINTER(ctypes.c_int))
    return [dict(precision=flat[5 * k], NT=flat[5 * k + 1], nvp=flat[5 * k + 2], threads=flat[5 * k + 3],
                 blocks_per_cu=flat[5 * k + 4]) for k in range(n)]


def hb_batch_use_graph(b, on):
    return _check(load_library().hb_batch_use_graph(b, int(on)), "hb_batch_use_graph")


def hb_batch_set_cache_bytes(b, nbytes):
    return _check(load_library().hb_batch_set_cache_bytes(b, int(nbytes)), "hb_batch_set_cache_bytes")


def hb_batch_pool_info(b):
    c, u, f = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().hb_batch_pool_info(b, ctypes.byref(c), ctypes.byref(u), ctypes.byref(f)),
           "hb_batch_pool_info")
    return c.value, u.value, f.value


def hb_batch_destroy(b):
    load_library().hb_batch_destroy(b)


class BatchCase:
    """Queries on one case of a batch (the batch owns and steps it)."""

    def __init__(self, batch, cid):
        self.batch, self.cid = batch, cid

    def _h(self):
        return hb_batch_case(self.batch.b, self.cid)

    def residual(self):
        rc, r, k = hb_ugks_residual(self._h())
        _check(rc, "hb_ugks_residual")
        return r

    def step_index(self):
        return hb_ugks_residual(self._h())[2]

    def state(self):
        return hb_ugks_state_out(self._h())

    def set_state(self, W, h, b):
        hb_ugks_state_in(self._h(), W, h, b)

    def harmonics(self, var_mask=0x7F):
        return hb_ugks_harmonics_out(self._h(), var_mask)


class Batch:
    """Many cases on one GPU, stepped together (see the batched section of hb_ugks.h)."""

    def __init__(self, device=0, stream=None, pool_bytes=0, max_cases=64, hbm_budget_bytes=0):
        self.b = hb_batch_create(device, stream, pool_bytes, max_cases, hbm_budget_bytes)

    def close(self):
        if getattr(self, "b", None):
            hb_batch_destroy(self.b)
            self.b = None

    __del__ = close

    def case_bytes(self, case, precision=HB_FP64):
        return hb_batch_case_bytes(self.b, case, precision)

    def add(self, case, precision=HB_FP64):
        return BatchCase(self, hb_batch_add(self.b, case, precision))

    def remove(self, bc):
        hb_batch_remove(self.b, bc.cid)

    def set_active(self, bc, on):
        hb_batch_set_active(self.b, bc.cid, on)

    def step(self, n=1):
        hb_batch_step(self.b, n)

    def residuals(self):
        return hb_batch_residuals(self.b)

    def tune(self, reps=3):
        hb_batch_tune(self.b, reps)

    def shapes(self):
        return hb_batch_shapes(self.b)

    def use_graph(self, on):
        hb_batch_use_graph(self.b, on)

    def set_cache_bytes(self, nbytes):
        hb_batch_set_cache_bytes(self.b, nbytes)

    def pool_info(self):
        return hb_batch_pool_info(self.b)


# ------------------------------------------------------------- serving
def serve(batch, cases, arrivals, precision=HB_MIXED, tol=1e-8, check_every=100, max_steps=200000,
          var_mask=0x7F, max_wall_s=0.0):
    """Run the serving loop (hb_serve_run) on an empty Batch.  Returns
    (results: list of dicts, harmonics: list of (re, im) or None, wall seconds).
    max_wall_s > 0 caps the run (resident cases then retire unconverged)."""
    n = len(cases)
    reqs = (hb_request * n)()
    keep = []
    harm = []
    for k, (c, t) in enumerate(zip(cases, arrivals)):
        g, walls, vg, nm, kk = _case_args(c)
        keep.append(kk)
        nsel = bin(var_mask & 0x7F).count("1")
        re = np.zeros((nsel, c.NH + 1, c.nx * c.ny))
        im = np.zeros_like(re)
        harm.append((re, im))
        r = reqs[k]
        r.geo = g
        r.Kn, r.St, r.n_harmonics = c.Kn, c.St, c.NH
        for w in range(4):
            r.walls[w] = walls[w]
        r.vg = vg
        r.has_numerics = 1
        r.num = nm
        r.precision = precision
        r.arrival_s = float(t)
        r.var_mask = var_mask
        r.re, r.im, r.capacity = _dp(re), _dp(im), re.size
    out = (hb_result * n)()
    wall = ctypes.c_double()
    _check(load_library().hb_serve_run(batch.b, reqs, n, float(tol), int(check_every), int(max_steps),
                                       float(max_wall_s), out, ctypes.byref(wall)), "hb_serve_run")
    res = [dict(status=o.status, steps=o.steps, residual=list(o.residual), t_admit=o.t_admit, t_done=o.t_done,
                arrival=float(t), bytes=o.bytes) for o, t in zip(out, arrivals)]
    return res, [h if r["status"] == HB_OK else None for h, r in zip(harm, res)], wall.value
