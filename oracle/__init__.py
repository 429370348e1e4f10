"""FP64 CPU oracle of the HB-UGKS pseudo-time step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU path
(``paper_2605_03479_amd``) and neither imports the other.

The arithmetic lives in ``hbref.c`` (plain C, FP64), which follows Section 2
of the HB-UGKS paper (arXiv 2605.03479); see the header of that file for the
equation map.  This module only marshals arguments through ctypes.

Layouts: W[c][n][4], h/b[c][n][alpha], c = j*nx + i, alpha = iv*M + iu.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _p(a):
    return a.ctypes.data_as(_D) if a is not None else None


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.hbref_new.restype = ctypes.c_void_p
        L.hbref_free.argtypes = [ctypes.c_void_p]
        L.hbref_setup.restype = ctypes.c_int
        L.hbref_setup.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, _D, _D, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, _D,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, _D, _D, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  _D, _D]
        L.hbref_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.hbref_td_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        L.hbref_residual.argtypes = [ctypes.c_void_p, _D]
        L.hbref_step_index.restype = ctypes.c_long
        L.hbref_step_index.argtypes = [ctypes.c_void_p]
        L.hbref_get_state.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.hbref_set_state.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.hbref_get_debug.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.hbref_harmonics.argtypes = [ctypes.c_void_p, _D, _D]
        L.hbref_sizes.argtypes = [ctypes.c_void_p, _I]
        L.hbref_constants.argtypes = [ctypes.c_void_p, _D]
        L.hbref_max_nu.restype = ctypes.c_double
        L.hbref_max_nu.argtypes = [ctypes.c_void_p]
        L.hbref_threads.restype = ctypes.c_int
        L.hbref_set_dt_scale.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.hbref_time.restype = ctypes.c_double
        L.hbref_time.argtypes = [ctypes.c_void_p]
        L.hbref_E.argtypes = [ctypes.c_int, _D]
        L.hbref_ccoef.argtypes = [ctypes.c_double, ctypes.c_double, _D]
        L.hbref_velocity_grid.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D]
        L.hbref_moments_normal.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, _D]
        L.hbref_slope_solve.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, _D, _D]
        L.hbref_moment_vec.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, _D]
        L.hbref_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, ctypes.c_int, _D,
                                        _D, _D, _D, _D, _D]
        _LIB = L
    return _LIB


def threads():
    """OpenMP threads the oracle uses."""
    return lib().hbref_threads()


# ---------------------------------------------------------------- unit-level
def E_matrix(NT):
    """Spectral operator E of Eq. (17)."""
    E = np.zeros(NT * NT)
    lib().hbref_E(NT, _p(E))
    return E.reshape(NT, NT)


def ccoef(tau, dG):
    """(C1..C5) of Eq. (22)."""
    C = np.zeros(5)
    lib().hbref_ccoef(float(tau), float(dG), _p(C))
    return C


def velocity_grid(M, umax):
    u1 = np.zeros(M)
    w1 = np.zeros(M)
    lib().hbref_velocity_grid(M, float(umax), _p(u1), _p(w1))
    return u1, w1


def moments_normal(U, lam, which, nmax):
    m = np.zeros(nmax + 1)
    lib().hbref_moments_normal(float(U), float(lam), int(which), int(nmax), _p(m))
    return m


def slope_solve(Un, Ut, lam, K, d):
    d = np.ascontiguousarray(d, dtype=np.float64)
    a = np.zeros(4)
    lib().hbref_slope_solve(float(Un), float(Ut), float(lam), int(K), _p(d), _p(a))
    return a


def moment_vec(a, pn, pt, Un, Ut, lam, K, which):
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros(4)
    lib().hbref_moment_vec(_p(a), pn, pt, float(Un), float(Ut), float(lam), int(K), int(which),
                           _p(out))
    return out


def equilibrium(K, Pr, prim, q, u, v):
    """Per-velocity (H, B, H+, B+) of the reduced Shakhov equilibrium."""
    prim = np.ascontiguousarray(prim, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    n = u.size
    H, B, Hp, Bp = (np.zeros(n) for _ in range(4))
    lib().hbref_equilibrium(int(K), float(Pr), _p(prim), _p(q), n, _p(u), _p(v), _p(H), _p(B),
                            _p(Hp), _p(Bp))
    return H, B, Hp, Bp


def gauss_hermite(M):
    """M-point Gauss-Hermite rule for the weight exp(-u^2) (the velocity
    quadrature of Sec. 3.1.1 for Kn <= 0.1), with the weight folded into the
    returned weights, w_k exp(u_k^2), so that sum_k w_k f(u_k) approximates
    the plain integral of f.  Nodes and Gauss weights from numpy."""
    x, w = np.polynomial.hermite.hermgauss(int(M))
    return np.ascontiguousarray(x), np.ascontiguousarray(w * np.exp(x * x))


def velocity_rule(case):
    """1-D nodes and weights of a case's velocity rule along u."""
    if getattr(case, "vrule", 0) == 1:
        return gauss_hermite(case.M)
    return velocity_grid(case.M, case.umax)


def velocity_rule_v(case):
    """1-D nodes and weights of a case's velocity rule along v (M_v nodes; the
    trapezoid on [-vmax, vmax])."""
    Mv = getattr(case, "Mv", 0) or case.M
    if getattr(case, "vrule", 0) == 1:
        return gauss_hermite(Mv)
    vmax = getattr(case, "vmax", 0.0)
    return velocity_grid(Mv, vmax if vmax > 0.0 else case.umax)


# ---------------------------------------------------------------- solver
class Oracle:
    """One HB-UGKS case on the CPU (FP64).  ``case`` is an ``hbcases.Case``."""

    def __init__(self, case, td=False):
        self.case = case
        self._h = lib().hbref_new()
        walls = np.ascontiguousarray(case.walls, dtype=np.float64).reshape(4, 6)
        xf = None if case.x_faces is None else np.ascontiguousarray(case.x_faces, np.float64)
        yf = None if case.y_faces is None else np.ascontiguousarray(case.y_faces, np.float64)
        NH = 0 if td else case.NH
        dt_mode = 1 if td else case.dt_mode
        u1, w1 = velocity_rule(case) if getattr(case, "vrule", 0) else (None, None)
        Mv = getattr(case, "Mv", 0) or case.M
        vmax = getattr(case, "vmax", 0.0)
        v1, w1v = velocity_rule_v(case) if getattr(case, "vrule", 0) else (None, None)
        rc = lib().hbref_setup(self._h, case.nx, case.ny, case.L, case.H, _p(xf), _p(yf), case.M,
                               case.umax, case.Kn, case.St, NH, _p(walls), case.cfl,
                               case.face_dt, case.Pr, case.omega_vss, case.alpha_vss, case.K,
                               case.macro_mode, dt_mode, case.dt_fixed, _p(u1), _p(w1),
                               int(getattr(case, "level_mass", 1)), Mv, float(vmax), _p(v1), _p(w1v))
        if rc != 0:
            lib().hbref_free(self._h)
            self._h = None
            raise ValueError("oracle rejected the case")
        s = np.zeros(6, dtype=np.int32)
        lib().hbref_sizes(self._h, s.ctypes.data_as(_I))
        self.nx, self.ny, self.nc, self.M, self.nv, self.NT = (int(x) for x in s)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().hbref_free(self._h)
            self._h = None

    def constants(self):
        c = np.zeros(3)
        lib().hbref_constants(self._h, _p(c))
        return {"mu_ref": c[0], "omega": c[1], "gamma": c[2]}

    def step(self, n=1):
        lib().hbref_step(self._h, int(n))

    def td_step(self, n, omega):
        lib().hbref_td_step(self._h, int(n), float(omega))

    def time(self):
        return lib().hbref_time(self._h)

    def set_dt_scale(self, s):
        """Test hook: multiply every local pseudo step by s."""
        lib().hbref_set_dt_scale(self._h, float(s))

    def max_nu(self):
        return lib().hbref_max_nu(self._h)

    def residual(self):
        r = np.zeros(4)
        lib().hbref_residual(self._h, _p(r))
        return r

    def step_index(self):
        return lib().hbref_step_index(self._h)

    def state(self):
        W = np.zeros((self.nc, self.NT, 4))
        h = np.zeros((self.nc, self.NT, self.nv))
        b = np.zeros((self.nc, self.NT, self.nv))
        lib().hbref_get_state(self._h, _p(W), _p(h), _p(b))
        return W, h, b

    def set_state(self, W, h, b):
        W = np.ascontiguousarray(W, dtype=np.float64)
        h = np.ascontiguousarray(h, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        assert W.size == self.nc * self.NT * 4 and h.size == b.size == self.nc * self.NT * self.nv
        lib().hbref_set_state(self._h, _p(W), _p(h), _p(b))

    def debug(self):
        """(local steps of the last step, x-face macro fluxes, y-face macro fluxes)."""
        dtc = np.zeros(self.nc)
        Fx = np.zeros((self.ny, self.nx + 1, self.NT, 4))
        Fy = np.zeros((self.ny + 1, self.nx, self.NT, 4))
        lib().hbref_get_debug(self._h, _p(dtc), _p(Fx), _p(Fy))
        return dtc, Fx, Fy

    def harmonics(self):
        """re, im with shape [7 vars][NH+1][nc]: rho, U, V, T, P_xy, q_x, q_y (Eq. 40)."""
        NH = (self.NT - 1) // 2
        re = np.zeros((7, NH + 1, self.nc))
        im = np.zeros((7, NH + 1, self.nc))
        lib().hbref_harmonics(self._h, _p(re), _p(im))
        return re, im
