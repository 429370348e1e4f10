"""Near-continuum pin: oscillating Stokes layers against the analytic profile.

At Kn = 0.01 the gas next to a wall oscillating tangentially as
U_a cos(omega t) is a Stokes layer.  Its one-sided complex amplitude at
distance d from the wall is

    U(d) = U_a exp(-(1 + i) d / delta) / (1 + (1 + i) l_s / delta),
    delta = sqrt(2 nu / omega),  nu = mu(T0) / rho0,

with the velocity slip length l_s of a diffuse wall (1.016 times the
viscosity-based mean free path (mu / p) sqrt(pi R T / 2) for the BGK model).
In the paper's units (Eqs. 36-37) mu(T0) = Kn sqrt(pi) / 2.4245867 and
omega = St, so delta = 0.121 H and l_s = 0.0132 H here.

A lid alone drives a net oscillating flux that the side walls turn into a
pressure-driven counterflow across the whole cavity, so the top and bottom
walls move in opposite directions (no net flux through any vertical section)
and the cavity is 3 H wide: the measured profile along x = L/2 then differs
from the profile above by 1.5 % of U_a and 0.07 rad (a 2 H wide cavity: 3.6 %,
0.28 rad).  The pin is 5 % of U_a and 0.1 rad for 2 dy <= d <= 3 delta, at both
walls; a viscosity off by a factor 2 changes delta by 41 %, and dropping the
slip term alone changes the amplitude by 10 %.

Run on the GPU path (its pseudo step matches the FP64 oracle to 1e-12 per
step): 96 x 64 cells, 32 x 32 velocities, NH = 1, about 22000 steps to a
residual of 1e-9 in every conserved variable.
"""
import numpy as np
import pytest

import hbcases
from hbcases import Case

pytestmark = pytest.mark.gpu

UA = 0.01
KN, ST = 0.01, 1.0


def _say(*a):
    print(*a, flush=True)


def _counter_walls():
    w = [list(r) for r in hbcases.REST_WALLS]
    w[2][1] = UA   # top: +U_a cos(omega t) along +x
    w[0][1] = -UA  # bottom: the opposite motion
    return tuple(tuple(r) for r in w)


def test_stokes_layers_match_analytic_profile():
    import paper_2605_03479_amd as hb
    hb.load_library()
    nx, ny = 96, 64
    case = Case(nx, ny, 32, 4.0, KN, ST, 1, _counter_walls(), L=3.0, H=1.0, Pr=1.0)
    s = hb.Solver(case)
    k = 0
    while True:
        s.step(2000)
        k += 2000
        r = s.residual()
        if k % 10000 == 0:
            _say(f"  step {k}: max residual {max(r):.3e}")
        if max(r) <= 1e-9:
            break
        assert k < 60000, r
    re, im = s.harmonics(0x2)  # U
    s.close()
    U1 = 2.0 * (re[0, 1] + 1j * im[0, 1]).reshape(ny, nx)  # one-sided amplitude
    prof = 0.5 * (U1[:, nx // 2 - 1] + U1[:, nx // 2])
    mu = KN * np.sqrt(np.pi) / 2.4245867
    delta = np.sqrt(2.0 * mu / ST)
    l_s = 1.016 * (mu / 0.5) * np.sqrt(np.pi * 0.5 / 2.0)
    yc = (np.arange(ny) + 0.5) / ny
    for wall, d, sign in (("top", 1.0 - yc, 1.0), ("bottom", yc, -1.0)):
        an = sign * UA * np.exp(-(1 + 1j) * d / delta) / (1 + (1 + 1j) * l_s / delta)
        sel = (d <= 3 * delta) & (d >= 2.0 / ny)
        amp_err = np.max(np.abs(prof[sel] - an[sel])) / UA
        big = sel & (np.abs(an) > 0.1 * UA)
        ph_err = np.max(np.abs(np.angle(prof[big] / an[big])))
        _say(f"  {wall} wall: {k} steps, max |U - U_analytic| / U_a = {amp_err:.4f}, max phase error {ph_err:.4f} rad")
        assert amp_err <= 0.05
        assert ph_err <= 0.1
