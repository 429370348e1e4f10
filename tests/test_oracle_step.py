"""Whole-step pins of the oracle: invariants and special cases that the paper
and the mathematics fix for the pseudo-time map (Secs. 2.2-2.4)."""
import numpy as np
import pytest

import hbcases
from hbcases import Case


def _wide(**kw):
    """A velocity grid wide and fine enough that the trapezoid rule integrates
    Maxwellians near T0 exactly to round-off (truncation erfc(7) ~ 4e-23)."""
    base = dict(nx=6, ny=5, M=28, umax=7.0, Kn=0.1, St=2.0, NH=1)
    base.update(kw)
    return Case(**base)


@pytest.mark.parametrize("Kn,St,NH,Pr,vrule", [(0.01, 1.0, 1, 2 / 3, 0), (1.0, 3.0, 2, 1.0, 0),
                                               (10.0, 0.3, 3, 2 / 3, 0), (0.1, 10.0, 0, 2 / 3, 0),
                                               (0.1, 2.0, 1, 2 / 3, 1)])
def test_resting_maxwellian_is_fixed_point(oracle_mod, Kn, St, NH, Pr, vrule):
    """A uniform rest Maxwellian between stationary walls at T0 stays at rest:
    every flux cancels, the spectral source vanishes, collisions are in
    equilibrium (Sec. 2.4; Eqs. 27-29).  vrule 1: the 28-point Gauss-Hermite
    grid of Sec. 3.1.1, exact for the rest Maxwellian's moments."""
    o = oracle_mod.Oracle(_wide(Kn=Kn, St=St, NH=NH, Pr=Pr, vrule=vrule))
    W0, h0, b0 = o.state()
    for _ in range(3):
        o.step(20)
        assert np.all(o.residual() < 1e-15)
    W, h, b = o.state()
    np.testing.assert_allclose(W, W0, atol=1e-14)
    np.testing.assert_allclose(h, h0, atol=1e-14)


def _forced(dt_mode=0, **kw):
    w = [list(r) for r in hbcases.lid_walls(0.05)]
    w[0][4] = 0.2   # bottom wall T = T0 (1 + 0.2 cos wt)
    w[3][1] = -0.03  # left wall slides too
    base = dict(nx=6, ny=5, M=12, umax=4.0, Kn=0.2, St=1.5, NH=2, walls=tuple(map(tuple, w)))
    base.update(kw)
    c = Case(**base)
    if dt_mode:
        c = c.with_(dt_mode=1, dt_fixed=2e-3)
    return c


def test_mass_conservation_with_global_step(oracle_mod):
    """With one global pseudo step, sum_n sum_i |Omega_i| rho_i,n is constant:
    interior fluxes telescope, walls are impermeable (Eq. 28), and the columns
    of E sum to zero (E is skew with zero row sums)."""
    c = _forced(dt_mode=1, x_faces=[0, .1, .3, .45, .7, .85, 1.0])
    o = oracle_mod.Oracle(c)
    dx = np.diff(c.x_faces)
    dy = np.full(c.ny, 1.0 / c.ny)
    area = np.outer(dy, dx).ravel()

    def mass():
        W, _, _ = o.state()
        return np.sum(area[:, None] * W[:, :, 0])

    m0 = mass()
    for _ in range(5):
        o.step(10)
        assert abs(mass() - m0) < 1e-13 * m0
    W, _, _ = o.state()
    assert np.max(np.abs(W[:, :, 0] - 1.0)) > 1e-5  # the forcing did move mass around


def test_walls_are_impermeable(oracle_mod):
    """Zero net mass flux through every wall face at every level (Eq. 28)."""
    o = oracle_mod.Oracle(_forced())
    o.step(15)
    _, Fx, Fy = o.debug()
    walls = np.concatenate([Fx[:, 0, :, 0].ravel(), Fx[:, -1, :, 0].ravel(),
                            Fy[0, :, :, 0].ravel(), Fy[-1, :, :, 0].ravel()])
    interior = np.abs(Fx[:, 1:-1, :, 1]).max()
    assert interior > 1e-4
    assert np.max(np.abs(walls)) < 1e-15


def test_mirror_symmetry_thermal_cavity(oracle_mod):
    """A cavity heated from the bottom is symmetric under x -> L - x:
    rho, V, E even and rho U odd."""
    c = Case(8, 6, 12, 4.5, 0.3, 2.0, 2, hbcases.thermal_walls(0.4, 0, "sin"))
    o = oracle_mod.Oracle(c)
    o.step(40)
    W, h, _ = o.state()
    W = W.reshape(c.ny, c.nx, c.NT, 4)
    Wm = W[:, ::-1]
    scale = np.abs(W - W[0, 0, 0]).max()
    assert scale > 1e-4
    np.testing.assert_allclose(W[..., 0], Wm[..., 0], atol=1e-12 * scale)
    np.testing.assert_allclose(W[..., 1], -Wm[..., 1], atol=1e-12 * scale)
    np.testing.assert_allclose(W[..., 2], Wm[..., 2], atol=1e-12 * scale)
    np.testing.assert_allclose(W[..., 3], Wm[..., 3], atol=1e-12 * scale)
    # the distribution mirrors too: h(x, u, v) = h(L - x, -u, v)
    H = h.reshape(c.ny, c.nx, c.NT, c.M, c.M)  # [.., iv, iu]
    np.testing.assert_allclose(H, H[:, ::-1, :, :, ::-1], atol=1e-12 * np.abs(H).max())


def test_transpose_symmetry(oracle_mod):
    """Swapping x and y maps a top lid sliding along x onto a right wall sliding
    along y; the x-face and y-face paths must then agree (rho U <-> rho V)."""
    a = Case(6, 6, 12, 4.0, 0.5, 1.0, 1, hbcases.lid_walls(0.05))
    w = [list(r) for r in hbcases.REST_WALLS]
    w[1][1] = 0.05
    bcase = a.with_(walls=tuple(map(tuple, w)))
    oa, ob = oracle_mod.Oracle(a), oracle_mod.Oracle(bcase)
    oa.step(30)
    ob.step(30)
    Wa = oa.state()[0].reshape(6, 6, 3, 4)
    Wb = ob.state()[0].reshape(6, 6, 3, 4)
    Wat = np.transpose(Wa, (1, 0, 2, 3))[..., [0, 2, 1, 3]]
    scale = np.abs(Wa[..., 1]).max()
    assert scale > 1e-4
    np.testing.assert_allclose(Wb, Wat, atol=1e-12 * scale)


def _transposed(c):
    """The case with x and y swapped: walls (bottom, right, top, left) become
    (left, top, right, bottom), each keeping its tangential velocity (along +x
    on bottom/top, +y on left/right), and the two velocity axes swap."""
    w = c.walls
    return c.with_(nx=c.ny, ny=c.nx, L=c.H, H=c.L, M=c.Mv_, Mv=c.M, umax=c.vmax_, vmax=c.umax,
                   walls=(w[3], w[2], w[1], w[0]))


def test_transpose_symmetry_rectangular_velocity_grid(oracle_mod):
    """Rectangular cells, a rectangular velocity grid (10 nodes on [-4, 4]
    along u, 14 on [-5, 5] along v), a sliding lid and a heated wall: swapping
    x and y (and u and v) maps the state onto itself transposed, which fixes
    which axis of the grid each face, slope and CFL bound takes."""
    w = [list(r) for r in hbcases.lid_walls(0.06)]
    w[0][4] = 0.15
    a = Case(7, 5, 10, 4.0, 0.4, 1.5, 1, tuple(map(tuple, w)), L=1.4, H=1.0, Mv=14, vmax=5.0)
    b = _transposed(a)
    oa, ob = oracle_mod.Oracle(a), oracle_mod.Oracle(b)
    assert oa.nv == ob.nv == 140
    oa.step(30)
    ob.step(30)
    Wa, ha, _ = oa.state()
    Wb, hb, _ = ob.state()
    Wa = Wa.reshape(a.ny, a.nx, a.NT, 4)
    Wb = Wb.reshape(b.ny, b.nx, b.NT, 4)
    scale = np.abs(Wa[..., 1]).max()
    assert scale > 1e-4
    np.testing.assert_allclose(Wb, np.transpose(Wa, (1, 0, 2, 3))[..., [0, 2, 1, 3]], atol=1e-12 * scale)
    Ha = ha.reshape(a.ny, a.nx, a.NT, a.Mv_, a.M)  # [j, i, n, iv, iu]
    Hb = hb.reshape(b.ny, b.nx, b.NT, b.Mv_, b.M)
    np.testing.assert_allclose(Hb, np.transpose(Ha, (1, 0, 2, 4, 3)), atol=1e-12 * np.abs(Ha).max())


def test_rectangular_grid_layout_and_rest_state(oracle_mod):
    """On a rectangular grid (28 nodes on [-7, 7] along u, 30 on [-7.5, 7.5]
    along v) the initial state is the rest Maxwellian exp(-u^2 - v^2)/pi at
    a = iv*M + iu, and it stays a fixed point (Sec. 2.4)."""
    c = _wide(M=28, Mv=30, vmax=7.5)
    o = oracle_mod.Oracle(c)
    assert o.nv == 28 * 30
    u = np.linspace(-7.0, 7.0, 28)
    v = np.linspace(-7.5, 7.5, 30)
    H0 = np.exp(-u[None, :] ** 2 - v[:, None] ** 2) / np.pi
    W0, h0, _ = o.state()
    np.testing.assert_allclose(h0.reshape(c.nc, c.NT, 30, 28), np.broadcast_to(H0, (c.nc, c.NT, 30, 28)),
                               rtol=1e-13, atol=1e-300)
    o.step(20)
    assert np.all(o.residual() < 1e-15)
    np.testing.assert_allclose(o.state()[1], h0, atol=1e-14)


def test_local_step_takes_each_axis_extent(oracle_mod):
    """Eq. (32) at rest on a rectangular velocity grid (10 nodes on [-4, 4]
    along u, 14 on [-6, 6] along v) and non-uniform cells: the local step is
    CFL / ((u_max + c_s)/dx + (v_max + c_s)/dy + omega N_H), c_s = sqrt(gamma/2),
    with each axis's own extent against its own cell width."""
    xf = (0.0, 0.1, 0.3, 0.6, 0.8, 1.0)
    yf = (0.0, 0.2, 0.35, 0.5, 0.75, 0.9, 1.0)
    c = Case(5, 6, 10, 4.0, 0.5, 1.5, 2, hbcases.REST_WALLS, x_faces=xf, y_faces=yf, Mv=14, vmax=6.0)
    o = oracle_mod.Oracle(c)
    o.step(1)
    dtc, _, _ = o.debug()
    cs = np.sqrt((c.K + 4.0) / (c.K + 2.0) / 2.0)
    dx, dy = np.diff(xf), np.diff(yf)
    want = c.cfl / ((4.0 + cs) / dx[None, :] + (6.0 + cs) / dy[:, None] + c.St * c.NH)
    np.testing.assert_allclose(dtc.reshape(c.ny, c.nx), want, rtol=1e-14)


def test_harmonics_of_a_known_state(oracle_mod):
    """Eq. (40): qhat_k = (1/NT) sum_n q_n exp(-i k w t_n).  A state whose
    levels carry rho_n = 1 + A cos(w t_n + phi) has rhohat_1 = (A/2) e^{i phi}."""
    c = Case(4, 3, 12, 5.0, 1.0, 1.0, 2)
    o = oracle_mod.Oracle(c)
    W, h, b = o.state()
    t = 2 * np.pi * np.arange(c.NT) / c.NT
    A = 0.01 * (1 + np.arange(c.nc))
    phi = 0.3 * np.arange(c.nc)
    fac = 1 + A[:, None] * np.cos(t[None, :] + phi[:, None]) + 0.002 * np.cos(2 * t)[None, :]
    W = W * fac[:, :, None]   # density scales, U = V = 0, T unchanged
    o.set_state(W, h * fac[:, :, None], b * fac[:, :, None])
    re, im = o.harmonics()
    np.testing.assert_allclose(re[0, 0], 1.0, atol=1e-14)
    np.testing.assert_allclose(re[0, 1] + 1j * im[0, 1], A / 2 * np.exp(1j * phi), atol=1e-14)
    np.testing.assert_allclose(re[0, 2] + 1j * im[0, 2], 0.001, atol=1e-14)
    np.testing.assert_allclose(re[3], np.array([1.0, 0.0, 0.0])[:, None] * np.ones(c.nc), atol=1e-13)


def test_residual_definition(oracle_mod):
    """Eq. (43): RMS over cells of the level-0 change of each conservative
    variable, on the step as printed (with the level-mass projection the
    residual is the step's increment before the scaling)."""
    o = oracle_mod.Oracle(_forced(level_mass=0))
    o.step(3)
    W0 = o.state()[0]
    o.step(1)
    W1 = o.state()[0]
    ref = np.sqrt(np.mean((W1[:, 0, :] - W0[:, 0, :]) ** 2, axis=0))
    np.testing.assert_allclose(o.residual(), ref, rtol=1e-14)


@pytest.mark.parametrize("Kn", [1e-4, 1e-5])
def test_continuum_limit_viscous_flux(oracle_mod, Kn):
    """For tau << dG the UGKS interface flux of a linear shear U = s y (uniform
    rho, T, equilibrium data) tends to the Navier-Stokes stress -mu s, carried
    by the C2 term of Eq. (24); the error is O(tau/dG)."""
    s = 0.02
    c = Case(6, 8, 24, 6.0, Kn, 1.0, 0, Pr=1.0)
    o = oracle_mod.Oracle(c)
    mu = o.constants()["mu_ref"]
    W, h, b = o.state()
    yc = (np.arange(c.ny) + 0.5) / c.ny
    u1, _ = oracle_mod.velocity_grid(c.M, c.umax)
    uu, vv = np.meshgrid(u1, u1, indexing="xy")
    for j in range(c.ny):
        U = s * (yc[j] - 0.5)
        H, B, _, _ = oracle_mod.equilibrium(1, 1.0, [1.0, U, 0.0, 1.0], [0, 0], uu.ravel(), vv.ravel())
        for i in range(c.nx):
            cc = j * c.nx + i
            W[cc, :, :] = [1.0, U, 0.0, 0.75 + 0.5 * U * U]
            h[cc, :, :] = H
            b[cc, :, :] = B
    o.set_state(W, h, b)
    o.step(1)
    dtc, Fx, Fy = o.debug()
    tau = mu * 2.0  # tau = mu / p with p = 1/2
    ratio = Fy[c.ny // 2, c.nx // 2, 0, 1] / (-mu * s)
    assert abs(ratio - 1.0) < 3 * tau / dtc.min() + 1e-3, (ratio, tau / dtc.min())


CONVERGED_TOL = 1e-10


def _harm_signal_errors(a, b):
    out = []
    for v in range(7):
        dev = b[v].copy()
        if v in (0, 3):
            dev[0] -= 1.0
        out.append(np.max(np.abs(a[v] - b[v])) / np.max(np.abs(dev)))
    return np.array(out)


@pytest.mark.slow
def test_converged_state_roundoff_floor(oracle_mod):
    """At convergence the agreement of two FP64 implementations is floored by
    the conditioning of the fixed point: one ulp more on every local step
    (the oracle against itself) moves the converged harmonics of the small
    shear case by more than 1e-12 of their signal for some variables.  The
    GPU comparison at convergence is held to CONVERGED_TOL, a few times this
    measured floor; comparisons after a fixed, smaller number of steps keep
    the 1e-12 bound."""
    case = hbcases.shear_small()
    res = []
    for s in (1.0, 1.0 + 2.0 ** -52):
        o = oracle_mod.Oracle(case)
        o.set_dt_scale(s)
        o.step(1500)
        re, im = o.harmonics()
        res.append(re + 1j * im)
    floor = _harm_signal_errors(res[1], res[0])
    print("one-ulp sensitivity per variable:", floor)
    assert floor.max() > 1e-12
    assert floor.max() < CONVERGED_TOL / 4
