"""GPU parity: the HIP pseudo step (through the C ABI) against the FP64 CPU
oracle on the same seeded inputs, element by element.

Tolerance: relative L-inf <= 1e-12 in FP64, where "relative" divides the
largest absolute difference by the largest deviation of the oracle's result
from the uniform rest state (the signal the step computes; the rest state
itself is common to both sides), floored at 1% of the state's magnitude.  Harmonics compare per variable: the largest
|difference| over k and cells against the variable's harmonic signal, the
largest |qhat_k| over k and cells (k = 0 of rho and T: deviation from rest).
Per-k normalisation is not used because a small harmonic (the O(amplitude)
mean flow, say) carries the absolute round-off of the whole variable."""
import numpy as np
import pytest

import hbcases
from hbcases import Case

pytestmark = pytest.mark.gpu
TOL = 1e-12
CONVERGED_TOL = 1e-10  # conditioning floor at convergence, measured in test_oracle_step


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import paper_2605_03479_amd as hb
    hb.load_library()
    return hb


def _rest_like(oracle_state):
    W, h, b = oracle_state
    return W[:, :1, :].copy(), h[:, :1, :].copy(), b[:, :1, :].copy()


def _rel(a, r, rest):
    """max |a - r| over the signal max |r - rest|, but never over less than 1%
    of the state itself: 1e-12 of a signal that is 1e-3 of |h| would ask for
    agreement below an ulp of h."""
    scale = max(np.max(np.abs(r - rest)), 1e-2 * np.max(np.abs(r)))
    return np.max(np.abs(a - r)) / scale, scale


def _compare_states(sg, so, rest, tol=TOL, what="", signal_tol=None):
    """tol against the floored scale of _rel; signal_tol (if given) against
    the signal max |r - rest| itself, without the floor."""
    for name, a, r, r0 in zip("Whb", sg, so, rest):
        err, scale = _rel(a, r, r0)
        sig = np.max(np.abs(r - r0))
        err_sig = np.max(np.abs(a - r)) / sig if sig > 0 else 0.0
        _say(f"  {what} {name}: rel err {err:.3e} (scale {scale:.3e}); against the signal alone {err_sig:.3e}")
        assert scale > 0
        assert err <= tol, (what, name, err)
        if signal_tol is not None:
            assert err_sig <= signal_tol, (what, name, err_sig)


def _perturbed(oracle_mod, case, seed, amp=0.05):
    """Rest Maxwellian times (1 + amp * noise), different per level, with W
    set to its moments perturbed as well (W and moments of h need not agree)."""
    o = oracle_mod.Oracle(case)
    W, h, b = o.state()
    h = h * (1.0 + amp * hbcases.uniform(h.shape, seed))
    b = b * (1.0 + amp * hbcases.uniform(b.shape, seed + 1))
    W = W * (1.0 + 0.5 * amp * hbcases.uniform(W.shape, seed + 2))
    W[..., 1:3] = 0.02 * hbcases.uniform(W[..., 1:3].shape, seed + 3)
    return W, h, b


def _run_pair(gpu, oracle_mod, case, state, steps):
    _say(f"case {case}, steps {steps}")
    o = oracle_mod.Oracle(case)
    s = gpu.Solver(case)
    if state is not None:
        o.set_state(*state)
        s.set_state(*state)
    rest = _rest_like(o.state())
    out = []
    done = 0
    for k in steps:
        o.step(k - done)
        s.step(k - done)
        done = k
        out.append((k, s.state(), o.state(), s.residual(), o.residual()))
    s.close()
    return rest, out


# -------------------------------------------------------------------- cases
SMALL = hbcases.shear_small()


def _ragged():
    """7 x 5 cells on non-uniform x faces, 12^2 velocities (36 per quadrant,
    padded to 64), NH = 2, Shakhov, moving lid + sliding left wall + heated
    bottom wall, harmonic-mean face steps."""
    w = [list(r) for r in hbcases.lid_walls(0.03)]
    w[0][4] = 0.15
    w[0][5] = -0.05
    w[3][1] = 0.02
    w[3][2] = 0.01
    return Case(7, 5, 12, 4.5, 0.3, 2.0, 2, tuple(map(tuple, w)),
                x_faces=(0.0, 0.1, 0.25, 0.45, 0.6, 0.8, 0.9, 1.0), face_dt=1, name="ragged")


def test_small_from_rest(gpu, oracle_mod):
    # from rest the signal after one step is ~1e-4 of |h|, below what FP64
    # round-off resolves at 1e-12; compare once it has grown.  Against the
    # signal alone (no floor) the bound is 1e-10: each step rounds at 2^-53 of
    # |h|, and the signal is 1e-3 to 1e-2 of |h| after 10 to 60 steps, so a few
    # tens of roundings per step over 60 steps stay below 1e-11 of it
    rest, out = _run_pair(gpu, oracle_mod, SMALL, None, [10, 60])
    for k, sg, so, rg, ro in out:
        _compare_states(sg, so, rest, what=f"step {k}", signal_tol=1e-10)
        # residuals are RMS of increments: compare on the scale of the largest one
        np.testing.assert_allclose(rg, ro, rtol=0, atol=1e-10 * np.max(ro))


@pytest.mark.parametrize("Kn,St", [(0.01, 1.0), (1.0, 10.0), (10.0, 0.1)])
def test_perturbed_regimes(gpu, oracle_mod, Kn, St):
    case = Case(6, 6, 16, 4.0, Kn, St, 1, hbcases.lid_walls(0.02))
    st = _perturbed(oracle_mod, case, 1000 + int(Kn * 100))
    rest, out = _run_pair(gpu, oracle_mod, case, st, [1, 4])
    for k, sg, so, rg, ro in out:
        _compare_states(sg, so, rest, what=f"Kn {Kn} St {St} step {k}")


def test_ragged_nonuniform_shakhov(gpu, oracle_mod):
    case = _ragged()
    st = _perturbed(oracle_mod, case, 77)
    rest, out = _run_pair(gpu, oracle_mod, case, st, [1, 3, 12])
    for k, sg, so, rg, ro in out:
        _compare_states(sg, so, rest, what=f"ragged step {k}")


def test_global_step_mode(gpu, oracle_mod):
    case = _ragged().with_(dt_mode=1, dt_fixed=1.5e-3, face_dt=0, Pr=1.0)
    st = _perturbed(oracle_mod, case, 91)
    rest, out = _run_pair(gpu, oracle_mod, case, st, [2, 5])
    for k, sg, so, rg, ro in out:
        _compare_states(sg, so, rest, what=f"global step {k}")


def test_state_roundtrip_bitwise(gpu, oracle_mod):
    case = _ragged()
    st = _perturbed(oracle_mod, case, 5)
    s = gpu.Solver(case)
    s.set_state(*st)
    W, h, b = s.state()
    for a, r in zip((W, h, b), st):
        assert np.array_equal(a, r)
    s.close()


def test_small_converged_harmonics(gpu, oracle_mod):
    """Same number of steps as the oracle needs to reach R_rho <= 1e-8.  At
    convergence the bound is CONVERGED_TOL: one ulp of perturbation inside the
    oracle itself moves this fixed point by up to ~3e-12 of the signal, and
    independent rounding over 1500 steps by ~3e-11 (heat flux, a small
    difference of O(1) moments; see
    test_converged_state_roundoff_floor), so 1e-12 is below what two FP64
    implementations can share there."""
    o = oracle_mod.Oracle(SMALL)
    s = gpu.Solver(SMALL)
    k = 0
    while True:
        o.step(100)
        s.step(100)
        k += 100
        r = o.residual()
        if r[0] <= 1e-8 or k >= 4000:
            break
    _say(f"converged after {k} steps, oracle R = {r}")
    assert r[0] <= 1e-8
    np.testing.assert_allclose(s.residual(), r, rtol=1e-8)
    re_o, im_o = o.harmonics()
    re_g, im_g = s.harmonics()
    ho = re_o + 1j * im_o
    hg = re_g + 1j * im_g
    rest0 = {0: 1.0, 3: 1.0}
    for v in range(7):
        dev = ho[v].copy()
        dev[0] -= rest0.get(v, 0.0)
        scale = np.max(np.abs(dev))  # the variable's harmonic signal, all k
        diff = np.max(np.abs(hg[v] - ho[v]))
        err = diff / scale
        _say(f"  var {v}: rel err {err:.3e} (abs {diff:.2e}, signal {scale:.3e}; per k "
             + ", ".join(f"{np.max(np.abs(hg[v, k] - ho[v, k])):.1e}/{np.max(np.abs(dev[k])):.1e}"
                         for k in range(ho.shape[1])) + ")")
        assert err <= CONVERGED_TOL, (v, err)
    s.close()


def test_full_size_one_step(gpu, oracle_mod):
    """The benchmark workload (64 x 64 cells, 32 x 32 velocities, NH = 1),
    one step from a seeded perturbed state, every element compared."""
    case = hbcases.shear_cavity(1.0, 1.0)
    st = _perturbed(oracle_mod, case, 2024, amp=0.02)
    rest, out = _run_pair(gpu, oracle_mod, case, st, [1])
    for k, sg, so, rg, ro in out:
        _compare_states(sg, so, rest, what=f"64x64 step {k}")


@pytest.mark.parametrize("prec,tol", [(0, TOL), (1, 1e-6)], ids=["fp64", "mixed"])
def test_gauss_hermite_grid(gpu, oracle_mod, prec, tol):
    """The Gauss-Hermite velocity rule of Sec. 3.1.1 (14 nodes per axis, up to
    |u| = 4.30): the library computes its own nodes, the oracle takes
    numpy's; every element after 1 and 6 steps."""
    case = Case(7, 6, 14, 0.0, 0.1, 2.0, 1, hbcases.lid_walls(0.02), vrule=1, name="gh14")
    st = _perturbed(oracle_mod, case, 313)
    o = oracle_mod.Oracle(case)
    o.set_state(*st)
    s = gpu.Solver(case, precision=prec)
    s.set_state(*st)
    rest = _rest_like(o.state())
    done = 0
    for k in (1, 6):
        o.step(k - done)
        s.step(k - done)
        done = k
        _compare_states(s.state(), o.state(), rest, tol=tol, what=f"GH prec {prec} step {k}")
    s.close()


@pytest.mark.parametrize("prec,tol", [(0, TOL), (1, 1e-6)], ids=["fp64", "mixed"])
@pytest.mark.parametrize("grid", [dict(M=10, umax=4.0, Mv=16, vmax=5.0), dict(M=18, umax=5.0, Mv=8, vmax=4.0),
                                  dict(M=12, umax=0.0, Mv=16, vrule=1)], ids=["v-wider", "u-wider", "gh12x16"])
def test_rectangular_velocity_grid(gpu, oracle_mod, prec, tol, grid):
    """Velocity grids with a different node count and range along u and v
    (the trapezoid rule, and the Gauss-Hermite rule of 12 x 16 nodes): the
    face tables take the normal axis of each face, the collision tables both,
    the CFL bound each axis's extent.  A lid, a sliding wall and a heated
    wall on rectangular cells; every element after 1 and 6 steps."""
    w = [list(r) for r in hbcases.lid_walls(0.03)]
    w[0][4] = 0.12
    w[3][1] = 0.02
    case = Case(7, 6, Kn=0.2, St=2.0, NH=1, walls=tuple(map(tuple, w)), L=1.3,
                y_faces=(0.0, 0.1, 0.3, 0.55, 0.75, 0.9, 1.0), name="rect", **grid)
    st = _perturbed(oracle_mod, case, 5150 + case.M)
    o = oracle_mod.Oracle(case)
    o.set_state(*st)
    s = gpu.Solver(case, precision=prec)
    s.set_state(*st)
    assert s.sizes[4] == case.M * case.Mv_
    rest = _rest_like(o.state())
    done = 0
    for k in (1, 6):
        o.step(k - done)
        s.step(k - done)
        done = k
        _compare_states(s.state(), o.state(), rest, tol=tol, what=f"{grid} prec {prec} step {k}")
    s.close()


@pytest.mark.parametrize("nx,ny,M,NH", [(3, 3, 4, 0), (4, 3, 6, 5), (5, 5, 4, 3), (3, 6, 8, 1)])
def test_degenerate_sizes(gpu, oracle_mod, nx, ny, M, NH):
    """The smallest grids (every cell in the boundary ring, or one interior
    cell), the smallest velocity grids (4 or 9 velocities per quadrant, padded
    to 64 lanes) and the most levels (N_T = 11), forced by a lid, a sliding
    wall and a heated wall, against the oracle after 1 and 7 steps."""
    w = [list(r) for r in hbcases.lid_walls(0.03)]
    w[0][4] = 0.1
    w[1][2] = 0.02
    case = Case(nx, ny, M, 4.0, 0.5, 2.0, NH, tuple(map(tuple, w)))
    st = _perturbed(oracle_mod, case, 900 + nx * 10 + ny)
    rest, out = _run_pair(gpu, oracle_mod, case, st, [1, 7])
    for k, sg, so, rg, ro in out:
        _compare_states(sg, so, rest, what=f"{nx}x{ny} M={M} NH={NH} step {k}")


@pytest.mark.parametrize("level_mass,macro_mode", [(0, 0), (1, 1), (0, 1)], ids=["as-printed", "discrete-macro",
                                                                                "as-printed-discrete-macro"])
def test_step_options(gpu, oracle_mod, level_mass, macro_mode):
    """The step as printed (no level-mass projection) and the all-discrete
    macro flux (velocity sum of the micro flux), on the ragged heated cavity,
    every element after 1, 3 and 12 steps."""
    case = _ragged().with_(level_mass=level_mass, macro_mode=macro_mode)
    st = _perturbed(oracle_mod, case, 4711)
    rest, out = _run_pair(gpu, oracle_mod, case, st, [1, 3, 12])
    for k, sg, so, rg, ro in out:
        _compare_states(sg, so, rest, what=f"level_mass {level_mass} macro {macro_mode} step {k}")
        np.testing.assert_allclose(rg, ro, rtol=0, atol=1e-10 * np.max(ro))
