"""Time-domain UGKS on the GPU (the paper's comparison solver, Sec. 3.1.4)
against the FP64 CPU oracle's time-domain march.

The time-domain step is a pseudo step with one level and one global physical
step, the walls taken at the mid-step phase.  States are compared element by
element after a few steps and after one forcing period, with the same
tolerances as the pseudo step: 1e-12 of the signal in FP64, 1e-6 in the mixed
form.  The period residual of Eq. (43), second line, is checked against the
RMS change of the oracle's W over the same period."""
import numpy as np
import pytest

import hbcases
from hbcases import Case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import paper_2605_03479_amd as hb
    hb.load_library()
    return hb


def _rel(a, r, rest):
    """largest difference over the signal, max |r - rest|, floored at 1% of
    max |r| (as in the pseudo-step parity tests)"""
    scale = max(np.max(np.abs(r - rest)), 1e-2 * np.max(np.abs(r)))
    return np.max(np.abs(a - r)) / scale


def _ragged_td(dt):
    """7 x 5 cells on non-uniform x faces, 12^2 velocities, Shakhov, lid
    oscillating in phase and quadrature, bottom wall heated periodically."""
    w = [list(r) for r in hbcases.lid_walls(0.03)]
    w[2][2] = 0.01
    w[0][4] = 0.15
    w[0][5] = -0.05
    return Case(7, 5, 12, 4.5, 0.3, 6.0, 0, tuple(map(tuple, w)),
                x_faces=(0.0, 0.1, 0.25, 0.45, 0.6, 0.8, 0.9, 1.0), dt_mode=1, dt_fixed=dt, name="ragged_td")


def _perturbed(oracle_mod, case, seed, amp=0.05):
    o = oracle_mod.Oracle(case)
    W, h, b = o.state()
    h = h * (1.0 + amp * hbcases.uniform(h.shape, seed))
    b = b * (1.0 + amp * hbcases.uniform(b.shape, seed + 1))
    W = W * (1.0 + 0.5 * amp * hbcases.uniform(W.shape, seed + 2))
    return W, h, b


@pytest.mark.parametrize("grid", [{}, dict(Mv=16, vmax=5.5)], ids=["square", "rect12x16"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)], ids=["fp64", "mixed"])
def test_td_steps_match_oracle(gpu, oracle_mod, prec, tol, grid):
    """The ragged heated case (12^2 velocities on [-4.5, 4.5], or 12 along u and
    16 on [-5.5, 5.5] along v) after 1, 4 and 30 time-domain steps."""
    case = _ragged_td(1.2e-3).with_(**grid)
    st = _perturbed(oracle_mod, case, 404)
    o = oracle_mod.Oracle(case, td=True)
    rest = [x.copy() for x in o.state()]  # the uniform rest state: the signal is the deviation from it
    o.set_state(*st)
    s = gpu.Solver(case, precision=prec)
    s.set_state(*st)
    done = 0
    for k in (1, 4, 30):
        o.td_step(k - done, case.St)
        s.td_step(k - done)
        done = k
        assert s.time() == pytest.approx(o.time(), rel=1e-15)
        for name, a, r, r0 in zip("Whb", s.state(), o.state(), rest):
            err = _rel(a, r, r0)
            _say(f"  prec {prec} step {k} {name}: rel err {err:.3e}")
            assert err <= tol, (k, name, err)
    s.close()


def test_td_period_residual(gpu, oracle_mod):
    """One forcing period from rest on an 8 x 8 cavity with an oscillating
    lid: the state and the residual of Eq. (43), second line."""
    base = Case(8, 8, 16, 4.0, 1.0, 4.0, 0, hbcases.lid_walls(0.01), Pr=1.0)
    ns = 120
    case = base.with_(dt_mode=1, dt_fixed=2.0 * np.pi / base.St / ns)
    o = oracle_mod.Oracle(case, td=True)
    s = gpu.Solver(case)
    W0 = o.state()[0][:, 0, :]
    rest = [x.copy() for x in o.state()]
    for period in range(2):
        r = s.td_period(ns)
        o.td_step(ns, case.St)
        W1 = o.state()[0][:, 0, :]
        ref = np.sqrt(np.mean((W1 - W0) ** 2, axis=0))
        _say(f"  period {period}: R_TD gpu {r} oracle {ref}")
        np.testing.assert_allclose(r, ref, rtol=0, atol=1e-10 * np.max(ref))
        assert s.time() == pytest.approx(2.0 * np.pi / base.St * (period + 1), rel=1e-12)
        for name, a, b_, r0 in zip("Whb", s.state(), o.state(), rest):
            err = _rel(a, b_, r0)
            _say(f"  period {period} {name}: rel err {err:.3e}")
            assert err <= 1e-12
        W0 = W1
    s.close()


def test_td_refuses_harmonic_cases(gpu):
    s = gpu.Solver(Case(6, 6, 8, 4.0, 1.0, 1.0, 1, hbcases.lid_walls(0.01), dt_mode=1, dt_fixed=1e-3))
    with pytest.raises(gpu.HBError) as e:
        s.td_step(1)
    assert e.value.code == gpu.HB_ESTATE
    s.close()
    s = gpu.Solver(Case(6, 6, 8, 4.0, 1.0, 1.0, 0, hbcases.lid_walls(0.01)))  # local pseudo steps
    with pytest.raises(gpu.HBError) as e:
        s.td_period(10)
    assert e.value.code == gpu.HB_ESTATE
    s.close()
