"""GPU mixed form (FP32 storage of the deviation of h, b from the rest
Maxwellian and FP32 per-velocity flux, source and collision arithmetic on
those deviations; FP64 face and cell records, moment sums, W and residual)
against the FP64 CPU oracle.

Bounds: per step, every FP32 product carries a factor of the size of the
deviation, so each rounding is 2^-24 of the deviation; the update sums a few
tens of them, so states agree to 1e-6 of the signal; at convergence the
macroscopic harmonics agree to 1e-5 of each variable's harmonic signal (the
stated mixed-precision tolerance), each side converged on its own to
R_rho <= 1e-8."""
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


def _perturbed(oracle_mod, case, seed, amp=0.05):
    o = oracle_mod.Oracle(case)
    W, h, b = o.state()
    h = h * (1.0 + amp * hbcases.uniform(h.shape, seed))
    b = b * (1.0 + amp * hbcases.uniform(b.shape, seed + 1))
    W = W * (1.0 + 0.5 * amp * hbcases.uniform(W.shape, seed + 2))
    W[..., 1:3] = 0.02 * hbcases.uniform(W[..., 1:3].shape, seed + 3)
    return W, h, b


def _rel(a, r, rest):
    scale = max(np.max(np.abs(r - rest)), 1e-2 * np.max(np.abs(r)))
    return np.max(np.abs(a - r)) / scale


def test_mixed_state_roundtrip(gpu, oracle_mod):
    case = Case(7, 5, 12, 4.5, 0.3, 2.0, 2, hbcases.lid_walls(0.03))
    W, h, b = _perturbed(oracle_mod, case, 3)
    s = gpu.Solver(case, precision=gpu.HB_MIXED)
    s.set_state(W, h, b)
    W2, h2, b2 = s.state()
    s.close()
    assert np.array_equal(W2, W)  # W is FP64 in every form
    rest = h[:, :1, :]
    dev = np.max(np.abs(h - rest))
    assert np.max(np.abs(h2 - h)) <= 2.0 ** -23 * np.max(np.abs(h)) + 1e-300
    assert np.max(np.abs(h2 - h)) > 0.0 or dev == 0.0


@pytest.mark.parametrize("case", [
    Case(6, 6, 16, 4.0, 0.05, 1.0, 1, hbcases.lid_walls(0.02)),
    Case(7, 5, 12, 5.0, 1.0, 10.0, 4, hbcases.thermal_walls(0.5, 0, "sin")),
], ids=["shear", "thermal_nh4"])
def test_mixed_steps_match_oracle(gpu, oracle_mod, case):
    st = _perturbed(oracle_mod, case, 17)
    o = oracle_mod.Oracle(case)
    o.set_state(*st)
    s = gpu.Solver(case, precision=gpu.HB_MIXED)
    s.set_state(*st)
    rest = [x[:, :1, :] for x in o.state()]
    for k in (1, 5):
        o.step(k if k == 1 else 4)
        s.step(k if k == 1 else 4)
        for name, a, r, r0 in zip("Whb", s.state(), o.state(), rest):
            err = _rel(a, r, r0)
            _say(f"  {case.name or 'case'} step {k} {name}: rel err {err:.3e}")
            assert err <= 1e-6, (k, name, err)
    s.close()


def test_mixed_converged_harmonics(gpu, oracle_mod):
    """Each side converges on its own to R_rho <= 1e-8 (16 x 16 shear case,
    Kn = 1, St = 1); macroscopic harmonics agree within 1e-5."""
    case = hbcases.shear_small()
    o = oracle_mod.Oracle(case)
    k = 0
    while o.residual()[0] > 1e-8 or k == 0:
        o.step(100)
        k += 100
        assert k <= 5000
    s = gpu.Solver(case, precision=gpu.HB_MIXED)
    kg = 0
    while True:
        s.step(100)
        kg += 100
        r = s.residual()
        if r[0] <= 1e-8:
            break
        assert kg <= 6000, r
    _say(f"oracle converged in {k} steps, mixed GPU in {kg}")
    re_o, im_o = o.harmonics()
    re_g, im_g = s.harmonics()
    s.close()
    ho, hg = re_o + 1j * im_o, re_g + 1j * im_g
    for v in range(4):  # rho, U, V, T
        dev = ho[v].copy()
        if v in (0, 3):
            dev[0] -= 1.0
        err = np.max(np.abs(hg[v] - ho[v])) / np.max(np.abs(dev))
        _say(f"  var {v}: rel err {err:.3e}")
        assert err <= 1e-5, (v, err)


def test_mixed_converged_harmonics_thermal_nh4(gpu):
    """The mixed form at the heated-cavity benchmark's velocity grid and level
    count (48^2 velocities on [-5, 5], N_H = 4, Shakhov, bottom wall
    T0 (1 + 0.5 sin wt)) on 12 x 12 cells, converged from rest to
    R_rho <= 1e-8, against the oracle's converged harmonics stored in
    tests/golden/thermal12_v48_nh4_harmonics.txt (written by
    tests/golden/make_thermal12.py, the oracle at R_rho = 6e-10): rho, U, V, T
    within 1e-5 of each variable's harmonic signal."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "thermal12_v48_nh4_harmonics.txt")
    case = Case(12, 12, 48, 5.0, 1.0, 1.0, 4, hbcases.thermal_walls(0.5, 0, "sin"), name="thermal12_v48_nh4")
    g = np.loadtxt(path).reshape(4, case.NH + 1, 2, case.nc)
    ho = g[:, :, 0] + 1j * g[:, :, 1]
    s = gpu.Solver(case, precision=gpu.HB_MIXED)
    k = 0
    while True:
        s.step(100)
        k += 100
        r = s.residual()
        if r[0] <= 1e-8:
            break
        assert k <= 8000, r
    re, im = s.harmonics(0xF)
    s.close()
    hg = re + 1j * im
    _say(f"  mixed GPU converged in {k} steps (the oracle took 2800 to 6e-10)")
    for v in range(4):
        dev = ho[v].copy()
        if v in (0, 3):
            dev[0] -= 1.0
        err = np.max(np.abs(hg[v] - ho[v])) / np.max(np.abs(dev))
        _say(f"  var {v}: rel err {err:.3e}")
        assert err <= 1e-5, (v, err)
