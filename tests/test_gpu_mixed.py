"""GPU mixed form (FP32 storage of the deviation of h, b from the rest
Maxwellian and FP32 per-velocity flux, source and collision arithmetic on
those deviations; FP64 face and cell records, moment sums, W and residual)
against the FP64 CPU oracle.

Bounds: per step, every FP32 product carries a factor of the size of the
deviation, so each rounding is 2^-24 of the deviation; the update sums a few
tens of them, so states agree to 1e-6 of the signal; at convergence the
macroscopic harmonics agree to 1e-5 in the relative L-infinity norm over the
stacked harmonics of rho, U, V, T (the stated mixed-precision tolerance; see
harmerr.py), each side converged on its own."""
import numpy as np
import pytest

import hbcases
from harmerr import macro_errors
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
    Kn = 1, St = 1); macroscopic harmonics agree within 1e-5 (relative
    L-infinity over the stacked rho, U, V, T harmonics)."""
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
    err, per = macro_errors(hg, ho)
    _say(f"  rel err {err:.3e}; per variable (rho, U, V, T) " + " ".join(f"{e:.2e}" for e in per))
    assert err <= 1e-5, (err, per)


def test_mixed_converged_harmonics_thermal_nh4(gpu):
    """The mixed form at the heated-cavity benchmark's velocity grid and level
    count (48^2 velocities on [-5, 5], N_H = 4, Shakhov, bottom wall
    T0 (1 + 0.5 sin wt)) on 12 x 12 cells, stepped from rest 8000 pseudo steps,
    against the oracle's converged harmonics stored in
    tests/golden/thermal12_v48_nh4_harmonics.txt (written by
    tests/golden/make_thermal12.py, the oracle at R_rho <= 1e-11 after 4600
    steps): relative L-infinity error over the stacked rho, U, V, T harmonics
    within 1e-5.  (Against its own signal the x velocity is off by about 1e-4:
    its thermal-creep signal is 1e-2 of the temperature's, and the FP32
    rounding of the temperature-sized deviations reaches it.)

    Both sides go past the usual R_rho <= 1e-8 because this case contracts
    slowly (about 0.9966 per step): at 1e-8 it is still about 3e-5 of its
    density signal from the fixed point, which would hide the precision
    comparison under convergence error.  The mixed form cannot reach the
    oracle's 1e-11: its FP32 rounding of the deviations makes every step change
    the state by about 1e-9 of the density, so the residual levels off there.
    8000 steps takes the iteration error below that floor (the oracle's
    contraction reaches 1e-11 in 4600), and the test asks that the floor is
    below 1e-8."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "thermal12_v48_nh4_harmonics.txt")
    case = Case(12, 12, 48, 5.0, 1.0, 1.0, 4, hbcases.thermal_walls(0.5, 0, "sin"), name="thermal12_v48_nh4")
    g = np.loadtxt(path).reshape(4, case.NH + 1, 2, case.nc)
    ho = g[:, :, 0] + 1j * g[:, :, 1]
    s = gpu.Solver(case, precision=gpu.HB_MIXED)
    for k in range(1000, 8001, 1000):
        s.step(1000)
        r = s.residual()
        _say(f"  step {k}: R_rho {r[0]:.2e}")
    assert r[0] <= 1e-8, r
    re, im = s.harmonics(0xF)
    s.close()
    hg = re + 1j * im
    err, per = macro_errors(hg, ho)
    _say(f"  rel err {err:.3e}; per variable (rho, U, V, T) " + " ".join(f"{e:.2e}" for e in per))
    assert err <= 1e-5, (err, per)
