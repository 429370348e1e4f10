"""The path at the workload sizes the benchmark and the serving run use.

- The 64 x 64-cell, 48 x 48-velocity, N_T = 9 thermal cavity: one step from
  a seeded perturbed state, every element against the oracle (1e-12 of the
  signal in FP64, 1e-6 in the mixed form).
- The serving outlier, 128 x 128 cells, 64 x 64 velocities, N_T = 11 (the
  per-block tables then need more than 64 KB of LDS): too large for the
  oracle's whole-grid step, so it is checked by properties that hold at any
  size: a resting Maxwellian between walls at rest stays at rest, and a
  bottom wall heated uniformly keeps the solution mirror-symmetric in x.
- The same per-block tables (64 x 64 velocities, N_T = 11: 88 KB of
  dynamic LDS) on a 6 x 6-cell cavity, which the oracle steps in seconds:
  every element against the oracle after two steps from a perturbed state,
  with interior cells (the update kernel of the large grids) among them.
- The largest velocity grid with the most levels (128^2, N_T = 11) needs
  180 KB of tables per block, more than a CU's LDS: set-up refuses it.
- The 64-case seeded sweep as one tuned mixed batch (40 GB of state, the
  benchmark's launch shapes): sampled cases, the smallest, the largest and
  two seeded others, are bit-identical to the same case stepped alone, and
  the smallest one matches the oracle to the mixed bound."""
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
    scale = max(np.max(np.abs(r - rest)), 1e-2 * np.max(np.abs(r)))
    return np.max(np.abs(a - r)) / scale


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)], ids=["fp64", "mixed"])
def test_thermal_full_size_one_step(gpu, oracle_mod, prec, tol):
    case = hbcases.thermal_cavity(1.0, 1.0)
    o = oracle_mod.Oracle(case)
    W, h, b = o.state()
    rest = (W[:, :1, :].copy(), h[:, :1, :].copy(), b[:, :1, :].copy())
    h = h * (1.0 + 0.02 * hbcases.uniform(h.shape, 4242))
    b = b * (1.0 + 0.02 * hbcases.uniform(b.shape, 4243))
    W = W * (1.0 + 0.01 * hbcases.uniform(W.shape, 4244))
    o.set_state(W, h, b)
    s = gpu.Solver(case, precision=prec)
    s.set_state(W, h, b)
    del W, h, b
    _say(f"  {case.name}: one step, prec {prec}")
    o.step(1)
    s.step(1)
    for name, a, r, r0 in zip("Whb", s.state(), o.state(), rest):
        err = _rel(a, r, r0)
        _say(f"  {name}: rel err {err:.3e}")
        assert err <= tol, (name, err)
    s.close()


OUTLIER = dict(nx=128, ny=128, M=64, umax=5.0, Kn=1.0, St=1.0, NH=5)


def test_outlier_size_rest_state(gpu):
    # velocities on [-7, 7] so the trapezoid rule integrates the rest
    # Maxwellian to round-off (truncation erfc(7) ~ 4e-23)
    s = gpu.Solver(Case(**dict(OUTLIER, umax=7.0), walls=hbcases.REST_WALLS), precision=gpu.HB_MIXED)
    s.step(3)
    r = s.residual()
    _say(f"  128^2 x 64^2 x 11 at rest: R = {r}")
    assert np.all(r <= 1e-14)
    W = s.macro()
    assert np.max(np.abs(W[..., 0] - 1.0)) <= 1e-13 and np.max(np.abs(W[..., 1:3])) <= 1e-13
    s.close()


def test_outlier_size_mirror_symmetry(gpu):
    """Bottom wall T0 (1 + 0.3 sin omega t), other walls at T0: the problem is
    symmetric under x -> L - x, so rho, rho V, rho E are even and rho U odd."""
    case = Case(**OUTLIER, walls=hbcases.thermal_walls(0.3, 0, "sin"))
    s = gpu.Solver(case)
    s.step(4)
    W = s.macro().reshape(case.ny, case.nx, case.NT, 4)
    s.close()
    Wm = W[:, ::-1]
    sig = np.max(np.abs(W[..., 0] - 1.0))
    assert sig > 1e-6
    for k, sign in ((0, 1), (1, -1), (2, 1), (3, 1)):
        d = np.max(np.abs(W[..., k] - sign * Wm[..., k]))
        _say(f"  component {k}: mirror difference {d:.2e} (signal {sig:.2e})")
        assert d <= 1e-12 * max(sig, np.max(np.abs(W[..., k] - (W[..., k].mean() if sign > 0 else 0.0))))


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)], ids=["fp64", "mixed"])
def test_outlier_tables_against_oracle(gpu, oracle_mod, prec, tol):
    case = Case(6, 6, 64, 5.0, 0.5, 2.0, 5, hbcases.thermal_walls(0.3, 0, "sin"), name="lds88k_6x6")
    o = oracle_mod.Oracle(case)
    W, h, b = o.state()
    rest = (W[:, :1, :].copy(), h[:, :1, :].copy(), b[:, :1, :].copy())
    h = h * (1.0 + 0.03 * hbcases.uniform(h.shape, 5151))
    b = b * (1.0 + 0.03 * hbcases.uniform(b.shape, 5152))
    W = W * (1.0 + 0.01 * hbcases.uniform(W.shape, 5153))
    W[..., 1:3] = 0.01 * hbcases.uniform(W[..., 1:3].shape, 5154)
    o.set_state(W, h, b)
    s = gpu.Solver(case, precision=prec)
    s.set_state(W, h, b)
    _say(f"  {case.name}: 6x6 cells, 64^2 velocities, N_T = 11, two steps, prec {prec}")
    o.step(2)
    s.step(2)
    for name, a, r, r0 in zip("Whb", s.state(), o.state(), rest):
        err = _rel(a, r, r0)
        _say(f"  {name}: rel err {err:.3e}")
        assert err <= tol, (name, err)
    s.close()


def test_largest_tables_refused(gpu):
    with pytest.raises(gpu.HBError) as e:
        gpu.Solver(Case(8, 8, 128, 5.0, 1.0, 1.0, 5, hbcases.lid_walls(0.01)))
    assert e.value.code == gpu.HB_EINVAL


def test_full_sweep_sampled_cases(gpu, oracle_mod):
    cases = hbcases.batch_sweep()
    steps = 2
    B = gpu.Batch(max_cases=len(cases))
    hs = [B.add(c, gpu.HB_MIXED) for c in cases]
    B.tune(2)  # takes one batch step
    B.step(steps)
    res = B.residuals()
    assert all(res[h.cid][1] == steps + 1 and not res[h.cid][2] for h in hs)
    order = sorted(range(len(cases)), key=lambda k: cases[k].updates)
    rng = np.random.Generator(np.random.PCG64(2605))
    pick = [order[0], order[-1]] + [int(k) for k in rng.choice(order[1:-1], 2, replace=False)]
    for k in pick:
        c = cases[k]
        _say(f"  {c.name}: {c.nx}x{c.ny}, M={c.M}, NH={c.NH}, {c.updates:.3g} updates/step")
        s = gpu.Solver(c, precision=gpu.HB_MIXED)
        s.step(steps + 1)
        solo = s.state()
        assert all(np.array_equal(x, y) for x, y in zip(hs[k].state(), solo)), c.name
        assert np.array_equal(res[hs[k].cid][0], s.residual()), c.name
        if k == order[0]:
            o = oracle_mod.Oracle(c)
            rest = [x.copy() for x in o.state()]
            o.step(steps + 1)
            for name, a, r, r0 in zip("Whb", solo, o.state(), rest):
                err = _rel(a, r, r0)
                _say(f"    {name} against the oracle: rel err {err:.3e}")
                assert err <= 1e-6, (name, err)
        s.close()
        del solo
    B.close()
