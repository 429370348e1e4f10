"""Host checks of the case builders (no GPU): the wall-refined mesh law and
the paper's cavity setups."""
import numpy as np

import hbcases


def test_stretched_faces():
    for n, L, ds in ((90, 1.0, 1e-3), (180, 2.0, 1e-3), (45, 0.5, 1e-3), (9, 1.0, 0.03)):
        x = np.array(hbcases.stretched_faces(n, L, ds))
        d = np.diff(x)
        assert len(x) == n + 1 and x[0] == 0.0 and x[-1] == L
        assert np.all(d > 0)
        np.testing.assert_allclose([d[0], d[-1]], ds, rtol=1e-9)
        np.testing.assert_allclose(d, d[::-1], rtol=1e-9)  # symmetric about the centre
        h = n // 2
        assert np.all(np.diff(d[:h]) > 0)  # cells grow towards the centre


def test_paper_cases():
    c = hbcases.shear_paper(30.0, Kn=0.1, A=2.0)
    assert (c.nx, c.ny, c.M, c.NH, c.vrule) == (180, 90, 28, 1, 1)
    assert c.L == 2.0 and c.walls[2][1] == 0.0015 and c.omega_vss == 0.81
    t = hbcases.thermal_paper(2.0)
    assert (t.nx, t.ny, t.NH) == (90, 90, 2) and t.walls[2][3:] == (1.0, 0.3, 0.0)
    assert all(w[:3] == (0.0, 0.0, 0.0) for w in t.walls)


def test_time_domain_step_size():
    """The time-domain comparison step: CFL 0.5 of Eqs. (31)-(32) on the
    smallest cell at the hottest wall temperature, a whole number of steps per
    forcing period."""
    import bench
    import paper_2605_03479_amd as hb
    from paper_2605_03479_amd import build as hb_build
    if hb_build.stale():
        hb_build.build()
    for case in (hbcases.shear_paper(30.0), hbcases.thermal_paper(2.0)):
        dt, ns = bench.td_step_size(hb, case)
        assert abs(ns * dt - 2.0 * np.pi / case.St) <= 1e-12
        u, _ = hb.hb_vgrid_nodes(case.M, case.umax, case.vrule)
        tmax = max(w[3] + np.hypot(w[4], w[5]) for w in case.walls)
        ut = u[-1] + np.sqrt((case.K + 4.0) / (case.K + 2.0) * tmax / 2.0)
        nu = 2.0 * ut / np.min(np.diff(case.x_faces))
        assert nu * dt <= case.cfl * (1.0 + 1e-12)
        assert nu * 2.0 * np.pi / case.St / (ns - 1) > case.cfl  # one step fewer would break the bound
