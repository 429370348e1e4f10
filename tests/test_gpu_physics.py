"""Physics checks of the GPU solver against the closed forms the paper
quotes.

Collisionless high-frequency limit (Sec. 3.1, St = 30, Kn = 0.1): next to
the oscillating lid the gas is a half-Maxwellian from the bulk at rest plus
the diffusely re-emitted half-Maxwellian moving with the lid, so its
velocity amplitude is half the lid's (U~ = 0.5) and the shear-stress
amplitude is rho0 U_a sqrt(R T0 / (2 pi)), i.e. tau~ = 1/sqrt(pi).  The
paper's HB solutions come within 2 % for aspect ratios 0.5, 1 and 2; here on
its setup (90 cells across the height refined to 0.001 H at the walls by a
tanh law, 28 x 28 Gauss-Hermite velocities, U_a = 0.0015, N_H = 1).

U~ and tau~ (Eqs. 41-42) are the cell-width-weighted lid averages of the
fundamental amplitudes; the amplitude of a cos(omega t) is twice the
Eq. (40) coefficient |qhat_1|."""
import numpy as np
import pytest

import hbcases

pytestmark = pytest.mark.gpu

UA = 0.0015
P0 = 0.5  # rho0 R T0 with 2 R T0 = 1
STEPS = 6000


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import paper_2605_03479_amd as hb
    hb.load_library()
    return hb


@pytest.mark.parametrize("A", [1.0, 0.5, 2.0])
def test_collisionless_limit_st30(gpu, A):
    case = hbcases.shear_paper(30.0, Kn=0.1, A=A)
    s = gpu.Solver(case)
    for k in range(0, STEPS, 2000):
        s.step(2000)
        _say(f"  A {A}: step {k + 2000}, R = {s.residual()}")
    assert s.residual()[0] < 1e-9
    U = 2.0 * abs(s.wall_harmonic(2, 1, 1)) / UA
    tau = 2.0 * abs(s.wall_harmonic(2, 4, 1)) / (P0 * UA)
    s.close()
    _say(f"  A {A}: U~ = {U:.5f} (limit 0.5), tau~ = {tau:.5f} (limit {1 / np.sqrt(np.pi):.5f})")
    assert abs(U - 0.5) <= 0.02 * 0.5
    assert abs(tau - 1.0 / np.sqrt(np.pi)) <= 0.02 / np.sqrt(np.pi)


def test_wall_harmonic_is_width_weighted_average(gpu):
    """hb_ugks_wall_harmonic against the plain weighted average of
    hb_ugks_harmonics_out over the cells along each wall."""
    case = hbcases.Case(9, 7, 12, 4.0, 0.3, 2.0, 2, hbcases.lid_walls(0.02),
                        x_faces=hbcases.stretched_faces(9, 1.0, 0.03), y_faces=hbcases.stretched_faces(7, 1.0, 0.05))
    s = gpu.Solver(case)
    s.step(40)
    re, im = s.harmonics(0x7F)
    q = re + 1j * im  # [var][k][c]
    xf, yf = np.array(case.x_faces), np.array(case.y_faces)
    dx, dy = np.diff(xf), np.diff(yf)
    nx, ny = case.nx, case.ny
    cells = {0: np.arange(nx), 2: (ny - 1) * nx + np.arange(nx), 1: np.arange(ny) * nx + nx - 1, 3: np.arange(ny) * nx}
    for wall in range(4):
        ds = dx if wall in (0, 2) else dy
        for var in (1, 4, 5):
            for k in range(case.NH + 1):
                ref = np.sum(q[var, k, cells[wall]] * ds) / np.sum(ds)
                got = s.wall_harmonic(wall, var, k)
                assert abs(got - ref) <= 1e-14 * max(1e-300, np.max(np.abs(q[var, k]))), (wall, var, k)
    s.close()
