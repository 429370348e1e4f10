"""Case definitions and seeded synthetic inputs shared by the tests, the smoke
check and the benchmark.

This module holds no arithmetic of the method: only problem parameters (the
cavity workloads of the HB-UGKS paper's Section 3 at the sizes the benchmark
uses) and seeded random numbers.  Both the CPU oracle and the GPU path take
their inputs from here; neither is imported by this module.

Units: rho0 = H = sqrt(2 R T0) = 1 (T in units of T0, velocities in
sqrt(2 R T0)).  Walls are ordered bottom (y=0), right (x=L), top (y=H),
left (x=0); each wall row is (ut_mean, ut_re, ut_im, T_mean, T_re, T_im), so
the wall value is mean + Re(hat * exp(i omega t)) as in Eqs. (25)-(26).
"""
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import numpy as np

REST_WALLS = ((0.0, 0.0, 0.0, 1.0, 0.0, 0.0),) * 4


def lid_walls(amplitude=0.01):
    """Top lid moving tangentially with amplitude * cos(omega t); walls at T0."""
    w = [list(r) for r in REST_WALLS]
    w[2][1] = amplitude
    return tuple(tuple(r) for r in w)


def thermal_walls(dT=0.5, wall=0, phase="sin"):
    """One wall with T = T0 (1 + dT sin(omega t)) (or cos), others at T0, all at rest."""
    w = [list(r) for r in REST_WALLS]
    if phase == "sin":
        w[wall][5] = -dT  # Re(-i dT e^{i wt}) = dT sin(wt)
    else:
        w[wall][4] = dT
    return tuple(tuple(r) for r in w)


@dataclass(frozen=True)
class Case:
    nx: int
    ny: int
    M: int
    umax: float
    Kn: float
    St: float
    NH: int
    walls: tuple = REST_WALLS
    L: float = 1.0
    H: float = 1.0
    x_faces: Optional[Sequence[float]] = None
    y_faces: Optional[Sequence[float]] = None
    cfl: float = 0.5
    face_dt: int = 0          # 0 = min of the two cells, 1 = harmonic mean (Eq. 33)
    Pr: float = 2.0 / 3.0     # Shakhov; 1.0 = BGK
    omega_vss: float = 0.81
    alpha_vss: float = 1.0
    K: int = 1                # internal degrees of freedom
    macro_mode: int = 0       # 0 = macro flux of Eq. (24); 1 = all-discrete sum of the micro flux
    level_mass: int = 1       # 1 = level-mass projection after each pseudo step (convergence aid), 0 = off
    dt_mode: int = 0          # 0 = local pseudo step (Eqs. 31-32); 1 = global step dt_fixed
    dt_fixed: float = 0.0
    vrule: int = 0            # 1-D velocity rule: 0 = trapezoid on [-umax, umax], 1 = Gauss-Hermite
    Mv: int = 0               # nodes along v; 0 = M (square grid)
    vmax: float = 0.0         # trapezoid range along v; 0 = umax
    name: str = field(default="", compare=False)

    @property
    def NT(self):
        return 2 * self.NH + 1

    @property
    def nc(self):
        return self.nx * self.ny

    @property
    def Mv_(self):
        """Nodes along v."""
        return self.Mv or self.M

    @property
    def vmax_(self):
        """Trapezoid range along v."""
        return self.vmax if self.vmax > 0.0 else self.umax

    @property
    def nv(self):
        return self.M * self.Mv_

    @property
    def updates(self):
        """cell x velocity x level updates per pseudo step."""
        return self.nc * self.nv * self.NT

    def with_(self, **kw):
        return replace(self, **kw)


def stretched_faces(n, length, ds_min):
    """n + 1 face coordinates on [0, length], refined symmetrically towards both
    ends by a tanh law, x(s) = length/2 (1 + tanh(beta (2s - 1)) / tanh(beta)),
    s = i/n, with beta chosen so that the first and last cells are ds_min wide.
    (The paper refines its 90 x 90 cavity mesh to 0.001 H at every wall without
    giving the law; this one is a choice.)"""
    if not 0.0 < ds_min < length / n:
        raise ValueError("ds_min must lie in (0, length/n)")

    def first(beta):
        return 0.5 * length * (1.0 + np.tanh(beta * (2.0 / n - 1.0)) / np.tanh(beta))

    lo, hi = 1e-6, 50.0  # first() falls monotonically from ~length/n to 0 as beta grows
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if first(mid) > ds_min:
            lo = mid
        else:
            hi = mid
    beta = 0.5 * (lo + hi)
    s = np.arange(n + 1) / n
    x = 0.5 * length * (1.0 + np.tanh(beta * (2.0 * s - 1.0)) / np.tanh(beta))
    x[0], x[-1] = 0.0, length
    return tuple(float(v) for v in x)


# ----------------------------------------------------------------- workloads
def shear_small():
    """FP64 correctness case: 16x16 cells, 16x16 velocities on [-4,4], BGK,
    NH=1, Kn=1, St=1, lid 0.01 cos(wt), isothermal walls."""
    return Case(16, 16, 16, 4.0, 1.0, 1.0, 1, lid_walls(0.01), Pr=1.0, name="shear16_v16_nh1")


def shear_cavity(Kn=1.0, St=1.0):
    """Benchmark case: 64x64 cells, 32x32 velocities on [-4,4], NH=1, lid 0.01, Shakhov."""
    return Case(64, 64, 32, 4.0, Kn, St, 1, lid_walls(0.01),
                name=f"shear64_v32_nh1_kn{Kn:g}_st{St:g}")


def shear_paper(St, Kn=0.1, A=1.0, NH=1, ny=90, ds_min=1e-3, M=28):
    """The shear-driven cavity as the paper sets it up (Sec. 3.1): aspect
    ratio A = L/H, ny = 90 cells refined to ds_min = 0.001 H at every wall
    (nx = 90 A), lid U_a cos(omega t) with U_a = 0.0015, walls at T0, VSS
    argon (omega 0.81, alpha 1, Shakhov Pr 2/3), 28 x 28 Gauss-Hermite
    velocities (the rule it uses for Kn <= 0.1)."""
    nx = int(round(ny * A))
    return Case(nx, ny, M, 0.0, Kn, St, NH, lid_walls(0.0015), L=A,
                x_faces=stretched_faces(nx, A, ds_min), y_faces=stretched_faces(ny, 1.0, ds_min),
                vrule=1, name=f"shear_paper_{nx}x{ny}_gh{M}_nh{NH}_kn{Kn:g}_st{St:g}")


def thermal_paper(St, Kn=0.1, NH=2, ny=90, ds_min=1e-3, M=28):
    """The thermally driven cavity as the paper sets it up (Sec. 3.2): the
    mesh of the shear case, top wall T = T0 (1 + 0.3 cos(omega t)), other
    walls at T0, all at rest, N_H = 2, 28 x 28 Gauss-Hermite velocities.
    (Kn of its timing runs is not stated; Kn = 0.1 is the reading.)"""
    w = [list(r) for r in REST_WALLS]
    w[2][4] = 0.3
    f = stretched_faces(ny, 1.0, ds_min)
    return Case(ny, ny, M, 0.0, Kn, St, NH, tuple(tuple(r) for r in w), x_faces=f, y_faces=f, vrule=1,
                name=f"thermal_paper_{ny}x{ny}_gh{M}_nh{NH}_kn{Kn:g}_st{St:g}")


SHEAR_KN = (0.01, 0.1, 1.0, 10.0)
SHEAR_ST = (0.1, 1.0, 10.0)


def thermal_cavity(Kn=1.0, St=1.0):
    """Mixed-precision case: 64x64 cells, 48x48 velocities on [-5,5], NH=4,
    bottom wall T = T0 (1 + 0.5 sin wt), Shakhov."""
    return Case(64, 64, 48, 5.0, Kn, St, 4, thermal_walls(0.5, 0, "sin"),
                name=f"thermal64_v48_nh4_kn{Kn:g}_st{St:g}")


THERMAL_KN = (0.05, 1.0)
THERMAL_ST = (1.0, 10.0)


def batch_sweep(n=64, seed=260503479):
    """Seeded heterogeneous sweep: grid side U{24..96}, velocity side U{24..48}
    (rounded up to even), NH U{1..4}, Kn log-uniform [0.01, 10], St log-uniform
    [0.1, 10]; half shear (lid 0.01, [-4,4]) and half thermal (bottom wall,
    dT U(0.1, 0.5), [-5,5])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        N = int(rng.integers(24, 97))
        M = int(rng.integers(24, 49))
        M += M % 2
        NH = int(rng.integers(1, 5))
        Kn = float(10.0 ** rng.uniform(-2.0, 1.0))
        St = float(10.0 ** rng.uniform(-1.0, 1.0))
        if k % 2 == 0:
            out.append(Case(N, N, M, 4.0, Kn, St, NH, lid_walls(0.01), name=f"batch{k}_shear"))
        else:
            dT = float(rng.uniform(0.1, 0.5))
            out.append(Case(N, N, M, 5.0, Kn, St, NH, thermal_walls(dT, 0, "sin"),
                            name=f"batch{k}_thermal"))
    return out


def serving_requests(n=48, seed=260503480, outlier_p=1.0 / 16.0):
    """Seeded frequency-response requests of the serving workload: each request
    is drawn as a case of the batched sweep (grid side U{24..96}, velocity side
    U{24..48} rounded up to even, NH U{1..4}, Kn log-uniform [0.01, 10], St
    log-uniform [0.1, 10], even requests shear (lid 0.01, [-4, 4]) and odd ones
    thermal (bottom wall, dT U(0.1, 0.5), [-5, 5])); with probability outlier_p
    it is instead an outlier of 128 x 128 cells, 64 x 64 velocities and NH = 5
    with the same Kn, St and forcing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        outlier = bool(rng.uniform() < outlier_p)
        N = int(rng.integers(24, 97))
        M = int(rng.integers(24, 49))
        M += M % 2
        NH = int(rng.integers(1, 5))
        Kn = float(10.0 ** rng.uniform(-2.0, 1.0))
        St = float(10.0 ** rng.uniform(-1.0, 1.0))
        if outlier:
            N, M, NH = 128, 64, 5
        tag = "outlier_" if outlier else ""
        if k % 2 == 0:
            out.append(Case(N, N, M, 4.0, Kn, St, NH, lid_walls(0.01), name=f"req{k}_{tag}shear"))
        else:
            dT = float(rng.uniform(0.1, 0.5))
            out.append(Case(N, N, M, 5.0, Kn, St, NH, thermal_walls(dT, 0, "sin"), name=f"req{k}_{tag}thermal"))
    return out


def poisson_arrivals(n, rate, seed=260503481):
    """Arrival times (s) of a Poisson process of the given rate (1/s)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))


# ----------------------------------------------------------------- seeded noise
def noise(shape, seed, scale=1.0):
    """Seeded standard-normal numbers times `scale` (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal(shape)


def uniform(shape, seed, lo=-1.0, hi=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, shape)
