"""Pins of the oracle's building blocks against what the paper and the
mathematics fix, computed here by independent means (definitions written out,
numerical quadrature, hand-derived values) -- never by re-calling the oracle's
own formula."""
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


# ------------------------------------------------------------ spectral operator E
def test_E_worked_examples(oracle_mod):
    np.testing.assert_allclose(oracle_mod.E_matrix(3), _golden("E_NT3.txt"), atol=1e-15)
    row0 = _golden("E_NT5.txt")
    E5 = oracle_mod.E_matrix(5)
    np.testing.assert_allclose(E5[0], row0, atol=1e-13)
    for n in range(5):  # circulant
        np.testing.assert_allclose(E5[n], np.roll(row0, n), atol=1e-13)


@pytest.mark.parametrize("NH", [0, 1, 2, 3, 4, 5])
def test_E_is_spectral_derivative(oracle_mod, NH):
    """E = i D^-1 K D (Eq. 15) with D^-1 of Eq. (14); E differentiates the
    sampled harmonics exactly; E is real, skew, annihilates constants, and
    its eigenvalues are i k for k = -NH..NH."""
    NT = 2 * NH + 1
    E = oracle_mod.E_matrix(NT)
    t = 2 * np.pi * np.arange(NT) / NT  # omega t_n of Eq. (12), omega = 1
    ks = np.array(list(range(0, NH + 1)) + list(range(-NH, 0)))
    Dinv = np.exp(1j * np.outer(t, ks))          # Eq. (14)
    D = np.linalg.inv(Dinv)
    Edef = 1j * Dinv @ np.diag(ks) @ D           # Eq. (15)
    assert np.max(np.abs(Edef.imag)) < 1e-13
    np.testing.assert_allclose(E, Edef.real, atol=1e-13)
    np.testing.assert_allclose(E, -E.T, atol=0)
    np.testing.assert_allclose(E @ np.ones(NT), 0.0, atol=1e-13)
    for k in range(1, NH + 1):
        np.testing.assert_allclose(E @ np.sin(k * t), k * np.cos(k * t), atol=1e-13)
        np.testing.assert_allclose(E @ np.cos(k * t), -k * np.sin(k * t), atol=1e-13)
    ev = np.sort(np.linalg.eigvals(E).imag)
    np.testing.assert_allclose(ev, np.sort(ks.astype(float)), atol=1e-12)


# ------------------------------------------------------------ C1..C5
def _c_brute(tau, dG):
    """Time average over [0, dG] of the integral solution, Eq. (21), written out
    term by term: equilibrium g0 (1 + a.(x'-x_f) + A G'), x'-x_f = -u (G-G'),
    initial data h0 + sigma.(x_f - u G - x_f).  Returns the coefficients of
    g0, (u.a) g0, A g0, h0 and u.sigma, by 30-digit quadrature."""
    mp.mp.dps = 30
    tau = mp.mpf(tau)
    dG = mp.mpf(dG)

    def eq(f):
        inner = lambda G: mp.quad(lambda s: mp.exp(-(G - s) / tau) * f(G, s), [0, G]) / tau
        return mp.quad(inner, [0, dG])

    c1 = eq(lambda G, s: 1)
    c2 = eq(lambda G, s: -(G - s))
    c3 = eq(lambda G, s: s)
    c4 = mp.quad(lambda G: mp.exp(-G / tau), [0, dG])
    c5 = mp.quad(lambda G: -G * mp.exp(-G / tau), [0, dG])
    return np.array([float(c) for c in (c1, c2, c3, c4, c5)])


@pytest.mark.parametrize("tau,dG", [(1.0, 1e-4), (2.0, 3e-3), (1.0, 0.05), (0.3, 0.29),
                                    (1.0, 0.99), (1.0, 1.01), (0.01, 0.2), (1e-4, 0.01),
                                    (7.31, 1.6e-3)])
def test_ccoef_against_integral_solution(oracle_mod, tau, dG):
    C = oracle_mod.ccoef(tau, dG)
    Cb = _c_brute(tau, dG)
    np.testing.assert_allclose(C, Cb, rtol=2e-13, atol=1e-300)


def test_ccoef_limits(oracle_mod):
    dG = 0.01
    # tau -> 0 (continuum): C -> (dG, 0, dG^2/2, 0, 0); first corrections by hand
    # from Eq. (22) with exp(-dG/tau) = 0: (-tau, -tau dG + 2 tau^2, -tau dG + tau^2, tau, -tau^2)
    t = 1e-9
    C = oracle_mod.ccoef(t, dG)
    np.testing.assert_allclose(C, [dG - t, -t * dG + 2 * t * t, dG ** 2 / 2 - t * dG + t * t, t, -t * t],
                               rtol=1e-14, atol=1e-30)
    # tau -> inf (free transport): C -> (0, 0, 0, dG, -dG^2/2); leading terms by
    # expanding exp(-x), x = dG/tau: (dG^2/(2 tau), -dG^3/(6 tau), dG^3/(6 tau),
    # dG - dG^2/(2 tau), -dG^2/2 + dG^3/(3 tau))
    t = 1e9
    C = oracle_mod.ccoef(t, dG)
    np.testing.assert_allclose(C, [dG ** 2 / (2 * t), -dG ** 3 / (6 * t), dG ** 3 / (6 * t),
                                   dG - dG ** 2 / (2 * t), -dG ** 2 / 2 + dG ** 3 / (3 * t)],
                               rtol=1e-9, atol=1e-30)
    for tau in (1e-3, 0.1, 1.0, 10.0):
        C = oracle_mod.ccoef(tau, dG)
        assert abs(C[0] + C[3] - dG) < 1e-17


# ------------------------------------------------------------ Maxwellian moments
@pytest.mark.parametrize("U,lam", [(0.0, 1.0), (0.3, 0.7), (-0.8, 2.5), (2.0, 1.3)])
def test_half_space_moments(oracle_mod, U, lam):
    M = lambda u: np.sqrt(lam / np.pi) * np.exp(-lam * (u - U) ** 2)
    for which, (a, b) in ((0, (-np.inf, np.inf)), (1, (0, np.inf)), (2, (-np.inf, 0))):
        m = oracle_mod.moments_normal(U, lam, which, 7)
        for k in range(8):
            ref = integrate.quad(lambda u: u ** k * M(u), a, b, epsabs=1e-15, epsrel=1e-14,
                                 limit=200)[0]
            assert abs(m[k] - ref) <= 1e-13 * max(1.0, abs(ref)), (which, k, m[k], ref)


def _gh(n=40):
    x, w = np.polynomial.hermite.hermgauss(n)
    return x, w / np.sqrt(np.pi)


def _maxwell_avg(f, Un, Ut, lam, half=0, nleg=400):
    """<f(un, ut, xi)> of the normalised Maxwellian (K = 1), by quadrature:
    Gauss-Hermite in u_t and xi; Gauss-Hermite or Gauss-Legendre on a half
    line in u_n."""
    x, w = _gh()
    ut = Ut + x / np.sqrt(lam)
    xi = x / np.sqrt(lam)
    if half == 0:
        un = Un + x / np.sqrt(lam)
        wn = w
    else:
        g, gw = np.polynomial.legendre.leggauss(nleg)
        top = abs(Un) + 14.0 / np.sqrt(lam)
        if half == 1:
            un = 0.5 * top * (g + 1)
        else:
            un = -0.5 * top * (g + 1)
        wn = 0.5 * top * gw * np.sqrt(lam / np.pi) * np.exp(-lam * (un - Un) ** 2)
    UN, UT, XI = np.meshgrid(un, ut, xi, indexing="ij")
    WW = wn[:, None, None] * w[None, :, None] * w[None, None, :]
    return np.sum(WW * f(UN, UT, XI))


def _psi(i, un, ut, xi):
    return [np.ones_like(un), un, ut, 0.5 * (un ** 2 + ut ** 2 + xi ** 2)][i]


def _apsi(a, un, ut, xi):
    return a[0] + a[1] * un + a[2] * ut + 0.5 * a[3] * (un ** 2 + ut ** 2 + xi ** 2)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_slope_solve_recomposes(oracle_mod, seed):
    """a solves <psi (a.psi)> = dw (the Taylor-slope solve of Sec. 2.2)."""
    import hbcases
    r = hbcases.uniform(7, seed)
    Un, Ut, lam = 0.3 * r[0], 0.3 * r[1], 1.0 + 0.4 * r[2]
    dw = r[3:7]
    a = oracle_mod.slope_solve(Un, Ut, lam, 1, dw)
    got = [_maxwell_avg(lambda un, ut, xi: _psi(i, un, ut, xi) * _apsi(a, un, ut, xi), Un, Ut, lam)
           for i in range(4)]
    np.testing.assert_allclose(got, dw, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("pn,pt,half", [(1, 0, 1), (1, 0, 2), (0, 1, 0), (2, 0, 1), (2, 0, 2),
                                        (1, 1, 0), (1, 0, 0)])
def test_moment_vec_quadrature(oracle_mod, pn, pt, half):
    """<u_n^pn u_t^pt psi (a.psi)> over full / half spaces: the moments of the
    compatibility condition and of the C2/C3 part of Eq. (24)."""
    import hbcases
    r = hbcases.uniform(7, 100 + pn * 10 + pt + half)
    Un, Ut, lam = 0.4 * r[0], 0.4 * r[1], 1.0 + 0.5 * r[2]
    a = r[3:7]
    got = oracle_mod.moment_vec(a, pn, pt, Un, Ut, lam, 1, half)
    ref = [_maxwell_avg(lambda un, ut, xi: un ** pn * ut ** pt * _psi(i, un, ut, xi) *
                        _apsi(a, un, ut, xi), Un, Ut, lam, half) for i in range(4)]
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13)


# ------------------------------------------------------------ equilibria
def test_reduced_equilibrium_is_xi_integral_of_shakhov(oracle_mod):
    """H, B, H+, B+ equal the xi-integrals of g (Eq. 3) and g+ - g (Eq. 4) with
    D = 2, K = 1 (Eqs. 7-10), computed here by quadrature over xi."""
    rho, U, V, lam, Pr = 1.3, 0.2, -0.1, 0.8, 2.0 / 3.0
    q = np.array([0.05, -0.03])
    u = np.array([-1.1, 0.0, 0.4, 2.2])
    v = np.array([0.7, -0.5, 0.0, 1.9])
    H, B, Hp, Bp = oracle_mod.equilibrium(1, Pr, [rho, U, V, lam], q, u, v)
    RT = 1.0 / (2 * lam)
    p = rho * RT
    x, w = np.polynomial.hermite.hermgauss(60)
    xi = x / np.sqrt(lam)          # integrate over xi with weight exp(-lam xi^2)
    wx = w / np.sqrt(lam)
    for k in range(u.size):
        c2 = (u[k] - U) ** 2 + (v[k] - V) ** 2
        cq = (u[k] - U) * q[0] + (v[k] - V) * q[1]
        g = rho * (lam / np.pi) ** 1.5 * np.exp(-lam * c2)  # times exp(-lam xi^2) in the weight
        corr = (1 - Pr) * cq / (5 * p * RT) * ((c2 + xi ** 2) / RT - 5)
        assert abs(H[k] - np.sum(wx * g)) < 1e-15
        assert abs(B[k] - np.sum(wx * g * xi ** 2)) < 1e-15
        assert abs(Hp[k] - np.sum(wx * g * corr)) < 1e-15
        assert abs(Bp[k] - np.sum(wx * g * corr * xi ** 2)) < 1e-15


@pytest.mark.parametrize("seed", [11, 12])
def test_equilibrium_moments_on_wide_grid(oracle_mod, seed):
    """On a velocity grid wide and fine enough that the trapezoid rule is exact
    to round-off, sum w psi (H, B) = W, the Shakhov correction carries no mass,
    momentum or energy, and its heat flux is (1 - Pr) q ("moments of f - g
    vanish")."""
    import hbcases
    r = hbcases.uniform(6, seed)
    rho, U, V, lam = 1.0 + 0.3 * r[0], 0.3 * r[1], 0.3 * r[2], 1.0 + 0.4 * r[3]
    q = 0.05 * r[4:6]
    Pr = 2.0 / 3.0
    u1, w1 = oracle_mod.velocity_grid(80, 9.0)
    u, v = np.meshgrid(u1, u1, indexing="xy")
    u, v = u.ravel(), v.ravel()
    w = np.outer(w1, w1).ravel()
    H, B, Hp, Bp = oracle_mod.equilibrium(1, Pr, [rho, U, V, lam], q, u, v)
    W = [np.sum(w * H), np.sum(w * u * H), np.sum(w * v * H), 0.5 * np.sum(w * ((u * u + v * v) * H + B))]
    E = rho * (U * U + V * V) / 2 + 3 * rho / (4 * lam)
    np.testing.assert_allclose(W, [rho, rho * U, rho * V, E], rtol=1e-13, atol=1e-14)
    Wp = [np.sum(w * Hp), np.sum(w * u * Hp), np.sum(w * v * Hp), 0.5 * np.sum(w * ((u * u + v * v) * Hp + Bp))]
    np.testing.assert_allclose(Wp, 0.0, atol=1e-14)
    cu, cv = u - U, v - V
    e = (cu * cu + cv * cv)
    qp = 0.5 * np.array([np.sum(w * cu * (e * Hp + Bp)), np.sum(w * cv * (e * Hp + Bp))])
    np.testing.assert_allclose(qp, (1 - Pr) * q, rtol=1e-12, atol=1e-15)
    q0 = 0.5 * np.array([np.sum(w * cu * (e * H + B)), np.sum(w * cv * (e * H + B))])
    np.testing.assert_allclose(q0, 0.0, atol=1e-14)


def test_velocity_grid_trapezoid(oracle_mod):
    u1, w1 = oracle_mod.velocity_grid(16, 4.0)
    h = 8.0 / 15
    np.testing.assert_allclose(u1, -4.0 + h * np.arange(16), atol=1e-15)
    np.testing.assert_allclose(w1[1:-1], h, atol=1e-15)
    np.testing.assert_allclose(w1[[0, -1]], h / 2, atol=1e-15)
    np.testing.assert_allclose(u1, -u1[::-1], atol=1e-15)


@pytest.mark.parametrize("M", [4, 16, 28, 64])
def test_gauss_hermite_moments(oracle_mod, M):
    """The M-point Gauss-Hermite rule (Sec. 3.1.1) is exact for polynomials of
    degree <= 2M - 1 against exp(-u^2): with the weight folded into w,
    sum w u^(2j) exp(-u^2) = Gamma(j + 1/2) and odd moments vanish.  A wrong
    node, a weight without the exp(u^2) factor or a mirrored half fails."""
    u, w = oracle_mod.gauss_hermite(M)
    assert np.all(np.diff(u) > 0) and np.all(w > 0)
    np.testing.assert_allclose(u, -u[::-1], atol=1e-14)
    g = w * np.exp(-u * u)
    for j in range(M):
        ref = float(mp.gamma(j + 0.5))
        assert abs(np.sum(g * u ** (2 * j)) - ref) <= 1e-13 * ref * max(1.0, 2.0 ** j), j
        assert abs(np.sum(g * u ** (2 * j + 1))) <= 1e-13 * ref * max(1.0, 2.0 ** j)


def test_gauss_hermite_rest_state_moments(oracle_mod):
    """On the 28 x 28 Gauss-Hermite grid the oracle's rest Maxwellian has
    density 1 and energy (2 + K)/4 to round-off (the rule is exact for it)."""
    import hbcases
    case = hbcases.Case(4, 4, 28, 0.0, 0.1, 1.0, 0, vrule=1)
    o = oracle_mod.Oracle(case)
    W, h, b = o.state()
    u, w1 = oracle_mod.gauss_hermite(28)
    uu, vv = np.meshgrid(u, u)
    w = np.outer(w1, w1).ravel()
    e2 = (uu * uu + vv * vv).ravel()
    np.testing.assert_allclose(np.sum(w * h[0, 0]), 1.0, rtol=1e-14)
    np.testing.assert_allclose(0.5 * np.sum(w * (e2 * h[0, 0] + b[0, 0])), (2 + case.K) / 4.0, rtol=1e-14)
