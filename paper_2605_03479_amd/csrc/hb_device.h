// Device-side helpers of the HB-UGKS pseudo step (gfx950).
//
// Everything here is scalar per-face / per-cell arithmetic: primitives,
// relaxation time, the UGKS time coefficients, the Taylor-slope solve, the
// Maxwellian moments of the compatibility condition and of the macro flux,
// and cubic polynomials in the face-frame velocities (n, t).
#pragma once
#include <hip/hip_runtime.h>

#define HB_NTMAX 11
#define HB_PI 3.14159265358979323846

namespace hb {

// Pointers typed in the global address space.  Kernel arguments are known to
// be global, but pointers read from memory (the per-case tables of the batched
// form) are not, and the compiler would access them with flat instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ inline gptr<T> G(T *p)
{
    return (gptr<T>)p;
}
template <class T>
__device__ inline gptr<T> G(gptr<T> p)
{
    return p;
}

struct Params {
    // velocity grid: M nodes along u (Mh = M/2), Mv along v (Mvh = Mv/2),
    // Mt = max(M, Mv) the stride of the per-axis tables
    int nx, ny, nc, M, Mh, Mv, Mvh, Mt, Q, Qp, nvp, NT, NH, K, face_dt, dt_mode;
    int macro_mode;  // 0: macro flux of Eq. (24); 1: the velocity sum of the micro flux
    int level_mass;  // 1: level-mass projection after each step (see resid_block)
    int ls;  // level stride of h, b in words (nvp plus padding)
    int stream_out;  // 1: the update stores h, b past the caches (the state exceeds the last-level cache)
    double omega, mu_ref, omega_vss, Pr, cfl, gamma, umax, vmax, dt_fixed;
    double E[HB_NTMAX * HB_NTMAX];
    double wall_ut[4][HB_NTMAX], wall_T[4][HB_NTMAX];
    // geometry
    const double *xf, *yf, *xc, *yc, *rdx, *rdy, *rcx, *rcy;
    // velocity grid: 1-D nodes/weights and per-alpha (internal order) values
    const double *u1, *w1, *v1, *w1v, *vu, *vv, *vw;  // 1-D rules along u (M) and v (Mv)
    const int *viu, *viv;
    const double *vref;  // rest Maxwellian per velocity (mixed storage reference)
    const double *rmom;  // per quadrant, sum of w u^a v^b H_ref over its velocities, a + b <= 3 (10 each)
    double *lscale;      // per-level scale factors of the level-mass projection [HB_NTMAX]
    // mixed form only (null otherwise): FP32 face and collision records, the
    // projection factors s_n and (s_n - 1)/pi in FP32, E(u_k) = exp(-u_k^2)
    // in FP64 and FP32, and E of Eq. (17) in FP32
    float *rx32, *ry32, *cr32, *lscale32;
    const double *ex64, *ex64v;  // exp(-x^2) at the u nodes, at the v nodes
    const float *er32, *er32v;
    const float *vel32;  // vu, vv, vw rounded to FP32 (multipliers of the deviations in the moment sums)
    float Ef[HB_NTMAX * HB_NTMAX];
};

// W = (rho, rho Un, rho Ut, rho E) -> (rho, Un, Ut, lambda); rho E = rho |U|^2/2 + (2+K) rho/(4 lambda)
__host__ __device__ inline void prim4(int K, const double *W, double *p)
{
    double rho = W[0];
    double U = W[1] / rho, V = W[2] / rho;
    double e = W[3] - 0.5 * rho * (U * U + V * V);
    p[0] = rho;
    p[1] = U;
    p[2] = V;
    p[3] = (2.0 + K) * rho / (4.0 * e);
}

// tau = mu / p, mu = mu_ref (T/T0)^omega_vss, p = rho/(2 lambda), T/T0 = 1/lambda
__device__ inline double tau_of(const Params &P, double rho, double lam)
{
    return P.mu_ref * pow(1.0 / lam, P.omega_vss) * 2.0 * lam / rho;
}

// UGKS time coefficients of the interface integral solution, x = dG/tau.
// The tau^2 brackets (and C1) are summed as power series below x = 1, where
// the closed forms lose digits to cancellation.
__device__ inline void ccoef(double tau, double dG, double C[5])
{
    double x = dG / tau;
    double e1 = -expm1(-x);
    double p2, p3, p5, p1;
    if (x < 1.0) {
        double t = 0.5 * x * x;  // x^k / k! at k = 2
        p2 = 0.0;
        p3 = 0.0;
        p5 = -t;
        double sgn = 1.0;  // (-1)^(k+1) at k = 3
#pragma unroll
        for (int k = 3; k <= 30; k++) {
            t *= x * (1.0 / k);  // unrolled: 1/k is a constant, no division in the chain
            p3 += sgn * t;
            p2 += sgn * (2.0 - k) * t;
            p5 += sgn * (k - 1.0) * t;
            sgn = -sgn;
        }
        p1 = 0.5 * x * x - p3;
    } else {
        double ex = exp(-x);
        p3 = 0.5 * x * x - x + e1;
        p2 = 2.0 * e1 - x - x * ex;
        p5 = x * ex - e1;
        p1 = x - e1;
    }
    C[0] = tau * p1;
    C[1] = tau * tau * p2;
    C[2] = tau * tau * p3;
    C[3] = tau * e1;
    C[4] = tau * tau * p5;
}

// Closed-form solve of <psi (a.psi)>_g = dw for a normalised Maxwellian with
// mean (Un, Ut), inverse temperature lam, K internal dofs.
__device__ inline void slope_solve(double Un, double Ut, double lam, int K, const double dw[4], double a[4])
{
    const double rk = 1.0 / (K + 2.0);
    double s = Un * Un + Ut * Ut + 0.5 * (K + 2.0) / lam;
    double R2 = dw[1] - Un * dw[0];
    double R3 = dw[2] - Ut * dw[0];
    double R4 = 2.0 * dw[3] - s * dw[0];
    double a4 = 4.0 * lam * lam * (R4 - 2.0 * Un * R2 - 2.0 * Ut * R3) * rk;
    double a2 = 2.0 * lam * R2 - Un * a4;
    double a3 = 2.0 * lam * R3 - Ut * a4;
    a[0] = dw[0] - Un * a2 - Ut * a3 - 0.5 * a4 * s;
    a[1] = a2;
    a[2] = a3;
    a[3] = a4;
}

// Moment tables of a Maxwellian: normal direction over `which` (0 full, 1 u>0, 2 u<0),
// tangential full, xi^(2g).  N[0..7], T[0..7], X[0..2].
struct MomTab {
    double N[8], T[8], X[3];
};

__device__ inline void normal_moments(double U, double lam, int which, double *m, int nmax)
{
    double e = exp(-lam * U * U) * (0.5 / sqrt(HB_PI * lam));
    if (which == 0) {
        m[0] = 1.0;
        m[1] = U;
    } else if (which == 1) {
        m[0] = 0.5 * erfc(-sqrt(lam) * U);
        m[1] = U * m[0] + e;
    } else {
        m[0] = 0.5 * erfc(sqrt(lam) * U);
        m[1] = U * m[0] - e;
    }
    double r = 0.5 / lam;
    for (int k = 2; k <= nmax; k++) m[k] = U * m[k - 1] + (k - 1) * r * m[k - 2];
}

__device__ inline void momtab(double Un, double Ut, double lam, int K, int which, MomTab &t)
{
    normal_moments(Un, lam, which, t.N, 7);
    normal_moments(Ut, lam, 0, t.T, 7);
    t.X[0] = 1.0;
    t.X[1] = K / (2.0 * lam);
    t.X[2] = K * (K + 2.0) / (4.0 * lam * lam);
}

// <n^p t^r (xi^2)^g (a.psi)>, a.psi = a0 + a1 n + a2 t + a3 (n^2 + t^2 + xi^2)/2
__device__ inline double m_apsi(const MomTab &t, int p, int r, int g, const double a[4])
{
    return a[0] * t.N[p] * t.T[r] * t.X[g] + a[1] * t.N[p + 1] * t.T[r] * t.X[g] +
           a[2] * t.N[p] * t.T[r + 1] * t.X[g] +
           0.5 * a[3] * (t.N[p + 2] * t.T[r] * t.X[g] + t.N[p] * t.T[r + 2] * t.X[g] + t.N[p] * t.T[r] * t.X[g + 1]);
}

// out_i = <n^p t^r psi_i (a.psi)>, psi = (1, n, t, (n^2+t^2+xi^2)/2)
__device__ inline void mpsi_apsi(const MomTab &t, int p, int r, const double a[4], double out[4])
{
    out[0] = m_apsi(t, p, r, 0, a);
    out[1] = m_apsi(t, p + 1, r, 0, a);
    out[2] = m_apsi(t, p, r + 1, 0, a);
    out[3] = 0.5 * (m_apsi(t, p + 2, r, 0, a) + m_apsi(t, p, r + 2, 0, a) + m_apsi(t, p, r, 1, a));
}

// Cubic polynomial in (n, t); monomial order 1, n, t, nn, nt, tt, nnn, nnt, ntt, ttt.
struct P3 {
    double c[10];
};
__device__ inline void p3_zero(P3 &p)
{
#pragma unroll
    for (int k = 0; k < 10; k++) p.c[k] = 0.0;
}
// (l0 + l1 n + l2 t) * (q0 + q1 n + q2 t + q3 nn + q4 nt + q5 tt)
__device__ inline void p3_lin_quad(const double l[3], const double q[6], P3 &o)
{
    o.c[0] = l[0] * q[0];
    o.c[1] = l[0] * q[1] + l[1] * q[0];
    o.c[2] = l[0] * q[2] + l[2] * q[0];
    o.c[3] = l[0] * q[3] + l[1] * q[1];
    o.c[4] = l[0] * q[4] + l[1] * q[2] + l[2] * q[1];
    o.c[5] = l[0] * q[5] + l[2] * q[2];
    o.c[6] = l[1] * q[3];
    o.c[7] = l[1] * q[4] + l[2] * q[3];
    o.c[8] = l[1] * q[5] + l[2] * q[4];
    o.c[9] = l[2] * q[5];
}
__device__ inline void p3_axpy(double s, const P3 &x, P3 &y)
{
#pragma unroll
    for (int k = 0; k < 10; k++) y.c[k] += s * x.c[k];
}
// exponents of the monomials
__device__ constexpr int P3_N[10] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0};
__device__ constexpr int P3_T[10] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};

// sum_alpha w n^a t^b P(n, t) e_n(n) e_t(t) from 1-D sums Gn[k] = sum w n^k e_n, Gt likewise
__device__ inline double p3_sum(const P3 &p, int a, int b, const double *Gn, const double *Gt)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 10; k++) s += p.c[k] * Gn[a + P3_N[k]] * Gt[b + P3_T[k]];
    return s;
}

// Shakhov factor S = s (c.q) (2 lam |c|^2 + kappa), c = (n - Un, t - Ut), as a cubic in (n, t)
__device__ inline void shakhov_poly(double s, double qn, double qt, double Un, double Ut, double lam, double kappa,
                                    P3 &o)
{
    double l[3] = {-s * (qn * Un + qt * Ut), s * qn, s * qt};
    double q[6] = {2.0 * lam * (Un * Un + Ut * Ut) + kappa, -4.0 * lam * Un, -4.0 * lam * Ut, 2.0 * lam, 0.0,
                   2.0 * lam};
    p3_lin_quad(l, q, o);
}

// a . psi reduced over xi against the h (xx = K/(2 lam)) or b (xx = (K+2)/(2 lam)) weight:
// a0 + a1 n + a2 t + a3 (n^2 + t^2 + xx)/2, as the quadratic coefficients q[6]
__device__ inline void apsi_quad(const double a[4], double xx, double q[6])
{
    q[0] = a[0] + 0.5 * a[3] * xx;
    q[1] = a[1];
    q[2] = a[2];
    q[3] = 0.5 * a[3];
    q[4] = 0.0;
    q[5] = 0.5 * a[3];
}

}  // namespace hb
