/*
 * hbref.c -- plain, slow FP64 CPU oracle of the HB-UGKS pseudo-time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU path, and it imports nothing from it.
 *
 * What it computes follows the HB-UGKS paper (arXiv 2605.03479), Section 2:
 *   Sec. 2.1  BGK/Shakhov model: Eqs. (1)-(10)  (Maxwellian, Shakhov g+,
 *             moments, heat flux, reduced distributions h, b, h+, b+)
 *   Sec. 2.2  harmonic balance: Eqs. (12), (17) (collocation, spectral operator E);
 *             UGKS interface flux: Eqs. (21)-(24) (integral solution, C1..C5,
 *             micro flux, macro flux)
 *   Sec. 2.3  walls: Eqs. (25)-(28) (harmonic wall state, diffuse wall, rho_w)
 *   Sec. 2.4  finite volume + pseudo time: Eqs. (29)-(33)
 *   Sec. 3.1  Kn, St (Eqs. 36, 37), shear stress (Eq. 39), DFT (Eq. 40),
 *   Sec. 3.1.4 residual (Eq. 43)
 * Where the paper is silent the reading taken is stated at the point of use
 * (limiter, wall-adjacent slopes, slope sources, heat flux at k+1, the wall
 * incident state, the velocity quadrature, CFL).
 *
 * Units: rho0 = H = sqrt(2 R T0) = 1, so R T0 = 1/2, lambda0 = 1, Ttilde = 1/lambda.
 * Layouts (row-major, last index fastest):
 *   W[c][n][4] with c = j*nx + i;   h, b [c][n][alpha] with alpha = iv*M + iu.
 * Everything is plain loops; OpenMP only splits independent rows/cells.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define NTMAX 11
#define PN 8 /* polynomial degree bound in u_n (0..7) */
#define PT 6 /* in u_t (0..5) */
#define PX 3 /* in xi^2 (0..2) */

typedef struct {
    /* geometry */
    int nx, ny, nc;
    double *xf, *yf, *xc, *yc, *dx, *dy;
    /* velocity grid: tensor product of a 1-D rule of M nodes along u and one
     * of Mv nodes along v */
    int M, Mv, nv;
    double umax, vmax;
    double *u1, *w1, *v1, *w1v;
    double *u, *v, *w;
    /* physics and numerics */
    int NH, NT, K;
    double Kn, St, omega, mu_ref, Pr, omega_vss, gamma, cfl;
    int face_dt, macro_mode, dt_mode, level_mass;
    double dt_fixed;
    double E[NTMAX * NTMAX];
    double wall_ut[4][NTMAX], wall_T[4][NTMAX];
    double walls_in[4][6];
    /* state */
    double *W, *h, *b;
    long step;
    double res[4];
    /* work arrays */
    double *Wn, *dtc, *divH, *divB, *divF, *q;
    double *sxh, *syh, *sxb, *syb;
    double *Fx, *Fy; /* macro fluxes [face][n][4], x-faces (nx+1)*ny, y-faces nx*(ny+1) */
    double t_phys;   /* time-domain mode: physical time */
    double dt_scale; /* test hook: multiplies every local step (1 by default) */
} hbref;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */

static double sq(double a) { return a * a; }

/* van Leer limiter (the paper asks for "a monotonicity-preserving limiter",
 * Sec. 2.2 after Eq. 21; van Leer is the reading taken). */
static double vanleer(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return 2.0 * a * b / (a + b);
}

/* 1-D closed composite trapezoid rule on [-umax, umax] with M nodes: the
 * Newton-Cotes rule of Sec. 3.1.1 read as its two-point member. */
void hbref_velocity_grid(int M, double umax, double *u1, double *w1)
{
    double du = 2.0 * umax / (M - 1);
    for (int k = 0; k < M; k++) {
        u1[k] = -umax + k * du;
        w1[k] = (k == 0 || k == M - 1) ? 0.5 * du : du;
    }
}

/* Spectral operator E of Eq. (17), Sec. 2.2: E_nm = 1/2 (-1)^(n-m) csc(pi (n-m)/NT). */
void hbref_E(int NT, double *E)
{
    for (int n = 0; n < NT; n++)
        for (int m = 0; m < NT; m++) {
            if (n == m) {
                E[n * NT + m] = 0.0;
            } else {
                int d = n - m;
                double sgn = (abs(d) % 2 == 0) ? 1.0 : -1.0;
                E[n * NT + m] = 0.5 * sgn / sin(M_PI * d / NT);
            }
        }
}

/* Viscosity reference from Kn, Eq. (36) with rho0 = H = 1 and sqrt(2 pi R T0) = sqrt(pi). */
static double mu_ref_from_kn(double Kn, double omega_vss, double alpha_vss)
{
    double a = alpha_vss, w = omega_vss;
    double coef = 4.0 * a * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) / (5.0 * (a + 1.0) * (a + 2.0));
    return Kn * sqrt(M_PI) / coef;
}

/* tau = mu/p (Sec. 2.1, Eq. 2), mu = mu_ref Ttilde^omega_vss (Sec. 3.1.1),
 * p = rho/(2 lambda), Ttilde = 1/lambda. */
static double tau_of(const hbref *o, double rho, double lam)
{
    double mu = o->mu_ref * pow(1.0 / lam, o->omega_vss);
    return mu * 2.0 * lam / rho;
}

/* Conservative W = (rho, rho U, rho V, rho E) -> primitives (rho, U, V, lambda).
 * rho E = rho |U|^2 / 2 + (2 + K) rho / (4 lambda). */
static void prim_of(int K, const double *W, double *p)
{
    double rho = W[0];
    double U = W[1] / rho, V = W[2] / rho;
    double eint = W[3] - 0.5 * rho * (U * U + V * V);
    p[0] = rho;
    p[1] = U;
    p[2] = V;
    p[3] = (2.0 + K) * rho / (4.0 * eint);
}

/* ------------------------------------------------------------------ */
/* UGKS time coefficients C1..C5, Eq. (22), Sec. 2.2.
 * With x = dG/tau the printed forms equal
 *   C1 = dG - tau e1,  C4 = tau e1,  e1 = 1 - exp(-x)
 *   C2 = tau^2 (2 e1 - x - x exp(-x)),  C3 = tau^2 (x^2/2 - x + e1),
 *   C5 = tau^2 (x exp(-x) - e1).
 * For x < 1 the three tau^2 brackets are summed as their Taylor series, and
 * C1 = tau (x - e1) = tau (x^2/2 - p3), because the printed differences cancel
 * catastrophically when dG << tau. */
void hbref_ccoef(double tau, double dG, double *C)
{
    double x = dG / tau;
    double e1 = -expm1(-x);
    double ex = exp(-x);
    double p2, p3, p5;
    if (x < 1.0) {
        /* p3 = sum_{k>=3} (-1)^(k+1) x^k/k!
         * p2 = sum_{k>=3} (-1)^(k+1) (2-k) x^k/k!
         * p5 = sum_{k>=2} (-1)^(k+1) (k-1) x^k/k!          */
        double term = x * x / 2.0; /* x^k/k! at k = 2 */
        p2 = 0.0;
        p3 = 0.0;
        p5 = -term; /* k = 2: (-1)^3 * 1 * x^2/2 */
        for (int k = 3; k <= 30; k++) {
            term *= x / k;
            double s = (k % 2 == 1) ? 1.0 : -1.0; /* (-1)^(k+1) */
            p3 += s * term;
            p2 += s * (2.0 - k) * term;
            p5 += s * (k - 1.0) * term;
        }
    } else {
        p3 = x * x / 2.0 - x + e1;
        p2 = 2.0 * e1 - x - x * ex;
        p5 = x * ex - e1;
    }
    C[0] = (x < 1.0) ? tau * (0.5 * x * x - p3) : dG - tau * e1;
    C[1] = tau * tau * p2;
    C[2] = tau * tau * p3;
    C[3] = tau * e1;
    C[4] = tau * tau * p5;
}

/* ------------------------------------------------------------------ */
/* Maxwellian moments, used for the slope solves, the compatibility
 * condition and the C2/C3 parts of the macro flux (Eq. 24).
 * A polynomial in (u_n, u_t, xi^2) is a list of terms c u_n^pn u_t^pt (xi^2)^px. */
#define PTERMS 64
typedef struct {
    int n;
    int pn[PTERMS], pt[PTERMS], px[PTERMS];
    double c[PTERMS];
} poly;

static void poly_zero(poly *p) { p->n = 0; }

static void poly_add(poly *p, int pn, int pt, int px, double c)
{
    p->pn[p->n] = pn;
    p->pt[p->n] = pt;
    p->px[p->n] = px;
    p->c[p->n] = c;
    p->n++;
}

static void poly_mul(const poly *x, const poly *y, poly *z)
{
    poly r;
    poly_zero(&r);
    for (int i = 0; i < x->n; i++)
        for (int j = 0; j < y->n; j++)
            poly_add(&r, x->pn[i] + y->pn[j], x->pt[i] + y->pt[j], x->px[i] + y->px[j], x->c[i] * y->c[j]);
    *z = r;
}

/* Normal-velocity moments <u^k> of the 1-D normalised Maxwellian with mean U
 * and inverse temperature lam, over the full line (which = 0), u > 0 (1) or
 * u < 0 (2).  Recursion <u^{k+2}> = U <u^{k+1}> + (k+1)/(2 lam) <u^k>, from
 * integration by parts; the half-line starts carry the boundary term. */
void hbref_moments_normal(double U, double lam, int which, int nmax, double *m)
{
    double e = exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
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
    for (int k = 0; k + 2 <= nmax; k++) m[k + 2] = U * m[k + 1] + (k + 1) / (2.0 * lam) * m[k];
}

/* <p> for the normalised Maxwellian (rho = 1) with face-frame mean (Un, Ut),
 * inverse temperature lam and K internal degrees of freedom; the normal
 * direction is restricted by `which`. */
static double poly_moment(const poly *p, double Un, double Ut, double lam, int K, int which)
{
    double mn[PN], mt[PT], mx[PX];
    hbref_moments_normal(Un, lam, which, PN - 1, mn);
    hbref_moments_normal(Ut, lam, 0, PT - 1, mt);
    mx[0] = 1.0;
    mx[1] = K / (2.0 * lam);
    mx[2] = K * (K + 2.0) / (4.0 * lam * lam);
    double s = 0.0;
    for (int i = 0; i < p->n; i++) {
        if (p->pn[i] >= PN || p->pt[i] >= PT || p->px[i] >= PX) abort(); /* degree bound */
        s += p->c[i] * mn[p->pn[i]] * mt[p->pt[i]] * mx[p->px[i]];
    }
    return s;
}

/* psi_i, the collision invariants (1, u_n, u_t, (u_n^2 + u_t^2 + xi^2)/2) of Eq. (5). */
static void psi_poly(int i, poly *p)
{
    poly_zero(p);
    if (i == 0) poly_add(p, 0, 0, 0, 1.0);
    if (i == 1) poly_add(p, 1, 0, 0, 1.0);
    if (i == 2) poly_add(p, 0, 1, 0, 1.0);
    if (i == 3) {
        poly_add(p, 2, 0, 0, 0.5);
        poly_add(p, 0, 2, 0, 0.5);
        poly_add(p, 0, 0, 1, 0.5);
    }
}

/* a . psi as a polynomial. */
static void apsi_poly(const double *a, poly *p)
{
    poly_zero(p);
    poly_add(p, 0, 0, 0, a[0]);
    poly_add(p, 1, 0, 0, a[1]);
    poly_add(p, 0, 1, 0, a[2]);
    poly_add(p, 2, 0, 0, 0.5 * a[3]);
    poly_add(p, 0, 2, 0, 0.5 * a[3]);
    poly_add(p, 0, 0, 1, 0.5 * a[3]);
}

/* <m psi_i (a . psi)> for i = 0..3, where m = u_n^pn u_t^pt. */
static void moment_vec(const double *a, int pn, int pt, double Un, double Ut, double lam, int K,
                       int which, double *out)
{
    poly ap, mp, t, ps;
    apsi_poly(a, &ap);
    poly_zero(&mp);
    poly_add(&mp, pn, pt, 0, 1.0);
    for (int i = 0; i < 4; i++) {
        psi_poly(i, &ps);
        poly_mul(&mp, &ps, &t);
        poly_mul(&t, &ap, &t);
        out[i] = poly_moment(&t, Un, Ut, lam, K, which);
    }
}

/* Solve <psi (a . psi)> = d for a (4x4 system of Maxwellian moments,
 * Gaussian elimination with partial pivoting).  This is how the spatial
 * slopes a_n, a_t and the time slope A of the equilibrium expansion in
 * Sec. 2.2 (after Eq. 21) are found. */
void hbref_slope_solve(double Un, double Ut, double lam, int K, const double *d, double *a)
{
    double Mx[4][5];
    for (int i = 0; i < 4; i++) {
        for (int j = 0; j < 4; j++) {
            poly pi, pj, t;
            psi_poly(i, &pi);
            psi_poly(j, &pj);
            poly_mul(&pi, &pj, &t);
            Mx[i][j] = poly_moment(&t, Un, Ut, lam, K, 0);
        }
        Mx[i][4] = d[i];
    }
    for (int col = 0; col < 4; col++) {
        int piv = col;
        for (int r = col + 1; r < 4; r++)
            if (fabs(Mx[r][col]) > fabs(Mx[piv][col])) piv = r;
        if (piv != col)
            for (int k = 0; k < 5; k++) {
                double tmp = Mx[col][k];
                Mx[col][k] = Mx[piv][k];
                Mx[piv][k] = tmp;
            }
        for (int r = col + 1; r < 4; r++) {
            double f = Mx[r][col] / Mx[col][col];
            for (int k = col; k < 5; k++) Mx[r][k] -= f * Mx[col][k];
        }
    }
    for (int r = 3; r >= 0; r--) {
        double s = Mx[r][4];
        for (int k = r + 1; k < 4; k++) s -= Mx[r][k] * a[k];
        a[r] = s / Mx[r][r];
    }
}

/* Exported for the pins: <u_n^pn u_t^pt psi_i (a . psi)>, i = 0..3. */
void hbref_moment_vec(const double *a, int pn, int pt, double Un, double Ut, double lam, int K, int which,
                      double *out)
{
    moment_vec(a, pn, pt, Un, Ut, lam, K, which, out);
}

/* ------------------------------------------------------------------ */
/* Reduced equilibria, Eqs. (3), (4), (9), (10) integrated over the K internal
 * velocities:
 *   H  = rho (lam/pi) exp(-lam |c|^2),  B = K/(2 lam) H
 *   H+ = (1-Pr) 4 lam^2/(5 rho) (c.q) (2 lam |c|^2 + K - 5) H
 *   B+ = (1-Pr) 4 lam^2/(5 rho) (c.q) (2 lam |c|^2 + K - 3) B
 * prim = (rho, U, V, lam); q in the same frame as (u, v). */
static void equilibrium(int K, double Pr, const double *prim, const double *q, double u, double v,
                        double *Hout, double *Bout, double *Hp, double *Bp)
{
    double rho = prim[0], lam = prim[3];
    double cu = u - prim[1], cv = v - prim[2];
    double c2 = cu * cu + cv * cv;
    double H = rho * (lam / M_PI) * exp(-lam * c2);
    double B = K / (2.0 * lam) * H;
    double s = (1.0 - Pr) * 4.0 * lam * lam / (5.0 * rho) * (cu * q[0] + cv * q[1]);
    *Hout = H;
    *Bout = B;
    *Hp = s * (2.0 * lam * c2 + K - 5.0) * H;
    *Bp = s * (2.0 * lam * c2 + K - 3.0) * B;
}

/* Exported for the equilibrium pins: per-velocity H, B, H+, B+. */
void hbref_equilibrium(int K, double Pr, const double *prim, const double *q, int n, const double *u,
                       const double *v, double *H, double *B, double *Hp, double *Bp)
{
    for (int k = 0; k < n; k++) equilibrium(K, Pr, prim, q, u[k], v[k], &H[k], &B[k], &Hp[k], &Bp[k]);
}

/* Heat flux q = 1/2 sum_a w c (|c|^2 h + b), Eq. (6) reduced by Eqs. (7)-(8),
 * about the velocity (U, V). */
static void heat_flux(int nv, const double *u, const double *v, const double *w, const double *h,
                      const double *b, double U, double V, double *q)
{
    double qx = 0.0, qy = 0.0;
    for (int a = 0; a < nv; a++) {
        double cu = u[a] - U, cv = v[a] - V;
        double e = (cu * cu + cv * cv) * h[a] + b[a];
        qx += w[a] * cu * e;
        qy += w[a] * cv * e;
    }
    q[0] = 0.5 * qx;
    q[1] = 0.5 * qy;
}

/* W = sum_a w psi (h, b), Eq. (5) reduced by Eqs. (7)-(8). */
static void moments_W(int nv, const double *u, const double *v, const double *w, const double *h,
                      const double *b, double *W)
{
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int a = 0; a < nv; a++) {
        s0 += w[a] * h[a];
        s1 += w[a] * u[a] * h[a];
        s2 += w[a] * v[a] * h[a];
        s3 += w[a] * 0.5 * ((u[a] * u[a] + v[a] * v[a]) * h[a] + b[a]);
    }
    W[0] = s0;
    W[1] = s1;
    W[2] = s2;
    W[3] = s3;
}

/* ------------------------------------------------------------------ */
/* setup                                                                 */

void *hbref_new(void) { return calloc(1, sizeof(hbref)); }

static void free_arrays(hbref *o)
{
    double **ptrs[] = {&o->xf,  &o->yf,  &o->xc,  &o->yc,  &o->dx,   &o->dy,   &o->u1, &o->w1,
                       &o->v1,  &o->w1v, &o->u,   &o->v,   &o->w,   &o->W,   &o->h,    &o->b,    &o->Wn, &o->dtc,
                       &o->divH, &o->divB, &o->divF, &o->q, &o->sxh, &o->syh, &o->sxb, &o->syb,
                       &o->Fx,  &o->Fy};
    for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); k++) {
        free(*ptrs[k]);
        *ptrs[k] = NULL;
    }
}

void hbref_free(void *p)
{
    if (!p) return;
    free_arrays((hbref *)p);
    free(p);
}

/* Harmonic wall state at phase theta = omega t, Eqs. (25)-(26):
 * value = mean + Re(hat e^{i theta}). */
static void wall_state_at(const hbref *o, int wl, double theta, double *ut, double *T)
{
    const double *p = o->walls_in[wl];
    *ut = p[0] + p[1] * cos(theta) - p[2] * sin(theta);
    *T = p[3] + p[4] * cos(theta) - p[5] * sin(theta);
}

/* walls: 4 x 6 doubles, wall order bottom (y=0), right (x=L), top (y=H),
 * left (x=0); per wall (ut_mean, ut_re, ut_im, T_mean, T_re, T_im), ut the
 * wall-tangential velocity along +x (bottom/top) or +y (left/right), T in T0.
 * dt_mode 0: local pseudo step of Eqs. (31)-(32); 1: one global step dt_fixed.
 * u1in, w1in: NULL for the closed trapezoid rule on [-umax, umax], else M
 * increasing 1-D nodes and their weights (umax is then the last node).
 * Mv, vmax, v1in, w1vin: the same for the v axis (Mv = 0 takes M and the u
 * rule, vmax <= 0 takes umax). */
int hbref_setup(void *p, int nx, int ny, double L, double Hh, const double *xf, const double *yf, int M,
                double umax, double Kn, double St, int NH, const double *walls, double cfl, int face_dt,
                double Pr, double omega_vss, double alpha_vss, int K, int macro_mode, int dt_mode,
                double dt_fixed, const double *u1in, const double *w1in, int level_mass, int Mv, double vmax,
                const double *v1in, const double *w1vin)
{
    hbref *o = (hbref *)p;
    if (Mv == 0) {
        Mv = M;
        v1in = u1in;
        w1vin = w1in;
    }
    if (!(vmax > 0.0)) vmax = umax;
    if (nx < 3 || ny < 3 || M < 2 || (M % 2) != 0 || Mv < 2 || (Mv % 2) != 0 || NH < 0 || 2 * NH + 1 > NTMAX ||
        Kn <= 0.0)
        return -1;
    free_arrays(o);
    o->nx = nx;
    o->ny = ny;
    o->nc = nx * ny;
    o->M = M;
    o->Mv = Mv;
    o->nv = M * Mv;
    o->umax = umax;
    o->vmax = vmax;
    o->NH = NH;
    o->NT = 2 * NH + 1;
    o->K = K;
    o->Kn = Kn;
    o->St = St;
    o->omega = St; /* Eq. (37) with H = sqrt(2 R T0) = 1 */
    o->Pr = Pr;
    o->omega_vss = omega_vss;
    o->gamma = (K + 4.0) / (K + 2.0); /* D = 2 translational + K internal */
    o->cfl = cfl;
    o->face_dt = face_dt;
    o->macro_mode = macro_mode;
    o->level_mass = level_mass;
    o->dt_mode = dt_mode;
    o->dt_fixed = dt_fixed;
    o->mu_ref = mu_ref_from_kn(Kn, omega_vss, alpha_vss);

    o->xf = malloc(sizeof(double) * (nx + 1));
    o->yf = malloc(sizeof(double) * (ny + 1));
    o->xc = malloc(sizeof(double) * nx);
    o->yc = malloc(sizeof(double) * ny);
    o->dx = malloc(sizeof(double) * nx);
    o->dy = malloc(sizeof(double) * ny);
    for (int i = 0; i <= nx; i++) o->xf[i] = xf ? xf[i] : L * i / nx;
    for (int j = 0; j <= ny; j++) o->yf[j] = yf ? yf[j] : Hh * j / ny;
    for (int i = 0; i < nx; i++) {
        o->xc[i] = 0.5 * (o->xf[i] + o->xf[i + 1]);
        o->dx[i] = o->xf[i + 1] - o->xf[i];
        if (o->dx[i] <= 0.0) return -1;
    }
    for (int j = 0; j < ny; j++) {
        o->yc[j] = 0.5 * (o->yf[j] + o->yf[j + 1]);
        o->dy[j] = o->yf[j + 1] - o->yf[j];
        if (o->dy[j] <= 0.0) return -1;
    }

    o->u1 = malloc(sizeof(double) * M);
    o->w1 = malloc(sizeof(double) * M);
    if (u1in && w1in) { /* a given 1-D rule (Gauss-Hermite, Sec. 3.1.1): its largest node bounds Eq. (32) */
        memcpy(o->u1, u1in, sizeof(double) * M);
        memcpy(o->w1, w1in, sizeof(double) * M);
        o->umax = u1in[M - 1];
    } else {
        hbref_velocity_grid(M, umax, o->u1, o->w1);
    }
    o->v1 = malloc(sizeof(double) * Mv);
    o->w1v = malloc(sizeof(double) * Mv);
    if (v1in && w1vin) {
        memcpy(o->v1, v1in, sizeof(double) * Mv);
        memcpy(o->w1v, w1vin, sizeof(double) * Mv);
        o->vmax = v1in[Mv - 1];
    } else {
        hbref_velocity_grid(Mv, vmax, o->v1, o->w1v);
    }
    int nv = o->nv;
    o->u = malloc(sizeof(double) * nv);
    o->v = malloc(sizeof(double) * nv);
    o->w = malloc(sizeof(double) * nv);
    for (int iv = 0; iv < Mv; iv++)
        for (int iu = 0; iu < M; iu++) {
            int a = iv * M + iu;
            o->u[a] = o->u1[iu];
            o->v[a] = o->v1[iv];
            o->w[a] = o->w1[iu] * o->w1v[iv];
        }

    hbref_E(o->NT, o->E);
    memcpy(o->walls_in, walls, sizeof(double) * 24);
    for (int wl = 0; wl < 4; wl++)
        for (int n = 0; n < o->NT; n++)
            wall_state_at(o, wl, 2.0 * M_PI * n / o->NT, &o->wall_ut[wl][n], &o->wall_T[wl][n]);

    size_t ncn = (size_t)o->nc * o->NT;
    size_t nel = ncn * nv;
    o->W = calloc(ncn * 4, sizeof(double));
    o->Wn = calloc(ncn * 4, sizeof(double));
    o->h = calloc(nel, sizeof(double));
    o->b = calloc(nel, sizeof(double));
    o->divH = calloc(nel, sizeof(double));
    o->divB = calloc(nel, sizeof(double));
    o->sxh = calloc(nel, sizeof(double));
    o->syh = calloc(nel, sizeof(double));
    o->sxb = calloc(nel, sizeof(double));
    o->syb = calloc(nel, sizeof(double));
    o->divF = calloc(ncn * 4, sizeof(double));
    o->q = calloc(ncn * 2, sizeof(double));
    o->dtc = calloc(o->nc, sizeof(double));
    o->Fx = calloc((size_t)(nx + 1) * ny * o->NT * 4, sizeof(double));
    o->Fy = calloc((size_t)nx * (ny + 1) * o->NT * 4, sizeof(double));

    /* uniform rest state rho = 1, U = 0, T = T0 at every level; h = H, b = B */
    double prim[4] = {1.0, 0.0, 0.0, 1.0}, q0[2] = {0.0, 0.0};
    for (int c = 0; c < o->nc; c++)
        for (int n = 0; n < o->NT; n++) {
            double *Wc = o->W + ((size_t)c * o->NT + n) * 4;
            Wc[0] = 1.0;
            Wc[1] = 0.0;
            Wc[2] = 0.0;
            Wc[3] = (2.0 + K) / 4.0;
            for (int a = 0; a < nv; a++) {
                double H, B, Hp, Bp;
                equilibrium(K, 1.0, prim, q0, o->u[a], o->v[a], &H, &B, &Hp, &Bp);
                o->h[((size_t)c * o->NT + n) * nv + a] = H;
                o->b[((size_t)c * o->NT + n) * nv + a] = B;
            }
        }
    o->step = 0;
    o->t_phys = 0.0;
    o->dt_scale = 1.0;
    memset(o->res, 0, sizeof(o->res));
    return 0;
}

/* ------------------------------------------------------------------ */
/* one pseudo step                                                      */

#define IDX(c, n) ((size_t)(c) * o->NT + (n))

/* Local pseudo step of cell c from W^k, Eqs. (31)-(32): one value per cell,
 * the largest convective spectral radius over the levels. */
static double local_dt(const hbref *o, int c)
{
    if (o->dt_mode == 1) return o->dt_fixed;
    int i = c % o->nx, j = c / o->nx;
    double nu = 0.0;
    for (int n = 0; n < o->NT; n++) {
        double p[4];
        prim_of(o->K, o->W + IDX(c, n) * 4, p);
        double cs = sqrt(o->gamma / (2.0 * p[3]));
        double ut = fmax(o->umax, fabs(p[1])) + cs;
        double vt = fmax(o->vmax, fabs(p[2])) + cs;
        double nc = (o->dy[j] * ut + o->dx[i] * vt) / (o->dx[i] * o->dy[j]);
        if (nc > nu) nu = nc;
    }
    return o->cfl / (nu + o->omega * o->NH);
}

/* One-sided or limited slope along a line of cells: values f[k], centres x[k],
 * k = 0..len-1, at position k. */
static double line_slope(const double *f, const double *x, int k, int len, long stride)
{
    if (k == 0) return (f[stride] - f[0]) / (x[1] - x[0]);
    if (k == len - 1) return (f[k * stride] - f[(k - 1) * stride]) / (x[k] - x[k - 1]);
    double sm = (f[k * stride] - f[(k - 1) * stride]) / (x[k] - x[k - 1]);
    double sp = (f[(k + 1) * stride] - f[k * stride]) / (x[k + 1] - x[k]);
    return vanleer(sm, sp);
}

static void compute_slopes(hbref *o)
{
    int nx = o->nx, ny = o->ny, NT = o->NT, nv = o->nv;
    long sx = (long)NT * nv;      /* stride between x-neighbours */
    long sy = (long)nx * NT * nv; /* stride between y-neighbours */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; c++) {
        int i = c % nx, j = c / nx;
        for (int n = 0; n < NT; n++)
            for (int a = 0; a < nv; a++) {
                size_t e = IDX(c, n) * nv + a;
                /* pointers to the start of the line through this cell */
                const double *hx = o->h + e - (long)i * sx, *bx = o->b + e - (long)i * sx;
                const double *hy = o->h + e - (long)j * sy, *by = o->b + e - (long)j * sy;
                o->sxh[e] = line_slope(hx, o->xc, i, nx, sx);
                o->sxb[e] = line_slope(bx, o->xc, i, nx, sx);
                o->syh[e] = line_slope(hy, o->yc, j, ny, sy);
                o->syb[e] = line_slope(by, o->yc, j, ny, sy);
            }
    }
}

/* Face-frame quantities of one interior face and level, built per velocity
 * from the upwind side.  un/ut are the face-normal/tangential velocity per
 * alpha; the caller provides them for its orientation. */
typedef struct {
    double *h0, *b0, *snh, *sth, *snb, *stb; /* per alpha */
} face_work;

/* Interior face flux, Eqs. (21)-(24) of Sec. 2.2.
 * Inputs per alpha: un, ut, upwind-reconstructed h0, b0 and upwind slopes.
 * WL/WR are the cells' macroscopic W^k in the face frame, dL = x_f - x_L,
 * dR = x_R - x_f.  Outputs: micro fluxes Hh, Hb per alpha (normal direction)
 * and the macro flux F in the face frame. */
static void interior_face_flux(const hbref *o, const double *un, const double *ut, const face_work *fw,
                               const double *WL, const double *WR, double dL, double dR, double dGf,
                               double *Hh, double *Hb, double *F)
{
    int nv = o->nv, K = o->K;
    const double *w = o->w;
    /* "kinetic averaging" of the reconstructed states: W0 = sum w psi h0 */
    double W0[4];
    moments_W(nv, un, ut, w, fw->h0, fw->b0, W0);
    double p0[4];
    prim_of(K, W0, p0);
    double rho0 = p0[0], Un = p0[1], Ut = p0[2], lam = p0[3];
    double tau0 = tau_of(o, rho0, lam);
    double q0[2];
    heat_flux(nv, un, ut, w, fw->h0, fw->b0, Un, Ut, q0);
    double C[5];
    hbref_ccoef(tau0, dGf, C);

    /* spatial slopes of W: normal from the cell averages to W0, tangential
     * from the upwind tangential slopes of h, b */
    double dWL[4], dWR[4], dWt[4];
    for (int k = 0; k < 4; k++) {
        dWL[k] = (W0[k] - WL[k]) / dL / rho0;
        dWR[k] = (WR[k] - W0[k]) / dR / rho0;
    }
    moments_W(nv, un, ut, w, fw->sth, fw->stb, dWt);
    for (int k = 0; k < 4; k++) dWt[k] /= rho0;
    double aL[4], aR[4], at[4], A[4];
    hbref_slope_solve(Un, Ut, lam, K, dWL, aL);
    hbref_slope_solve(Un, Ut, lam, K, dWR, aR);
    hbref_slope_solve(Un, Ut, lam, K, dWt, at);
    /* time slope from the compatibility condition */
    double m1[4], m2[4], m3[4], rhs[4];
    moment_vec(aL, 1, 0, Un, Ut, lam, K, 1, m1);
    moment_vec(aR, 1, 0, Un, Ut, lam, K, 2, m2);
    moment_vec(at, 0, 1, Un, Ut, lam, K, 0, m3);
    for (int k = 0; k < 4; k++) rhs[k] = -(m1[k] + m2[k] + m3[k]);
    hbref_slope_solve(Un, Ut, lam, K, rhs, A);

    /* micro flux, Eq. (23), for h and b */
    double xh = K / (2.0 * lam), xb = (K + 2.0) / (2.0 * lam);
    double s1[4] = {0, 0, 0, 0}, s4[4] = {0, 0, 0, 0}, s5[4] = {0, 0, 0, 0};
    for (int a = 0; a < nv; a++) {
        double H, B, Hp, Bp;
        equilibrium(K, o->Pr, p0, q0, un[a], ut[a], &H, &B, &Hp, &Bp);
        const double *an = (un[a] > 0.0) ? aL : aR;
        double r2 = un[a] * un[a] + ut[a] * ut[a];
        double Pn_h = an[0] + an[1] * un[a] + an[2] * ut[a] + 0.5 * an[3] * (r2 + xh);
        double Pt_h = at[0] + at[1] * un[a] + at[2] * ut[a] + 0.5 * at[3] * (r2 + xh);
        double PA_h = A[0] + A[1] * un[a] + A[2] * ut[a] + 0.5 * A[3] * (r2 + xh);
        double Pn_b = an[0] + an[1] * un[a] + an[2] * ut[a] + 0.5 * an[3] * (r2 + xb);
        double Pt_b = at[0] + at[1] * un[a] + at[2] * ut[a] + 0.5 * at[3] * (r2 + xb);
        double PA_b = A[0] + A[1] * un[a] + A[2] * ut[a] + 0.5 * A[3] * (r2 + xb);
        double gh = C[0] * (H + Hp) + C[1] * (un[a] * Pn_h + ut[a] * Pt_h) * H + C[2] * PA_h * H +
                    C[3] * fw->h0[a] + C[4] * (un[a] * fw->snh[a] + ut[a] * fw->sth[a]);
        double gb = C[0] * (B + Bp) + C[1] * (un[a] * Pn_b + ut[a] * Pt_b) * B + C[2] * PA_b * B +
                    C[3] * fw->b0[a] + C[4] * (un[a] * fw->snb[a] + ut[a] * fw->stb[a]);
        Hh[a] = un[a] / dGf * gh;
        Hb[a] = un[a] / dGf * gb;
        /* discrete sums for the C1, C4, C5 parts of the macro flux */
        double wu = w[a] * un[a];
        double eh = H + Hp, eb = B + Bp;
        s1[0] += wu * eh;
        s1[1] += wu * un[a] * eh;
        s1[2] += wu * ut[a] * eh;
        s1[3] += wu * 0.5 * (r2 * eh + eb);
        s4[0] += wu * fw->h0[a];
        s4[1] += wu * un[a] * fw->h0[a];
        s4[2] += wu * ut[a] * fw->h0[a];
        s4[3] += wu * 0.5 * (r2 * fw->h0[a] + fw->b0[a]);
        double sh = un[a] * fw->snh[a] + ut[a] * fw->sth[a];
        double sb = un[a] * fw->snb[a] + ut[a] * fw->stb[a];
        s5[0] += wu * sh;
        s5[1] += wu * un[a] * sh;
        s5[2] += wu * ut[a] * sh;
        s5[3] += wu * 0.5 * (r2 * sh + sb);
    }
    if (o->macro_mode == 1) {
        /* all-discrete variant: F = sum w psi (Hh, Hb) */
        double f[4] = {0, 0, 0, 0};
        for (int a = 0; a < nv; a++) {
            f[0] += w[a] * Hh[a];
            f[1] += w[a] * un[a] * Hh[a];
            f[2] += w[a] * ut[a] * Hh[a];
            f[3] += w[a] * 0.5 * ((un[a] * un[a] + ut[a] * ut[a]) * Hh[a] + Hb[a]);
        }
        for (int k = 0; k < 4; k++) F[k] = f[k];
        return;
    }
    /* macro flux, Eq. (24): C2 and C3 parts as Maxwellian moments, the
     * normal slope taken from a^L over u_n > 0 and a^R over u_n < 0 */
    double c2a[4], c2b[4], c2c[4], c3[4];
    moment_vec(aL, 2, 0, Un, Ut, lam, K, 1, c2a);
    moment_vec(aR, 2, 0, Un, Ut, lam, K, 2, c2b);
    moment_vec(at, 1, 1, Un, Ut, lam, K, 0, c2c);
    moment_vec(A, 1, 0, Un, Ut, lam, K, 0, c3);
    for (int k = 0; k < 4; k++)
        F[k] = (C[0] * s1[k] + C[1] * rho0 * (c2a[k] + c2b[k] + c2c[k]) + C[2] * rho0 * c3[k] +
                C[3] * s4[k] + C[4] * s5[k]) /
               dGf;
}

/* Diffuse isothermal wall, Sec. 2.3, Eqs. (27)-(28).
 * Face frame: normal along +x (vertical walls) or +y (horizontal walls);
 * sin = +1 if the inward normal points along +normal (wall at the low end),
 * -1 otherwise.  hI, bI: interior reconstruction at the wall (per alpha);
 * snh.. : slopes of the adjacent cell in the face frame.
 * Wall state: tangential velocity Uw_t (face frame), temperature Tw.
 * Reading taken for the incident state (the paper refers to the integral
 * solution without printing it): an auxiliary wall state W0 is formed from the
 * incident hI and the reflected rho_w0 H_w, and the incident time average is
 * (C1 h0+ + C4 hI + C5 u.sigma)/dG; rho_w then follows from Eq. (28). */
static void wall_face_flux(const hbref *o, const double *un, const double *ut, const face_work *fw,
                           double sin_, double Uw_t, double Tw, double dGf, double *Hh, double *Hb,
                           double *F)
{
    int nv = o->nv, K = o->K;
    const double *w = o->w;
    double lw = 1.0 / Tw;
    double pw[4] = {1.0, 0.0, Uw_t, lw}, qz[2] = {0.0, 0.0};
    double *Hw = malloc(sizeof(double) * nv), *Bw = malloc(sizeof(double) * nv);
    double *h0 = malloc(sizeof(double) * nv), *b0 = malloc(sizeof(double) * nv);
    for (int a = 0; a < nv; a++) {
        double Hp, Bp;
        equilibrium(K, 1.0, pw, qz, un[a], ut[a], &Hw[a], &Bw[a], &Hp, &Bp);
    }
    /* rho_w0 from the reconstructed incident distribution */
    double num = 0.0, den = 0.0;
    for (int a = 0; a < nv; a++) {
        double cn = sin_ * un[a]; /* u . n_in */
        if (cn < 0.0) num += w[a] * cn * fw->h0[a];
        if (cn > 0.0) den += w[a] * cn * Hw[a];
    }
    double rw0 = -num / den;
    for (int a = 0; a < nv; a++) {
        double cn = sin_ * un[a];
        if (cn > 0.0) {
            h0[a] = rw0 * Hw[a];
            b0[a] = rw0 * Bw[a];
        } else {
            h0[a] = fw->h0[a];
            b0[a] = fw->b0[a];
        }
    }
    double W0[4], p0[4], q0[2], C[5];
    moments_W(nv, un, ut, w, h0, b0, W0);
    prim_of(K, W0, p0);
    double tau0 = tau_of(o, p0[0], p0[3]);
    heat_flux(nv, un, ut, w, h0, b0, p0[1], p0[2], q0);
    hbref_ccoef(tau0, dGf, C);
    /* incident time-averaged distribution and rho_w, Eq. (28) */
    double num2 = 0.0;
    for (int a = 0; a < nv; a++) {
        double cn = sin_ * un[a];
        if (cn < 0.0) {
            double H, B, Hp, Bp;
            equilibrium(K, o->Pr, p0, q0, un[a], ut[a], &H, &B, &Hp, &Bp);
            double hin = (C[0] * (H + Hp) + C[3] * fw->h0[a] + C[4] * (un[a] * fw->snh[a] + ut[a] * fw->sth[a])) / dGf;
            double bin = (C[0] * (B + Bp) + C[3] * fw->b0[a] + C[4] * (un[a] * fw->snb[a] + ut[a] * fw->stb[a])) / dGf;
            h0[a] = hin;
            b0[a] = bin;
            num2 += w[a] * cn * hin;
        }
    }
    double rw = -num2 / den;
    double f[4] = {0, 0, 0, 0};
    for (int a = 0; a < nv; a++) {
        double cn = sin_ * un[a];
        double hh, bb;
        if (cn > 0.0) {
            hh = rw * Hw[a];
            bb = rw * Bw[a];
        } else if (cn < 0.0) {
            hh = h0[a];
            bb = b0[a];
        } else {
            hh = 0.0;
            bb = 0.0;
        }
        Hh[a] = un[a] * hh;
        Hb[a] = un[a] * bb;
        double wu = w[a] * un[a];
        f[0] += wu * hh;
        f[1] += wu * un[a] * hh;
        f[2] += wu * ut[a] * hh;
        f[3] += wu * 0.5 * ((un[a] * un[a] + ut[a] * ut[a]) * hh + bb);
    }
    for (int k = 0; k < 4; k++) F[k] = f[k];
    free(Hw);
    free(Bw);
    free(h0);
    free(b0);
}

/* All face fluxes of one level-set; accumulates divH, divB, divF. */
static void all_fluxes(hbref *o)
{
    int nx = o->nx, ny = o->ny, NT = o->NT, nv = o->nv;
    size_t nel = (size_t)o->nc * NT * nv;
    memset(o->divH, 0, nel * sizeof(double));
    memset(o->divB, 0, nel * sizeof(double));
    memset(o->divF, 0, (size_t)o->nc * NT * 4 * sizeof(double));

    /* x-faces (normal +x, tangential +y); rows are independent */
#pragma omp parallel
    {
        face_work fw;
        double *buf = malloc(sizeof(double) * nv * 8);
        fw.h0 = buf;
        fw.b0 = buf + nv;
        fw.snh = buf + 2 * nv;
        fw.sth = buf + 3 * nv;
        fw.snb = buf + 4 * nv;
        fw.stb = buf + 5 * nv;
        double *Hh = buf + 6 * nv, *Hb = buf + 7 * nv;
#pragma omp for schedule(static)
        for (int j = 0; j < ny; j++) {
            for (int fi = 0; fi <= nx; fi++) {
                int cL = j * nx + fi - 1, cR = j * nx + fi;
                for (int n = 0; n < NT; n++) {
                    double F[4];
                    if (fi == 0 || fi == nx) {
                        int c = (fi == 0) ? cR : cL;
                        int wl = (fi == 0) ? 3 : 1;
                        double sgn = (fi == 0) ? 1.0 : -1.0;
                        double xw = o->xf[fi], xcc = o->xc[c % nx];
                        for (int a = 0; a < nv; a++) {
                            size_t e = IDX(c, n) * nv + a;
                            fw.h0[a] = o->h[e] + o->sxh[e] * (xw - xcc);
                            fw.b0[a] = o->b[e] + o->sxb[e] * (xw - xcc);
                            fw.snh[a] = o->sxh[e];
                            fw.sth[a] = o->syh[e];
                            fw.snb[a] = o->sxb[e];
                            fw.stb[a] = o->syb[e];
                        }
                        wall_face_flux(o, o->u, o->v, &fw, sgn, o->wall_ut[wl][n], o->wall_T[wl][n], o->dtc[c], Hh,
                                       Hb, F);
                    } else {
                        double xf = o->xf[fi];
                        double xL = o->xc[fi - 1], xR = o->xc[fi];
                        for (int a = 0; a < nv; a++) {
                            int up = (o->u[a] > 0.0) ? cL : cR;
                            double xu = (o->u[a] > 0.0) ? xL : xR;
                            size_t e = IDX(up, n) * nv + a;
                            fw.h0[a] = o->h[e] + o->sxh[e] * (xf - xu);
                            fw.b0[a] = o->b[e] + o->sxb[e] * (xf - xu);
                            fw.snh[a] = o->sxh[e];
                            fw.sth[a] = o->syh[e];
                            fw.snb[a] = o->sxb[e];
                            fw.stb[a] = o->syb[e];
                        }
                        double dGL = o->dtc[cL], dGR = o->dtc[cR];
                        double dGf = (o->face_dt == 1) ? 2.0 * dGL * dGR / (dGL + dGR) : fmin(dGL, dGR);
                        interior_face_flux(o, o->u, o->v, &fw, o->W + IDX(cL, n) * 4, o->W + IDX(cR, n) * 4,
                                           xf - xL, xR - xf, dGf, Hh, Hb, F);
                    }
                    double *Fs = o->Fx + (((size_t)j * (nx + 1) + fi) * NT + n) * 4;
                    for (int k = 0; k < 4; k++) Fs[k] = F[k];
                    if (fi > 0) {
                        double r = 1.0 / o->dx[fi - 1];
                        for (int a = 0; a < nv; a++) {
                            o->divH[IDX(cL, n) * nv + a] += Hh[a] * r;
                            o->divB[IDX(cL, n) * nv + a] += Hb[a] * r;
                        }
                        for (int k = 0; k < 4; k++) o->divF[IDX(cL, n) * 4 + k] += F[k] * r;
                    }
                    if (fi < nx) {
                        double r = 1.0 / o->dx[fi];
                        for (int a = 0; a < nv; a++) {
                            o->divH[IDX(cR, n) * nv + a] -= Hh[a] * r;
                            o->divB[IDX(cR, n) * nv + a] -= Hb[a] * r;
                        }
                        for (int k = 0; k < 4; k++) o->divF[IDX(cR, n) * 4 + k] -= F[k] * r;
                    }
                }
            }
        }
        free(buf);
    }

    /* y-faces (normal +y, tangential +x); columns are independent.  Face-frame
     * momentum components (n, t) = (V, U) are rotated back to (U, V). */
#pragma omp parallel
    {
        face_work fw;
        double *buf = malloc(sizeof(double) * nv * 8);
        fw.h0 = buf;
        fw.b0 = buf + nv;
        fw.snh = buf + 2 * nv;
        fw.sth = buf + 3 * nv;
        fw.snb = buf + 4 * nv;
        fw.stb = buf + 5 * nv;
        double *Hh = buf + 6 * nv, *Hb = buf + 7 * nv;
#pragma omp for schedule(static)
        for (int i = 0; i < nx; i++) {
            for (int fj = 0; fj <= ny; fj++) {
                int cL = (fj - 1) * nx + i, cR = fj * nx + i;
                for (int n = 0; n < NT; n++) {
                    double Fl[4];
                    if (fj == 0 || fj == ny) {
                        int c = (fj == 0) ? cR : cL;
                        int wl = (fj == 0) ? 0 : 2;
                        double sgn = (fj == 0) ? 1.0 : -1.0;
                        double yw = o->yf[fj], ycc = o->yc[c / nx];
                        for (int a = 0; a < nv; a++) {
                            size_t e = IDX(c, n) * nv + a;
                            fw.h0[a] = o->h[e] + o->syh[e] * (yw - ycc);
                            fw.b0[a] = o->b[e] + o->syb[e] * (yw - ycc);
                            fw.snh[a] = o->syh[e];
                            fw.sth[a] = o->sxh[e];
                            fw.snb[a] = o->syb[e];
                            fw.stb[a] = o->sxb[e];
                        }
                        wall_face_flux(o, o->v, o->u, &fw, sgn, o->wall_ut[wl][n], o->wall_T[wl][n], o->dtc[c], Hh,
                                       Hb, Fl);
                    } else {
                        double yf = o->yf[fj];
                        double yL = o->yc[fj - 1], yR = o->yc[fj];
                        for (int a = 0; a < nv; a++) {
                            int up = (o->v[a] > 0.0) ? cL : cR;
                            double yu = (o->v[a] > 0.0) ? yL : yR;
                            size_t e = IDX(up, n) * nv + a;
                            fw.h0[a] = o->h[e] + o->syh[e] * (yf - yu);
                            fw.b0[a] = o->b[e] + o->syb[e] * (yf - yu);
                            fw.snh[a] = o->syh[e];
                            fw.sth[a] = o->sxh[e];
                            fw.snb[a] = o->syb[e];
                            fw.stb[a] = o->sxb[e];
                        }
                        double WL[4], WR[4];
                        const double *wl_ = o->W + IDX(cL, n) * 4, *wr_ = o->W + IDX(cR, n) * 4;
                        WL[0] = wl_[0];
                        WL[1] = wl_[2];
                        WL[2] = wl_[1];
                        WL[3] = wl_[3];
                        WR[0] = wr_[0];
                        WR[1] = wr_[2];
                        WR[2] = wr_[1];
                        WR[3] = wr_[3];
                        double dGL = o->dtc[cL], dGR = o->dtc[cR];
                        double dGf = (o->face_dt == 1) ? 2.0 * dGL * dGR / (dGL + dGR) : fmin(dGL, dGR);
                        interior_face_flux(o, o->v, o->u, &fw, WL, WR, yf - yL, yR - yf, dGf, Hh, Hb, Fl);
                    }
                    double F[4] = {Fl[0], Fl[2], Fl[1], Fl[3]};
                    double *Fs = o->Fy + (((size_t)fj * nx + i) * NT + n) * 4;
                    for (int k = 0; k < 4; k++) Fs[k] = F[k];
                    if (fj > 0) {
                        double r = 1.0 / o->dy[fj - 1];
                        for (int a = 0; a < nv; a++) {
                            o->divH[IDX(cL, n) * nv + a] += Hh[a] * r;
                            o->divB[IDX(cL, n) * nv + a] += Hb[a] * r;
                        }
                        for (int k = 0; k < 4; k++) o->divF[IDX(cL, n) * 4 + k] += F[k] * r;
                    }
                    if (fj < ny) {
                        double r = 1.0 / o->dy[fj];
                        for (int a = 0; a < nv; a++) {
                            o->divH[IDX(cR, n) * nv + a] -= Hh[a] * r;
                            o->divB[IDX(cR, n) * nv + a] -= Hb[a] * r;
                        }
                        for (int k = 0; k < 4; k++) o->divF[IDX(cR, n) * 4 + k] -= F[k] * r;
                    }
                }
            }
        }
        free(buf);
    }
}

/* One pseudo step k -> k+1 (Sec. 2.4).  In time-domain mode (NT = 1, no E
 * term) the same step is one explicit physical step of size dt_fixed. */
/* Level-mass projection (a convergence aid; not in the paper).  The spectral
 * source of Eq. (29) only moves mass between the sub-time levels, and with
 * local pseudo steps (Eq. 31) the flux terms of the cells no longer cancel in
 * the sum over the cavity, so each level's total mass M_n drifts during the
 * transient.  The part of (M_n) that is not level-independent then rotates
 * under the explicit source term without decaying: the density residual
 * stalls.  Every fixed point of the step has M_n equal at all levels (sum
 * Eq. (29) over the cells: the fluxes cancel at impermeable walls and
 * omega E M = 0 leaves only constants), so the step is followed by a scaling
 * of W, h and b at each level n by s_n = 1 + (Mbar - M_n) / M_n, Mbar the mean
 * level mass: s_n = 1 exactly when the masses agree, and the fixed points of
 * the projected step are those of the step itself.  M_n = sum_i |Omega_i|
 * rho_{i,n}; the residual of Eq. (43) is the step's increment before the
 * scaling. */
static void level_mass_projection(hbref *o)
{
    int nc = o->nc, NT = o->NT, nv = o->nv;
    double M[NTMAX];
    for (int n = 0; n < NT; n++) {
        M[n] = 0.0;
        for (int c = 0; c < nc; c++) M[n] += o->dx[c % o->nx] * o->dy[c / o->nx] * o->W[IDX(c, n) * 4];
    }
    double d = 0.0;
    for (int n = 0; n < NT; n++) d += M[n] - M[0];
    double mean = M[0] + d / NT;
    for (int n = 0; n < NT; n++) {
        double s_n = 1.0 + (mean - M[n]) / M[n];
        for (int c = 0; c < nc; c++) {
            for (int k = 0; k < 4; k++) o->W[IDX(c, n) * 4 + k] *= s_n;
            for (int a = 0; a < nv; a++) {
                o->h[IDX(c, n) * nv + a] *= s_n;
                o->b[IDX(c, n) * nv + a] *= s_n;
            }
        }
    }
}

static void one_step(hbref *o, int with_E)
{
    int nc = o->nc, NT = o->NT, nv = o->nv, K = o->K;
    double om = with_E ? o->omega : 0.0;

    /* local pseudo steps from W^k, Eqs. (31)-(32) */
    for (int c = 0; c < nc; c++) o->dtc[c] = local_dt(o, c) * o->dt_scale;
    /* heat flux q^k of h^k, b^k about U^k (Shakhov term of h+^k) */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; c++)
        for (int n = 0; n < NT; n++) {
            double p[4];
            prim_of(K, o->W + IDX(c, n) * 4, p);
            heat_flux(nv, o->u, o->v, o->w, o->h + IDX(c, n) * nv, o->b + IDX(c, n) * nv, p[1], p[2],
                      o->q + IDX(c, n) * 2);
        }
    compute_slopes(o);
    all_fluxes(o);

    /* macroscopic update, Eq. (29) */
    for (int c = 0; c < nc; c++)
        for (int n = 0; n < NT; n++)
            for (int k = 0; k < 4; k++) {
                double src = 0.0;
                for (int m = 0; m < NT; m++) src += o->E[n * NT + m] * o->W[IDX(c, m) * 4 + k];
                o->Wn[IDX(c, n) * 4 + k] =
                    o->W[IDX(c, n) * 4 + k] - o->dtc[c] * (o->divF[IDX(c, n) * 4 + k] + om * src);
            }

    /* microscopic update, Eq. (30): explicit flux and spectral source,
     * trapezoidal collision with h+^{k+1} from W^{k+1}.  The heat flux in
     * h+^{k+1} is the moment of h^k, b^k about U^{k+1} (the paper says only
     * that h+^{k+1} follows from W^{k+1}; q is not part of W). */
#pragma omp parallel
    {
        double *hn = malloc(sizeof(double) * NT * nv), *bn = malloc(sizeof(double) * NT * nv);
#pragma omp for schedule(static)
        for (int c = 0; c < nc; c++) {
            double dG = o->dtc[c];
            for (int n = 0; n < NT; n++) {
                double pk[4], pk1[4], qk1[2];
                prim_of(K, o->W + IDX(c, n) * 4, pk);
                prim_of(K, o->Wn + IDX(c, n) * 4, pk1);
                double tk = tau_of(o, pk[0], pk[3]), tk1 = tau_of(o, pk1[0], pk1[3]);
                const double *hc = o->h + IDX(c, n) * nv, *bc = o->b + IDX(c, n) * nv;
                heat_flux(nv, o->u, o->v, o->w, hc, bc, pk1[1], pk1[2], qk1);
                const double *qk = o->q + IDX(c, n) * 2;
                for (int a = 0; a < nv; a++) {
                    double Hk, Bk, Hpk, Bpk, Hk1, Bk1, Hpk1, Bpk1;
                    equilibrium(K, o->Pr, pk, qk, o->u[a], o->v[a], &Hk, &Bk, &Hpk, &Bpk);
                    equilibrium(K, o->Pr, pk1, qk1, o->u[a], o->v[a], &Hk1, &Bk1, &Hpk1, &Bpk1);
                    double Eh = 0.0, Eb = 0.0;
                    for (int m = 0; m < NT; m++) {
                        Eh += o->E[n * NT + m] * o->h[IDX(c, m) * nv + a];
                        Eb += o->E[n * NT + m] * o->b[IDX(c, m) * nv + a];
                    }
                    size_t e = IDX(c, n) * nv + a;
                    double hk = o->h[e], bk = o->b[e];
                    double numh = hk - dG * o->divH[e] - dG * om * Eh +
                                  0.5 * dG * ((Hk1 + Hpk1) / tk1 + ((Hk + Hpk) - hk) / tk);
                    double numb = bk - dG * o->divB[e] - dG * om * Eb +
                                  0.5 * dG * ((Bk1 + Bpk1) / tk1 + ((Bk + Bpk) - bk) / tk);
                    double den = 1.0 + 0.5 * dG / tk1;
                    hn[n * nv + a] = numh / den;
                    bn[n * nv + a] = numb / den;
                }
            }
            for (int n = 0; n < NT; n++)
                for (int a = 0; a < nv; a++) {
                    o->h[IDX(c, n) * nv + a] = hn[n * nv + a];
                    o->b[IDX(c, n) * nv + a] = bn[n * nv + a];
                }
        }
        free(hn);
        free(bn);
    }

    /* residual, Eq. (43): RMS over cells of the level-0 increment */
    double r[4] = {0, 0, 0, 0};
    for (int c = 0; c < nc; c++)
        for (int k = 0; k < 4; k++) r[k] += sq(o->Wn[IDX(c, 0) * 4 + k] - o->W[IDX(c, 0) * 4 + k]);
    for (int k = 0; k < 4; k++) o->res[k] = sqrt(r[k] / nc);
    double *t = o->W;
    o->W = o->Wn;
    o->Wn = t;
    o->step++;
    if (o->level_mass) level_mass_projection(o);
}

void hbref_step(void *p, int nsteps)
{
    hbref *o = (hbref *)p;
    for (int s = 0; s < nsteps; s++) one_step(o, 1);
}

void hbref_residual(void *p, double *out)
{
    hbref *o = (hbref *)p;
    for (int k = 0; k < 4; k++) out[k] = o->res[k];
}

long hbref_step_index(void *p) { return ((hbref *)p)->step; }

void hbref_get_state(void *p, double *W, double *h, double *b)
{
    hbref *o = (hbref *)p;
    size_t ncn = (size_t)o->nc * o->NT;
    if (W) memcpy(W, o->W, ncn * 4 * sizeof(double));
    if (h) memcpy(h, o->h, ncn * o->nv * sizeof(double));
    if (b) memcpy(b, o->b, ncn * o->nv * sizeof(double));
}

void hbref_set_state(void *p, const double *W, const double *h, const double *b)
{
    hbref *o = (hbref *)p;
    size_t ncn = (size_t)o->nc * o->NT;
    if (W) memcpy(o->W, W, ncn * 4 * sizeof(double));
    if (h) memcpy(o->h, h, ncn * o->nv * sizeof(double));
    if (b) memcpy(o->b, b, ncn * o->nv * sizeof(double));
}

/* Last step's local steps and macro face fluxes (for sub-step checks). */
void hbref_get_debug(void *p, double *dtc, double *Fx, double *Fy)
{
    hbref *o = (hbref *)p;
    if (dtc) memcpy(dtc, o->dtc, sizeof(double) * o->nc);
    if (Fx) memcpy(Fx, o->Fx, sizeof(double) * (o->nx + 1) * o->ny * o->NT * 4);
    if (Fy) memcpy(Fy, o->Fy, sizeof(double) * o->nx * (o->ny + 1) * o->NT * 4);
}

/* Test hook: scale every local pseudo step by s (e.g. 1 + 2^-52 to measure
 * how strongly the converged state reacts to one ulp of perturbation). */
void hbref_set_dt_scale(void *p, double s) { ((hbref *)p)->dt_scale = s; }

/* ------------------------------------------------------------------ */
/* Harmonics, Eq. (40): qhat_k = (1/NT) sum_n q_n exp(-i k omega t_n), for
 * k = 0..NH and the variables
 *   0 rho, 1 U, 2 V, 3 T/T0 (from W), 4 P_xy (Eq. 39, from h about U_n, V_n),
 *   5 q_x, 6 q_y (Eq. 6, from h and b about U_n, V_n).
 * Layout re/im [var][k][cell]. */
void hbref_harmonics(void *p, double *re, double *im)
{
    hbref *o = (hbref *)p;
    int nc = o->nc, NT = o->NT, NH = o->NH, nv = o->nv;
    double *val = malloc(sizeof(double) * 7 * NT);
    for (int c = 0; c < nc; c++) {
        for (int n = 0; n < NT; n++) {
            double pr[4], qq[2];
            prim_of(o->K, o->W + IDX(c, n) * 4, pr);
            const double *hc = o->h + IDX(c, n) * nv, *bc = o->b + IDX(c, n) * nv;
            double pxy = 0.0;
            for (int a = 0; a < nv; a++) pxy += o->w[a] * (o->u[a] - pr[1]) * (o->v[a] - pr[2]) * hc[a];
            heat_flux(nv, o->u, o->v, o->w, hc, bc, pr[1], pr[2], qq);
            val[0 * NT + n] = pr[0];
            val[1 * NT + n] = pr[1];
            val[2 * NT + n] = pr[2];
            val[3 * NT + n] = 1.0 / pr[3];
            val[4 * NT + n] = pxy;
            val[5 * NT + n] = qq[0];
            val[6 * NT + n] = qq[1];
        }
        for (int var = 0; var < 7; var++)
            for (int k = 0; k <= NH; k++) {
                double sr = 0.0, si = 0.0;
                for (int n = 0; n < NT; n++) {
                    double th = 2.0 * M_PI * k * n / NT;
                    sr += val[var * NT + n] * cos(th);
                    si -= val[var * NT + n] * sin(th);
                }
                re[((size_t)var * (NH + 1) + k) * nc + c] = sr / NT;
                im[((size_t)var * (NH + 1) + k) * nc + c] = si / NT;
            }
    }
    free(val);
}

/* ------------------------------------------------------------------ */
/* Explicit time-domain UGKS (the paper's comparison solver, Sec. 3.1.4):
 * the same flux with the physical step dt for every face, no spectral
 * source, one time level, walls evaluated at mid-step.  The handle must have
 * been set up with NH = 0, dt_mode = 1 and dt_fixed = dt.  Advances nsteps
 * steps from the handle's physical time. */
void hbref_td_step(void *p, int nsteps, double omega_forcing)
{
    hbref *o = (hbref *)p;
    for (int s = 0; s < nsteps; s++) {
        double th = omega_forcing * (o->t_phys + 0.5 * o->dt_fixed);
        for (int wl = 0; wl < 4; wl++) wall_state_at(o, wl, th, &o->wall_ut[wl][0], &o->wall_T[wl][0]);
        one_step(o, 0);
        o->t_phys += o->dt_fixed;
    }
}

double hbref_time(void *p) { return ((hbref *)p)->t_phys; }

/* Largest convective spectral radius of Eq. (32) over cells, without the
 * spectral term (used to size the physical step of the time-domain solver). */
double hbref_max_nu(void *p)
{
    hbref *o = (hbref *)p;
    double m = 0.0;
    double save = o->omega;
    int mode = o->dt_mode;
    o->dt_mode = 0;
    o->omega = 0.0;
    for (int c = 0; c < o->nc; c++) {
        double d = local_dt(o, c);
        double nu = o->cfl / d;
        if (nu > m) m = nu;
    }
    o->omega = save;
    o->dt_mode = mode;
    return m;
}

/* OpenMP threads the oracle's parallel loops use. */
int hbref_threads(void) { return omp_get_max_threads(); }

/* Integer sizes of the handle: nx, ny, nc, M, nv, NT. */
void hbref_sizes(void *p, int *out)
{
    hbref *o = (hbref *)p;
    out[0] = o->nx;
    out[1] = o->ny;
    out[2] = o->nc;
    out[3] = o->M;
    out[4] = o->nv;
    out[5] = o->NT;
}

/* Derived constants: mu_ref, omega, gamma. */
void hbref_constants(void *p, double *out)
{
    hbref *o = (hbref *)p;
    out[0] = o->mu_ref;
    out[1] = o->omega;
    out[2] = o->gamma;
}
