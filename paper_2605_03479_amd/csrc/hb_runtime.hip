// Host runtime and C ABI of the HB-UGKS pseudo-step library (see hb_ugks.h).
//
// The handle owns the device state of one case: geometry and velocity
// tables, the double-buffered (h, b), W and local steps, the per-step
// moment/face/cell records and a residual ring buffer.  A pseudo step is
// five kernel launches on the handle's stream (moments, faces, cells,
// residual, update) followed by a buffer swap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "hb_handle.h"

// One mixed-form state (h and b of every cell and level) above this size is
// not kept by the 256 MB last-level cache between the update and the next
// moments pass (which also holds the state being read), so the update streams
// its stores past the caches (Params::stream_out).  Measured: streaming slows
// a 101 MB state's step by 4 % and speeds a 168 MB one's by 2 %.
#define HB_STREAM_OUT_BYTES (128.0 * 1024 * 1024)

namespace {
const char *KNAMES[HB_NKERN] = {"moments", "faces", "cells", "dt_resid", "update_int", "update_bnd"};
}

static void free_case(hb_ugks *H)
{
    for (auto &b : H->bufs) {
        if (H->pool) H->pool->release(b.p);
        else (void)hipFree(b.p);
    }
    H->bufs.clear();
    H->bytes = 0;
    H->has_case = false;
}

static int dalloc(hb_ugks *H, void **p, size_t nbytes)
{
    if (H->count_only) {
        *p = nullptr;
        H->bytes += HbPool::round(nbytes);
        return HB_OK;
    }
    if (H->budget && H->bytes + nbytes > H->budget) return HB_ENOMEM;
    if (H->pool) {
        *p = H->pool->take(nbytes);
        if (!*p) return HB_ENOMEM;
    } else if (hipMalloc(p, nbytes) != hipSuccess) {
        (void)hipGetLastError();
        return HB_ENOMEM;
    }
    H->bufs.push_back({*p, nbytes});
    H->bytes += nbytes;
    return HB_OK;
}

// Orthonormal Hermite functions psi_k(x) = H_k(x) exp(-x^2/2) / sqrt(2^k k! sqrt(pi)),
// k = n-1 and n, by their three-term recurrence (values stay O(1) for any x).
static void hermite_fn(int n, double x, double &pm1, double &pn)
{
    double a = 0.0, b = std::pow(M_PI, -0.25) * std::exp(-0.5 * x * x);  // psi_{-1}, psi_0
    for (int k = 0; k < n; k++) {
        const double c = std::sqrt(2.0 / (k + 1)) * x * b - std::sqrt((double)k / (k + 1)) * a;
        a = b;
        b = c;
    }
    pm1 = a;
    pn = b;
}

// 1-D velocity rule of Sec. 3.1.1.  Trapezoid: m equally spaced nodes on
// [-umax, umax], closed composite trapezoid weights.  Gauss-Hermite: the m
// roots x_k of H_m (the Maxwellian at rest in these units is exp(-u^2)/pi, the
// weight the rule is exact for) with the weight folded back in,
// w_k = 1 / (m psi_{m-1}(x_k)^2) = (Gauss weight) * exp(x_k^2), so that
// sum_k w_k f(u_k) approximates the plain integral of f.  Positive roots are
// bracketed by a scan finer than a tenth of the smallest root spacing
// (about pi / sqrt(2 m)), then bisected to the last bit.
static int velocity_rule(int m, double umax, int rule, double *u, double *w)
{
    if (m < 4 || m > 128 || (m & 1)) return HB_EINVAL;
    if (rule == HB_RULE_TRAPEZOID) {
        if (!(umax > 0.0)) return HB_EINVAL;
        const double du = 2.0 * umax / (m - 1);
        for (int k = 0; k < m; k++) {
            u[k] = -umax + k * du;
            w[k] = (k == 0 || k == m - 1) ? 0.5 * du : du;
        }
        return HB_OK;
    }
    if (rule != HB_RULE_GAUSS_HERMITE) return HB_EINVAL;
    const int half = m / 2;
    const double xend = std::sqrt(2.0 * m + 1.0) + 1.0, step = 0.1 * M_PI / std::sqrt(2.0 * m + 1.0);
    int found = 0;
    double pm1, p0, x0 = 0.0;
    hermite_fn(m, x0, pm1, p0);
    while (x0 < xend && found < half) {
        double x1 = std::min(x0 + step, xend), p1;
        hermite_fn(m, x1, pm1, p1);
        if ((p0 < 0.0) != (p1 < 0.0)) {
            double lo = x0, hi = x1, plo = p0;
            for (int it = 0; it < 200 && hi - lo > 0.0; it++) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double q, pmid;
                hermite_fn(m, mid, q, pmid);
                if ((pmid < 0.0) == (plo < 0.0)) {
                    lo = mid;
                    plo = pmid;
                } else {
                    hi = mid;
                }
            }
            const double r = 0.5 * (lo + hi);
            double q, pr;
            hermite_fn(m, r, q, pr);
            u[half + found] = r;
            w[half + found] = 1.0 / (m * q * q);
            found++;
        }
        x0 = x1;
        p0 = p1;
    }
    if (found != half) return HB_EINVAL;
    for (int k = 0; k < half; k++) {
        u[half - 1 - k] = -u[half + k];
        w[half - 1 - k] = w[half + k];
    }
    return HB_OK;
}

// the update kernels are compiled for each admissible number of levels
template <int NT, typename TS, bool SO>
static int set_update_lds_so(size_t bytes)
{
    if (hipFuncSetAttribute((const void *)hb::k_update_int<NT, TS, SO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes) != hipSuccess ||
        hipFuncSetAttribute((const void *)hb::k_update_bnd<NT, TS, SO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes) != hipSuccess)
        return HB_EDEVICE;
    return HB_OK;
}
// the mixed form has a cached and a streaming-store instance of each update
template <int NT, typename TS>
static int set_update_lds_t(size_t bytes)
{
    if (bytes <= 64 * 1024) return HB_OK;
    const int rc = set_update_lds_so<NT, TS, false>(bytes);
    if constexpr (sizeof(TS) == 4) {
        if (rc == HB_OK) return set_update_lds_so<NT, TS, true>(bytes);
    }
    return rc;
}

template <typename TS>
static int update_lds_attr_t(int NT, size_t bytes)
{
    switch (NT) {
    case 1: return set_update_lds_t<1, TS>(bytes);
    case 3: return set_update_lds_t<3, TS>(bytes);
    case 5: return set_update_lds_t<5, TS>(bytes);
    case 7: return set_update_lds_t<7, TS>(bytes);
    case 9: return set_update_lds_t<9, TS>(bytes);
    default: return set_update_lds_t<11, TS>(bytes);
    }
}

static int update_lds_attr(int precision, int NT, size_t bytes)
{
    return precision == HB_MIXED ? update_lds_attr_t<float>(NT, bytes) : update_lds_attr_t<double>(NT, bytes);
}

template <int NT, typename TS, bool SO>
static void launch_update_so(hb_ugks *H, const hb::Params &P, int c, int x, hipEvent_t mid)
{
    const TS *h = (const TS *)H->h[c], *b = (const TS *)H->b[c];
    TS *hn = (TS *)H->h[x], *bn = (TS *)H->b[x];
    // The two kernels write disjoint cells from the same inputs.  The ring's
    // launch is small (a few hundred blocks): on the side stream it fills the
    // slots the interior launch leaves free instead of running after it.
    const bool fork = H->n_int > 0 && H->n_bnd > 0 && H->side;
    hipStream_t sb = fork ? H->side : H->stream;
    if (fork) {
        (void)hipEventRecord(H->fork, H->stream);
        (void)hipStreamWaitEvent(H->side, H->fork, 0);
    }
    if (fork)
        hipLaunchKernelGGL((hb::k_update_bnd<NT, TS, SO>), dim3(H->n_bnd), dim3(256), H->upd_lds, sb, P, H->bnd_cells, h,
                           b, H->recx, H->recy, H->crec, H->dt[c], hn, bn, H->W[x]);
    if (H->n_int > 0)
        hipLaunchKernelGGL((hb::k_update_int<NT, TS, SO>), dim3(H->n_int), dim3(256), H->upd_lds, H->stream, P, h, b,
                           H->recx, H->recy, H->crec, H->dt[c], hn, bn, H->W[x]);
    if (mid) (void)hipEventRecord(mid, H->stream);
    if (fork) {
        (void)hipEventRecord(H->join, H->side);
        (void)hipStreamWaitEvent(H->stream, H->join, 0);
    } else if (H->n_bnd > 0) {
        hipLaunchKernelGGL((hb::k_update_bnd<NT, TS, SO>), dim3(H->n_bnd), dim3(256), H->upd_lds, H->stream, P,
                           H->bnd_cells, h, b, H->recx, H->recy, H->crec, H->dt[c], hn, bn, H->W[x]);
    }
}
// the mixed form streams its stores when its state exceeds the last-level cache
template <int NT, typename TS>
static void launch_update_t(hb_ugks *H, const hb::Params &P, int c, int x, hipEvent_t mid)
{
    if constexpr (sizeof(TS) == 4) {
        if (P.stream_out) {
            launch_update_so<NT, TS, true>(H, P, c, x, mid);
            return;
        }
    }
    launch_update_so<NT, TS, false>(H, P, c, x, mid);
}

template <typename TS>
static void launch_update_p(hb_ugks *H, const hb::Params &P, int c, int x, hipEvent_t mid)
{
    switch (P.NT) {
    case 1: launch_update_t<1, TS>(H, P, c, x, mid); break;
    case 3: launch_update_t<3, TS>(H, P, c, x, mid); break;
    case 5: launch_update_t<5, TS>(H, P, c, x, mid); break;
    case 7: launch_update_t<7, TS>(H, P, c, x, mid); break;
    case 9: launch_update_t<9, TS>(H, P, c, x, mid); break;
    default: launch_update_t<11, TS>(H, P, c, x, mid); break;
    }
}

// interior then boundary-ring update; `mid` (may be null) is recorded between them
static void launch_update(hb_ugks *H, const hb::Params &P, int c, int x, hipEvent_t mid)
{
    if (H->precision == HB_MIXED) launch_update_p<float>(H, P, c, x, mid);
    else launch_update_p<double>(H, P, c, x, mid);
}

static void launch_moments(hb_ugks *H, const hb::Params &P, int c)
{
    if (H->precision == HB_MIXED)
        hipLaunchKernelGGL(hb::k_moments<float>, dim3(P.nc), dim3(256), 0, H->stream, P, (const float *)H->h[c],
                           (const float *)H->b[c], H->feed);
    else
        hipLaunchKernelGGL(hb::k_moments<double>, dim3(P.nc), dim3(256), 0, H->stream, P, (const double *)H->h[c],
                           (const double *)H->b[c], H->feed);
}

static size_t elem_bytes(const hb_ugks *H) { return H->precision == HB_MIXED ? sizeof(float) : sizeof(double); }

extern "C" {

void hb_ugks_default_numerics(hb_numerics *o)
{
    if (!o) return;
    o->cfl = 0.5;
    o->face_dt = 0;
    o->Pr = 2.0 / 3.0;
    o->omega_vss = 0.81;
    o->alpha_vss = 1.0;
    o->K_int = 1;
    o->dt_mode = 0;
    o->dt_fixed = 0.0;
    o->macro_flux_mode = 0;
    o->level_mass = 1;
}

const char *hb_ugks_strerror(int s)
{
    switch (s) {
    case HB_OK: return "ok";
    case HB_EINVAL: return "invalid argument";
    case HB_ENOMEM: return "device memory exhausted or over budget";
    case HB_ESTATE: return "call out of order (no case set)";
    case HB_EDIVERGED: return "non-finite residual: the iteration diverged";
    case HB_EDEVICE: return "HIP runtime error or no gfx950 device";
    case HB_ECAPACITY: return "output buffer too small";
    default: return "unknown status";
    }
}

int hb_vgrid_nodes(const hb_vgrid *vg, double *u, double *w)
{
    if (!vg || !u || !w) return HB_EINVAL;
    return velocity_rule(vg->m, vg->umax, vg->rule, u, w);
}

int hb_ugks_create(const hb_create_opts *opts, hb_handle *out)
{
    if (!out) return HB_EINVAL;
    *out = nullptr;
    hb_create_opts o{0, nullptr, HB_FP64, 0};
    if (opts) o = *opts;
    if (o.precision != HB_FP64 && o.precision != HB_MIXED) return HB_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o.device < 0 || o.device >= ndev) {
        (void)hipGetLastError();
        return HB_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) != hipSuccess) return HB_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HB_EDEVICE;
    hb_ugks *H = new (std::nothrow) hb_ugks();
    if (!H) return HB_ENOMEM;
    H->device = o.device;
    H->stream = (hipStream_t)o.stream;
    H->precision = o.precision;
    H->budget = o.hbm_budget_bytes;
    *out = H;
    return HB_OK;
}

void hb_ugks_destroy(hb_handle H)
{
    if (!H) return;
    (void)hipSetDevice(H->device);
    if (H->stream) (void)hipStreamSynchronize(H->stream);
    else (void)hipDeviceSynchronize();
    if (H->side) {
        (void)hipStreamSynchronize(H->side);
        (void)hipStreamDestroy(H->side);
        (void)hipEventDestroy(H->fork);
        (void)hipEventDestroy(H->join);
    }
    free_case(H);
    for (auto &e : H->tev) (void)hipEventDestroy(e);
    delete H;
}

int hb_ugks_set_case(hb_handle H, const hb_geometry *g, double Kn, double St, int NH, const hb_wall walls[4],
                     const hb_vgrid *vg, const hb_numerics *num)
{
    if (!H || !g || !walls || !vg) return HB_EINVAL;
    hb_numerics nm;
    hb_ugks_default_numerics(&nm);
    if (num) nm = *num;
    const int nx = g->nx, ny = g->ny, M = vg->m, Mv = vg->m_v ? vg->m_v : vg->m;
    const double vmax = vg->vmax > 0.0 ? vg->vmax : vg->umax;
    if (nx < 3 || ny < 3 || M < 4 || M > 128 || (M & 1) || Mv < 4 || Mv > 128 || (Mv & 1) || NH < 0 ||
        2 * NH + 1 > HB_NTMAX || !(Kn > 0.0) ||
        !(St >= 0.0) || (vg->rule != HB_RULE_TRAPEZOID && vg->rule != HB_RULE_GAUSS_HERMITE) ||
        (vg->rule == HB_RULE_TRAPEZOID && !(vg->umax > 0.0)) || !(nm.cfl > 0.0) || nm.K_int < 0 || !(nm.Pr > 0.0) ||
        (nm.dt_mode == 1 && !(nm.dt_fixed > 0.0)) || !(g->L > 0.0) || !(g->H > 0.0) ||
        (nm.macro_flux_mode != 0 && nm.macro_flux_mode != 1) || (nm.level_mass != 0 && nm.level_mass != 1))
        return HB_EINVAL;
    for (int w = 0; w < 4; w++)
        if (!(walls[w].T_mean - std::hypot(walls[w].T_hat_re, walls[w].T_hat_im) > 0.0)) return HB_EINVAL;
    std::vector<double> xf(nx + 1), yf(ny + 1);
    for (int i = 0; i <= nx; i++) xf[i] = g->x_faces ? g->x_faces[i] : g->L * i / nx;
    for (int j = 0; j <= ny; j++) yf[j] = g->y_faces ? g->y_faces[j] : g->H * j / ny;
    for (int i = 0; i < nx; i++)
        if (!(xf[i + 1] > xf[i])) return HB_EINVAL;
    for (int j = 0; j < ny; j++)
        if (!(yf[j + 1] > yf[j])) return HB_EINVAL;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    if (H->stream) (void)hipStreamSynchronize(H->stream);
    free_case(H);

    hb::Params &P = H->P;
    P = hb::Params{};
    P.nx = nx;
    P.ny = ny;
    P.nc = nx * ny;
    P.M = M;
    P.Mh = M / 2;
    P.Mv = Mv;
    P.Mvh = Mv / 2;
    P.Mt = std::max(M, Mv);
    P.Q = P.Mh * P.Mvh;
    P.Qp = (P.Q + 63) / 64 * 64;
    P.nvp = 4 * P.Qp;
    P.ls = P.nvp;
    P.NH = NH;
    P.NT = 2 * NH + 1;
    P.K = nm.K_int;
    P.face_dt = nm.face_dt;
    P.macro_mode = nm.macro_flux_mode;
    P.level_mass = nm.level_mass;
    P.dt_mode = nm.dt_mode;
    P.dt_fixed = nm.dt_fixed;
    P.omega = St;  // Eq. (37) with H = sqrt(2 R T0) = 1
    {
        const double a = nm.alpha_vss, w = nm.omega_vss;
        const double coef = 4.0 * a * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) / (5.0 * (a + 1.0) * (a + 2.0));
        P.mu_ref = Kn * std::sqrt(M_PI) / coef;  // Eq. (36), rho0 = H = 1, sqrt(2 pi R T0) = sqrt(pi)
    }
    P.omega_vss = nm.omega_vss;
    P.Pr = nm.Pr;
    P.cfl = nm.cfl;
    P.gamma = (P.K + 4.0) / (P.K + 2.0);
    P.umax = vg->umax;  // the Gauss-Hermite rule replaces both by their largest nodes below
    P.vmax = vmax;
    const int NT = P.NT;
    for (int n = 0; n < NT; n++)
        for (int m = 0; m < NT; m++) {
            const int d = n - m;
            P.E[n * NT + m] = d == 0 ? 0.0 : 0.5 * ((d % 2 == 0) ? 1.0 : -1.0) / std::sin(M_PI * d / NT);  // Eq. (17)
        }
    for (int w = 0; w < 4; w++) H->walls[w] = walls[w];
    H->t_phys = 0.0;
    H->Wp = H->tdres = nullptr;
    for (int w = 0; w < 4; w++)
        for (int n = 0; n < NT; n++) {
            const double th = 2.0 * M_PI * n / NT;  // omega t_n, Eq. (12)
            P.wall_ut[w][n] = walls[w].ut_mean + walls[w].ut_hat_re * std::cos(th) - walls[w].ut_hat_im * std::sin(th);
            P.wall_T[w][n] = walls[w].T_mean + walls[w].T_hat_re * std::cos(th) - walls[w].T_hat_im * std::sin(th);
        }

    // host tables
    std::vector<double> geo;
    geo.insert(geo.end(), xf.begin(), xf.end());
    geo.insert(geo.end(), yf.begin(), yf.end());
    std::vector<double> xc(nx), yc(ny), rdx(nx), rdy(ny), rcx(nx, 0.0), rcy(ny, 0.0), u1(M), w1(M), v1(Mv), w1v(Mv);
    for (int i = 0; i < nx; i++) {
        xc[i] = 0.5 * (xf[i] + xf[i + 1]);
        rdx[i] = 1.0 / (xf[i + 1] - xf[i]);
    }
    for (int j = 0; j < ny; j++) {
        yc[j] = 0.5 * (yf[j] + yf[j + 1]);
        rdy[j] = 1.0 / (yf[j + 1] - yf[j]);
    }
    for (int i = 1; i < nx; i++) rcx[i] = 1.0 / (xc[i] - xc[i - 1]);
    for (int j = 1; j < ny; j++) rcy[j] = 1.0 / (yc[j] - yc[j - 1]);
    if (velocity_rule(M, vg->umax, vg->rule, u1.data(), w1.data()) != HB_OK ||
        velocity_rule(Mv, vmax, vg->rule, v1.data(), w1v.data()) != HB_OK)
        return HB_EINVAL;
    if (vg->rule == HB_RULE_GAUSS_HERMITE) {
        P.umax = u1[M - 1];
        P.vmax = v1[Mv - 1];
    }
    // a square grid keeps one 1-D rule for both axes
    const bool square = Mv == M && v1 == u1;
    const size_t ox_xc = geo.size();
    geo.insert(geo.end(), xc.begin(), xc.end());
    const size_t ox_yc = geo.size();
    geo.insert(geo.end(), yc.begin(), yc.end());
    const size_t ox_rdx = geo.size();
    geo.insert(geo.end(), rdx.begin(), rdx.end());
    const size_t ox_rdy = geo.size();
    geo.insert(geo.end(), rdy.begin(), rdy.end());
    const size_t ox_rcx = geo.size();
    geo.insert(geo.end(), rcx.begin(), rcx.end());
    const size_t ox_rcy = geo.size();
    geo.insert(geo.end(), rcy.begin(), rcy.end());
    const size_t ox_u1 = geo.size();
    geo.insert(geo.end(), u1.begin(), u1.end());
    const size_t ox_w1 = geo.size();
    geo.insert(geo.end(), w1.begin(), w1.end());
    const size_t ox_v1 = square ? ox_u1 : geo.size();
    if (!square) geo.insert(geo.end(), v1.begin(), v1.end());
    const size_t ox_w1v = square ? ox_w1 : geo.size();
    if (!square) geo.insert(geo.end(), w1v.begin(), w1v.end());

    // internal velocity order: quadrant q = (u>0) + 2 (v>0), then (iv, iu) inside it, 64-padded
    const int Mh = P.Mh, Qp = P.Qp, nvp = P.nvp;
    std::vector<double> vel(3 * (size_t)nvp, 0.0);
    std::vector<int> veli(2 * (size_t)nvp, 0);
    H->perm.assign((size_t)M * Mv, -1);
    for (int q = 0; q < 4; q++)
        for (int r = 0; r < Qp; r++) {
            const int rr = r < P.Q ? r : 0;  // padding repeats the first velocity with zero weight
            const int il = rr % Mh, jl = rr / Mh;
            const int iu = (q & 1) ? Mh + il : il, iv = (q & 2) ? P.Mvh + jl : jl;
            const int ap = q * Qp + r;
            vel[ap] = u1[iu];
            vel[nvp + ap] = v1[iv];
            vel[2 * (size_t)nvp + ap] = r < P.Q ? w1[iu] * w1v[iv] : 0.0;
            veli[ap] = iu;
            veli[nvp + ap] = iv;
            if (r < P.Q) H->perm[(size_t)iv * M + iu] = ap;
        }

    const size_t nel = (size_t)P.nc * NT * P.ls;
    P.stream_out = H->precision == HB_MIXED && 2.0 * (double)nel * 4.0 > HB_STREAM_OUT_BYTES;
    const size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
    H->cells_blocks = (P.nc * NT + 127) / 128;
    H->upd_lds = (H->precision == HB_MIXED ? sizeof(float) : sizeof(double)) * 16 * (size_t)NT * P.Mt;
    if (H->upd_lds > 160 * 1024) return HB_EINVAL;
    int rc = HB_OK;
#define ALLOC(ptr, count, T)                                            \
    do {                                                                \
        rc = dalloc(H, (void **)&(ptr), sizeof(T) * (size_t)(count));  \
        if (rc != HB_OK) {                                              \
            free_case(H);                                               \
            return rc;                                                  \
        }                                                               \
    } while (0)
    ALLOC(H->geo, geo.size(), double);
    ALLOC(H->vel, vel.size(), double);
    ALLOC(H->veli, veli.size(), int);
    for (int s = 0; s < 2; s++) {
        if (H->precision == HB_MIXED) {
            ALLOC(H->h[s], nel, float);
            ALLOC(H->b[s], nel, float);
        } else {
            ALLOC(H->h[s], nel, double);
            ALLOC(H->b[s], nel, double);
        }
        ALLOC(H->W[s], (size_t)P.nc * NT * 4, double);
        ALLOC(H->dt[s], P.nc, double);
    }
    ALLOC(H->feed, (size_t)P.nc * NT * hb::FEED, double);
    ALLOC(H->recx, nfx * NT * hb::REC, double);
    ALLOC(H->recy, nfy * NT * hb::REC, double);
    ALLOC(H->crec, (size_t)P.nc * NT * hb::CREC, double);
    ALLOC(H->rpart, (size_t)H->cells_blocks * hb::RPART, double);
    // level-mass factors: HB_NTMAX doubles, then (mixed form) s_n and (s_n - 1)/pi in FP32
    ALLOC(H->lscale, 2 * HB_NTMAX, double);
    if (H->precision == HB_MIXED) {
        ALLOC(H->rx32, nfx * NT * hb::REC32, float);
        ALLOC(H->ry32, nfy * NT * hb::REC32, float);
        ALLOC(H->cr32, (size_t)P.nc * NT * hb::CREC32, float);
        ALLOC(H->ex64, M + Mv, double);
        ALLOC(H->er32, M + Mv, float);
        ALLOC(H->vel32, vel.size(), float);
    }
    ALLOC(H->ring, (size_t)HB_RING * 4, double);
    ALLOC(H->flag, 1, int);
    // rest Maxwellian per velocity, then its per-quadrant moment sums (4 x 10)
    ALLOC(H->vref, nvp + 40, double);
    {
        const size_t nh = (size_t)(P.NH + 1) * P.nc * 7;
        ALLOC(H->hvars, (size_t)P.nc * NT * 7, double);
        ALLOC(H->hre, nh, double);
        ALLOC(H->him, nh, double);
    }
    // The boundary ring (cells within two of a wall), listed as a walk around
    // the cavity: each cell is keyed by the perimeter position of its nearest
    // wall, then by its depth.  Contiguous ranges of the list, one per XCD,
    // are then stretches of the ring whose stencils overlap.
    std::vector<int> bnd;
    {
        std::vector<std::tuple<long, int, int>> key;
        for (int jj = 0; jj < ny; jj++)
            for (int ii = 0; ii < nx; ii++)
                if (ii < 2 || ii > nx - 3 || jj < 2 || jj > ny - 3) {
                    const int d[4] = {jj, nx - 1 - ii, ny - 1 - jj, ii};
                    const long sp[4] = {ii, (long)nx + jj, (long)nx + ny + (nx - 1 - ii), 2L * nx + ny + (ny - 1 - jj)};
                    int w = 0;
                    for (int k = 1; k < 4; k++)
                        if (d[k] < d[w]) w = k;
                    key.emplace_back(sp[w], d[w], jj * nx + ii);
                }
        std::sort(key.begin(), key.end());
        for (const auto &t : key) bnd.push_back(std::get<2>(t));
    }
    H->n_bnd = (int)bnd.size();
    H->n_int = P.nc - H->n_bnd;
    ALLOC(H->bnd_cells, bnd.size(), int);
    if (NT == 1 && P.dt_mode == 1 && !H->pool) {
        ALLOC(H->Wp, (size_t)P.nc * 4, double);
        ALLOC(H->tdres, 4, double);
    }
#undef ALLOC
    H->bnd_host = bnd;
    H->xf_host = xf;
    H->yf_host = yf;
    if (H->count_only) return HB_OK;
    HIPOK(hipMemcpy(H->geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(H->vel, vel.data(), vel.size() * sizeof(double), hipMemcpyHostToDevice));
    if (H->precision == HB_MIXED) {
        std::vector<float> v32(vel.begin(), vel.end());
        HIPOK(hipMemcpy(H->vel32, v32.data(), v32.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    HIPOK(hipMemcpy(H->veli, veli.data(), veli.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPOK(hipMemset(H->flag, 0, sizeof(int)));
    HIPOK(hipMemcpy(H->bnd_cells, bnd.data(), bnd.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPOK(hipMemset(H->ring, 0, sizeof(double) * HB_RING * 4));
    P.xf = H->geo;
    P.yf = H->geo + (nx + 1);
    P.xc = H->geo + ox_xc;
    P.yc = H->geo + ox_yc;
    P.rdx = H->geo + ox_rdx;
    P.rdy = H->geo + ox_rdy;
    P.rcx = H->geo + ox_rcx;
    P.rcy = H->geo + ox_rcy;
    P.u1 = H->geo + ox_u1;
    P.w1 = H->geo + ox_w1;
    P.v1 = H->geo + ox_v1;
    P.w1v = H->geo + ox_w1v;
    P.vu = H->vel;
    P.vv = H->vel + nvp;
    P.vw = H->vel + 2 * (size_t)nvp;
    P.viu = H->veli;
    P.viv = H->veli + nvp;
    P.vref = H->vref;
    P.rmom = H->vref + nvp;
    P.lscale = H->lscale;
    if (H->precision == HB_MIXED) {
        P.rx32 = H->rx32;
        P.ry32 = H->ry32;
        P.cr32 = H->cr32;
        P.lscale32 = (float *)(H->lscale + HB_NTMAX);
        P.ex64 = H->ex64;
        P.er32 = H->er32;
        P.ex64v = H->ex64 + M;
        P.er32v = H->er32 + M;
        P.vel32 = H->vel32;
        for (int k = 0; k < NT * NT; k++) P.Ef[k] = static_cast<float>(P.E[k]);
    }
    {
        const int rcl = update_lds_attr(H->precision, NT, H->upd_lds);
        if (rcl != HB_OK) {
            free_case(H);
            return rcl;
        }
    }
    H->cur = 0;
    H->step = 0;
    const long tot = (long)nel;
    hipLaunchKernelGGL(hb::k_vref, dim3((nvp + 255) / 256), dim3(256), 0, H->stream, P, H->vref);
    hipLaunchKernelGGL(hb::k_restmom, dim3(1), dim3(256), 0, H->stream, P, H->vref + nvp);
    if (H->precision == HB_MIXED)
        hipLaunchKernelGGL(hb::k_etab, dim3(1), dim3(128), 0, H->stream, P, H->ex64, H->er32);
    for (int s = 0; s < 2; s++) {
        if (H->precision == HB_MIXED)
            hipLaunchKernelGGL(hb::k_init<float>, dim3((tot + 255) / 256), dim3(256), 0, H->stream, P,
                               (float *)H->h[s], (float *)H->b[s], H->W[s]);
        else
            hipLaunchKernelGGL(hb::k_init<double>, dim3((tot + 255) / 256), dim3(256), 0, H->stream, P,
                               (double *)H->h[s], (double *)H->b[s], H->W[s]);
    }
    hipLaunchKernelGGL(hb::k_dt, dim3((P.nc + 127) / 128), dim3(128), 0, H->stream, P, H->W[0], H->dt[0]);
    HIPOK(hipGetLastError());
    HIPOK(H->stream ? hipStreamSynchronize(H->stream) : hipDeviceSynchronize());
    H->vref_host.resize(nvp);
    HIPOK(hipMemcpy(H->vref_host.data(), H->vref, nvp * sizeof(double), hipMemcpyDeviceToHost));
    H->has_case = true;
    return HB_OK;
}

}  // extern "C"

// Queue one step of Sec. 2.4 on the handle's stream and swap the buffers.
// the side stream and its fork/join events, on the handle's device
static int side_stream(hb_ugks *H)
{
    if (H->side) return HB_OK;
    if (hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking) != hipSuccess) {
        H->side = nullptr;
        return HB_EDEVICE;
    }
    if (hipEventCreateWithFlags(&H->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&H->join, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(H->side);
        H->side = nullptr;
        return HB_EDEVICE;
    }
    return HB_OK;
}

static int enqueue_step(hb_ugks *H)
{
    const hb::Params &P = H->P;
    if (H->n_bnd > 0 && H->n_int > 0) {
        const int rc = side_stream(H);
        if (rc != HB_OK) return rc;
    }
    const int NT = P.NT;
    const int nfaces = (P.nx + 1) * P.ny + P.nx * (P.ny + 1);
    const int c = H->cur, x = 1 - c;
    const int slot = (int)(H->step % HB_RING);
    hipEvent_t *ev = nullptr;
    if (H->timing) {
        if (H->tused + HB_NKERN + 1 > H->tev.size()) {
            for (int k = 0; k <= HB_NKERN; k++) {
                hipEvent_t e;
                HIPOK(hipEventCreate(&e));
                H->tev.push_back(e);
            }
        }
        ev = H->tev.data() + H->tused;
        H->tused += HB_NKERN + 1;
        HIPOK(hipEventRecord(ev[0], H->stream));
    }
    launch_moments(H, P, c);
    if (ev) HIPOK(hipEventRecord(ev[1], H->stream));
    hipLaunchKernelGGL(hb::k_faces, dim3((nfaces * NT + 127) / 128), dim3(128), 0, H->stream, P, H->feed, H->W[c],
                       H->dt[c], H->recx, H->recy);
    if (ev) HIPOK(hipEventRecord(ev[2], H->stream));
    hipLaunchKernelGGL(hb::k_cells, dim3(H->cells_blocks), dim3(128), 0, H->stream, P, H->feed, H->recx, H->recy,
                       H->W[c], H->dt[c], H->W[x], H->crec, H->rpart);
    if (ev) HIPOK(hipEventRecord(ev[3], H->stream));
    hipLaunchKernelGGL(hb::k_dt_resid, dim3((P.nc + 255) / 256 + 1), dim3(256), 0, H->stream, P, H->W[x], H->dt[x],
                       H->rpart, H->cells_blocks, H->ring, slot, H->flag);
    if (ev) HIPOK(hipEventRecord(ev[4], H->stream));
    launch_update(H, P, c, x, ev ? ev[5] : nullptr);
    if (ev) HIPOK(hipEventRecord(ev[6], H->stream));
    HIPOK(hipGetLastError());
    H->cur = x;
    H->step++;
    return HB_OK;
}

extern "C" {

int hb_ugks_pseudo_step(hb_handle H, int nsteps)
{
    if (!H) return HB_EINVAL;
    if (!H->has_case || H->batch_owned) return HB_ESTATE;
    if (nsteps < 0) return HB_EINVAL;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    for (int s = 0; s < nsteps; s++) {
        const int rc = enqueue_step(H);
        if (rc != HB_OK) return rc;
    }
    return HB_OK;
}

// Explicit time-domain UGKS: the wall state of Eqs. (25)-(26) is taken at the
// physical mid-step time, the spectral term vanishes with one level, and every
// cell advances by the same physical step dt_fixed.
static int td_steps(hb_ugks *H, int nsteps)
{
    hb::Params &P = H->P;
    const double dt = P.dt_fixed;
    for (int s = 0; s < nsteps; s++) {
        const double th = P.omega * (H->t_phys + 0.5 * dt);
        const double c = std::cos(th), sn = std::sin(th);
        for (int w = 0; w < 4; w++) {
            const hb_wall &wl = H->walls[w];
            P.wall_ut[w][0] = wl.ut_mean + wl.ut_hat_re * c - wl.ut_hat_im * sn;
            P.wall_T[w][0] = wl.T_mean + wl.T_hat_re * c - wl.T_hat_im * sn;
        }
        const int rc = enqueue_step(H);
        if (rc != HB_OK) return rc;
        H->t_phys += dt;
    }
    return HB_OK;
}

static bool td_ready(const hb_ugks *H) { return H->has_case && !H->batch_owned && H->Wp && H->P.NT == 1; }

int hb_ugks_td_step(hb_handle H, int nsteps)
{
    if (!H) return HB_EINVAL;
    if (!td_ready(H)) return HB_ESTATE;
    if (nsteps < 0) return HB_EINVAL;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    return td_steps(H, nsteps);
}

int hb_ugks_td_period(hb_handle H, int nsteps, double out[4])
{
    if (!H || !out) return HB_EINVAL;
    if (!td_ready(H)) return HB_ESTATE;
    if (nsteps < 1) return HB_EINVAL;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    const size_t wb = (size_t)H->P.nc * 4 * sizeof(double);
    HIPOK(hipMemcpyAsync(H->Wp, H->W[H->cur], wb, hipMemcpyDeviceToDevice, H->stream));
    const int rc = td_steps(H, nsteps);
    if (rc != HB_OK) return rc;
    hipLaunchKernelGGL(hb::k_period_diff, dim3(1), dim3(256), 0, H->stream, H->W[H->cur], H->Wp, H->P.nc, H->tdres);
    HIPOK(hipGetLastError());
    HIPOK(hipMemcpyAsync(out, H->tdres, 4 * sizeof(double), hipMemcpyDeviceToHost, H->stream));
    HIPOK(H->stream ? hipStreamSynchronize(H->stream) : hipDeviceSynchronize());
    int flag = 0;
    HIPOK(hipMemcpy(&flag, H->flag, sizeof(int), hipMemcpyDeviceToHost));
    for (int k = 0; k < 4; k++)
        if (!std::isfinite(out[k])) flag = 1;
    return flag ? HB_EDIVERGED : HB_OK;
}

int hb_ugks_time(hb_handle H, double *t)
{
    if (!H || !t) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    *t = H->t_phys;
    return HB_OK;
}

// fold the recorded event sets into the per-kernel sums
static int collect_times(hb_ugks *H)
{
    if (!H->tused) return HB_OK;
    HIPOK(hipEventSynchronize(H->tev[H->tused - 1]));
    for (size_t s = 0; s < H->tused; s += HB_NKERN + 1)
        for (int k = 0; k < HB_NKERN; k++) {
            float ms = 0.f;
            HIPOK(hipEventElapsedTime(&ms, H->tev[s + k], H->tev[s + k + 1]));
            H->kms[k] += ms;
            H->klaunch[k]++;
        }
    H->tused = 0;
    return HB_OK;
}

int hb_ugks_residual(hb_handle H, double out[4], long *step_index)
{
    if (!H || !out) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    HIPOK(H->stream ? hipStreamSynchronize(H->stream) : hipDeviceSynchronize());
    if (step_index) *step_index = H->step;
    if (H->step == 0) {
        for (int k = 0; k < 4; k++) out[k] = 0.0;
        return HB_OK;
    }
    const int slot = (int)((H->step - 1) % HB_RING);
    HIPOK(hipMemcpy(out, H->ring + slot * 4, 4 * sizeof(double), hipMemcpyDeviceToHost));
    int flag = 0;
    HIPOK(hipMemcpy(&flag, H->flag, sizeof(int), hipMemcpyDeviceToHost));
    return flag ? HB_EDIVERGED : HB_OK;
}

int hb_ugks_sizes(hb_handle H, int out[6])
{
    if (!H || !out) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    out[0] = H->P.nx;
    out[1] = H->P.ny;
    out[2] = H->P.nc;
    out[3] = H->P.M;
    out[4] = H->P.M * H->P.Mv;
    out[5] = H->P.NT;
    return HB_OK;
}

size_t hb_ugks_device_bytes(hb_handle H) { return H ? H->bytes : 0; }

int hb_ugks_state_out(hb_handle H, double *W, double *hh, double *bb, size_t capacity)
{
    if (!H) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    const hb::Params &P = H->P;
    const size_t ncn = (size_t)P.nc * P.NT, nv = (size_t)P.M * P.Mv;
    if ((hh || bb) && capacity < ncn * nv) return HB_ECAPACITY;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    HIPOK(H->stream ? hipStreamSynchronize(H->stream) : hipDeviceSynchronize());
    if (W) HIPOK(hipMemcpy(W, H->W[H->cur], ncn * 4 * sizeof(double), hipMemcpyDeviceToHost));
    const bool mixed = H->precision == HB_MIXED;
    const size_t eb = elem_bytes(H);
    std::vector<unsigned char> tmp;
    void *src[2] = {H->h[H->cur], H->b[H->cur]};
    double *dst[2] = {hh, bb};
    for (int s = 0; s < 2; s++) {
        if (!dst[s]) continue;
        tmp.resize(ncn * P.ls * eb);
        HIPOK(hipMemcpy(tmp.data(), src[s], tmp.size(), hipMemcpyDeviceToHost));
        const double fac = s == 0 ? 1.0 : 0.5 * P.K;
        for (size_t e = 0; e < ncn; e++)
            for (size_t a = 0; a < nv; a++) {
                const size_t k = e * P.ls + H->perm[a];
                dst[s][e * nv + a] = mixed ? (double)((const float *)tmp.data())[k] + fac * H->vref_host[H->perm[a]]
                                           : ((const double *)tmp.data())[k];
            }
    }
    return HB_OK;
}

int hb_ugks_state_in(hb_handle H, const double *W, const double *hh, const double *bb)
{
    if (!H) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    const hb::Params &P = H->P;
    const size_t ncn = (size_t)P.nc * P.NT, nv = (size_t)P.M * P.Mv;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    HIPOK(H->stream ? hipStreamSynchronize(H->stream) : hipDeviceSynchronize());
    if (W) HIPOK(hipMemcpy(H->W[H->cur], W, ncn * 4 * sizeof(double), hipMemcpyHostToDevice));
    const bool mixed = H->precision == HB_MIXED;
    const size_t eb = elem_bytes(H);
    std::vector<unsigned char> tmp;
    void *dst[2] = {H->h[H->cur], H->b[H->cur]};
    const double *src[2] = {hh, bb};
    for (int s = 0; s < 2; s++) {
        if (!src[s]) continue;
        tmp.assign(ncn * P.ls * eb, 0);
        const double fac = s == 0 ? 1.0 : 0.5 * P.K;
        for (size_t e = 0; e < ncn; e++)
            for (size_t a = 0; a < nv; a++) {
                const size_t k = e * P.ls + H->perm[a];
                if (mixed)
                    ((float *)tmp.data())[k] = (float)(src[s][e * nv + a] - fac * H->vref_host[H->perm[a]]);
                else
                    ((double *)tmp.data())[k] = src[s][e * nv + a];
            }
        HIPOK(hipMemcpy(dst[s], tmp.data(), tmp.size(), hipMemcpyHostToDevice));
    }
    if (W) {
        hipLaunchKernelGGL(hb::k_dt, dim3((P.nc + 127) / 128), dim3(128), 0, H->stream, P, H->W[H->cur], H->dt[H->cur]);
        HIPOK(hipGetLastError());
        HIPOK(H->stream ? hipStreamSynchronize(H->stream) : hipDeviceSynchronize());
    }
    return HB_OK;
}

}  // extern "C"

// Harmonics of Eq. (40) into re/im (selected variables in bit order, host
// memory) through the device scratch vars [nc][NT][7], dre, dim [7][NH+1][nc].
static int harmonics_into(hb_ugks *H, unsigned var_mask, double *re, double *im, double *vars, double *dre,
                          double *dim_)
{
    const hb::Params &P = H->P;
    const size_t per = (size_t)(P.NH + 1) * P.nc, nout = 7 * per;
    const int c = H->cur;
    if (H->precision == HB_MIXED)
        hipLaunchKernelGGL(hb::k_harm_vars<float>, dim3(P.nc), dim3(256), 0, H->stream, P, (const float *)H->h[c],
                           (const float *)H->b[c], H->W[c], vars);
    else
        hipLaunchKernelGGL(hb::k_harm_vars<double>, dim3(P.nc), dim3(256), 0, H->stream, P, (const double *)H->h[c],
                           (const double *)H->b[c], H->W[c], vars);
    hipLaunchKernelGGL(hb::k_harm_dft, dim3((nout + 255) / 256), dim3(256), 0, H->stream, P, vars, dre, dim_);
    HIPOK(hipGetLastError());
    HIPOK(H->stream ? hipStreamSynchronize(H->stream) : hipDeviceSynchronize());
    size_t o = 0;
    for (int v = 0; v < 7; v++) {
        if (!((var_mask >> v) & 1)) continue;
        HIPOK(hipMemcpy(re + o, dre + v * per, per * sizeof(double), hipMemcpyDeviceToHost));
        HIPOK(hipMemcpy(im + o, dim_ + v * per, per * sizeof(double), hipMemcpyDeviceToHost));
        o += per;
    }
    return HB_OK;
}

static int harmonics_check(hb_ugks *H, unsigned var_mask, const double *re, const double *im, size_t capacity)
{
    if (!H || !re || !im || (var_mask & ~0x7Fu) || !var_mask) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    int nsel = 0;
    for (int v = 0; v < 7; v++) nsel += (var_mask >> v) & 1;
    if (capacity < nsel * (size_t)(H->P.NH + 1) * H->P.nc) return HB_ECAPACITY;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    return HB_OK;
}

// Device scratch of hb_ugks_harmonics_out_noalloc: a file-scope array, so each
// GPU the library runs on holds its own copy until the process ends.  Host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device (the array's name is a host-side stand-in).
static __device__ __align__(256) double scratch[HB_NOALLOC_DOUBLES];
static std::mutex scratch_mu;
static double *scratch_dev[HB_MAX_DEVICES];

// The scratch address on the current device `dev`, taken once per device.
static double *scratch_on(int dev)
{
    if (dev < 0 || dev >= HB_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        double *p = nullptr;
        if (hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_dev[dev] = p;
    }
    return scratch_dev[dev];
}

extern "C" {

int hb_ugks_harmonics_out(hb_handle H, unsigned var_mask, double *re, double *im, size_t capacity)
{
    const int rc = harmonics_check(H, var_mask, re, im, capacity);
    if (rc != HB_OK) return rc;
    // scratch of the handle (allocated with the case, from its pool or budget)
    return harmonics_into(H, var_mask, re, im, H->hvars, H->hre, H->him);
}

int hb_ugks_harmonics_out_noalloc(hb_handle H, unsigned var_mask, double *re, double *im, size_t capacity)
{
    const int rc = harmonics_check(H, var_mask, re, im, capacity);
    if (rc != HB_OK) return rc;
    const hb::Params &P = H->P;
    const size_t nvars = (size_t)P.nc * P.NT * 7, nout = 7 * (size_t)(P.NH + 1) * P.nc;
    if (nvars + 2 * nout > HB_NOALLOC_DOUBLES) return HB_ENOMEM;
    double *base = scratch_on(H->device);
    if (!base) return HB_EDEVICE;
    return harmonics_into(H, var_mask, re, im, base, base + nvars, base + nvars + nout);
}

int hb_ugks_wall_harmonic(hb_handle H, int wall, int var, int k, double out[2])
{
    if (!H || !out || wall < 0 || wall > 3 || var < 0 || var > 6 || k < 0) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    const hb::Params &P = H->P;
    if (k > P.NH) return HB_EINVAL;
    const size_t per = (size_t)(P.NH + 1) * P.nc;
    std::vector<double> re(per), im(per);
    const int rc = hb_ugks_harmonics_out(H, 1u << var, re.data(), im.data(), per);
    if (rc != HB_OK) return rc;
    const bool horiz = wall == 0 || wall == 2;  // bottom/top run along x
    const int n = horiz ? P.nx : P.ny;
    const std::vector<double> &f = horiz ? H->xf_host : H->yf_host;
    double sr = 0.0, si = 0.0;
    for (int i = 0; i < n; i++) {
        const int c = wall == 0 ? i : wall == 2 ? (P.ny - 1) * P.nx + i : wall == 1 ? i * P.nx + P.nx - 1 : i * P.nx;
        const double ds = f[i + 1] - f[i];
        sr += re[(size_t)k * P.nc + c] * ds;
        si += im[(size_t)k * P.nc + c] * ds;
    }
    const double len = f[n] - f[0];
    out[0] = sr / len;
    out[1] = si / len;
    return HB_OK;
}

int hb_ugks_enable_timing(hb_handle H, int on)
{
    if (!H) return HB_EINVAL;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    if (H->tused) HIPOK(hipEventSynchronize(H->tev[H->tused - 1]));
    H->tused = 0;
    H->timing = on != 0;
    for (int k = 0; k < HB_NKERN; k++) {
        H->kms[k] = 0.0;
        H->klaunch[k] = 0;
    }
    return HB_OK;
}

int hb_ugks_kernel_times(hb_handle H, const char **names, long *launches, double *ms, int capacity)
{
    if (!H) return HB_EINVAL;
    if (!H->has_case) return HB_ESTATE;
    if (capacity < HB_NKERN) return HB_ECAPACITY;
    if (hipSetDevice(H->device) != hipSuccess) return HB_EDEVICE;
    const int rc = collect_times(H);
    if (rc != HB_OK) return rc;
    for (int k = 0; k < HB_NKERN; k++) {
        if (names) names[k] = KNAMES[k];
        if (launches) launches[k] = H->klaunch[k];
        if (ms) ms[k] = H->kms[k];
    }
    return HB_NKERN;
}

}  // extern "C"
