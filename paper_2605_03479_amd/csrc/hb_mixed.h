// Mixed form of the update kernels: FP32 per-velocity arithmetic on the
// stored deviations dh = h - H_ref, db = b - K/2 H_ref from the rest
// Maxwellian H_ref = E(u) E(v) / pi, E(x) = exp(-x^2) (Sec. 2.1, Eqs. 7-10).
//
// Flux (Eq. 23).  Every face flux is taken minus u_n H_ref; that term is the
// same at every face, so the flux divergence is unchanged.  With the face
// exponential e = (E_n + dn)(E_t + dt), dn = exp(-lam (x - U_n)^2) - E(x)
// (dt likewise) from FP32 tables built in FP64, and the record's
// Q' = Q - k0, k0 = (1 - c4)/pi (b: (1 - c4) K/(2 pi)):
//   u_n [e Q + c4 h0 + c5 s] - u_n H_ref = u_n [e Q' + (e - E_n E_t) k0 + c4 dh0 + c5 s].
// Collision (Eq. 30): with the equilibrium amplitude A and A - 1/pi (b: B,
// B - K/(2 pi)) from the FP32 record, h+ - H_ref = A e (1 + S) - E_u E_v/pi
//   = A (e S + (e - E_u E_v)) + E_u E_v (A - 1/pi),  S the Shakhov factor.
// Each product then carries a factor of the size of the deviation, so FP32
// rounding stays relative to the deviation, not to the distribution.  The
// moment sums, W and the residual stay in FP64 (moments kernel, cells kernel).
#pragma once

namespace hb {

typedef __attribute__((address_space(4))) const float cfloat;

__device__ inline cfloat *wave_uniform_f(const float *p)
{
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
    return (cfloat *)((static_cast<unsigned long long>(hi) << 32) | lo);
}

// van Leer slope 2ab/(a+b) for ab > 0, else 0; v_rcp_f32 is within 1 ulp
__device__ inline float vanleer_f(float a, float b)
{
    const float p = a * b;
    const float q = 2.0f * p * __builtin_amdgcn_rcpf(a + b);
    return p > 0.0f ? q : 0.0f;
}

// slope_c in FP32: mode 0 interior (limited), 1 at the low wall, 2 at the high wall
__device__ inline float slope_cf(float fm, float fc, float fp, int mode, float rm, float rp)
{
    if (mode == 1) return (fp - fc) * rp;
    if (mode == 2) return (fc - fm) * rm;
    return vanleer_f((fc - fm) * rm, (fp - fc) * rp);
}

// The velocity's monomials of degree 1..3 (global u, v order): every face's
// cubic is a sum of wave-uniform coefficients times these.
struct Mono {
    float u, v, uu, uv, vv, uuu, uuv, uvv, vvv;
};
__device__ inline Mono mono_of(float u, float v)
{
    Mono m;
    m.u = u;
    m.v = v;
    m.uu = u * u;
    m.uv = u * v;
    m.vv = v * v;
    m.uuu = m.uu * u;
    m.uuv = m.uu * v;
    m.uvv = u * m.vv;
    m.vvv = m.vv * v;
    return m;
}
__device__ inline float cubic_f(cfloat *c, const Mono &m)
{
    float a = m.u * c[1];
    a = fmaf(m.v, c[2], a);
    a = fmaf(m.uu, c[3], a);
    a = fmaf(m.uv, c[4], a);
    a = fmaf(m.vv, c[5], a);
    a = fmaf(m.uuu, c[6], a);
    a = fmaf(m.uuv, c[7], a);
    a = fmaf(m.uvv, c[8], a);
    a = fmaf(m.vvv, c[9], a);
    return a + c[0];
}

// Flux of one face without its u_n factor (the caller folds u_n into the
// divergence): g = e Q' + (e - E_n E_t) k0 + c4 dh0 + c5 s.
__device__ inline void face_g(cfloat *s, const Mono &m, float ern, float ert, float href, float dn, float dt, float h0,
                              float b0, float sh, float sb, float &gh, float &gb)
{
    const float cross = fmaf(ern, dt, dn * (ert + dt));  // e - E_n E_t
    const float e = href + cross;
    const float qh = cubic_f(s, m), qb = cubic_f(s + 10, m);
    gh = fmaf(s[23], sh, fmaf(s[22], h0, fmaf(e, qh, cross * s[20])));
    gb = fmaf(s[23], sb, fmaf(s[22], b0, fmaf(e, qb, cross * s[21])));
}

// FP32 deviation tables of one cell's block, built in FP64: per face and level
// the merged normal table and the two tangential ones, then per level the
// cell equilibria's u and v tables at k and k+1 (layout as build_tables).
template <int NT>
__device__ inline void build_tables_m(const Params &P, const gptr<const double> fr[4], gptr<const double> cr,
                                      float *tab)
{
    const int M = P.M, ftab = 12 * NT * M;
    for (int t = threadIdx.x; t < 16 * NT * M; t += blockDim.x) {
        const int k = t % M;
        const double x = G(P.u1)[k];
        double lam, U;
        if (t < ftab) {
            const int which = (t / M) % 3, fn = t / (3 * M), n = fn % NT, fs = fn / NT;
            const gptr<const double> sd =
                fr[fs] + n * REC + REC_SIDE + REC_SIDEW * (which == 0 ? (x > 0.0 ? 1 : 0) : which - 1);
            lam = sd[0];
            U = which == 0 ? sd[1] : sd[2];
        } else {
            const int tt = t - ftab, which = (tt / M) % 4, n = tt / (4 * M);
            const gptr<const double> cc = cr + n * CREC + (which >= 2 ? CREC_T : 0);
            lam = cc[0];
            U = (which & 1) ? cc[2] : cc[1];
        }
        tab[t] = static_cast<float>(exp(-lam * (x - U) * (x - U)) - G(P.ex64)[k]);
    }
}

// Spectral source and semi-implicit collision (Eq. 30) for one velocity at all
// levels in FP32, then the store of the deviations of h^{k+1}, b^{k+1} times
// the level-mass factor s_n: s_n (H_ref + d) - H_ref = s_n d + (s_n - 1) H_ref.
template <int NT>
__device__ inline void collide_store_m(const Params &P, cfloat *cc, const float *ctab, float dG, float dgw,
                                       const Mono &m, float eru, float erv, float href, int iu, int iv,
                                       const float *hk, const float *bk, const float *dh, const float *db,
                                       float *__restrict__ hn, float *__restrict__ bn, long e0)
{
    const int M = P.M;
    const float kh = P.K - 5.0f;
    cfloat *ls = wave_uniform_f(P.lscale32);
#pragma unroll
    for (int n = 0; n < NT; n++) {
        float Eh = 0.0f, Eb = 0.0f;
#pragma unroll
        for (int mm = 0; mm < NT; mm++) {
            Eh = fmaf(P.Ef[n * NT + mm], hk[mm], Eh);
            Eb = fmaf(P.Ef[n * NT + mm], bk[mm], Eb);
        }
        cfloat *q = cc + n * CREC32;
        const float *ct = ctab + n * 4 * M;
        float dheq[2], dbeq[2];
#pragma unroll
        for (int s2 = 0; s2 < 2; s2++) {
            cfloat *qq = q + CREC32_T * s2;
            const float du = ct[(2 * s2) * M + iu], dv = ct[(2 * s2 + 1) * M + iv];
            const float cross = fmaf(eru, dv, du * (erv + dv));  // e - E_u E_v
            const float e = href + cross;
            const float cu = m.u - qq[0], cv = m.v - qq[1];
            const float c2 = fmaf(cu, cu, cv * cv), cq = fmaf(cu, qq[7], cv * qq[8]);
            const float th = fmaf(qq[2], c2, kh);  // 2 lam c^2 + K - 5; the b factor is 2 more
            const float sh = cq * th, sb = cq * (th + 2.0f);
            dheq[s2] = fmaf(qq[3], fmaf(e, sh, cross), href * qq[4]);
            dbeq[s2] = fmaf(qq[5], fmaf(e, sb, cross), href * qq[6]);
        }
        const float a0 = q[18], a1 = q[19], om0 = q[20], rden = q[21];
        const float hnum = fmaf(hk[n], om0, fmaf(a1, dheq[1], fmaf(a0, dheq[0], -fmaf(dG, dh[n], dgw * Eh))));
        const float bnum = fmaf(bk[n], om0, fmaf(a1, dbeq[1], fmaf(a0, dbeq[0], -fmaf(dG, db[n], dgw * Eb))));
        const float sn = ls[n], sm = ls[HB_NTMAX + n];  // s_n, (s_n - 1)/pi
        G(hn)[e0 + (long)n * P.ls] = fmaf(sn, hnum * rden, sm * href);
        G(bn)[e0 + (long)n * P.ls] = fmaf(sn, bnum * rden, sm * (0.5f * P.K) * href);
    }
}

// Interior cell (2 <= i <= nx-3, 2 <= j <= ny-3) of the mixed form: the
// straight-line stencil of update_int_cell in FP32.
template <int NT>
__device__ inline void update_int_cell_m(const Params &P, const float *__restrict__ h, const float *__restrict__ b,
                                         const double *__restrict__ recx, const double *__restrict__ recy,
                                         const double *__restrict__ crec, const double *__restrict__ dtc,
                                         float *__restrict__ hn, float *__restrict__ bn, double *__restrict__ Wn,
                                         int ci)
{
    extern __shared__ float tabf[];
    const int nxi = P.nx - 4;
    const int i = 2 + ci % nxi, j = 2 + ci / nxi;
    const int M = P.M, nx = P.nx;
    const int c = j * nx + i;
    scale_w<NT>(P, Wn, c);
    const long fw = (long)(j * (nx + 1) + i) * NT, fe = fw + NT, fs = (long)(j * nx + i) * NT,
               fn = (long)((j + 1) * nx + i) * NT;
    const gptr<const double> fr[4] = {G(recx) + fw * REC, G(recx) + fe * REC, G(recy) + fs * REC, G(recy) + fn * REC};
    build_tables_m<NT>(P, fr, G(crec) + (long)c * NT * CREC, tabf);
    __syncthreads();
    const float *ctab = tabf + 12 * NT * M;
    const long sx = (long)NT * P.ls, sy = (long)nx * NT * P.ls;
    const double dGd = dtc[c];
    const float dG = static_cast<float>(dGd), dgw = static_cast<float>(dGd * P.omega);
    const float rdx = static_cast<float>(G(P.rdx)[i]), rdy = static_cast<float>(G(P.rdy)[j]);
    // limiter reciprocal centre distances rc[i-1..i+2] and face distances of
    // the cell and of its two possible upwind neighbours in each direction
    const gptr<const double> rcx = G(P.rcx), rcy = G(P.rcy), xf = G(P.xf), xc = G(P.xc), yf = G(P.yf),
                             yc = G(P.yc);
    const float rx0 = rcx[i - 1], rx1 = rcx[i], rx2 = rcx[i + 1], rx3 = rcx[i + 2];
    const float ry0 = rcy[j - 1], ry1 = rcy[j], ry2 = rcy[j + 1], ry3 = rcy[j + 2];
    const float dxe = xf[i + 1] - xc[i], dxw = xf[i] - xc[i], dye = yf[j + 1] - yc[j], dyw = yf[j] - yc[j];
    const float dxiW = xf[i] - xc[i - 1], dxiE = xf[i + 1] - xc[i + 1];
    const float dyiS = yf[j] - yc[j - 1], dyiN = yf[j + 1] - yc[j + 1];
    cfloat *cc = wave_uniform_f(P.cr32 + (long)c * NT * CREC32);
    const float *rxw = P.rx32 + fw * REC32, *rxe = P.rx32 + fe * REC32, *rys = P.ry32 + fs * REC32,
                *ryn = P.ry32 + fn * REC32;

    for (int ap = threadIdx.x; ap < P.nvp; ap += blockDim.x) {
        const int r = ap % P.Qp;
        if (r >= P.Q) continue;
        const float u = static_cast<float>(G(P.vu)[ap]), v = static_cast<float>(G(P.vv)[ap]);
        const int iu = G(P.viu)[ap], iv = G(P.viv)[ap];
        const float eru = G(P.er32)[iu], erv = G(P.er32)[iv], href = eru * erv;
        const Mono m = mono_of(u, v);
        const int su = __builtin_amdgcn_readfirstlane(u > 0.0f ? 1 : 0);
        const int sv = __builtin_amdgcn_readfirstlane(v > 0.0f ? 1 : 0);
        // downwind (o) and upwind (i) faces of this quadrant, and their records
        const int fxo = su ? 1 : 0, fxi = 1 - fxo, fyo = sv ? 3 : 2, fyi = 5 - fyo;
        const float *bxo = su ? rxe : rxw, *bxi = su ? rxw : rxe, *byo = sv ? ryn : rys, *byi = sv ? rys : ryn;
        const long oU = su ? -sx : sx, oV = sv ? -sy : sy;
        const float dxo = su ? dxe : dxw, dyo = sv ? dye : dyw;
        const float dxi = su ? dxiW : dxiE, dyi = sv ? dyiS : dyiN;
        const float rUm = su ? rx0 : rx2, rUp = su ? rx1 : rx3, rVm = sv ? ry0 : ry2, rVp = sv ? ry1 : ry3;
        // |u| rdx, |v| rdy: the divergence is |u| (g_downwind - g_upwind) / dx + ...
        const float aur = fabsf(u) * rdx, avr = fabsf(v) * rdy;
        float hk[NT], bk[NT], dh[NT], db[NT];
        const long e0 = (long)c * NT * P.ls + ap;
        struct Lv {
            float hc, bc, hW, bW, hE, bE, hS, bS, hN, bN, hUF, bUF, hUs, bUs, hUn, bUn, hVF, bVF, hVw, bVw, hVe, bVe;
        };
        auto ld_level = [&](int n) {
            Lv L;
            const gptr<const float> hp = G(h + e0 + (long)n * P.ls), bp = G(b + e0 + (long)n * P.ls);
            L.hc = hp[0];
            L.bc = bp[0];
            L.hW = hp[-sx];
            L.bW = bp[-sx];
            L.hE = hp[sx];
            L.bE = bp[sx];
            L.hS = hp[-sy];
            L.bS = bp[-sy];
            L.hN = hp[sy];
            L.bN = bp[sy];
            L.hUF = hp[2 * oU];
            L.bUF = bp[2 * oU];
            L.hUs = hp[oU - sy];
            L.bUs = bp[oU - sy];
            L.hUn = hp[oU + sy];
            L.bUn = bp[oU + sy];
            L.hVF = hp[2 * oV];
            L.bVF = bp[2 * oV];
            L.hVw = hp[oV - sx];
            L.bVw = bp[oV - sx];
            L.hVe = hp[oV + sx];
            L.bVe = bp[oV + sx];
            return L;
        };
        // the next level's stencil is loaded before this level's arithmetic
        Lv nxt = ld_level(0);
#pragma unroll
        for (int n = 0; n < NT; n++) {
            const Lv L = nxt;
            if (n + 1 < NT) nxt = ld_level(n + 1);
            hk[n] = L.hc;
            bk[n] = L.bc;
            const float sxh = vanleer_f((L.hc - L.hW) * rx1, (L.hE - L.hc) * rx2);
            const float sxb = vanleer_f((L.bc - L.bW) * rx1, (L.bE - L.bc) * rx2);
            const float syh = vanleer_f((L.hc - L.hS) * ry1, (L.hN - L.hc) * ry2);
            const float syb = vanleer_f((L.bc - L.bS) * ry1, (L.bN - L.bc) * ry2);
            const float sh = fmaf(u, sxh, v * syh), sb = fmaf(u, sxb, v * syb);
            // upwind x-neighbour U: its x-slope from (U-1, U, U+1); for su the far value is U-1 and c is U+1
            const float hU = su ? L.hW : L.hE, bU = su ? L.bW : L.bE;
            const float xm_h = su ? L.hUF : L.hc, xp_h = su ? L.hc : L.hUF;
            const float xm_b = su ? L.bUF : L.bc, xp_b = su ? L.bc : L.bUF;
            const float sxhU = vanleer_f((hU - xm_h) * rUm, (xp_h - hU) * rUp);
            const float sxbU = vanleer_f((bU - xm_b) * rUm, (xp_b - bU) * rUp);
            const float syhU = vanleer_f((hU - L.hUs) * ry1, (L.hUn - hU) * ry2);
            const float sybU = vanleer_f((bU - L.bUs) * ry1, (L.bUn - bU) * ry2);
            const float hV = sv ? L.hS : L.hN, bV = sv ? L.bS : L.bN;
            const float ym_h = sv ? L.hVF : L.hc, yp_h = sv ? L.hc : L.hVF;
            const float ym_b = sv ? L.bVF : L.bc, yp_b = sv ? L.bc : L.bVF;
            const float syhV = vanleer_f((hV - ym_h) * rVm, (yp_h - hV) * rVp);
            const float sybV = vanleer_f((bV - ym_b) * rVm, (yp_b - bV) * rVp);
            const float sxhV = vanleer_f((hV - L.hVw) * rx1, (L.hVe - hV) * rx2);
            const float sxbV = vanleer_f((bV - L.bVw) * rx1, (L.bVe - bV) * rx2);
            const float *tbx = tabf + (fxo * NT + n) * 3 * M, *tbxi = tabf + (fxi * NT + n) * 3 * M;
            const float *tby = tabf + (fyo * NT + n) * 3 * M, *tbyi = tabf + (fyi * NT + n) * 3 * M;
            cfloat *rxo = wave_uniform_f(bxo + n * REC32 + REC32_SIDEW * su);
            cfloat *rxi = wave_uniform_f(bxi + n * REC32 + REC32_SIDEW * su);
            cfloat *ryo = wave_uniform_f(byo + n * REC32 + REC32_SIDEW * sv);
            cfloat *ryi = wave_uniform_f(byi + n * REC32 + REC32_SIDEW * sv);
            float gxo_h, gxo_b, gxi_h, gxi_b, gyo_h, gyo_b, gyi_h, gyi_b;
            face_g(rxo, m, eru, erv, href, tbx[iu], tbx[(1 + su) * M + iv], fmaf(sxh, dxo, L.hc),
                   fmaf(sxb, dxo, L.bc), sh, sb, gxo_h, gxo_b);
            face_g(ryo, m, erv, eru, href, tby[iv], tby[(1 + sv) * M + iu], fmaf(syh, dyo, L.hc),
                   fmaf(syb, dyo, L.bc), sh, sb, gyo_h, gyo_b);
            face_g(rxi, m, eru, erv, href, tbxi[iu], tbxi[(1 + su) * M + iv], fmaf(sxhU, dxi, hU),
                   fmaf(sxbU, dxi, bU), fmaf(u, sxhU, v * syhU), fmaf(u, sxbU, v * sybU), gxi_h, gxi_b);
            face_g(ryi, m, erv, eru, href, tbyi[iv], tbyi[(1 + sv) * M + iu], fmaf(syhV, dyi, hV),
                   fmaf(sybV, dyi, bV), fmaf(u, sxhV, v * syhV), fmaf(u, sxbV, v * sybV), gyi_h, gyi_b);
            dh[n] = fmaf(aur, gxo_h - gxi_h, avr * (gyo_h - gyi_h));
            db[n] = fmaf(aur, gxo_b - gxi_b, avr * (gyo_b - gyi_b));
            __builtin_amdgcn_sched_barrier(0);
        }
        collide_store_m<NT>(P, cc, ctab, dG, dgw, m, eru, erv, href, iu, iv, hk, bk, dh, db, hn, bn, e0);
    }
}

// Cells within two of a wall in the mixed form: update_bnd_cell in FP32, with
// one-sided wall slopes and the diffuse-wall inflow (the wall side of a wall
// face has c4 = c5 = 0 in its record, so its face value does not enter).
template <int NT>
__device__ inline void update_bnd_cell_m(const Params &P, const float *__restrict__ h, const float *__restrict__ b,
                                         const double *__restrict__ recx, const double *__restrict__ recy,
                                         const double *__restrict__ crec, const double *__restrict__ dtc,
                                         float *__restrict__ hn, float *__restrict__ bn, double *__restrict__ Wn,
                                         int c)
{
    extern __shared__ float tabf[];
    const int M = P.M, nx = P.nx, ny = P.ny;
    const int i = c % nx, j = c / nx;
    scale_w<NT>(P, Wn, c);
    const long fw = (long)(j * (nx + 1) + i) * NT, fe = fw + NT, fs = (long)(j * nx + i) * NT,
               fn = (long)((j + 1) * nx + i) * NT;
    const gptr<const double> fr[4] = {G(recx) + fw * REC, G(recx) + fe * REC, G(recy) + fs * REC, G(recy) + fn * REC};
    build_tables_m<NT>(P, fr, G(crec) + (long)c * NT * CREC, tabf);
    __syncthreads();
    const float *ctab = tabf + 12 * NT * M;
    const long sx = (long)NT * P.ls, sy = (long)nx * NT * P.ls;
    const double dGd = dtc[c];
    const float dG = static_cast<float>(dGd), dgw = static_cast<float>(dGd * P.omega);
    const float rdx = static_cast<float>(G(P.rdx)[i]), rdy = static_cast<float>(G(P.rdy)[j]);
    const gptr<const double> xf = G(P.xf), xc = G(P.xc), yf = G(P.yf), yc = G(P.yc);
    const float dxe = xf[i + 1] - xc[i], dxw = xf[i] - xc[i];
    const float dyn = yf[j + 1] - yc[j], dys = yf[j] - yc[j];
    // stencil offsets clamped to the cell itself at the walls: every load is
    // unconditional (the one-sided slopes never read a clamped value)
    const int mx = wall_mode(i, nx), my = wall_mode(j, ny);
    const long oW = mx == 1 ? 0 : -sx, oE = mx == 2 ? 0 : sx, oS = my == 1 ? 0 : -sy, oN = my == 2 ? 0 : sy;
    const float rxm = G(P.rcx)[i], rxp = G(P.rcx)[i + 1], rym = G(P.rcy)[j], ryp = G(P.rcy)[j + 1];
    cfloat *cc = wave_uniform_f(P.cr32 + (long)c * NT * CREC32);
    const float *rxw = P.rx32 + fw * REC32, *rxe = P.rx32 + fe * REC32, *rys = P.ry32 + fs * REC32,
                *ryn = P.ry32 + fn * REC32;

    for (int ap = threadIdx.x; ap < P.nvp; ap += blockDim.x) {
        const int r = ap % P.Qp;
        if (r >= P.Q) continue;
        const float u = static_cast<float>(G(P.vu)[ap]), v = static_cast<float>(G(P.vv)[ap]);
        const int iu = G(P.viu)[ap], iv = G(P.viv)[ap];
        const float eru = G(P.er32)[iu], erv = G(P.er32)[iv], href = eru * erv;
        const Mono m = mono_of(u, v);
        const int su = __builtin_amdgcn_readfirstlane(u > 0.0f ? 1 : 0);
        const int sv = __builtin_amdgcn_readfirstlane(v > 0.0f ? 1 : 0);
        const int fxo = su ? 1 : 0, fxi = su ? 0 : 1;
        const int fyo = sv ? 3 : 2, fyi = sv ? 2 : 3;
        const float *bxo = su ? rxe : rxw, *bxi = su ? rxw : rxe, *byo = sv ? ryn : rys, *byi = sv ? rys : ryn;
        const bool inx_wall = su ? (i == 0) : (i == nx - 1);
        const bool iny_wall = sv ? (j == 0) : (j == ny - 1);
        const int iU = su ? i - 1 : i + 1, jV = sv ? j - 1 : j + 1;
        const long oU = su ? -sx : sx, oV = sv ? -sy : sy;
        const float dxo = su ? dxe : dxw, dyo = sv ? dyn : dys;
        const float dxi = inx_wall ? 0.0f : static_cast<float>(su ? xf[i] - xc[iU] : xf[i + 1] - xc[iU]);
        const float dyi = iny_wall ? 0.0f : static_cast<float>(sv ? yf[j] - yc[jV] : yf[j + 1] - yc[jV]);
        // upwind neighbours U (x) and V (y), the cell itself where the wall is upwind
        const int iUc = inx_wall ? i : iU, jVc = iny_wall ? j : jV;
        const long oUc = inx_wall ? 0 : oU, oVc = iny_wall ? 0 : oV;
        const int mUx = wall_mode(iUc, nx), mVy = wall_mode(jVc, ny);
        const long oUF = (su ? mUx == 1 : mUx == 2) ? 0 : oU;  // far neighbour of U, relative to U
        const long oVF = (sv ? mVy == 1 : mVy == 2) ? 0 : oV;  // far neighbour of V, relative to V
        const float rUm = G(P.rcx)[iUc], rUp = G(P.rcx)[iUc + 1], rVm = G(P.rcy)[jVc], rVp = G(P.rcy)[jVc + 1];
        const float aur = fabsf(u) * rdx, avr = fabsf(v) * rdy;
        float hk[NT], bk[NT], dh[NT], db[NT];
        const long e0 = (long)c * NT * P.ls + ap;
        struct Lv {
            float hc, bc, hW, bW, hE, bE, hS, bS, hN, bN, hUF, bUF, hUs, bUs, hUn, bUn, hVF, bVF, hVw, bVw, hVe, bVe;
        };
        auto ld_level = [&](int n) {
            Lv L;
            const gptr<const float> hp = G(h + e0 + (long)n * P.ls), bp = G(b + e0 + (long)n * P.ls);
            L.hc = hp[0];
            L.bc = bp[0];
            L.hW = hp[oW];
            L.bW = bp[oW];
            L.hE = hp[oE];
            L.bE = bp[oE];
            L.hS = hp[oS];
            L.bS = bp[oS];
            L.hN = hp[oN];
            L.bN = bp[oN];
            L.hUF = hp[oUc + oUF];
            L.bUF = bp[oUc + oUF];
            L.hUs = hp[oUc + oS];
            L.bUs = bp[oUc + oS];
            L.hUn = hp[oUc + oN];
            L.bUn = bp[oUc + oN];
            L.hVF = hp[oVc + oVF];
            L.bVF = bp[oVc + oVF];
            L.hVw = hp[oVc + oW];
            L.bVw = bp[oVc + oW];
            L.hVe = hp[oVc + oE];
            L.bVe = bp[oVc + oE];
            return L;
        };
        Lv nxt = ld_level(0);
        constexpr int UNR = NT <= 3 ? NT : 1;
#pragma unroll UNR
        for (int n = 0; n < NT; n++) {
            const Lv L = nxt;
            if (n + 1 < NT) nxt = ld_level(n + 1);
            const float hc = L.hc, bc = L.bc;
            hk[n] = hc;
            bk[n] = bc;
            const float sxh = slope_cf(L.hW, hc, L.hE, mx, rxm, rxp), sxb = slope_cf(L.bW, bc, L.bE, mx, rxm, rxp);
            const float syh = slope_cf(L.hS, hc, L.hN, my, rym, ryp), syb = slope_cf(L.bS, bc, L.bN, my, rym, ryp);
            const float sh = fmaf(u, sxh, v * syh), sb = fmaf(u, sxb, v * syb);
            const float *tbx = tabf + (fxo * NT + n) * 3 * M, *tbxi = tabf + (fxi * NT + n) * 3 * M;
            const float *tby = tabf + (fyo * NT + n) * 3 * M, *tbyi = tabf + (fyi * NT + n) * 3 * M;
            cfloat *rxo = wave_uniform_f(bxo + n * REC32 + REC32_SIDEW * su);
            cfloat *rxi = wave_uniform_f(bxi + n * REC32 + REC32_SIDEW * su);
            cfloat *ryo = wave_uniform_f(byo + n * REC32 + REC32_SIDEW * sv);
            cfloat *ryi = wave_uniform_f(byi + n * REC32 + REC32_SIDEW * sv);
            float gxo_h, gxo_b, gxi_h, gxi_b, gyo_h, gyo_b, gyi_h, gyi_b;
            face_g(rxo, m, eru, erv, href, tbx[iu], tbx[(1 + su) * M + iv], fmaf(sxh, dxo, hc), fmaf(sxb, dxo, bc),
                   sh, sb, gxo_h, gxo_b);
            face_g(ryo, m, erv, eru, href, tby[iv], tby[(1 + sv) * M + iu], fmaf(syh, dyo, hc), fmaf(syb, dyo, bc),
                   sh, sb, gyo_h, gyo_b);
            if (inx_wall) {
                face_g(rxi, m, eru, erv, href, tbxi[iu], tbxi[(1 + su) * M + iv], 0.0f, 0.0f, 0.0f, 0.0f, gxi_h,
                       gxi_b);
            } else {
                const float hU = su ? L.hW : L.hE, bU = su ? L.bW : L.bE;
                const float sxhU = su ? slope_cf(L.hUF, hU, hc, mUx, rUm, rUp) : slope_cf(hc, hU, L.hUF, mUx, rUm, rUp);
                const float sxbU = su ? slope_cf(L.bUF, bU, bc, mUx, rUm, rUp) : slope_cf(bc, bU, L.bUF, mUx, rUm, rUp);
                const float syhU = slope_cf(L.hUs, hU, L.hUn, my, rym, ryp);
                const float sybU = slope_cf(L.bUs, bU, L.bUn, my, rym, ryp);
                face_g(rxi, m, eru, erv, href, tbxi[iu], tbxi[(1 + su) * M + iv], fmaf(sxhU, dxi, hU),
                       fmaf(sxbU, dxi, bU), fmaf(u, sxhU, v * syhU), fmaf(u, sxbU, v * sybU), gxi_h, gxi_b);
            }
            if (iny_wall) {
                face_g(ryi, m, erv, eru, href, tbyi[iv], tbyi[(1 + sv) * M + iu], 0.0f, 0.0f, 0.0f, 0.0f, gyi_h,
                       gyi_b);
            } else {
                const float hV = sv ? L.hS : L.hN, bV = sv ? L.bS : L.bN;
                const float syhV = sv ? slope_cf(L.hVF, hV, hc, mVy, rVm, rVp) : slope_cf(hc, hV, L.hVF, mVy, rVm, rVp);
                const float sybV = sv ? slope_cf(L.bVF, bV, bc, mVy, rVm, rVp) : slope_cf(bc, bV, L.bVF, mVy, rVm, rVp);
                const float sxhV = slope_cf(L.hVw, hV, L.hVe, mx, rxm, rxp);
                const float sxbV = slope_cf(L.bVw, bV, L.bVe, mx, rxm, rxp);
                face_g(ryi, m, erv, eru, href, tbyi[iv], tbyi[(1 + sv) * M + iu], fmaf(syhV, dyi, hV),
                       fmaf(sybV, dyi, bV), fmaf(u, sxhV, v * syhV), fmaf(u, sxbV, v * sybV), gyi_h, gyi_b);
            }
            dh[n] = fmaf(aur, gxo_h - gxi_h, avr * (gyo_h - gyi_h));
            db[n] = fmaf(aur, gxo_b - gxi_b, avr * (gyo_b - gyi_b));
            __builtin_amdgcn_sched_barrier(0);
        }
        collide_store_m<NT>(P, cc, ctab, dG, dgw, m, eru, erv, href, iu, iv, hk, bk, dh, db, hn, bn, e0);
    }
}

}  // namespace hb
