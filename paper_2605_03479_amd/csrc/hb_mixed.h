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
    const int M = P.Mt, ftab = 12 * NT * M;
    for (int t = threadIdx.x; t < 16 * NT * M; t += blockDim.x) {
        const int k = t % M;
        bool onv;  // the row runs over the v nodes
        int which, n, fs = 0;
        if (t < ftab) {
            which = (t / M) % 3;
            const int fn = t / (3 * M);
            n = fn % NT;
            fs = fn / NT;
            onv = (fs >= 2) == (which == 0);  // x-faces: normal u, tangential v; y-faces the reverse
        } else {
            which = ((t - ftab) / M) % 4;
            n = (t - ftab) / (4 * M);
            onv = which & 1;
        }
        if (k >= (onv ? P.Mv : P.M)) {
            tab[t] = 0.0f;  // stride padding of the shorter axis, never read
            continue;
        }
        const double x = onv ? G(P.v1)[k] : G(P.u1)[k];
        double lam, U;
        if (t < ftab) {
            const gptr<const double> sd =
                fr[fs] + n * REC + REC_SIDE + REC_SIDEW * (which == 0 ? (x > 0.0 ? 1 : 0) : which - 1);
            lam = sd[0];
            U = which == 0 ? sd[1] : sd[2];
        } else {
            const gptr<const double> cc = cr + n * CREC + (which >= 2 ? CREC_T : 0);
            lam = cc[0];
            U = (which & 1) ? cc[2] : cc[1];
        }
        tab[t] = static_cast<float>(exp(-lam * (x - U) * (x - U)) - (onv ? G(P.ex64v)[k] : G(P.ex64)[k]));
    }
}

// Spectral source and semi-implicit collision (Eq. 30) for one velocity at all
// levels in FP32, then the store of the deviations of h^{k+1}, b^{k+1} times
// the level-mass factor s_n: s_n (H_ref + d) - H_ref = s_n d + (s_n - 1) H_ref.
template <int NT, int OUT>
__device__ inline void collide_store_m(const Params &P, cfloat *cc, const float *ctab, float dG, float dgw,
                                       const Mono &m, float eru, float erv, float href, int iu, int iv,
                                       const float *hk, const float *bk, const float *dh, const float *db,
                                       float *__restrict__ hn, float *__restrict__ bn, long cb, int ap)
{
    // the cell's block of the outputs (cb: its first word), the lane's velocity ap
    const OutStore<OUT> out(hn, bn, cb, ap);
    const int M = P.Mt;  // table row stride
    const float kh = P.K - 5.0f;
    cfloat *ls = wave_uniform_f(P.lscale32);
#pragma unroll
    for (int n = 0; n < NT; n++) {
        // E of Eq. (17) is circulant with a zero diagonal: E_nm = e_d for
        // d = (n - m) mod N_T, e_d = E_d0, so the sum takes N_T - 1 wave-uniform
        // coefficients
        float Eh = 0.0f, Eb = 0.0f;
#pragma unroll
        for (int d = 1; d < NT; d++) {
            const int mm = (n - d + NT) % NT;
            Eh = fmaf(P.Ef[d * NT], hk[mm], Eh);
            Eb = fmaf(P.Ef[d * NT], bk[mm], Eb);
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
        out.put(n * P.ls, fmaf(sn, hnum * rden, sm * href), fmaf(sn, bnum * rden, sm * (0.5f * P.K) * href));
    }
}

// Moments of the mixed form (the sums of the moments kernel, Sec. 2.2).  The
// FEED sums are linear in the reconstructed face values h0 = h_c + sigma d, so
// each quadrant's sums split into sums over its velocities of the ten
// monomials w u^a v^b (a + b <= 3) times the stored deviation, times its x
// slope and times its y slope, plus the rest Maxwellian's share (the same for
// every cell: P.rmom).  The slopes of h equal the slopes of its deviation
// (H_ref is the same in every cell) and are taken in FP32 like the update's.
// The monomials multiply deviations only, so they are formed from the
// velocities rounded to FP32 (a relative error of 2^-24 of the deviation sums,
// the size of the deviations' own storage rounding; the rest share uses the
// FP64 velocities); every product and sum is FP64.  Per lane and level 41 sums:
//   S[0..9]   w m_k dh      S[10..19] w m_k sx_h    S[20..29] w m_k sy_h
//   S[30..32] w m_k db      S[33..35] w m_k sx_b    S[36..38] w m_k sy_b  (k < 3)
//   S[39]     w u (r^2 s_h + s_b)     S[40] w v (r^2 s_h + s_b)
// with s = u sx + v sy and r^2 = u^2 + v^2; the 55 per-quadrant rows of the
// FP64 form follow from them (mom_row).
constexpr int NMOM_M = 41;

// Row k (0..54) of quadrant q's sums in the layout of the FP64 moments kernel
// from the 41 reduced sums S, the rest shares R (10) and the face distances.
__device__ inline double mom_row(const double *S, const double *R, double kb, double dxo, double dyo, int k)
{
    if (k < 10) return (S[k] + dxo * S[10 + k]) + R[k];
    if (k < 13) return (S[30 + k - 10] + dxo * S[33 + k - 10]) + kb * R[k - 10];
    if (k < 16) return S[20 + k - 13];
    if (k == 16) return 0.5 * ((S[23] + S[25]) + S[36]);
    if (k == 17) return S[13] + S[24];
    if (k == 18) return S[16] + S[27];
    if (k == 19) return S[17] + S[28];
    if (k == 20) return 0.5 * S[39];
    if (k < 31) return (S[k - 21] + dyo * S[20 + k - 21]) + R[k - 21];
    if (k < 34) return (S[30 + k - 31] + dyo * S[36 + k - 31]) + kb * R[k - 31];
    if (k < 37) return S[10 + k - 34];
    if (k == 37) return 0.5 * ((S[13] + S[15]) + S[33]);
    if (k == 38) return S[14] + S[25];
    if (k == 39) return S[17] + S[28];
    if (k == 40) return S[18] + S[29];
    if (k == 41) return 0.5 * S[40];
    if (k < 52) return S[k - 42] + R[k - 42];
    return S[30 + k - 52] + kb * R[k - 52];
}

__device__ inline void moments_cell_m(const Params &P, const float *__restrict__ h, const float *__restrict__ b,
                                      double *__restrict__ feed, int c)
{
    // LDS rows per reduction pass: 14 (three passes), 31 KB per block, so that
    // four blocks fit a CU's 160 KB of LDS (the kernel runs four waves per SIMD)
    constexpr int RPP = 14, NPASS = (NMOM_M + RPP - 1) / RPP;
    __shared__ double red[4][RPP * K1_ROW];
    __shared__ double wsum[4][NMOM_M];
    const int i = c % P.nx, j = c / P.nx;
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int NT = P.NT;
    const long sx = (long)NT * P.ls, sy = (long)P.nx * NT * P.ls;
    // neighbour offsets clamped to the cell itself at the walls (the one-sided
    // slope there does not read them)
    const int mx = wall_mode(i, P.nx), my = wall_mode(j, P.ny);
    const long oW = mx == 1 ? 0 : -sx, oE = mx == 2 ? 0 : sx, oS = my == 1 ? 0 : -sy, oN = my == 2 ? 0 : sy;
    const float rxm = G(P.rcx)[i], rxp = G(P.rcx)[i + 1], rym = G(P.rcy)[j], ryp = G(P.rcy)[j + 1];
    const int nch = P.Qp / 64;
    const float *vu = P.vel32, *vv = P.vel32 + P.nvp, *vw = P.vel32 + 2 * (long)P.nvp;
    // One lane's stencil and velocity for (level n, chunk ch).  (Loading the
    // next pair ahead needs registers the four waves per SIMD do not leave:
    // it spills and measured slower.)
    struct Ld {
        float u, v, w, hc, bc, hW, bW, hE, bE, hS, bS, hN, bN;
    };
    auto load = [&](int n, int ch) {
        Ld d;
        const int ap = q * P.Qp + lane + 64 * ch;
        d.u = vu[ap];
        d.v = vv[ap];
        d.w = vw[ap];
        const long e = ((long)c * NT + n) * P.ls + ap;
        const gptr<const float> hp = G(h + e), bp = G(b + e);
        d.hc = hp[0];
        d.bc = bp[0];
        d.hW = hp[oW];
        d.bW = bp[oW];
        d.hE = hp[oE];
        d.bE = bp[oE];
        d.hS = hp[oS];
        d.bS = bp[oS];
        d.hN = hp[oN];
        d.bN = bp[oN];
        return d;
    };
    // interior cells (limited slopes both ways) take a copy of the loop
    // without the wall cases' branches
    const bool inner = mx == 0 && my == 0;

    for (int n = 0; n < NT; n++) {
        double S[NMOM_M];
#pragma unroll
        for (int k = 0; k < NMOM_M; k++) S[k] = 0.0;
        auto body = [&](int ch, auto interior) {
            const Ld d = load(n, ch);

            const float hc = d.hc, bc = d.bc;
            double sxh, sxb, syh, syb;
            if constexpr (decltype(interior)::value) {
                sxh = vanleer_f((hc - d.hW) * rxm, (d.hE - hc) * rxp);
                sxb = vanleer_f((bc - d.bW) * rxm, (d.bE - bc) * rxp);
                syh = vanleer_f((hc - d.hS) * rym, (d.hN - hc) * ryp);
                syb = vanleer_f((bc - d.bS) * rym, (d.bN - bc) * ryp);
            } else {
                sxh = slope_cf(d.hW, hc, d.hE, mx, rxm, rxp);
                sxb = slope_cf(d.bW, bc, d.bE, mx, rxm, rxp);
                syh = slope_cf(d.hS, hc, d.hN, my, rym, ryp);
                syb = slope_cf(d.bS, bc, d.bN, my, rym, ryp);
            }
            const double u = d.u, v = d.v, w = d.w;
            const double dh = hc, db = bc;
            const double uu = u * u, uv = u * v, vv2 = v * v;
            const double wm[10] = {w, w * u, w * v, w * uu, w * uv, w * vv2, w * uu * u, w * uu * v, w * u * vv2,
                                   w * vv2 * v};
#pragma unroll
            for (int k = 0; k < 10; k++) {
                S[k] += wm[k] * dh;
                S[10 + k] += wm[k] * sxh;
                S[20 + k] += wm[k] * syh;
            }
#pragma unroll
            for (int k = 0; k < 3; k++) {
                S[30 + k] += wm[k] * db;
                S[33 + k] += wm[k] * sxb;
                S[36 + k] += wm[k] * syb;
            }
            const double t = (uu + vv2) * (u * sxh + v * syh) + (u * sxb + v * syb);
            S[39] += wm[1] * t;
            S[40] += wm[2] * t;
        };
        if (inner)
            for (int ch = 0; ch < nch; ch++) body(ch, std::true_type{});
        else
            for (int ch = 0; ch < nch; ch++) body(ch, std::false_type{});
        // wave reduction through LDS as in the FP64 kernel: RPP rows per pass,
        // two lanes per row; the wave writes and reads only its own rows
        double *rb = red[q];
#pragma unroll
        for (int half = 0; half < NPASS; half++) {
            const int k0 = half * RPP, kn = NMOM_M - k0 < RPP ? NMOM_M - k0 : RPP;
#pragma unroll
            for (int k = 0; k < RPP; k++)
                if (k < kn) rb[k * K1_ROW + lane] = S[k0 + k];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int rk = lane & 31;
            double part = 0.0;
            if (rk < kn) {
                const double2 *row = reinterpret_cast<const double2 *>(rb + rk * K1_ROW + (lane & 32));
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
                for (int l = 0; l < 16; l += 2) {
                    const double2 x0 = row[l], x1 = row[l + 1];
                    s0 += x0.x;
                    s1 += x0.y;
                    s2 += x1.x;
                    s3 += x1.y;
                }
                part = (s0 + s1) + (s2 + s3);
            }
            const double other = __shfl_down(part, 32);
            if (lane < kn) wsum[q][k0 + lane] = part + other;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // quadrant rows, then the faces: E = q1 + q3, W = q0 + q2, N = q2 + q3,
        // S = q0 + q1, cell moments over all four
        const double kb = 0.5 * P.K;
        const double dxe = G(P.xf)[i + 1] - G(P.xc)[i], dxw = G(P.xf)[i] - G(P.xc)[i];
        const double dyn = G(P.yf)[j + 1] - G(P.yc)[j], dys = G(P.yf)[j] - G(P.yc)[j];
        auto row = [&](int qq, int k) {
            return mom_row(wsum[qq], P.rmom + 10 * qq, kb, (qq & 1) ? dxe : dxw, (qq & 2) ? dyn : dys, k);
        };
        const gptr<double> out = G(feed) + ((long)c * NT + n) * FEED;
        for (int t = threadIdx.x; t < FEED; t += blockDim.x) {
            double val;
            if (t < 21) val = row(1, t) + row(3, t);
            else if (t < 42) val = row(0, t - 21) + row(2, t - 21);
            else if (t < 63) val = row(2, t - 42 + 21) + row(3, t - 42 + 21);
            else if (t < 84) val = row(0, t - 63 + 21) + row(1, t - 63 + 21);
            else val = ((row(0, t - 84 + 42) + row(1, t - 84 + 42)) + row(2, t - 84 + 42)) + row(3, t - 84 + 42);
            out[t] = val;
        }
        __syncthreads();
    }
}

// van Leer slope of the differences d1 = f_i - f_{i-1}, d2 = f_{i+1} - f_i with
// reciprocal centre distances r1, r2, divided by 2 r1 r2 (the caller folds
// that constant into the slope's uses): d1 d2 / (r1 d1 + r2 d2) for d1 d2 > 0.
__device__ inline float vlslope(float d1, float d2, float r1, float r2)
{
    const float p = d1 * d2;
    const float q = p * __builtin_amdgcn_rcpf(fmaf(r1, d1, r2 * d2));
    return p > 0.0f ? q : 0.0f;
}

// Interior cell (2 <= i <= nx-3, 2 <= j <= ny-3) of the mixed form: the
// straight-line stencil of update_int_cell in FP32.  The stencil is read with
// buffer loads (one descriptor per array at the cell's lowest stencil element,
// the velocity as the lane offset, level and neighbour as a wave-uniform
// offset).  The upwind neighbour U's limited slope is taken on the differences
// away from the cell, dA = f_U - f_UU and dB = f_c - f_U, whatever the
// quadrant: for u < 0 that negates both differences, so the slope changes sign
// and the sign goes into the constants that multiply it.
template <int NT, int OUT>
__device__ inline void update_int_cell_m(const Params &P, const float *__restrict__ h, const float *__restrict__ b,
                                         const double *__restrict__ recx, const double *__restrict__ recy,
                                         const double *__restrict__ crec, const double *__restrict__ dtc,
                                         float *__restrict__ hn, float *__restrict__ bn, double *__restrict__ Wn,
                                         int ci)
{
    extern __shared__ float tabf[];
    const int nxi = P.nx - 4;
    const int i = 2 + ci % nxi, j = 2 + ci / nxi;
    const int M = P.Mt, nx = P.nx;
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
    // the stencil of an interior cell reaches two rows down at most
    const long lo = (long)c * NT * P.ls - 2 * sy;
    const __amdgpu_buffer_rsrc_t rsh = uniform_rsrc(h + lo);
    const __amdgpu_buffer_rsrc_t rsb = uniform_rsrc(b + lo);
    // the folded van Leer constants 2 r1 r2 of the cell's own slopes
    const float kx = 2.0f * rx1 * rx2, ky = 2.0f * ry1 * ry2;

    for (int ap = threadIdx.x; ap < P.nvp; ap += blockDim.x) {
        const int r = ap % P.Qp;
        if (r >= P.Q) continue;
        const float u = static_cast<float>(G(P.vu)[ap]), v = static_cast<float>(G(P.vv)[ap]);
        const int iu = G(P.viu)[ap], iv = G(P.viv)[ap];
        const float eru = G(P.er32)[iu], erv = G(P.er32v)[iv], href = eru * erv;
        const Mono m = mono_of(u, v);
        const int su = __builtin_amdgcn_readfirstlane(u > 0.0f ? 1 : 0);
        const int sv = __builtin_amdgcn_readfirstlane(v > 0.0f ? 1 : 0);
        // downwind (o) and upwind (i) faces of this quadrant, and their records
        const int fxo = su ? 1 : 0, fxi = 1 - fxo, fyo = sv ? 3 : 2, fyi = 5 - fyo;
        const float *bxo = su ? rxe : rxw, *bxi = su ? rxw : rxe, *byo = sv ? ryn : rys, *byi = sv ? rys : ryn;
        const long oU = su ? -sx : sx, oV = sv ? -sy : sy;
        // reciprocal centre distances of U's far (UU to U) and near (U to c)
        // differences, and V's
        const float rUf = su ? rx0 : rx3, rUn = su ? rx1 : rx2, rVf = sv ? ry0 : ry3, rVn = sv ? ry1 : ry2;
        // slopes come as slope / (2 r1 r2); their uses take the factor, with
        // the upwind neighbours' sign
        const float kU = (su ? 2.0f : -2.0f) * rUf * rUn, kV = (sv ? 2.0f : -2.0f) * rVf * rVn;
        const float dxo = (su ? dxe : dxw) * kx, dyo = (sv ? dye : dyw) * ky;
        const float dxi = (su ? dxiW : dxiE) * kU, dyi = (sv ? dyiS : dyiN) * kV;
        const float ukx = u * kx, vky = v * ky, ukU = u * kU, vkV = v * kV;
        // |u| rdx, |v| rdy: the divergence is |u| (g_downwind - g_upwind) / dx + ...
        const float aur = fabsf(u) * rdx, avr = fabsf(v) * rdy;
        float hk[NT], bk[NT], dh[NT], db[NT];
        const unsigned vo = (unsigned)ap * 4u;
        struct Lv {
            float hc, bc, hW, bW, hE, bE, hS, bS, hN, bN, hUU, bUU, hUs, bUs, hUn, bUn, hVV, bVV, hVw, bVw, hVe, bVe;
        };
        auto ld_level = [=](int n) {
            Lv L;
            const int cn = (int)((long)n * P.ls + 2 * sy);
            auto at = [=](__amdgpu_buffer_rsrc_t rs, long off) -> float {
                return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (int)((cn + off) * 4), 0));
            };
            L.hc = at(rsh, 0);
            L.bc = at(rsb, 0);
            L.hW = at(rsh, -sx);
            L.bW = at(rsb, -sx);
            L.hE = at(rsh, sx);
            L.bE = at(rsb, sx);
            L.hS = at(rsh, -sy);
            L.bS = at(rsb, -sy);
            L.hN = at(rsh, sy);
            L.bN = at(rsb, sy);
            L.hUU = at(rsh, 2 * oU);
            L.bUU = at(rsb, 2 * oU);
            L.hUs = at(rsh, oU - sy);
            L.bUs = at(rsb, oU - sy);
            L.hUn = at(rsh, oU + sy);
            L.bUn = at(rsb, oU + sy);
            L.hVV = at(rsh, 2 * oV);
            L.bVV = at(rsb, 2 * oV);
            L.hVw = at(rsh, oV - sx);
            L.bVw = at(rsb, oV - sx);
            L.hVe = at(rsh, oV + sx);
            L.bVe = at(rsb, oV + sx);
            return L;
        };
#pragma unroll
        for (int n = 0; n < NT; n++) {
            const Lv L = ld_level(n);
            hk[n] = L.hc;
            bk[n] = L.bc;
            const float sxh = vlslope(L.hc - L.hW, L.hE - L.hc, rx1, rx2);
            const float sxb = vlslope(L.bc - L.bW, L.bE - L.bc, rx1, rx2);
            const float syh = vlslope(L.hc - L.hS, L.hN - L.hc, ry1, ry2);
            const float syb = vlslope(L.bc - L.bS, L.bN - L.bc, ry1, ry2);
            const float sh = fmaf(ukx, sxh, vky * syh), sb = fmaf(ukx, sxb, vky * syb);
            const float hU = su ? L.hW : L.hE, bU = su ? L.bW : L.bE, hV = sv ? L.hS : L.hN, bV = sv ? L.bS : L.bN;
            const float sxhU = vlslope(hU - L.hUU, L.hc - hU, rUf, rUn);
            const float sxbU = vlslope(bU - L.bUU, L.bc - bU, rUf, rUn);
            const float syhU = vlslope(hU - L.hUs, L.hUn - hU, ry1, ry2);
            const float sybU = vlslope(bU - L.bUs, L.bUn - bU, ry1, ry2);
            const float syhV = vlslope(hV - L.hVV, L.hc - hV, rVf, rVn);
            const float sybV = vlslope(bV - L.bVV, L.bc - bV, rVf, rVn);
            const float sxhV = vlslope(hV - L.hVw, L.hVe - hV, rx1, rx2);
            const float sxbV = vlslope(bV - L.bVw, L.bVe - bV, rx1, rx2);
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
                   fmaf(sxbU, dxi, bU), fmaf(ukU, sxhU, vky * syhU), fmaf(ukU, sxbU, vky * sybU), gxi_h, gxi_b);
            face_g(ryi, m, erv, eru, href, tbyi[iv], tbyi[(1 + sv) * M + iu], fmaf(syhV, dyi, hV),
                   fmaf(sybV, dyi, bV), fmaf(ukx, sxhV, vkV * syhV), fmaf(ukx, sxbV, vkV * sybV), gyi_h, gyi_b);
            dh[n] = fmaf(aur, gxo_h - gxi_h, avr * (gyo_h - gyi_h));
            db[n] = fmaf(aur, gxo_b - gxi_b, avr * (gyo_b - gyi_b));
            // few levels: keep each level's loads and arithmetic together (the
            // scheduler's interleaving across levels measured slower there)
            if constexpr (NT <= 5) __builtin_amdgcn_sched_barrier(0);
        }
        collide_store_m<NT, OUT>(P, cc, ctab, dG, dgw, m, eru, erv, href, iu, iv, hk, bk, dh, db, hn, bn, (long)c * NT * P.ls, ap);
    }
}

// Cells within two of a wall in the mixed form: update_bnd_cell in FP32, with
// one-sided wall slopes and the diffuse-wall inflow (the wall side of a wall
// face has c4 = c5 = 0 in its record, so its face value does not enter).
template <int NT, int OUT>
__device__ inline void update_bnd_cell_m(const Params &P, const float *__restrict__ h, const float *__restrict__ b,
                                         const double *__restrict__ recx, const double *__restrict__ recy,
                                         const double *__restrict__ crec, const double *__restrict__ dtc,
                                         float *__restrict__ hn, float *__restrict__ bn, double *__restrict__ Wn,
                                         int c)
{
    extern __shared__ float tabf[];
    const int M = P.Mt, nx = P.nx, ny = P.ny;
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
    // buffer loads as in the interior update: one descriptor per array based
    // two rows below the cell (the lowest element a ring stencil can reach; the
    // descriptor's base may lie below the array, every address read is inside)
    const long lo = (long)c * NT * P.ls - 2 * sy;
    const __amdgpu_buffer_rsrc_t rsh = uniform_rsrc(h + lo);
    const __amdgpu_buffer_rsrc_t rsb = uniform_rsrc(b + lo);

    for (int ap = threadIdx.x; ap < P.nvp; ap += blockDim.x) {
        const int r = ap % P.Qp;
        if (r >= P.Q) continue;
        const float u = static_cast<float>(G(P.vu)[ap]), v = static_cast<float>(G(P.vv)[ap]);
        const int iu = G(P.viu)[ap], iv = G(P.viv)[ap];
        const float eru = G(P.er32)[iu], erv = G(P.er32v)[iv], href = eru * erv;
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
        const unsigned vo = (unsigned)ap * 4u;
        struct Lv {
            float hc, bc, hW, bW, hE, bE, hS, bS, hN, bN, hUF, bUF, hUs, bUs, hUn, bUn, hVF, bVF, hVw, bVw, hVe, bVe;
        };
        auto ld_level = [=](int n) {
            Lv L;
            const int cn = (int)((long)n * P.ls + 2 * sy);
            auto at = [=](__amdgpu_buffer_rsrc_t rs, long off) -> float {
                return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (int)((cn + off) * 4), 0));
            };
            L.hc = at(rsh, 0);
            L.bc = at(rsb, 0);
            L.hW = at(rsh, oW);
            L.bW = at(rsb, oW);
            L.hE = at(rsh, oE);
            L.bE = at(rsb, oE);
            L.hS = at(rsh, oS);
            L.bS = at(rsb, oS);
            L.hN = at(rsh, oN);
            L.bN = at(rsb, oN);
            L.hUF = at(rsh, oUc + oUF);
            L.bUF = at(rsb, oUc + oUF);
            L.hUs = at(rsh, oUc + oS);
            L.bUs = at(rsb, oUc + oS);
            L.hUn = at(rsh, oUc + oN);
            L.bUn = at(rsb, oUc + oN);
            L.hVF = at(rsh, oVc + oVF);
            L.bVF = at(rsb, oVc + oVF);
            L.hVw = at(rsh, oVc + oW);
            L.bVw = at(rsb, oVc + oW);
            L.hVe = at(rsh, oVc + oE);
            L.bVe = at(rsb, oVc + oE);
            return L;
        };
        constexpr int UNR = NT <= 3 ? NT : 1;
#pragma unroll UNR
        for (int n = 0; n < NT; n++) {
            const Lv L = ld_level(n);
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
        collide_store_m<NT, OUT>(P, cc, ctab, dG, dgw, m, eru, erv, href, iu, iv, hk, bk, dh, db, hn, bn, (long)c * NT * P.ls, ap);
    }
}

}  // namespace hb
