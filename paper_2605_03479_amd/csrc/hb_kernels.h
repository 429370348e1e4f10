// HIP kernels of one HB-UGKS pseudo step on gfx950 (FP64 form).
//
// Data layout (device):
//   h, b [cell][level][alpha']  alpha' = quadrant-major velocity order: each
//       quadrant (sign u, sign v) is a contiguous, 64-padded block, so every
//       wavefront holds velocities of one quadrant and all its lanes share the
//       upwind side of every face.  Adjacent lanes = adjacent velocities.
//   W    [cell][level][4]
//   feed [cell][level][FEED]   per-cell velocity moments for the faces it feeds
//   recx [x-face][level][REC], recy [y-face][level][REC]  face records
//   crec [cell][level][CREC]   equilibria of W^k and W^{k+1} for the collision
// Kernels per step: moments -> faces -> cells -> residual -> update.
#pragma once
#include "hb_device.h"
#include "hb_layout.h"

namespace hb {

// Block -> cell map that gives each XCD (blocks are dealt round-robin to the
// 8 XCDs) a contiguous range of cells, so stencil neighbours share its L2.
__device__ inline int xcd_cell(int b, int G)
{
    int x = b & 7, k = b >> 3;
    int per = G >> 3, rem = G & 7;
    return x * per + (x < rem ? x : rem) + k;
}

// Position p of a walk over an nx x ny grid in eight column strips (the
// first nx % 8 strips one column wider), each strip row by row -> row-major
// cell index.  Composed with xcd_cell, each XCD walks one strip down the
// grid, so the vertical stencil neighbours of a cell are revisited while they
// are still in that XCD's L2; in row-major order they are a whole row of
// cells apart.  The batched work lists use the same order.
__host__ __device__ inline int strip_cell(int p, int nx, int ny)
{
    const int q = nx >> 3, rem = nx & 7;
    const int big = rem * (q + 1) * ny;
    int w, c0, r;
    if (p < big) {
        const int s = p / ((q + 1) * ny);
        w = q + 1, c0 = s * (q + 1), r = p - s * (q + 1) * ny;
    } else {  // only reached when q > 0
        const int pp = p - big, s = pp / (q * ny);
        w = q, c0 = rem * (q + 1) + s * q, r = pp - s * q * ny;
    }
    return (r / w) * nx + c0 + r % w;
}

// Storage of (h, b): FP64 values, or FP32 deviations from the rest Maxwellian
// H_ref = exp(-|u|^2)/pi (B_ref = K/2 H_ref) for the mixed form.  All
// arithmetic below runs in FP64 either way.
template <typename TS, typename Ptr>
__device__ inline double ldv(Ptr p, long off, double ref)
{
    if constexpr (sizeof(TS) == 4) return static_cast<double>(G(p)[off]) + ref;
    else return G(p)[off];
}
template <typename TS, typename Ptr>
__device__ inline void stv(Ptr p, long off, double v, double ref)
{
    if constexpr (sizeof(TS) == 4) G(p)[off] = static_cast<float>(v - ref);
    else G(p)[off] = v;
}

// Buffer resource for raw loads and stores at a wave-uniform base (the first
// lane's address, moved to scalar registers)
template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t uniform_rsrc(T *p)
{
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)((static_cast<unsigned long long>(hi) << 32) | lo), 0, -1,
                                             0x00020000);
}

// How the mixed update writes h^{k+1}, b^{k+1} (a template parameter: the
// cache policy is an immediate of the store instruction).  OUT_NT: non-temporal
// stores, for a state larger than the last-level cache (Params::stream_out):
// the next pass cannot find it there, and cached stores would only evict the
// stencil the update is still reading.  OUT_BUF: stores through buffer
// resources at the cell's block (a wave-uniform base, the lane's velocity as
// the offset), which leaves the single-case kernels fewer address registers;
// the batched kernels, shorter of scalar registers, keep global stores.
enum : int { OUT_NT = 1, OUT_BUF = 2 };
template <int OUT, bool BUF = (OUT & OUT_BUF) != 0>
struct OutStore;
template <int OUT>
struct OutStore<OUT, true> {
    __amdgpu_buffer_rsrc_t rh, rb;
    unsigned vo;
    __device__ OutStore(float *hn, float *bn, long cb, int ap)
        : rh(uniform_rsrc(hn + cb)), rb(uniform_rsrc(bn + cb)), vo((unsigned)ap * 4u)
    {
    }
    // lw: the level's offset in words from the cell's block
    __device__ void put(int lw, float h, float b) const
    {
        constexpr int pol = (OUT & OUT_NT) ? 2 : 0;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, h), rh, vo, lw * 4, pol);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, b), rb, vo, lw * 4, pol);
    }
};
template <int OUT>
struct OutStore<OUT, false> {
    gptr<float> ph, pb;
    __device__ OutStore(float *hn, float *bn, long cb, int ap) : ph(G(hn + cb + ap)), pb(G(bn + cb + ap)) {}
    __device__ void put(int lw, float h, float b) const
    {
        if constexpr ((OUT & OUT_NT) != 0) {
            __builtin_nontemporal_store(h, &ph[lw]);
            __builtin_nontemporal_store(b, &pb[lw]);
        } else {
            ph[lw] = h;
            pb[lw] = b;
        }
    }
};

template <typename TS>
__device__ inline double href_of(const Params &P, int ap)
{
    if constexpr (sizeof(TS) == 4) return G(P.vref)[ap];
    else return 0.0;
}

// 1/x from v_rcp_f64 refined by two Newton steps (within an ulp of IEEE division)
__device__ inline double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// van Leer limited slope 2ab/(a+b) for ab > 0, else 0.  The reciprocal is
// v_rcp_f64 (about 2^-24 relative) with one Newton step: within 11 ulp of
// IEEE division over 4M samples spanning 2^-300..2^300, which the limited
// slope carries into the face values at 1e-15 relative.
__device__ inline double vanleer_fast(double a, double b)
{
    const double p = a * b;
    const double x = a + b, r0 = __builtin_amdgcn_rcp(x);
    const double r = fma(r0, fma(-x, r0, 1.0), r0);
    const double q = 2.0 * p * r;
    return p > 0.0 ? q : 0.0;
}

// slope at index i of a line from the values at i-1, i, i+1 (one-sided at the walls)
__device__ inline double slope3(double fm, double fc, double fp, int i, int len, const double *__restrict__ rc_)
{
    const gptr<const double> rc = G(rc_);
    if (i == 0) return (fp - fc) * rc[1];
    if (i == len - 1) return (fc - fm) * rc[i];
    return vanleer_fast((fc - fm) * rc[i], (fp - fc) * rc[i + 1]);
}

// The same slope from per-cell constants: mode 0 interior (limited), 1 at the
// low wall, 2 at the high wall; rm = rc[i], rp = rc[i+1].  fm (mode 1) or fp
// (mode 2) is not read, so the caller may pass any finite value there.
__device__ inline double slope_c(double fm, double fc, double fp, int mode, double rm, double rp)
{
    if (mode == 1) return (fp - fc) * rp;
    if (mode == 2) return (fc - fm) * rm;
    return vanleer_fast((fc - fm) * rm, (fp - fc) * rp);
}
__device__ inline int wall_mode(int i, int len) { return i == 0 ? 1 : (i == len - 1 ? 2 : 0); }

// ---------------------------------------------------------------- K1: moments
// One block per cell, wave q = velocity quadrant q (u>0: bit 0, v>0: bit 1).
// Per level, each lane accumulates over its velocities the FEED sums for the
// x-face and y-face its quadrant is upwind of, plus the cell moments; the
// wave reduces them through LDS (transpose + row sums) and the four waves
// combine into the per-face feeds.
#define K1_ROW 66
template <typename TS>
__device__ inline void moments_cell_d(const Params &P, const TS *__restrict__ h, const TS *__restrict__ b,
                                      double *__restrict__ feed, int c)
{
    // LDS rows per reduction pass: 24, so that three blocks' 52 KB buffers
    // fit a CU's 160 KB of LDS
    constexpr int RPP = 24, NPASS = (NMOM + RPP - 1) / RPP;
    __shared__ double red[4][RPP * K1_ROW];
    __shared__ double wsum[4][NMOM];
    const int i = c % P.nx, j = c / P.nx;
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int NT = P.NT;
    const long sx = (long)NT * P.ls;        // x-neighbour stride
    const long sy = (long)P.nx * NT * P.ls;  // y-neighbour stride
    const double dxo = (q & 1) ? (G(P.xf)[i + 1] - G(P.xc)[i]) : (G(P.xf)[i] - G(P.xc)[i]);
    const double dyo = (q & 2) ? (G(P.yf)[j + 1] - G(P.yc)[j]) : (G(P.yf)[j] - G(P.yc)[j]);
    // neighbour offsets clamped to the cell itself at the walls, so every load
    // of the stencil is unconditional and they all issue together
    const int mx = wall_mode(i, P.nx), my = wall_mode(j, P.ny);
    const long oW = mx == 1 ? 0 : -sx, oE = mx == 2 ? 0 : sx, oS = my == 1 ? 0 : -sy, oN = my == 2 ? 0 : sy;
    const double rxm = G(P.rcx)[i], rxp = G(P.rcx)[i + 1], rym = G(P.rcy)[j], ryp = G(P.rcy)[j + 1];

    // One lane's stencil values and velocity for (level n, quadrant row r).
    struct Ld {
        double hc, bc, hW, bW, hE, bE, hS, bS, hN, bN, u, v, w;
    };
    auto load = [&](int n, int r) {
        Ld d;
        const int ap = q * P.Qp + r;
        d.u = G(P.vu)[ap];
        d.v = G(P.vv)[ap];
        d.w = G(P.vw)[ap];
        const long e = ((long)c * NT + n) * P.ls + ap;
        const TS *hp = h + e, *bp = b + e;
        const double rh = href_of<TS>(P, ap), rb = 0.5 * P.K * rh;
        d.hc = ldv<TS>(hp, 0, rh);
        d.bc = ldv<TS>(bp, 0, rb);
        d.hW = ldv<TS>(hp, oW, rh);
        d.bW = ldv<TS>(bp, oW, rb);
        d.hE = ldv<TS>(hp, oE, rh);
        d.bE = ldv<TS>(bp, oE, rb);
        d.hS = ldv<TS>(hp, oS, rh);
        d.bS = ldv<TS>(bp, oS, rb);
        d.hN = ldv<TS>(hp, oN, rh);
        d.bN = ldv<TS>(bp, oN, rb);
        return d;
    };
    // Loads in place: the kernel runs three blocks per CU (three waves per
    // SIMD), which hides their latency better than loading the next (level,
    // row) pair ahead, whose registers cost the third block.
    const int nch = P.Qp / 64;
    for (int n = 0; n < NT; n++) {
        double acc[NMOM];
#pragma unroll
        for (int k = 0; k < NMOM; k++) acc[k] = 0.0;
        for (int ch = 0; ch < nch; ch++) {
            const Ld d = load(n, lane + 64 * ch);
            const double u = d.u, v = d.v, w = d.w;
            const double hc = d.hc, bc = d.bc;
            const double sxh = slope_c(d.hW, hc, d.hE, mx, rxm, rxp), sxb = slope_c(d.bW, bc, d.bE, mx, rxm, rxp);
            const double syh = slope_c(d.hS, hc, d.hN, my, rym, ryp), syb = slope_c(d.bS, bc, d.bN, my, rym, ryp);
            const double uu = u * u, uv = u * v, vv = v * v;
            const double wm[10] = {w, w * u, w * v, w * uu, w * uv, w * vv, w * uu * u, w * uu * v, w * u * vv,
                                   w * vv * v};
            const double r2 = uu + vv;
            const double sh = u * sxh + v * syh, sb = u * sxb + v * syb;
            // x-feed: face-normal u, tangential slope sigma_y
            const double h0x = hc + sxh * dxo, b0x = bc + sxb * dxo;
#pragma unroll
            for (int k = 0; k < 10; k++) acc[k] += wm[k] * h0x;
            acc[10] += wm[0] * b0x;
            acc[11] += wm[1] * b0x;
            acc[12] += wm[2] * b0x;
            acc[13] += wm[0] * syh;
            acc[14] += wm[1] * syh;
            acc[15] += wm[2] * syh;
            acc[16] += 0.5 * (w * r2 * syh + w * syb);
            acc[17] += wm[1] * sh;
            acc[18] += wm[3] * sh;
            acc[19] += wm[4] * sh;
            acc[20] += 0.5 * wm[1] * (r2 * sh + sb);
            // y-feed: face-normal v, tangential slope sigma_x
            const double h0y = hc + syh * dyo, b0y = bc + syb * dyo;
#pragma unroll
            for (int k = 0; k < 10; k++) acc[21 + k] += wm[k] * h0y;
            acc[31] += wm[0] * b0y;
            acc[32] += wm[1] * b0y;
            acc[33] += wm[2] * b0y;
            acc[34] += wm[0] * sxh;
            acc[35] += wm[1] * sxh;
            acc[36] += wm[2] * sxh;
            acc[37] += 0.5 * (w * r2 * sxh + w * sxb);
            acc[38] += wm[2] * sh;
            acc[39] += wm[4] * sh;
            acc[40] += wm[5] * sh;
            acc[41] += 0.5 * wm[2] * (r2 * sh + sb);
            // cell moments of h^k, b^k
#pragma unroll
            for (int k = 0; k < 10; k++) acc[42 + k] += wm[k] * hc;
            acc[52] += wm[0] * bc;
            acc[53] += wm[1] * bc;
            acc[54] += wm[2] * bc;
        }
        // wave reduction through LDS in passes of RPP rows (row k = sum k of
        // the 64 lanes), two lanes per row.  Each
        // wave works in its own rows, so a wave-level fence orders the writes
        // before the reads; only the quadrant combine below needs the block.
        double *rb = red[q];
#pragma unroll
        for (int half = 0; half < NPASS; half++) {
            const int k0 = half * RPP, kn = NMOM - k0 < RPP ? NMOM - k0 : RPP;
#pragma unroll
            for (int k = 0; k < RPP; k++)
                if (k < kn) rb[k * K1_ROW + lane] = acc[k0 + k];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // row k is summed by two lanes, k over its first 32 entries and
            // k + 32 over the last 32; lane k then adds its partner's part
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
        // combine quadrants: E = q1 + q3, W = q0 + q2, N = q2 + q3, S = q0 + q1
        const gptr<double> out = G(feed) + ((long)c * NT + n) * FEED;
        for (int t = threadIdx.x; t < FEED; t += blockDim.x) {
            double val;
            if (t < 21) val = wsum[1][t] + wsum[3][t];
            else if (t < 42) val = wsum[0][t - 21] + wsum[2][t - 21];
            else if (t < 63) val = wsum[2][t - 42 + 21] + wsum[3][t - 42 + 21];
            else if (t < 84) val = wsum[0][t - 63 + 21] + wsum[1][t - 63 + 21];
            else val = ((wsum[0][t - 84 + 42] + wsum[1][t - 84 + 42]) + wsum[2][t - 84 + 42]) + wsum[3][t - 84 + 42];
            out[t] = val;
        }
        __syncthreads();
    }
}

// the mixed form's moments (FP32 slopes of the stored deviations, FP64 sums)
__device__ inline void moments_cell_m(const Params &P, const float *__restrict__ h, const float *__restrict__ b,
                                      double *__restrict__ feed, int c);

template <typename TS>
__device__ inline void moments_cell(const Params &P, const TS *__restrict__ h, const TS *__restrict__ b,
                                    double *__restrict__ feed, int c)
{
    if constexpr (sizeof(TS) == 4) moments_cell_m(P, h, b, feed, c);
    else moments_cell_d<TS>(P, h, b, feed, c);
}

// Second __launch_bounds__ argument: hipcc reads it as the minimum number of
// waves per SIMD the kernel must fit, which sets its VGPR budget (512 / waves).
// The moments kernel: three waves per SIMD, 168 VGPRs (three 256-thread
// blocks per CU); the mixed form's, with 41 sums per lane, four (128 VGPRs).
#define HB_MOM_WAVES 3
#define HB_MOM_WAVES_MIXED 4

template <typename TS>
__global__ __launch_bounds__(256, sizeof(TS) == 4 ? HB_MOM_WAVES_MIXED : HB_MOM_WAVES) void k_moments(Params P, const TS *__restrict__ h, const TS *__restrict__ b,
                                                 double *__restrict__ feed)
{
    moments_cell<TS>(P, h, b, feed, strip_cell(xcd_cell(blockIdx.x, gridDim.x), P.nx, P.ny));
}

// ---------------------------------------------------------------- K2: faces
// Face-frame raw moments -> W0, primitives, heat flux.
struct FaceState {
    double rho, Un, Ut, lam, qn, qt, W[4];
};
__device__ inline void face_state(int K, const double m[10], const double mb[3], FaceState &s)
{
    s.W[0] = m[0];
    s.W[1] = m[1];
    s.W[2] = m[2];
    s.W[3] = 0.5 * (m[3] + m[5]) + 0.5 * mb[0];
    double p[4];
    prim4(K, s.W, p);
    s.rho = p[0];
    s.Un = p[1];
    s.Ut = p[2];
    s.lam = p[3];
    const double Un = s.Un, Ut = s.Ut;
    double mu30 = m[6] - 3.0 * Un * m[3] + 3.0 * Un * Un * m[1] - Un * Un * Un * m[0];
    double mu12 = m[8] - 2.0 * Ut * m[4] + Ut * Ut * m[1] - Un * (m[5] - 2.0 * Ut * m[2] + Ut * Ut * m[0]);
    double mu21 = m[7] - 2.0 * Un * m[4] + Un * Un * m[2] - Ut * (m[3] - 2.0 * Un * m[1] + Un * Un * m[0]);
    double mu03 = m[9] - 3.0 * Ut * m[5] + 3.0 * Ut * Ut * m[2] - Ut * Ut * Ut * m[0];
    s.qn = 0.5 * (mu30 + mu12 + mb[1] - Un * mb[0]);
    s.qt = 0.5 * (mu21 + mu03 + mb[2] - Ut * mb[0]);
}

// Read-only data every lane of the wave reads at the same address: typed in
// the constant address space so the loads are scalar (SMEM, into SGPRs) and
// never wait behind the vector loads of the stencil.
typedef __attribute__((address_space(4))) const double cdouble;

template <typename Ptr>
__device__ inline cdouble *wave_uniform(Ptr p)
{
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
    return (cdouble *)((static_cast<unsigned long long>(hi) << 32) | lo);
}

// One axis of the tensor velocity grid: nodes, weights, count
struct Axis {
    const double *x, *w;
    int m;
};
__device__ inline Axis axis_u(const Params &P) { return {P.u1, P.w1, P.M}; }
__device__ inline Axis axis_v(const Params &P) { return {P.v1, P.w1v, P.Mv}; }
// one 1-D rule serves both axes
__device__ inline bool square_grid(const Params &P) { return P.Mv == P.M && P.v1 == P.u1; }

// 1-D sums G[k] = sum_i w_i x_i^k exp(-lam (x_i - U)^2), k = 0..6, over m
// nodes with sign selection sel (0 all, 1 x>0, 2 x<0).
template <typename Ptr>
__device__ inline void gsums_at(Ptr u1, Ptr w1, int m, double lam, double U, int sel, double G[7])
{
#pragma unroll
    for (int k = 0; k < 7; k++) G[k] = 0.0;
#pragma unroll 4
    for (int k = 0; k < m; k++) {
        const double x = u1[k];
        if ((sel == 1 && !(x > 0.0)) || (sel == 2 && !(x < 0.0))) continue;
        double t = w1[k] * exp(-lam * (x - U) * (x - U));
#pragma unroll
        for (int p = 0; p < 7; p++) {
            G[p] += t;
            t *= x;
        }
    }
}

// gsums_at over the nodes of one axis.  The lanes of a wave can hold faces of
// both orientations, so the axis varies across the wave unless the grid is
// square; only then are the nodes read through the scalar unit.
__device__ inline void gsums(const Params &P, const Axis &A, double lam, double U, int sel, double S[7])
{
    if (square_grid(P))
        gsums_at(wave_uniform(A.x), wave_uniform(A.w), P.M, lam, U, sel, S);
    else
        gsums_at(G(A.x), G(A.w), A.m, lam, U, sel, S);
}

// Two full-range sums of gsums at once (normal and tangential mean of one
// Maxwellian): the exponentials of both, and of four nodes, are independent,
// which a one-thread-per-face kernel needs to keep its pipeline busy.  Each
// sum still accumulates in node order.  On a square grid both run over the
// same nodes; otherwise the normal sum runs over An, the tangential over At.
__device__ inline void gsums2(const Params &P, const Axis &An, const Axis &At, double lam, double Un, double Ut,
                              double Gn[7], double Gt[7])
{
    if (!square_grid(P)) {
        gsums(P, An, lam, Un, 0, Gn);
        gsums(P, At, lam, Ut, 0, Gt);
        return;
    }
#pragma unroll
    for (int k = 0; k < 7; k++) Gn[k] = Gt[k] = 0.0;
    cdouble *u1 = wave_uniform(P.u1), *w1 = wave_uniform(P.w1);
#pragma unroll 4
    for (int k = 0; k < P.M; k++) {
        const double x = u1[k], w = w1[k];
        double tn = w * exp(-lam * (x - Un) * (x - Un)), tt = w * exp(-lam * (x - Ut) * (x - Ut));
#pragma unroll
        for (int p = 0; p < 7; p++) {
            Gn[p] += tn;
            Gt[p] += tt;
            tn *= x;
            tt *= x;
        }
    }
}

// Moment table of the normalised face Maxwellian over the velocity grid
// instead of the plane: N[k] = sqrt(lam/pi) sum_i w_i x_i^k exp(-lam (x_i - Un)^2)
// from the 1-D sums Gn (over the selected half or all nodes), T likewise from
// Gt; the internal-energy moments stay analytic (the reduced h, b carry them).
__device__ inline void disc_momtab(const double Gn[7], const double Gt[7], double lam, int K, MomTab &t)
{
    const double r = sqrt(lam / HB_PI);
#pragma unroll
    for (int k = 0; k < 7; k++) {
        t.N[k] = r * Gn[k];
        t.T[k] = r * Gt[k];
    }
    t.N[7] = t.T[7] = 0.0;
    t.X[0] = 1.0;
    t.X[1] = K / (2.0 * lam);
    t.X[2] = K * (K + 2.0) / (4.0 * lam * lam);
}

// sum_alpha w u_n psi (H0 + H0+, B0 + B0+) from the 1-D sums of the face Maxwellian.
__device__ inline void equil_flux_sums(int K, double pref, double lam, const P3 &Ph, const P3 &Pb, const double *Gn,
                                       const double *Gt, double S[4])
{
    S[0] = pref * p3_sum(Ph, 1, 0, Gn, Gt);
    S[1] = pref * p3_sum(Ph, 2, 0, Gn, Gt);
    S[2] = pref * p3_sum(Ph, 1, 1, Gn, Gt);
    S[3] = pref * (0.5 * (p3_sum(Ph, 3, 0, Gn, Gt) + p3_sum(Ph, 1, 2, Gn, Gt)) +
                   0.5 * (K / (2.0 * lam)) * p3_sum(Pb, 1, 0, Gn, Gt));
}

__device__ inline void store_side(double *rec, int side, double lam, double Un, double Ut, const P3 &Qh, const P3 &Qb,
                                  double c4, double c5)
{
    double *s = rec + REC_SIDE + REC_SIDEW * side;
    s[0] = lam;
    s[1] = Un;
    s[2] = Ut;
#pragma unroll
    for (int k = 0; k < 10; k++) {
        s[3 + k] = Qh.c[k];
        s[13 + k] = Qb.c[k];
    }
    s[23] = c4;
    s[24] = c5;
}

// FP32 coefficients of one side for the mixed form (record layout in
// hb_layout.h): y-face cubics in (n, t) = (v, u) are stored in the global
// (u, v) monomial order, so every face of a cell evaluates them on the same
// per-velocity monomials.
__device__ inline void store_side32(float *rec32, int side, bool isx, int K, const P3 &Qh, const P3 &Qb, double c4,
                                    double c5)
{
    constexpr int p10y[10] = {0, 2, 1, 5, 4, 3, 9, 8, 7, 6};
    float *o = rec32 + REC32_SIDEW * side;
    const double k0h = (1.0 - c4) / HB_PI, k0b = k0h * 0.5 * K;
#pragma unroll
    for (int k = 0; k < 10; k++) {
        const double qh = isx ? Qh.c[k] : Qh.c[p10y[k]], qb = isx ? Qb.c[k] : Qb.c[p10y[k]];
        o[k] = static_cast<float>(k == 0 ? qh - k0h : qh);
        o[10 + k] = static_cast<float>(k == 0 ? qb - k0b : qb);
    }
    o[20] = static_cast<float>(k0h);
    o[21] = static_cast<float>(k0b);
    o[22] = static_cast<float>(c4);
    o[23] = static_cast<float>(c5);
}

// one (face, level) per thread t; x-faces first, then y-faces
// Face slot -> face index (x-faces row by row, then y-faces).  The slots list
// the interior faces first (x, then y) and the wall faces last, so that a
// wave runs either the interior or the wall branch of the face kernel, not
// both one after the other.
__device__ inline int face_of_slot(int s, int nx, int ny)
{
    const int nfx = (nx + 1) * ny, ix = (nx - 1) * ny, iy = nx * (ny - 1);
    if (s < ix) return (s / (nx - 1)) * (nx + 1) + 1 + s % (nx - 1);
    s -= ix;
    if (s < iy) return nfx + nx + s;
    s -= iy;
    if (s < 2 * ny) return (s >> 1) * (nx + 1) + ((s & 1) ? nx : 0);
    s -= 2 * ny;
    return nfx + (s < nx ? s : ny * nx + s - nx);
}

__device__ inline void faces_thread(const Params &P, const double *__restrict__ feed, const double *__restrict__ W,
                                    const double *__restrict__ dtc, double *__restrict__ recx,
                                    double *__restrict__ recy, int t)
{
    const int NT = P.NT, nx = P.nx, ny = P.ny, K = P.K;
    const int nfx = (nx + 1) * ny, nfy = nx * (ny + 1);
    if (t >= (nfx + nfy) * NT) return;
    const int n = t % NT;
    int f = face_of_slot(t / NT, nx, ny);
    bool isx = f < nfx;
    // the face's normal velocity axis is u on x-faces, v on y-faces
    const Axis An = isx ? axis_u(P) : axis_v(P), At = isx ? axis_v(P) : axis_u(P);
    int cL, cR, lo_end;  // cells on the low/high side (-1 if wall)
    double xL = 0, xF = 0, xR = 0;
    double *rec;
    float *rec32 = nullptr;  // mixed form only
    if (isx) {
        const int fi = f % (nx + 1), jj = f / (nx + 1);
        cL = fi > 0 ? jj * nx + fi - 1 : -1;
        cR = fi < nx ? jj * nx + fi : -1;
        xF = P.xf[fi];
        if (cL >= 0) xL = P.xc[fi - 1];
        if (cR >= 0) xR = P.xc[fi];
        lo_end = fi == 0;
        rec = recx + ((long)f * NT + n) * REC;
        if (P.rx32) rec32 = P.rx32 + ((long)f * NT + n) * REC32;
    } else {
        f -= nfx;
        const int ii = f % nx, fj = f / nx;
        cL = fj > 0 ? (fj - 1) * nx + ii : -1;
        cR = fj < ny ? fj * nx + ii : -1;
        xF = P.yf[fj];
        if (cL >= 0) xL = P.yc[fj - 1];
        if (cR >= 0) xR = P.yc[fj];
        lo_end = fj == 0;
        rec = recy + ((long)f * NT + n) * REC;
        if (P.ry32) rec32 = P.ry32 + ((long)f * NT + n) * REC32;
    }
    // global -> face-frame index maps (y-faces: n = v, t = u), applied with
    // compile-time indices so that no array is indexed at run time
    constexpr int p10y[10] = {0, 2, 1, 5, 4, 3, 9, 8, 7, 6}, p3y[3] = {0, 2, 1}, p4y[4] = {0, 2, 1, 3};
    // feeds: low cell feeds through its high face (E or N), high cell through its low face (W or S)
    const int offHi = isx ? FEED_E : FEED_N, offLo = isx ? FEED_W : FEED_S;
    double m[10], mb[3], ts[4], c5s[4];
    {
        const double *fa = cL >= 0 ? feed + ((long)cL * NT + n) * FEED + offHi : nullptr;
        const double *fb = cR >= 0 ? feed + ((long)cR * NT + n) * FEED + offLo : nullptr;
        double g[21];
#pragma unroll
        for (int k = 0; k < 21; k++) g[k] = (fa ? fa[k] : 0.0) + (fb ? fb[k] : 0.0);
#pragma unroll
        for (int k = 0; k < 10; k++) m[k] = isx ? g[k] : g[p10y[k]];
#pragma unroll
        for (int k = 0; k < 3; k++) mb[k] = isx ? g[10 + k] : g[10 + p3y[k]];
#pragma unroll
        for (int k = 0; k < 4; k++) ts[k] = isx ? g[13 + k] : g[13 + p4y[k]];
#pragma unroll
        for (int k = 0; k < 4; k++) c5s[k] = isx ? g[17 + k] : g[17 + p4y[k]];
    }
    const double S4[4] = {m[1], m[3], m[4], 0.5 * (m[6] + m[8]) + 0.5 * mb[1]};
    double F[4];

    if (cL >= 0 && cR >= 0) {
        // ---------------- interior face (Eqs. 21-24)
        FaceState fs;
        face_state(K, m, mb, fs);
        const double rho = fs.rho, Un = fs.Un, Ut = fs.Ut, lam = fs.lam;
        const double tau0 = tau_of(P, rho, lam);
        const double dGL = dtc[cL], dGR = dtc[cR];
        const double dGf = P.face_dt == 1 ? 2.0 * dGL * dGR / (dGL + dGR) : fmin(dGL, dGR);
        double C[5];
        ccoef(tau0, dGf, C);
        double WL[4], WR[4];
        {
            const double *a = W + ((long)cL * NT + n) * 4, *bb = W + ((long)cR * NT + n) * 4;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                WL[k] = a[isx ? k : p4y[k]];
                WR[k] = bb[isx ? k : p4y[k]];
            }
        }
        double dWL[4], dWR[4], dWt[4];
        const double dL = xF - xL, dR = xR - xF;
        // reciprocals once, products below (the divisions sat on the chain)
        const double rrho = 1.0 / rho, rLr = rrho / dL, rRr = rrho / dR, rdG = 1.0 / dGf;
        for (int k = 0; k < 4; k++) {
            dWL[k] = (fs.W[k] - WL[k]) * rLr;
            dWR[k] = (WR[k] - fs.W[k]) * rRr;
            dWt[k] = ts[k] * rrho;
        }
        double aL[4], aR[4], at[4], A[4];
        slope_solve(Un, Ut, lam, K, dWL, aL);
        slope_solve(Un, Ut, lam, K, dWR, aR);
        slope_solve(Un, Ut, lam, K, dWt, at);
        MomTab t0, tp, tm;
        momtab(Un, Ut, lam, K, 0, t0);
        momtab(Un, Ut, lam, K, 1, tp);
        momtab(Un, Ut, lam, K, 2, tm);
        double r1[4], r2[4], r3[4], rhs[4];
        mpsi_apsi(tp, 1, 0, aL, r1);
        mpsi_apsi(tm, 1, 0, aR, r2);
        mpsi_apsi(t0, 0, 1, at, r3);
        for (int k = 0; k < 4; k++) rhs[k] = -(r1[k] + r2[k] + r3[k]);
        slope_solve(Un, Ut, lam, K, rhs, A);
        double Gn[7], Gt[7];
        gsums2(P, An, At, lam, Un, Ut, Gn, Gt);
        // macro flux: the C2 and C3 parts as Maxwellian moments (Eq. 24), or
        // as the velocity sums of the micro flux's C2 and C3 parts
        double c2a[4], c2b[4], c2c[4], c3[4];
        if (P.macro_mode == 1) {
            double Gp[7], Gm[7];
            gsums(P, An, lam, Un, 1, Gp);
            gsums(P, An, lam, Un, 2, Gm);
            MomTab d0, dp, dm;
            disc_momtab(Gn, Gt, lam, K, d0);
            disc_momtab(Gp, Gt, lam, K, dp);
            disc_momtab(Gm, Gt, lam, K, dm);
            mpsi_apsi(dp, 2, 0, aL, c2a);
            mpsi_apsi(dm, 2, 0, aR, c2b);
            mpsi_apsi(d0, 1, 1, at, c2c);
            mpsi_apsi(d0, 1, 0, A, c3);
        } else {
            mpsi_apsi(tp, 2, 0, aL, c2a);
            mpsi_apsi(tm, 2, 0, aR, c2b);
            mpsi_apsi(t0, 1, 1, at, c2c);
            mpsi_apsi(t0, 1, 0, A, c3);
        }
        const double sq = (1.0 - P.Pr) * 4.0 * lam * lam / (5.0 * rho);
        P3 Ph, Pb;
        shakhov_poly(sq, fs.qn, fs.qt, Un, Ut, lam, K - 5.0, Ph);
        shakhov_poly(sq, fs.qn, fs.qt, Un, Ut, lam, K - 3.0, Pb);
        Ph.c[0] += 1.0;
        Pb.c[0] += 1.0;
        const double pref = rho * lam / HB_PI;
        double S1[4];
        equil_flux_sums(K, pref, lam, Ph, Pb, Gn, Gt, S1);
        for (int k = 0; k < 4; k++)
            F[k] = (C[0] * S1[k] + C[1] * rho * (c2a[k] + c2b[k] + c2c[k]) + C[2] * rho * c3[k] + C[3] * S4[k] +
                    C[4] * c5s[k]) *
                   rdG;
        // micro-flux records: side 1 (u_n > 0) uses a^L, side 0 uses a^R
        const double xh = K / (2.0 * lam), xb = (K + 2.0) / (2.0 * lam);
        const double ln[3] = {0.0, 1.0, 0.0}, lt[3] = {0.0, 0.0, 1.0}, l1[3] = {1.0, 0.0, 0.0};
        double qt_h[6], qt_b[6], qA_h[6], qA_b[6];
        apsi_quad(at, xh, qt_h);
        apsi_quad(at, xb, qt_b);
        apsi_quad(A, xh, qA_h);
        apsi_quad(A, xb, qA_b);
        P3 tTh, tTb, pAh, pAb;
        p3_lin_quad(lt, qt_h, tTh);
        p3_lin_quad(lt, qt_b, tTb);
        p3_lin_quad(l1, qA_h, pAh);
        p3_lin_quad(l1, qA_b, pAb);
        for (int side = 0; side < 2; side++) {
            const double *as = side ? aL : aR;
            double qs_h[6], qs_b[6];
            apsi_quad(as, xh, qs_h);
            apsi_quad(as, xb, qs_b);
            P3 nSh, nSb, Qh, Qb;
            p3_lin_quad(ln, qs_h, nSh);
            p3_lin_quad(ln, qs_b, nSb);
            p3_zero(Qh);
            p3_zero(Qb);
            p3_axpy(C[0], Ph, Qh);
            p3_axpy(C[1], nSh, Qh);
            p3_axpy(C[1], tTh, Qh);
            p3_axpy(C[2], pAh, Qh);
            p3_axpy(C[0], Pb, Qb);
            p3_axpy(C[1], nSb, Qb);
            p3_axpy(C[1], tTb, Qb);
            p3_axpy(C[2], pAb, Qb);
            const double sh = pref * rdG, sbq = pref * xh * rdG;
            for (int k = 0; k < 10; k++) {
                Qh.c[k] *= sh;
                Qb.c[k] *= sbq;
            }
            store_side(rec, side, lam, Un, Ut, Qh, Qb, C[3] * rdG, C[4] * rdG);
            if (rec32) store_side32(rec32, side, isx, K, Qh, Qb, C[3] * rdG, C[4] * rdG);
        }
    } else {
        // ---------------- diffuse isothermal wall (Eqs. 25-28)
        const int c = cL >= 0 ? cL : cR;
        const int inc_side = lo_end ? 0 : 1;  // incident velocities: u.n_in < 0
        const int refl_side = 1 - inc_side;
        int wl;
        if (isx) wl = lo_end ? 3 : 1;
        else wl = lo_end ? 0 : 2;
        const double Uw = P.wall_ut[wl][n], lw = 1.0 / P.wall_T[wl][n];
        double Gwn[7], Gwt[7];
        gsums(P, An, lw, 0.0, refl_side ? 1 : 2, Gwn);
        gsums(P, At, lw, Uw, 0, Gwt);
        const double pw = lw / HB_PI, xw = K / (2.0 * lw);
        // reflected half of the unit-density wall Maxwellian: R_ab = sum w n^a t^b H_w
        auto R = [&](int a, int bq) { return pw * Gwn[a] * Gwt[bq]; };
        const double rw0 = -m[1] / R(1, 0);
        double mc[10], mbc[3];
        const int EN[10] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0}, ET[10] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};
        for (int k = 0; k < 10; k++) mc[k] = m[k] + rw0 * R(EN[k], ET[k]);
        for (int k = 0; k < 3; k++) mbc[k] = mb[k] + rw0 * xw * R(EN[k], ET[k]);
        FaceState fs;
        face_state(K, mc, mbc, fs);
        const double rho = fs.rho, Un = fs.Un, Ut = fs.Ut, lam = fs.lam;
        const double tau0 = tau_of(P, rho, lam);
        const double dGf = dtc[c];
        double C[5];
        ccoef(tau0, dGf, C);
        const double sq = (1.0 - P.Pr) * 4.0 * lam * lam / (5.0 * rho);
        P3 Ph, Pb;
        shakhov_poly(sq, fs.qn, fs.qt, Un, Ut, lam, K - 5.0, Ph);
        shakhov_poly(sq, fs.qn, fs.qt, Un, Ut, lam, K - 3.0, Pb);
        Ph.c[0] += 1.0;
        Pb.c[0] += 1.0;
        double Gn[7], Gt[7];
        gsums(P, An, lam, Un, inc_side ? 1 : 2, Gn);
        gsums(P, At, lam, Ut, 0, Gt);
        const double pref = rho * lam / HB_PI;
        double S1[4];
        equil_flux_sums(K, pref, lam, Ph, Pb, Gn, Gt, S1);
        const double inflow = (C[0] * S1[0] + C[3] * m[1] + C[4] * c5s[0]) / dGf;
        const double rw = -inflow / R(1, 0);
        const double Sr[4] = {R(1, 0), R(2, 0), R(1, 1), 0.5 * (R(3, 0) + R(1, 2)) + 0.5 * xw * R(1, 0)};
        for (int k = 0; k < 4; k++) F[k] = rw * Sr[k] + (C[0] * S1[k] + C[3] * S4[k] + C[4] * c5s[k]) / dGf;
        // records
        P3 Qh, Qb;
        for (int k = 0; k < 10; k++) {
            Qh.c[k] = Ph.c[k] * pref * C[0] / dGf;
            Qb.c[k] = Pb.c[k] * pref * (K / (2.0 * lam)) * C[0] / dGf;
        }
        store_side(rec, inc_side, lam, Un, Ut, Qh, Qb, C[3] / dGf, C[4] / dGf);
        if (rec32) store_side32(rec32, inc_side, isx, K, Qh, Qb, C[3] / dGf, C[4] / dGf);
        p3_zero(Qh);
        p3_zero(Qb);
        Qh.c[0] = rw * pw;
        Qb.c[0] = rw * pw * xw;
        store_side(rec, refl_side, lw, 0.0, Uw, Qh, Qb, 0.0, 0.0);
        if (rec32) store_side32(rec32, refl_side, isx, K, Qh, Qb, 0.0, 0.0);
    }
    // macro flux in the global frame
    if (isx) {
        rec[0] = F[0];
        rec[1] = F[1];
        rec[2] = F[2];
        rec[3] = F[3];
    } else {
        rec[0] = F[0];
        rec[1] = F[2];
        rec[2] = F[1];
        rec[3] = F[3];
    }
}

// one thread per (face, level); x-faces first, then y-faces
__global__ __launch_bounds__(128) void k_faces(Params P, const double *__restrict__ feed,
                                               const double *__restrict__ W, const double *__restrict__ dtc,
                                               double *__restrict__ recx, double *__restrict__ recy)
{
    faces_thread(P, feed, W, dtc, recx, recy, blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------- K3: cells
__device__ inline void heat_flux_raw(const double *m, const double *mb, double U, double V, double q[2])
{
    double mu30 = m[6] - 3.0 * U * m[3] + 3.0 * U * U * m[1] - U * U * U * m[0];
    double mu12 = m[8] - 2.0 * V * m[4] + V * V * m[1] - U * (m[5] - 2.0 * V * m[2] + V * V * m[0]);
    double mu21 = m[7] - 2.0 * U * m[4] + U * U * m[2] - V * (m[3] - 2.0 * U * m[1] + U * U * m[0]);
    double mu03 = m[9] - 3.0 * V * m[5] + 3.0 * V * V * m[2] - V * V * V * m[0];
    q[0] = 0.5 * (mu30 + mu12 + mb[1] - U * mb[0]);
    q[1] = 0.5 * (mu21 + mu03 + mb[2] - V * mb[0]);
}

// local pseudo step of cell c from its W at all levels (Eqs. 31-32)
__device__ inline double local_dt(const Params &P, const double *Wc, int i, int j)
{
    if (P.dt_mode == 1) return P.dt_fixed;
    double nu = 0.0;
    for (int n = 0; n < P.NT; n++) {
        double p[4];
        prim4(P.K, Wc + n * 4, p);
        const double cs = sqrt(P.gamma / (2.0 * p[3]));
        const double ut = fmax(P.umax, fabs(p[1])) + cs, vt = fmax(P.vmax, fabs(p[2])) + cs;
        nu = fmax(nu, ut * P.rdx[i] + vt * P.rdy[j]);
    }
    return P.cfl / (nu + P.omega * P.NH);
}

__device__ inline void cell_eq(const Params &P, const double *Wc, const double *cm, double dG, double *out)
{
    double p[4], q[2];
    prim4(P.K, Wc, p);
    heat_flux_raw(cm, cm + 10, p[1], p[2], q);
    const double s = (1.0 - P.Pr) * 4.0 * p[3] * p[3] / (5.0 * p[0]);
    const double A = p[0] * p[3] / HB_PI;
    out[0] = p[3];
    out[1] = p[1];
    out[2] = p[2];
    out[3] = A;
    out[4] = A * P.K / (2.0 * p[3]);
    out[5] = 0.5 * dG / tau_of(P, p[0], p[3]);
    out[6] = s * q[0];
    out[7] = s * q[1];
}

// one thread per (cell, level): macro update (Eq. 29), collision records, and
// the level-0 residual terms (per-block partial sums, fixed order)
// (block blk of 128 threads within the case)
__device__ inline void cells_block(const Params &P, const double *__restrict__ feed, const double *__restrict__ recx,
                                   const double *__restrict__ recy, const double *__restrict__ Wk,
                                   const double *__restrict__ dtc, double *__restrict__ Wn, double *__restrict__ crec,
                                   double *__restrict__ rpart, int blk)
{
    __shared__ double red[4][128];
    __shared__ double mred[2][HB_NTMAX];
    const int NT = P.NT, nx = P.nx;
    const int t = blk * 128 + threadIdx.x;
    double d2[4] = {0, 0, 0, 0};
    double mass = 0.0;  // |Omega_i| rho^{k+1}_{i,n} of this thread's (cell, level)
    int lvl = -1;
    if (t < P.nc * NT) {
        const int c = t / NT, n = t % NT;
        const int i = c % nx, j = c / nx;
        const double dG = dtc[c];
        const double *Wc = Wk + (long)c * NT * 4;
        double *Wo = Wn + ((long)c * NT + n) * 4;
        const double *Fw = recx + ((long)(j * (nx + 1) + i) * NT + n) * REC;
        const double *Fe = recx + ((long)(j * (nx + 1) + i + 1) * NT + n) * REC;
        const double *Fs = recy + ((long)(j * nx + i) * NT + n) * REC;
        const double *Fn = recy + ((long)((j + 1) * nx + i) * NT + n) * REC;
        double Wnew[4];
        // spectral source sum_m E_nm W_m, each sum in level order.  The loop
        // runs to the largest level count so that all its loads issue at once;
        // indices past NT are clamped and their terms weighted by zero.
        double src[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int mm = 0; mm < HB_NTMAX; mm++) {
            const int m2 = mm < NT ? mm : NT - 1;
            const double e = P.E[n * NT + m2] * (mm < NT ? 1.0 : 0.0);
#pragma unroll
            for (int k = 0; k < 4; k++) src[k] += e * Wc[m2 * 4 + k];
        }
        for (int k = 0; k < 4; k++) {
            const double div = (Fe[k] - Fw[k]) * P.rdx[i] + (Fn[k] - Fs[k]) * P.rdy[j];
            Wnew[k] = Wc[n * 4 + k] - dG * (div + P.omega * src[k]);
            Wo[k] = Wnew[k];
        }
        const double *cm = feed + ((long)c * NT + n) * FEED + FEED_CM;
        double *cr = crec + ((long)c * NT + n) * CREC;
        cell_eq(P, Wc + n * 4, cm, dG, cr);
        cell_eq(P, Wnew, cm, dG, cr + CREC_T);
        cr[16] = 1.0 / (1.0 + cr[CREC_T + 5]);
        if (P.cr32) {
            // FP32 record of the mixed form: the amplitudes also as deviations
            // from the rest Maxwellian's (1/pi, K/(2 pi))
            float *o = P.cr32 + ((long)c * NT + n) * CREC32;
#pragma unroll
            for (int s2 = 0; s2 < 2; s2++) {
                const double *q = cr + CREC_T * s2;
                float *os = o + CREC32_T * s2;
                os[0] = static_cast<float>(q[1]);
                os[1] = static_cast<float>(q[2]);
                os[2] = static_cast<float>(2.0 * q[0]);
                os[3] = static_cast<float>(q[3]);
                os[4] = static_cast<float>(q[3] - 1.0 / HB_PI);
                os[5] = static_cast<float>(q[4]);
                os[6] = static_cast<float>(q[4] - 0.5 * P.K / HB_PI);
                os[7] = static_cast<float>(q[6]);
                os[8] = static_cast<float>(q[7]);
            }
            o[18] = static_cast<float>(cr[5]);
            o[19] = static_cast<float>(cr[CREC_T + 5]);
            o[20] = static_cast<float>(1.0 - cr[5]);
            o[21] = static_cast<float>(cr[16]);
        }
        // level 0 carries the residual of Eq. (43); the other levels add
        // 0 * W^{k+1}, which is +-0 for finite values (the sums are
        // unchanged) and NaN for NaN/Inf, so divergence at any level
        // reaches the residual and its flag in the same step
        for (int k = 0; k < 4; k++) {
            const double d = Wnew[k] - Wc[k];
            d2[k] = n == 0 ? d * d : 0.0 * Wnew[k];
        }
        mass = (P.xf[i + 1] - P.xf[i]) * (P.yf[j + 1] - P.yf[j]) * Wnew[0];
        lvl = n;
    }
    for (int k = 0; k < 4; k++) red[k][threadIdx.x] = d2[k];
    // per-level mass of the block: a fixed-order shuffle tree per wave, then
    // wave 0 + wave 1
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int m = 0; m < NT; m++) {
        double v = lvl == m ? mass : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (lane == 0) mred[wv][m] = v;
    }
    __syncthreads();
    for (int s = 64; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 4; k++) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) rpart[blk * RPART + threadIdx.x] = red[threadIdx.x][0];
    if (threadIdx.x < NT) rpart[blk * RPART + 4 + threadIdx.x] = mred[0][threadIdx.x] + mred[1][threadIdx.x];
}

__global__ __launch_bounds__(128) void k_cells(Params P, const double *__restrict__ feed, const double *__restrict__ recx,
                                               const double *__restrict__ recy, const double *__restrict__ Wk,
                                               const double *__restrict__ dtc, double *__restrict__ Wn,
                                               double *__restrict__ crec, double *__restrict__ rpart)
{
    cells_block(P, feed, recx, recy, Wk, dtc, Wn, crec, rpart, blockIdx.x);
}

// ---------------------------------------------------------------- K4: residual
// The residual of the step (Eq. 43) into the ring, and the scale factors of
// the level-mass projection (a convergence aid; not in the paper).  The
// spectral source only moves mass between levels, and with local pseudo
// steps the flux terms no longer cancel over the cavity, so each level's mass
// M_n drifts during the transient; the level-dependent part of (M_n) then
// rotates under the explicit source term without decaying and the residual
// stalls.  At every fixed point of the step the level masses agree (summing
// Eq. 29 over the cells leaves omega E M = 0), so scaling level n by
// s_n = 1 + (Mbar - M_n) / M_n (Mbar their mean; exactly 1 when they agree)
// keeps the fixed points and removes that rotation.  One block, fixed-order
// sums of the cells kernel's block partials.
__device__ inline void resid_block(const Params &P, const double *__restrict__ rpart, int nblk,
                                   double *__restrict__ ring, int slot, int *__restrict__ flag)
{
    __shared__ double red[RPART][256];
    const int nk = 4 + P.NT;
    double s[RPART];
#pragma unroll
    for (int k = 0; k < RPART; k++) s[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256)
#pragma unroll
        for (int k = 0; k < RPART; k++)
            if (k < nk) s[k] += rpart[b * RPART + k];
#pragma unroll
    for (int k = 0; k < RPART; k++) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int k = 0; k < nk; k++) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4) {
        const double r = sqrt(red[threadIdx.x][0] / P.nc);
        ring[slot * 4 + threadIdx.x] = r;
        if (!isfinite(r)) atomicOr(flag, 1);
    }
    if (threadIdx.x < P.NT) {
        const int n = threadIdx.x;
        double d = 0.0;
        for (int m = 0; m < P.NT; m++) d += red[4 + m][0] - red[4][0];
        const double mean = red[4][0] + d / P.NT, Mn = red[4 + n][0];
        const double sn = P.level_mass ? 1.0 + (mean - Mn) / Mn : 1.0;
        P.lscale[n] = sn;
        if (P.lscale32) {
            P.lscale32[n] = static_cast<float>(sn);
            P.lscale32[HB_NTMAX + n] = static_cast<float>((sn - 1.0) / HB_PI);
        }
    }
}

// Period residual of the time-domain solver, Eq. (43) second line: RMS over
// cells of W(nT) - W((n-1)T) for one level (W[c][4]); one block, fixed-order sums.
__global__ __launch_bounds__(256) void k_period_diff(const double *__restrict__ Wa, const double *__restrict__ Wb,
                                                     int nc, double *__restrict__ out)
{
    __shared__ double red[4][256];
    double s[4] = {0, 0, 0, 0};
    for (int c = threadIdx.x; c < nc; c += 256)
        for (int k = 0; k < 4; k++) {
            const double d = Wa[(long)c * 4 + k] - Wb[(long)c * 4 + k];
            s[k] += d * d;
        }
    for (int k = 0; k < 4; k++) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int k = 0; k < 4; k++) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = sqrt(red[threadIdx.x][0] / nc);
}

// ---------------------------------------------------------------- K5: update
// One block per cell, templated on the number of levels so the per-level
// state of a velocity lives in registers.  LDS holds the 1-D Maxwellian factor
// tables of the four faces (merged normal table + one tangential table per
// upwind side) and of the cell equilibria at k and k+1, for every level.

// a * b + c with c wave-uniform, as one VOP3 FMA reading c from scalar
// registers.  (Left to itself the compiler copies c into a vector register
// and uses the accumulating form: two extra moves per FP64 coefficient.)
__device__ inline double fma_s(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// Cubic c0 + c1 n + c2 t + c3 n^2 + c4 n t + c5 t^2 + c6 n^3 + c7 n^2 t + c8 n t^2
// + c9 t^3 in nested form, every step pairing one wave-uniform coefficient
// with per-lane values.
template <typename Ptr>
__device__ inline double p3_eval(Ptr c, double n, double t)
{
#pragma clang fp contract(off)
    const double a = n * c[6] + c[3];
    const double b = n * c[7] + c[4];
    const double d = __builtin_fma(t, c[9], n * c[8]);
    const double e = __builtin_fma(t, b, fma_s(n, a, c[1]));
    const double f = fma_s(t, d + c[5], c[2]);
    return __builtin_fma(t, f, fma_s(n, e, c[0]));
}


// micro flux through one face for this lane: u_n (e Q(n,t) + c4 f0 + c5 s)
template <typename Ptr>
__device__ inline void face_flux(Ptr s, double e, double un, double ut, double h0, double b0, double sh, double sb,
                                 double &Hh, double &Hb)
{
    const double qh = p3_eval(s + 3, un, ut), qb = p3_eval(s + 13, un, ut);
    Hh = un * (e * qh + s[23] * h0 + s[24] * sh);
    Hb = un * (e * qb + s[23] * b0 + s[24] * sb);
}

// Tables of one cell's block: 4 faces x NT levels x (merged normal, two
// tangential) + NT levels x (u, v) x (k, k+1) for the cell equilibria.
template <int NT>
__device__ inline void build_tables(const Params &P, const gptr<const double> fr[4], gptr<const double> cr, double *tab)
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
            tab[t] = 0.0;  // stride padding of the shorter axis, never read
            continue;
        }
        const double x = onv ? G(P.v1)[k] : G(P.u1)[k];
        double lam, U;
        if (t < ftab) {
            const gptr<const double> sd = fr[fs] + n * REC + REC_SIDE + REC_SIDEW * (which == 0 ? (x > 0.0 ? 1 : 0) : which - 1);
            lam = sd[0];
            U = which == 0 ? sd[1] : sd[2];
        } else {
            const gptr<const double> cc = cr + n * CREC + (which >= 2 ? CREC_T : 0);
            lam = cc[0];
            U = (which & 1) ? cc[2] : cc[1];
        }
        tab[t] = exp(-lam * (x - U) * (x - U));
    }
}

// W^{k+1} of cell c times the level-mass factors (the block that updates
// the cell's distributions also scales its macroscopic state; nothing else
// reads W^{k+1} during the update)
template <int NT>
__device__ inline void scale_w(const Params &P, double *__restrict__ Wn, int c)
{
    if (threadIdx.x < NT * 4) Wn[(long)c * NT * 4 + threadIdx.x] *= P.lscale[threadIdx.x >> 2];
}

// Spectral source and semi-implicit collision (Eq. 30) for one velocity at all
// levels, then the store of h^{k+1}, b^{k+1} (times the level-mass factor).
template <int NT, typename TS>
__device__ inline void collide_store(const Params &P, gptr<const double> cr, const double *ctab, double dG, double u,
                                     double v, int iu, int iv, const double *hk, const double *bk, const double *dh,
                                     const double *db, TS *hn, TS *bn, long e0, double rh, double rb)
{
    const int M = P.Mt;  // table row stride
    const double kh = P.K - 5.0, kb = P.K - 3.0, dgw = dG * P.omega;
#pragma unroll
    for (int n = 0; n < NT; n++) {
        // E of Eq. (17) is circulant with a zero diagonal: E_nm = e_d for
        // d = (n - m) mod N_T, e_d = E_d0
        double Eh = 0.0, Eb = 0.0;
#pragma unroll
        for (int d = 1; d < NT; d++) {
            const int m = (n - d + NT) % NT;
            Eh = fma(P.E[d * NT], hk[m], Eh);
            Eb = fma(P.E[d * NT], bk[m], Eb);
        }
        const gptr<const double> cc = cr + n * CREC;
        const double *ct = ctab + n * 4 * M;
        double heq[2], beq[2];
#pragma unroll
        for (int s2 = 0; s2 < 2; s2++) {
            const gptr<const double> q = cc + CREC_T * s2;
            const double lam2 = 2.0 * q[0];
            const double e = ct[(2 * s2) * M + iu] * ct[(2 * s2 + 1) * M + iv];
            const double cu = u - q[1], cv = v - q[2];
            const double c2 = cu * cu + cv * cv, cq = cu * q[6] + cv * q[7];
            heq[s2] = e * q[3] * (1.0 + cq * (lam2 * c2 + kh));
            beq[s2] = e * q[4] * (1.0 + cq * (lam2 * c2 + kb));
        }
        const double a0 = cc[5], a1 = cc[CREC_T + 5], rden = cc[16];
        const double hnew = (hk[n] - dG * dh[n] - dgw * Eh + a1 * heq[1] + a0 * (heq[0] - hk[n])) * rden;
        const double bnew = (bk[n] - dG * db[n] - dgw * Eb + a1 * beq[1] + a0 * (beq[0] - bk[n])) * rden;
        const double sc = wave_uniform(P.lscale)[n];  // level-mass projection
        stv<TS>(hn, e0 + (long)n * P.ls, hnew * sc, rh);
        stv<TS>(bn, e0 + (long)n * P.ls, bnew * sc, rb);
    }
}

// Interior cells (2 <= i <= nx-3, 2 <= j <= ny-3): every stencil value exists
// and every slope is limited, so the per-velocity work is straight-line code.
// Minimum waves per SIMD of the interior update (see HB_MOM_WAVES): two, so
// up to 256 VGPRs; at three levels the body needs 120 and runs at four.
#define HB_UPD_WAVES 2
// the mixed form's FP32 interior update: four waves per SIMD (128 VGPRs)
#define HB_UPD_WAVES_MIXED 4
template <int NT, typename TS>
__device__ inline void update_int_cell_d(const Params &P, const TS *__restrict__ h, const TS *__restrict__ b,
                                       const double *__restrict__ recx, const double *__restrict__ recy,
                                       const double *__restrict__ crec, const double *__restrict__ dtc,
                                       TS *__restrict__ hn, TS *__restrict__ bn, double *__restrict__ Wn, int ci)
{
    extern __shared__ double tab[];
    const int nxi = P.nx - 4;
    const int i = 2 + ci % nxi, j = 2 + ci / nxi;
    const int M = P.Mt, nx = P.nx;
    const int c = j * nx + i;
    scale_w<NT>(P, Wn, c);
    const gptr<const double> fr[4] = {G(recx) + (long)(j * (nx + 1) + i) * NT * REC, G(recx) + (long)(j * (nx + 1) + i + 1) * NT * REC,
                                      G(recy) + (long)(j * nx + i) * NT * REC,
                                      G(recy) + (long)((j + 1) * nx + i) * NT * REC};
    const gptr<const double> cr = G(crec) + (long)c * NT * CREC;
    build_tables<NT>(P, fr, cr, tab);
    __syncthreads();
    const double *ctab = tab + 12 * NT * M;
    const long sx = (long)NT * P.ls, sy = (long)nx * NT * P.ls;
    const double dG = dtc[c];
    const double rdx = G(P.rdx)[i], rdy = G(P.rdy)[j];
    const double *rcx = P.rcx, *rcy = P.rcy;

    for (int ap = threadIdx.x; ap < P.nvp; ap += blockDim.x) {
        const int r = ap % P.Qp;
        if (r >= P.Q) continue;
        const double u = G(P.vu)[ap], v = G(P.vv)[ap];
        const int iu = G(P.viu)[ap], iv = G(P.viv)[ap];
        const double rh = href_of<TS>(P, ap), rb = 0.5 * P.K * rh;
        const int su = __builtin_amdgcn_readfirstlane(u > 0.0 ? 1 : 0);
        const int sv = __builtin_amdgcn_readfirstlane(v > 0.0 ? 1 : 0);
        const int fxo = su ? 1 : 0, fxi = 1 - fxo, fyo = sv ? 3 : 2, fyi = 5 - fyo;
        const int iU = su ? i - 1 : i + 1, jV = sv ? j - 1 : j + 1;
        const long oU = su ? -sx : sx, oV = sv ? -sy : sy;
        const double dxo = su ? G(P.xf)[i + 1] - G(P.xc)[i] : G(P.xf)[i] - G(P.xc)[i];
        const double dyo = sv ? G(P.yf)[j + 1] - G(P.yc)[j] : G(P.yf)[j] - G(P.yc)[j];
        const double dxi = su ? G(P.xf)[i] - G(P.xc)[iU] : G(P.xf)[i + 1] - G(P.xc)[iU];
        const double dyi = sv ? G(P.yf)[j] - G(P.yc)[jV] : G(P.yf)[j + 1] - G(P.yc)[jV];
        // limiter reciprocal centre distances: own cell and the two upwind neighbours
        const double rxm = rcx[i], rxp = rcx[i + 1], rym = rcy[j], ryp = rcy[j + 1];
        const double rUm = rcx[iU], rUp = rcx[iU + 1], rVm = rcy[jV], rVp = rcy[jV + 1];
        double hk[NT], bk[NT], dh[NT], db[NT];
        const long e0 = (long)c * NT * P.ls + ap;
#pragma unroll
        for (int n = 0; n < NT; n++) {
            double hc, bc, hW, bW, hE, bE, hS, bS, hN, bN, hUF, bUF, hUs, bUs, hUn, bUn, hVF, bVF, hVw, bVw, hVe, bVe;
            const TS *hp = h + e0 + (long)n * P.ls, *bp = b + e0 + (long)n * P.ls;
            hc = ldv<TS>(hp, 0, rh), bc = ldv<TS>(bp, 0, rb);
            hW = ldv<TS>(hp, -sx, rh), bW = ldv<TS>(bp, -sx, rb), hE = ldv<TS>(hp, sx, rh), bE = ldv<TS>(bp, sx, rb);
            hS = ldv<TS>(hp, -sy, rh), bS = ldv<TS>(bp, -sy, rb), hN = ldv<TS>(hp, sy, rh), bN = ldv<TS>(bp, sy, rb);
            // upwind x-neighbour: far value and diagonals; upwind y-neighbour likewise
            const TS *hq = hp + oU, *bq = bp + oU;
            hUF = ldv<TS>(hq, oU, rh), bUF = ldv<TS>(bq, oU, rb), hUs = ldv<TS>(hq, -sy, rh), bUs = ldv<TS>(bq, -sy, rb);
            hUn = ldv<TS>(hq, sy, rh), bUn = ldv<TS>(bq, sy, rb);
            const TS *hr = hp + oV, *br = bp + oV;
            hVF = ldv<TS>(hr, oV, rh), bVF = ldv<TS>(br, oV, rb), hVw = ldv<TS>(hr, -sx, rh), bVw = ldv<TS>(br, -sx, rb);
            hVe = ldv<TS>(hr, sx, rh), bVe = ldv<TS>(br, sx, rb);
            hk[n] = hc;
            bk[n] = bc;
            const double sxh = vanleer_fast((hc - hW) * rxm, (hE - hc) * rxp);
            const double sxb = vanleer_fast((bc - bW) * rxm, (bE - bc) * rxp);
            const double syh = vanleer_fast((hc - hS) * rym, (hN - hc) * ryp);
            const double syb = vanleer_fast((bc - bS) * rym, (bN - bc) * ryp);
            const double sh = u * sxh + v * syh, sb = u * sxb + v * syb;
            const double hU = su ? hW : hE, bU = su ? bW : bE;
            // U's x-slope from (U-1, U, U+1): for su the far value is U-1 and c is U+1
            const double xm_h = su ? hUF : hc, xp_h = su ? hc : hUF;
            const double xm_b = su ? bUF : bc, xp_b = su ? bc : bUF;
            const double sxhU = vanleer_fast((hU - xm_h) * rUm, (xp_h - hU) * rUp);
            const double sxbU = vanleer_fast((bU - xm_b) * rUm, (xp_b - bU) * rUp);
            const double syhU = vanleer_fast((hU - hUs) * rym, (hUn - hU) * ryp);
            const double sybU = vanleer_fast((bU - bUs) * rym, (bUn - bU) * ryp);
            const double hV = sv ? hS : hN, bV = sv ? bS : bN;
            const double ym_h = sv ? hVF : hc, yp_h = sv ? hc : hVF;
            const double ym_b = sv ? bVF : bc, yp_b = sv ? bc : bVF;
            const double syhV = vanleer_fast((hV - ym_h) * rVm, (yp_h - hV) * rVp);
            const double sybV = vanleer_fast((bV - ym_b) * rVm, (yp_b - bV) * rVp);
            const double sxhV = vanleer_fast((hV - hVw) * rxm, (hVe - hV) * rxp);
            const double sxbV = vanleer_fast((bV - bVw) * rxm, (bVe - bV) * rxp);
            const double *tbx = tab + (fxo * NT + n) * 3 * M, *tbxi = tab + (fxi * NT + n) * 3 * M;
            const double *tby = tab + (fyo * NT + n) * 3 * M, *tbyi = tab + (fyi * NT + n) * 3 * M;
            cdouble *rxo = wave_uniform(fr[fxo] + n * REC + REC_SIDE + REC_SIDEW * su);
            cdouble *rxi = wave_uniform(fr[fxi] + n * REC + REC_SIDE + REC_SIDEW * su);
            cdouble *ryo = wave_uniform(fr[fyo] + n * REC + REC_SIDE + REC_SIDEW * sv);
            cdouble *ryi = wave_uniform(fr[fyi] + n * REC + REC_SIDE + REC_SIDEW * sv);
            double Hxo, Bxo, Hxi, Bxi, Hyo, Byo, Hyi, Byi;
            face_flux(rxo, tbx[iu] * tbx[(1 + su) * M + iv], u, v, hc + sxh * dxo, bc + sxb * dxo, sh, sb, Hxo, Bxo);
            face_flux(ryo, tby[iv] * tby[(1 + sv) * M + iu], v, u, hc + syh * dyo, bc + syb * dyo, sh, sb, Hyo, Byo);
            face_flux(rxi, tbxi[iu] * tbxi[(1 + su) * M + iv], u, v, hU + sxhU * dxi, bU + sxbU * dxi,
                      u * sxhU + v * syhU, u * sxbU + v * sybU, Hxi, Bxi);
            face_flux(ryi, tbyi[iv] * tbyi[(1 + sv) * M + iu], v, u, hV + syhV * dyi, bV + sybV * dyi,
                      u * sxhV + v * syhV, u * sxbV + v * sybV, Hyi, Byi);
            const double dxh = su ? (Hxo - Hxi) : (Hxi - Hxo), dxb = su ? (Bxo - Bxi) : (Bxi - Bxo);
            const double dyh = sv ? (Hyo - Hyi) : (Hyi - Hyo), dyb = sv ? (Byo - Byi) : (Byi - Byo);
            dh[n] = dxh * rdx + dyh * rdy;
            db[n] = dxb * rdx + dyb * rdy;
            __builtin_amdgcn_sched_barrier(0);
        }
        collide_store<NT, TS>(P, cr, ctab, dG, u, v, iu, iv, hk, bk, dh, db, hn, bn, e0, rh, rb);
    }
}


// Cells within two of a wall (listed in cells[]): the general stencil with
// one-sided wall slopes and the diffuse-wall inflow.
template <int NT, typename TS>
__device__ inline void update_bnd_cell_d(const Params &P, const TS *__restrict__ h, const TS *__restrict__ b,
                                       const double *__restrict__ recx, const double *__restrict__ recy,
                                       const double *__restrict__ crec, const double *__restrict__ dtc,
                                       TS *__restrict__ hn, TS *__restrict__ bn, double *__restrict__ Wn, int c)
{
    extern __shared__ double tab[];
    const int M = P.Mt, nx = P.nx, ny = P.ny;
    const int i = c % nx, j = c / nx;
    scale_w<NT>(P, Wn, c);
    const gptr<const double> fr[4] = {G(recx) + (long)(j * (nx + 1) + i) * NT * REC, G(recx) + (long)(j * (nx + 1) + i + 1) * NT * REC,
                                      G(recy) + (long)(j * nx + i) * NT * REC,
                                      G(recy) + (long)((j + 1) * nx + i) * NT * REC};
    const gptr<const double> cr = G(crec) + (long)c * NT * CREC;
    build_tables<NT>(P, fr, cr, tab);
    __syncthreads();
    const double *ctab = tab + 12 * NT * M;
    const long sx = (long)NT * P.ls, sy = (long)nx * NT * P.ls;
    const double dG = dtc[c];
    const double rdx = G(P.rdx)[i], rdy = G(P.rdy)[j];
    const double dxe = G(P.xf)[i + 1] - G(P.xc)[i], dxw = G(P.xf)[i] - G(P.xc)[i];
    const double dyn = G(P.yf)[j + 1] - G(P.yc)[j], dys = G(P.yf)[j] - G(P.yc)[j];
    // stencil offsets clamped to the cell itself at the walls: every load is
    // unconditional (the one-sided slopes never read a clamped value)
    const int mx = wall_mode(i, nx), my = wall_mode(j, ny);
    const long oW = mx == 1 ? 0 : -sx, oE = mx == 2 ? 0 : sx, oS = my == 1 ? 0 : -sy, oN = my == 2 ? 0 : sy;
    const double rxm = G(P.rcx)[i], rxp = G(P.rcx)[i + 1], rym = G(P.rcy)[j], ryp = G(P.rcy)[j + 1];

    for (int ap = threadIdx.x; ap < P.nvp; ap += blockDim.x) {
        const int r = ap % P.Qp;
        if (r >= P.Q) continue;
        const double u = G(P.vu)[ap], v = G(P.vv)[ap];
        const int iu = G(P.viu)[ap], iv = G(P.viv)[ap];
        const double rh = href_of<TS>(P, ap), rb = 0.5 * P.K * rh;
        const int su = __builtin_amdgcn_readfirstlane(u > 0.0 ? 1 : 0);
        const int sv = __builtin_amdgcn_readfirstlane(v > 0.0 ? 1 : 0);
        const int fxo = su ? 1 : 0, fxi = su ? 0 : 1;
        const int fyo = sv ? 3 : 2, fyi = sv ? 2 : 3;
        const bool inx_wall = su ? (i == 0) : (i == nx - 1);
        const bool iny_wall = sv ? (j == 0) : (j == ny - 1);
        const int iU = su ? i - 1 : i + 1, jV = sv ? j - 1 : j + 1;
        const long oU = su ? -sx : sx, oV = sv ? -sy : sy;
        const double dxo = su ? dxe : dxw, dyo = sv ? dyn : dys;
        const double dxi = inx_wall ? 0.0 : (su ? G(P.xf)[i] - G(P.xc)[iU] : G(P.xf)[i + 1] - G(P.xc)[iU]);
        const double dyi = iny_wall ? 0.0 : (sv ? G(P.yf)[j] - G(P.yc)[jV] : G(P.yf)[j + 1] - G(P.yc)[jV]);
        // upwind neighbours U (x) and V (y), the cell itself where the wall is upwind
        const int iUc = inx_wall ? i : iU, jVc = iny_wall ? j : jV;
        const long oUc = inx_wall ? 0 : oU, oVc = iny_wall ? 0 : oV;
        const int mUx = wall_mode(iUc, nx), mVy = wall_mode(jVc, ny);
        const long oUF = (su ? mUx == 1 : mUx == 2) ? 0 : oU;  // far neighbour of U, relative to U
        const long oVF = (sv ? mVy == 1 : mVy == 2) ? 0 : oV;  // far neighbour of V, relative to V
        const double rUm = G(P.rcx)[iUc], rUp = G(P.rcx)[iUc + 1], rVm = G(P.rcy)[jVc], rVp = G(P.rcy)[jVc + 1];
        double hk[NT], bk[NT], dh[NT], db[NT];
        const long e0 = (long)c * NT * P.ls + ap;
        // the level loop unrolled up to three levels (the compiler can then
        // interleave one level's record loads and tables with the previous
        // level's arithmetic), kept rolled above for code size
        constexpr int UNR = NT <= 3 ? NT : 1;
#pragma unroll UNR
        for (int n = 0; n < NT; n++) {
            double hc, bc, hW, bW, hE, bE, hS, bS, hN, bN, hUF, bUF, hUs, bUs, hUn, bUn, hVF, bVF, hVw, bVw, hVe, bVe;
            const TS *hp = h + e0 + (long)n * P.ls, *bp = b + e0 + (long)n * P.ls;
            hc = ldv<TS>(hp, 0, rh), bc = ldv<TS>(bp, 0, rb);
            hW = ldv<TS>(hp, oW, rh), bW = ldv<TS>(bp, oW, rb);
            hE = ldv<TS>(hp, oE, rh), bE = ldv<TS>(bp, oE, rb);
            hS = ldv<TS>(hp, oS, rh), bS = ldv<TS>(bp, oS, rb);
            hN = ldv<TS>(hp, oN, rh), bN = ldv<TS>(bp, oN, rb);
            const TS *hq = hp + oUc, *bq = bp + oUc, *hr = hp + oVc, *br = bp + oVc;
            hUF = ldv<TS>(hq, oUF, rh), bUF = ldv<TS>(bq, oUF, rb);
            hUs = ldv<TS>(hq, oS, rh), bUs = ldv<TS>(bq, oS, rb);
            hUn = ldv<TS>(hq, oN, rh), bUn = ldv<TS>(bq, oN, rb);
            hVF = ldv<TS>(hr, oVF, rh), bVF = ldv<TS>(br, oVF, rb);
            hVw = ldv<TS>(hr, oW, rh), bVw = ldv<TS>(br, oW, rb);
            hVe = ldv<TS>(hr, oE, rh), bVe = ldv<TS>(br, oE, rb);
            hk[n] = hc;
            bk[n] = bc;
            const double sxh = slope_c(hW, hc, hE, mx, rxm, rxp), sxb = slope_c(bW, bc, bE, mx, rxm, rxp);
            const double syh = slope_c(hS, hc, hN, my, rym, ryp), syb = slope_c(bS, bc, bN, my, rym, ryp);
            const double sh = u * sxh + v * syh, sb = u * sxb + v * syb;
            const double *tbx = tab + (fxo * NT + n) * 3 * M;
            const double *tbxi = tab + (fxi * NT + n) * 3 * M;
            const double *tby = tab + (fyo * NT + n) * 3 * M;
            const double *tbyi = tab + (fyi * NT + n) * 3 * M;
            cdouble *rxo = wave_uniform(fr[fxo] + n * REC + REC_SIDE + REC_SIDEW * su);
            cdouble *rxi = wave_uniform(fr[fxi] + n * REC + REC_SIDE + REC_SIDEW * su);
            cdouble *ryo = wave_uniform(fr[fyo] + n * REC + REC_SIDE + REC_SIDEW * sv);
            cdouble *ryi = wave_uniform(fr[fyi] + n * REC + REC_SIDE + REC_SIDEW * sv);
            double Hxo, Bxo, Hxi, Bxi, Hyo, Byo, Hyi, Byi;
            face_flux(rxo, tbx[iu] * tbx[(1 + su) * M + iv], u, v, hc + sxh * dxo, bc + sxb * dxo, sh, sb, Hxo, Bxo);
            face_flux(ryo, tby[iv] * tby[(1 + sv) * M + iu], v, u, hc + syh * dyo, bc + syb * dyo, sh, sb, Hyo, Byo);
            const double exi = tbxi[iu] * tbxi[(1 + su) * M + iv];
            if (inx_wall) {
                face_flux(rxi, exi, u, v, 0.0, 0.0, 0.0, 0.0, Hxi, Bxi);
            } else {
                const double hU = su ? hW : hE, bU = su ? bW : bE;
                const double sxhU = su ? slope_c(hUF, hU, hc, mUx, rUm, rUp) : slope_c(hc, hU, hUF, mUx, rUm, rUp);
                const double sxbU = su ? slope_c(bUF, bU, bc, mUx, rUm, rUp) : slope_c(bc, bU, bUF, mUx, rUm, rUp);
                const double syhU = slope_c(hUs, hU, hUn, my, rym, ryp), sybU = slope_c(bUs, bU, bUn, my, rym, ryp);
                face_flux(rxi, exi, u, v, hU + sxhU * dxi, bU + sxbU * dxi, u * sxhU + v * syhU, u * sxbU + v * sybU,
                          Hxi, Bxi);
            }
            const double eyi = tbyi[iv] * tbyi[(1 + sv) * M + iu];
            if (iny_wall) {
                face_flux(ryi, eyi, v, u, 0.0, 0.0, 0.0, 0.0, Hyi, Byi);
            } else {
                const double hV = sv ? hS : hN, bV = sv ? bS : bN;
                const double syhV = sv ? slope_c(hVF, hV, hc, mVy, rVm, rVp) : slope_c(hc, hV, hVF, mVy, rVm, rVp);
                const double sybV = sv ? slope_c(bVF, bV, bc, mVy, rVm, rVp) : slope_c(bc, bV, bVF, mVy, rVm, rVp);
                const double sxhV = slope_c(hVw, hV, hVe, mx, rxm, rxp), sxbV = slope_c(bVw, bV, bVe, mx, rxm, rxp);
                face_flux(ryi, eyi, v, u, hV + syhV * dyi, bV + sybV * dyi, u * sxhV + v * syhV, u * sxbV + v * sybV,
                          Hyi, Byi);
            }
            const double dxh = su ? (Hxo - Hxi) : (Hxi - Hxo), dxb = su ? (Bxo - Bxi) : (Bxi - Bxo);
            const double dyh = sv ? (Hyo - Hyi) : (Hyi - Hyo), dyb = sv ? (Byo - Byi) : (Byi - Byo);
            dh[n] = dxh * rdx + dyh * rdy;
            db[n] = dxb * rdx + dyb * rdy;
            __builtin_amdgcn_sched_barrier(0);
        }
        collide_store<NT, TS>(P, cr, ctab, dG, u, v, iu, iv, hk, bk, dh, db, hn, bn, e0, rh, rb);
    }
}

}  // namespace hb
#include "hb_mixed.h"
namespace hb {

// FP64 storage: the FP64 bodies above; mixed storage: the FP32 bodies of
// hb_mixed.h, with the output policy OUT (OutStore).
template <int NT, typename TS, int OUT>
__device__ inline void update_int_cell(const Params &P, const TS *__restrict__ h, const TS *__restrict__ b,
                                       const double *__restrict__ recx, const double *__restrict__ recy,
                                       const double *__restrict__ crec, const double *__restrict__ dtc,
                                       TS *__restrict__ hn, TS *__restrict__ bn, double *__restrict__ Wn, int ci)
{
    if constexpr (sizeof(TS) == 4)
        update_int_cell_m<NT, OUT>(P, h, b, recx, recy, crec, dtc, hn, bn, Wn, ci);
    else
        update_int_cell_d<NT, TS>(P, h, b, recx, recy, crec, dtc, hn, bn, Wn, ci);
}
template <int NT, typename TS, int OUT>
__device__ inline void update_bnd_cell(const Params &P, const TS *__restrict__ h, const TS *__restrict__ b,
                                       const double *__restrict__ recx, const double *__restrict__ recy,
                                       const double *__restrict__ crec, const double *__restrict__ dtc,
                                       TS *__restrict__ hn, TS *__restrict__ bn, double *__restrict__ Wn, int c)
{
    if constexpr (sizeof(TS) == 4)
        update_bnd_cell_m<NT, OUT>(P, h, b, recx, recy, crec, dtc, hn, bn, Wn, c);
    else
        update_bnd_cell_d<NT, TS>(P, h, b, recx, recy, crec, dtc, hn, bn, Wn, c);
}

template <int NT, typename TS, bool SO = false>
__global__ __launch_bounds__(256, sizeof(TS) == 4 ? HB_UPD_WAVES_MIXED : HB_UPD_WAVES) void k_update_int(Params P, const TS *__restrict__ h,
                                                       const TS *__restrict__ b, const double *__restrict__ recx,
                                                       const double *__restrict__ recy,
                                                       const double *__restrict__ crec,
                                                       const double *__restrict__ dtc, TS *__restrict__ hn,
                                                       TS *__restrict__ bn, double *__restrict__ Wn)
{
    update_int_cell<NT, TS, (SO ? OUT_NT : 0) | OUT_BUF>(P, h, b, recx, recy, crec, dtc, hn, bn, Wn,
                                strip_cell(xcd_cell(blockIdx.x, gridDim.x), P.nx - 4, P.ny - 4));
}

template <int NT, typename TS, bool SO = false>
__global__ __launch_bounds__(256, 2) void k_update_bnd(Params P, const int *__restrict__ cells,
                                                       const TS *__restrict__ h, const TS *__restrict__ b,
                                                       const double *__restrict__ recx, const double *__restrict__ recy,
                                                       const double *__restrict__ crec,
                                                       const double *__restrict__ dtc, TS *__restrict__ hn,
                                                       TS *__restrict__ bn, double *__restrict__ Wn)
{
    update_bnd_cell<NT, TS, (SO ? OUT_NT : 0) | OUT_BUF>(P, h, b, recx, recy, crec, dtc, hn, bn, Wn, cells[xcd_cell(blockIdx.x, gridDim.x)]);
}

// ---------------------------------------------------------------- set-up kernels
template <typename TS>
__global__ void k_init(Params P, TS *h, TS *b, double *W)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nel = (long)P.nc * P.NT * P.ls;
    if (t < nel) {
        const int ap = t % P.ls;
        const bool valid = ap < P.nvp && (ap % P.Qp) < P.Q;
        const double u = valid ? P.vu[ap] : 0.0, v = valid ? P.vv[ap] : 0.0;
        const double H = valid ? exp(-(u * u + v * v)) / HB_PI : 0.0;
        if constexpr (sizeof(TS) == 4) {
            h[t] = 0.0f;  // rest state: deviation from H_ref is zero
            b[t] = 0.0f;
        } else {
            h[t] = H;
            b[t] = 0.5 * P.K * H;
        }
    }
    if (t < (long)P.nc * P.NT) {
        W[t * 4 + 0] = 1.0;
        W[t * 4 + 1] = 0.0;
        W[t * 4 + 2] = 0.0;
        W[t * 4 + 3] = (2.0 + P.K) / 4.0;
    }
}

// rest Maxwellian per velocity (reference of the mixed storage)
__global__ void k_vref(Params P, double *vref)
{
    const int ap = blockIdx.x * blockDim.x + threadIdx.x;
    if (ap < P.nvp) {
        const double u = P.vu[ap], v = P.vv[ap];
        vref[ap] = ((ap % P.Qp) < P.Q) ? exp(-(u * u + v * v)) / HB_PI : 0.0;
    }
}

// Per quadrant q (one wave each), the sums over its velocities of
// w u^a v^b H_ref for the ten monomials of degree <= 3 in the order
// 1, u, v, uu, uv, vv, uuu, uuv, uvv, vvv: the rest Maxwellian's share of the
// moment sums, which the mixed form's moments kernel adds to the sums of the
// stored deviations.  Runs after k_vref.
__global__ void k_restmom(Params P, double *rmom)
{
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc[10];
    for (int k = 0; k < 10; k++) acc[k] = 0.0;
    for (int r = lane; r < P.Q; r += 64) {
        const int ap = q * P.Qp + r;
        const double u = P.vu[ap], v = P.vv[ap], wh = P.vw[ap] * P.vref[ap];
        const double m[10] = {1.0, u, v, u * u, u * v, v * v, u * u * u, u * u * v, u * v * v, v * v * v};
        for (int k = 0; k < 10; k++) acc[k] += wh * m[k];
    }
    for (int k = 0; k < 10; k++) {
        double x = acc[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) rmom[q * 10 + k] = x;
    }
}

// E(u_k) = exp(-u_k^2) of the 1-D nodes, in FP64 (the reference the mixed
// form's deviation tables subtract; the same expression as the tables' own
// exponential at lam = 1, U = 0) and rounded to FP32 (multipliers)
// (the u nodes, then the v nodes)
__global__ void k_etab(Params P, double *ex64, float *er32)
{
    for (int k = threadIdx.x; k < P.M + P.Mv; k += blockDim.x) {
        const double x = k < P.M ? P.u1[k] : P.v1[k - P.M], e = exp(-x * x);
        ex64[k] = e;
        er32[k] = static_cast<float>(e);
    }
}

__device__ inline void dt_thread(const Params &P, const double *W, double *dtc, int c)
{
    if (c < P.nc) dtc[c] = local_dt(P, W + (long)c * P.NT * 4, c % P.nx, c / P.nx);
}

__global__ void k_dt(Params P, const double *W, double *dtc)
{
    dt_thread(P, W, dtc, blockIdx.x * blockDim.x + threadIdx.x);
}

// The next local steps and the residual of the step in one launch: blocks
// 0 .. gridDim.x - 2 take 256 cells each, the last block the residual sum
// (two tiny kernels cost mostly their launch).
__global__ __launch_bounds__(256) void k_dt_resid(Params P, const double *__restrict__ W, double *__restrict__ dtc,
                                                  const double *__restrict__ rpart, int nblk, double *__restrict__ ring,
                                                  int slot, int *__restrict__ flag)
{
    if (blockIdx.x + 1 < gridDim.x)
        dt_thread(P, W, dtc, blockIdx.x * 256 + threadIdx.x);
    else
        resid_block(P, rpart, nblk, ring, slot, flag);
}

// ---------------------------------------------------------------- harmonics
// per (cell, level): rho, U, V, T/T0 from W; P_xy, q_x, q_y from h, b about U, V
template <typename TS>
__global__ __launch_bounds__(256) void k_harm_vars(Params P, const TS *__restrict__ h, const TS *__restrict__ b,
                                                   const double *__restrict__ W, double *__restrict__ vars)
{
    __shared__ double red[3][256];
    const int c = blockIdx.x;
    for (int n = 0; n < P.NT; n++) {
        double p[4];
        prim4(P.K, W + ((long)c * P.NT + n) * 4, p);
        double s0 = 0, s1 = 0, s2 = 0;
        for (int ap = threadIdx.x; ap < P.nvp; ap += blockDim.x) {
            const long e = ((long)c * P.NT + n) * P.ls + ap;
            const double w = P.vw[ap], cu = P.vu[ap] - p[1], cv = P.vv[ap] - p[2];
            const double rh = href_of<TS>(P, ap);
            const double hh = ldv<TS>(h, e, rh), en = (cu * cu + cv * cv) * hh + ldv<TS>(b, e, 0.5 * P.K * rh);
            s0 += w * cu * cv * hh;
            s1 += w * cu * en;
            s2 += w * cv * en;
        }
        red[0][threadIdx.x] = s0;
        red[1][threadIdx.x] = s1;
        red[2][threadIdx.x] = s2;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s)
                for (int k = 0; k < 3; k++) red[k][threadIdx.x] += red[k][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double *o = vars + ((long)c * P.NT + n) * 7;
            o[0] = p[0];
            o[1] = p[1];
            o[2] = p[2];
            o[3] = 1.0 / p[3];
            o[4] = red[0][0];
            o[5] = 0.5 * red[1][0];
            o[6] = 0.5 * red[2][0];
        }
        __syncthreads();
    }
}

// thread per (var, k, cell): qhat_k = (1/NT) sum_n q_n exp(-i k 2 pi n / NT)
__global__ void k_harm_dft(Params P, const double *__restrict__ vars, double *__restrict__ re, double *__restrict__ im)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int NH = P.NH, NT = P.NT, nc = P.nc;
    if (t >= (long)7 * (NH + 1) * nc) return;
    const int c = t % nc, k = (t / nc) % (NH + 1), var = t / ((long)nc * (NH + 1));
    double sr = 0.0, si = 0.0;
    for (int n = 0; n < NT; n++) {
        const double th = 2.0 * HB_PI * k * n / NT;
        const double val = vars[((long)c * NT + n) * 7 + var];
        sr += val * cos(th);
        si -= val * sin(th);
    }
    re[t] = sr / NT;
    im[t] = si / NT;
}

}  // namespace hb
