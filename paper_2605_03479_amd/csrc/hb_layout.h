// Record layouts shared by the HB-UGKS kernels and their host runtime.
#pragma once

namespace hb {

// per (cell, level) velocity moments, K1 -> K2/K3
constexpr int NMOM = 55;      // per-quadrant sums: x-feed 21, y-feed 21, cell 13
constexpr int FEED_E = 0;     // u > 0 velocities, reconstructed on the east face
constexpr int FEED_W = 21;    // u < 0, west face
constexpr int FEED_N = 42;    // v > 0, north face
constexpr int FEED_S = 63;    // v < 0, south face
constexpr int FEED_CM = 84;   // cell raw moments of h (10) and b (3)
constexpr int FEED = 97;
// one feed (21): sum w h0 {1,u,v,uu,uv,vv,uuu,uuv,uvv,vvv}, sum w b0 {1,u,v},
// tangential slope moments (4), C5 moments (4); global (u, v) order.

// per (face, level) record, K2 -> K3/K5
constexpr int REC_SIDE = 4;   // [0..3] macro flux F, global frame
constexpr int REC_SIDEW = 25; // per side: lam, Un, Ut, Qh[10], Qb[10], c4, c5
constexpr int REC = 56;       // side 0 = velocities with u_n < 0, side 1 = u_n > 0

// per (cell, level) collision record, K3 -> K5: for W^k at [0..7], W^{k+1} at [8..15]:
// lam, U, V, A = rho lam/pi, A K/(2 lam), dG/(2 tau), s q_x, s q_y
// (s = (1-Pr) 4 lam^2 / (5 rho)); then [16] = 1/(1 + dG/(2 tau^{k+1})).
constexpr int CREC_T = 8;
constexpr int CREC = 20;

// Mixed form (FP32 per-velocity arithmetic on the deviations dh = h - H_ref,
// db = b - K/2 H_ref from the rest Maxwellian H_ref = exp(-u^2 - v^2)/pi).
// Every face flux is taken minus u_n H_ref, which is the same at every face
// and leaves the divergence unchanged, so with the face exponential
// e = (E_n + dn)(E_t + dt), E(x) = exp(-x^2) and dn, dt from tables,
//   u_n [e Q + c4 h0 + c5 s] - u_n H_ref
//     = u_n [E_n E_t Q' + (e - E_n E_t)(Q' + k0) + c4 dh0 + c5 s],
// Q' = Q - k0, k0 = (1 - c4)/pi (b: (1 - c4) K/(2 pi)).
// FP32 face record per (face, level), per side at [REC32_SIDEW * side]:
//   Q'_h[10], Q'_b[10] in the global monomial order 1, u, v, uu, uv, vv, uuu,
//   uuv, uvv, vvv; k0_h, k0_b, c4, c5.
constexpr int REC32_SIDEW = 24;
constexpr int REC32 = 48;
// FP32 collision record per (cell, level): for W^k at [0..8] and W^{k+1} at
// [9..17]: U, V, 2 lam, A, A - 1/pi, B = A K/(2 lam), B - K/(2 pi), s q_x,
// s q_y; then a0 = dG/(2 tau^k), a1 = dG/(2 tau^{k+1}), 1 - a0, 1/(1 + a1).
constexpr int CREC32_T = 9;
constexpr int CREC32 = 24;

// per cells-kernel block partial sums, K3 -> K4: [0..3] level-0 squared
// increments of W (residual of Eq. 43), [4 + n] mass of level n
constexpr int RPART = 4 + 11;

}  // namespace hb
