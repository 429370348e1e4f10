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

}  // namespace hb
