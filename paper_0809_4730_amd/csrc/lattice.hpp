// Lattice constants for the gfx950 kernels: D3Q19 (flow) and D3Q7 (magnetic
// induction) velocity sets in the library's direction order.
//
// D3Q19 (Sec. 2, eq. velocityd3q19): 0 rest; 1..6 axis (+x,-x,+y,-y,+z,-z);
// 7..18 face diagonals, each followed by its opposite:
//   7 (+1,+1,0)  8 (-1,-1,0)  9 (+1,-1,0) 10 (-1,+1,0)
//  11 (+1,0,+1) 12 (-1,0,-1) 13 (+1,0,-1) 14 (-1,0,+1)
//  15 (0,+1,+1) 16 (0,-1,-1) 17 (0,+1,-1) 18 (0,-1,+1)
// Pairs (2k-1, 2k) are opposites, which the collision uses: even moments
// depend only on pair sums, odd moments only on pair differences.
//
// D3Q7 (Sec. 4): 0 rest, 1..6 axis in the same order; W0 = 1/4, W = 1/8,
// theta_m = 1/4 (N_m = 4).
//
// D2Q9 (Sec. 2, eq. velocityd2q9): 0 rest; 1..4 axis (+x,-x,+y,-y);
//   5 (+1,+1)  6 (-1,-1)  7 (+1,-1)  8 (-1,+1).
// D2Q5 (Sec. 4, eq. velocityd2q5): 0 rest, 1..4 axis as above; W0 = 1/3,
// W = 1/6, theta_m = 1/3 (N_m = 3).
#pragma once

#include <cstdint>

namespace lbm {

constexpr int Q19 = 19;
constexpr int Q7 = 7;

constexpr int8_t EX19[Q19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int8_t EY19[Q19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int8_t EZ19[Q19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

constexpr int OPP19(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

constexpr int8_t EX7[Q7] = {0, 1, -1, 0, 0, 0, 0};
constexpr int8_t EY7[Q7] = {0, 0, 0, 1, -1, 0, 0};
constexpr int8_t EZ7[Q7] = {0, 0, 0, 0, 0, 1, -1};
constexpr int OPP7(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

// Squared norms of the orthogonal moment basis rows (App. A order:
// rho, e, e2, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz,
// mx, my, mz).  T^-1 = T^T diag(1/norm).
constexpr double NORM19[Q19] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72,
                                12, 24, 4, 4, 4, 8, 8, 8};

constexpr int Q9 = 9;
constexpr int Q5 = 5;
constexpr int8_t EX9[Q9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int8_t EY9[Q9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
constexpr int OPP9(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
constexpr int8_t EX5[Q5] = {0, 1, -1, 0, 0};
constexpr int8_t EY5[Q5] = {0, 0, 0, 1, -1};
constexpr int OPP5(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
// Squared norms of the D2Q9 rows (rho, e, e2, jx, qx, jy, qy, pxx, pxy).
constexpr double NORM9[Q9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};
constexpr double W5_REST = 1.0 / 3.0;
constexpr double W5_AXIS = 1.0 / 6.0;
constexpr double THETA_M2 = 1.0 / 3.0;

constexpr double W7_REST = 0.25;
constexpr double W7_AXIS = 0.125;
constexpr double THETA_M = 0.25;

}  // namespace lbm
