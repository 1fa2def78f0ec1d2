// Preconditioned D2Q9 GLBE collision with forcing for one node, in registers
// (the 2D form of Sec. 3: D2Q9 equilibrium moments, preconditioned source
// moments and rates), on deviations d = f - w rho0.
//
// Moment rows at the library's velocities (0 rest, 1..4 = +x -x +y -y,
// 5..8 = (+,+) (-,-) (+,-) (-,+)):
//   e   = 3|c|^2 - 4          : rest -4, axis -1, diagonal 2
//   e2  = (9|c|^4-21|c|^2+8)/2: rest  4, axis -2, diagonal 1
//   q_x = (3|c|^2 - 5) c_x    : axis -2 c_x, diagonal c_x   (q_y alike)
//   p_xx = c_x^2 - c_y^2, p_xy = c_x c_y
// With opposite directions stored as pairs, e, e2, p_xx, p_xy use pair sums and
// j, q pair differences; T^-1 = T^T diag(1/|T_k|^2) scatters the changes back.
// The j change is F/gamma whatever the rate; rho is unchanged.
#pragma once

#include "collide.hpp"

namespace lbm {

template <typename R>
__host__ __device__ __forceinline__ void raw_moments9(const R (&f)[Q9], R& drho, R& jx, R& jy) {
  const R d1 = f[1] - f[2], d3 = f[3] - f[4], d5 = f[5] - f[6], d7 = f[7] - f[8];
  drho = f[0] + ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
  jx = d1 + d5 + d7;
  jy = d3 + d5 - d7;
}

// In-place collision; returns the node's macroscopic fields (jz = uz = 0).
template <typename R>
__host__ __device__ __forceinline__ NodeMacro<R> collide9(R (&f)[Q9], R Fx, R Fy,
                                                          const CollideArgs<R>& c) {
  const R a1 = f[1] + f[2], d1 = f[1] - f[2];
  const R a3 = f[3] + f[4], d3 = f[3] - f[4];
  const R a5 = f[5] + f[6], d5 = f[5] - f[6];
  const R a7 = f[7] + f[8], d7 = f[7] - f[8];
  const R ax = a1 + a3, dg = a5 + a7;
  NodeMacro<R> o;
  o.drho = f[0] + ax + dg;
  o.jx = d1 + d5 + d7 + Fx * c.half_inv_gamma;
  o.jy = d3 + d5 - d7 + Fy * c.half_inv_gamma;
  o.jz = R(0);
  const R rho = c.rho0 + o.drho;
  const R irho = R(1) / rho;
  o.ux = o.jx * irho;
  o.uy = o.jy * irho;
  o.uz = R(0);
  // non-conserved moments of d
  const R m1 = R(-4) * f[0] - ax + R(2) * dg;
  const R m2 = R(4) * f[0] - R(2) * ax + dg;
  const R m4 = R(-2) * d1 + d5 + d7;
  const R m6 = R(-2) * d3 + d5 - d7;
  const R m7 = a1 - a3;
  const R m8 = a5 - a7;
  // preconditioned equilibria, deviation form (T w rho0 = rho0 (1, -2, 1, 0, ...))
  const R ig = c.inv_gamma * irho;
  const R jj = (o.jx * o.jx + o.jy * o.jy) * ig;
  const R q1 = R(-2) * o.drho + R(3) * jj;
  const R q2 = o.drho - R(3) * jj;
  const R q7 = (o.jx * o.jx - o.jy * o.jy) * ig;
  const R q8 = o.jx * o.jy * ig;
  // preconditioned sources: 1/gamma^2 on e, e2, p (1/gamma in the naive form),
  // 1/gamma on j and q
  const R Fu = (Fx * o.ux + Fy * o.uy) * c.inv_gamma2;
  const R S7 = R(2) * (Fx * o.ux - Fy * o.uy) * c.inv_gamma2;
  const R S8 = (Fx * o.uy + Fy * o.ux) * c.inv_gamma2;
  const R Fxg = Fx * c.inv_gamma, Fyg = Fy * c.inv_gamma;
  // scaled changes k = dm / |T|^2 (A = s/|T|^2, B = (1 - s/2)/|T|^2)
  const R k1 = -c.A[1] * (m1 - q1) + c.B[1] * (R(6) * Fu);
  const R k2 = -c.A[2] * (m2 - q2) - c.B[2] * (R(6) * Fu);
  const R k4 = -c.A[4] * (m4 + o.jx) - c.B[4] * Fxg;
  const R k6 = -c.A[6] * (m6 + o.jy) - c.B[6] * Fyg;
  const R k7 = -c.A[7] * (m7 - q7) + c.B[7] * S7;
  const R k8 = -c.A[8] * (m8 - q8) + c.B[8] * S8;
  const R bx = Fxg * R(1.0 / 6.0), by = Fyg * R(1.0 / 6.0);
  f[0] += R(-4) * k1 + R(4) * k2;
  const R E = -k1 - R(2) * k2;
  {
    const R Ex = E + k7, Ox = bx - R(2) * k4;
    f[1] += Ex + Ox;
    f[2] += Ex - Ox;
    const R Ey = E - k7, Oy = by - R(2) * k6;
    f[3] += Ey + Oy;
    f[4] += Ey - Oy;
  }
  const R D = R(2) * k1 + k2;
  const R Px = bx + k4, Py = by + k6;
  f[5] += (D + k8) + (Px + Py);
  f[6] += (D + k8) - (Px + Py);
  f[7] += (D - k8) + (Px - Py);
  f[8] += (D - k8) - (Px - Py);
  return o;
}

}  // namespace lbm
