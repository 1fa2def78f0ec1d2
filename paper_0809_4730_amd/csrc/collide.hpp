// Preconditioned GLBE collision with forcing for one node, in registers.
//
// Implements f~ = f + T^-1 [ -Lambda* (f^ - f^eq*) + (I - Lambda*/2) P_S S^ ]
// (Sec. 3, eq. prelax_term) on deviations d = f - w rho0.  The moment
// transform is not a matrix product: with opposite directions stored as pairs,
// every even moment of the D3Q19 basis is an integer combination of pair sums
// and every odd moment of pair differences, and T^-1 = T^T diag(1/|T_k|^2)
// maps the scaled moment changes back the same way (the orthogonality and
// integer entries of T, Sec. 2).  About 270 flops per node.
//
// Conserved moments: rho is unchanged; the j_k change is F_k/gamma whatever the
// rate (m - m^eq = -F/(2 gamma) for j), so their rates never appear.
#pragma once

#include "common.hpp"

namespace lbm {

template <typename R>
struct NodeMacro {
  R drho;        // rho - rho0
  R jx, jy, jz;  // momentum including F/(2 gamma)
  R ux, uy, uz;  // j / rho
  R irho;        // 1 / rho
};

// Opposite directions are stored as adjacent pairs: their sums carry the even
// moments, their differences the odd ones.
template <typename R>
struct Pairs19 {
  R f0;
  R sx, dx, sy, dy, sz, dz;                      // axis pairs
  R sa, Ad, sb, Bd, sc, Cd, sd, Dd, se, Ed, sg, Gd;  // diagonal pairs
  R sax, sab, scd, seg, sdg;                     // partial sums of the pair sums
  R oxd, oyd, ozd;                               // diagonal parts of sum f e
  R drho;                                        // sum f (deviations)
};

template <typename R>
__host__ __device__ __forceinline__ Pairs19<R> pairs19(const R (&f)[Q19]) {
  Pairs19<R> p;
  p.f0 = f[0];
  p.sx = f[1] + f[2], p.dx = f[1] - f[2];
  p.sy = f[3] + f[4], p.dy = f[3] - f[4];
  p.sz = f[5] + f[6], p.dz = f[5] - f[6];
  p.sa = f[7] + f[8], p.Ad = f[7] - f[8];      // (+1,+1,0)
  p.sb = f[9] + f[10], p.Bd = f[9] - f[10];    // (+1,-1,0)
  p.sc = f[11] + f[12], p.Cd = f[11] - f[12];  // (+1,0,+1)
  p.sd = f[13] + f[14], p.Dd = f[13] - f[14];  // (+1,0,-1)
  p.se = f[15] + f[16], p.Ed = f[15] - f[16];  // (0,+1,+1)
  p.sg = f[17] + f[18], p.Gd = f[17] - f[18];  // (0,+1,-1)
  p.sax = p.sx + p.sy + p.sz;
  p.sab = p.sa + p.sb, p.scd = p.sc + p.sd, p.seg = p.se + p.sg;
  p.sdg = p.sab + p.scd + p.seg;
  p.drho = p.f0 + p.sax + p.sdg;
  p.oxd = p.Ad + p.Bd + p.Cd + p.Dd;
  p.oyd = p.Ad - p.Bd + p.Ed + p.Gd;
  p.ozd = p.Cd - p.Dd + p.Ed - p.Gd;
  return p;
}

// Density deviation and raw momentum sum_a f_a e_a (no force term).
template <typename R>
__host__ __device__ __forceinline__ void raw_moments(const R (&f)[Q19], R& drho, R& jx, R& jy, R& jz) {
  const Pairs19<R> p = pairs19<R>(f);
  drho = p.drho;
  jx = p.dx + p.oxd;
  jy = p.dy + p.oyd;
  jz = p.dz + p.ozd;
}

// Fields of a node under force F: j = sum f e + F/(2 gamma), u = j / rho
// (Sec. 3, preconditioned hydrodynamic fields).
template <typename R>
__host__ __device__ __forceinline__ NodeMacro<R> macro_of(const Pairs19<R>& p, R Fx, R Fy, R Fz,
                                                          const CollideArgs<R>& c) {
  NodeMacro<R> o;
  o.drho = p.drho;
  o.jx = p.dx + p.oxd + Fx * c.half_inv_gamma;
  o.jy = p.dy + p.oyd + Fy * c.half_inv_gamma;
  o.jz = p.dz + p.ozd + Fz * c.half_inv_gamma;
  o.irho = R(1) / (c.rho0 + p.drho);
  o.ux = o.jx * o.irho;
  o.uy = o.jy * o.irho;
  o.uz = o.jz * o.irho;
  return o;
}

template <typename R>
__host__ __device__ __forceinline__ NodeMacro<R> macro19(const R (&f)[Q19], R Fx, R Fy, R Fz,
                                                         const CollideArgs<R>& c) {
  return macro_of<R>(pairs19<R>(f), Fx, Fy, Fz, c);
}

// f_a += sum_k T_ka k_k for the scaled moment changes k_k (k_k = dm_k / |T_k|^2;
// bx, by, bz are the changes of j_x, j_y, j_z over |T_j|^2 = 10; rho is never
// changed).  T_ka is the value of row polynomial k at e_a (App. A basis).
template <typename R>
__host__ __device__ __forceinline__ void scatter_moments(R (&f)[Q19], R k1, R k2, R k4, R k6, R k8,
                                                         R k9, R k10, R k11, R k12, R k13, R k14,
                                                         R k15, R k16, R k17, R k18, R bx, R by,
                                                         R bz) {
  f[0] += R(-30) * k1 + R(12) * k2;
  const R e_ax = R(-11) * k1 - R(4) * k2;
  {
    const R E = e_ax + R(2) * k9 - R(4) * k10;
    const R O = bx - R(4) * k4;
    f[1] += E + O;
    f[2] += E - O;
  }
  {
    const R E = e_ax - k9 + R(2) * k10 + k11 - R(2) * k12;
    const R O = by - R(4) * k6;
    f[3] += E + O;
    f[4] += E - O;
  }
  {
    const R E = e_ax - k9 + R(2) * k10 - k11 + R(2) * k12;
    const R O = bz - R(4) * k8;
    f[5] += E + O;
    f[6] += E - O;
  }
  const R e_dg = R(8) * k1 + k2;
  {  // xy diagonals
    const R E = e_dg + k9 + k10 + k11 + k12;
    const R Px = bx + k4 + k16, Py = by + k6 - k17;
    f[7] += (E + k13) + (Px + Py);
    f[8] += (E + k13) - (Px + Py);
    f[9] += (E - k13) + (Px - Py);
    f[10] += (E - k13) - (Px - Py);
  }
  {  // xz diagonals
    const R E = e_dg + k9 + k10 - k11 - k12;
    const R Qx = bx + k4 - k16, Qz = bz + k8 + k18;
    f[11] += (E + k15) + (Qx + Qz);
    f[12] += (E + k15) - (Qx + Qz);
    f[13] += (E - k15) + (Qx - Qz);
    f[14] += (E - k15) - (Qx - Qz);
  }
  {  // yz diagonals
    const R E = e_dg - R(2) * (k9 + k10);
    const R Ry = by + k6 + k17, Rz = bz + k8 - k18;
    f[15] += (E + k14) + (Ry + Rz);
    f[16] += (E + k14) - (Ry + Rz);
    f[17] += (E - k14) + (Ry - Rz);
    f[18] += (E - k14) - (Ry - Rz);
  }
}

template <typename R>
__host__ __device__ __forceinline__ NodeMacro<R> collide19(R (&f)[Q19], R Fx, R Fy, R Fz,
                                                  const CollideArgs<R>& c) {
  const Pairs19<R> p = pairs19<R>(f);
  const NodeMacro<R> mac = macro_of<R>(p, Fx, Fy, Fz, c);
  const R sx = p.sx, dx = p.dx, sy = p.sy, dy = p.dy, sz = p.sz, dz = p.dz;
  const R sa = p.sa, Ad = p.Ad, sb = p.sb, Bd = p.Bd, sc = p.sc, Cd = p.Cd;
  const R sd = p.sd, Dd = p.Dd, se = p.se, Ed = p.Ed, sg = p.sg, Gd = p.Gd;
  const R sax = p.sax, sab = p.sab, scd = p.scd, seg = p.seg, sdg = p.sdg;
  const R oxd = p.oxd, oyd = p.oyd, ozd = p.ozd;
  const R drho = p.drho;
  const R jx = mac.jx, jy = mac.jy, jz = mac.jz;
  const R ux = mac.ux, uy = mac.uy, uz = mac.uz;
  const R igr = c.inv_gamma * mac.irho;  // 1/(gamma rho)

  // non-conserved moments of the deviations (T d)
  const R m1 = R(-30) * f[0] - R(11) * sax + R(8) * sdg;
  const R m2 = R(12) * f[0] - R(4) * sax + sdg;
  const R m4 = R(-4) * dx + oxd;
  const R m6 = R(-4) * dy + oyd;
  const R m8 = R(-4) * dz + ozd;
  const R m9 = R(2) * sx - sy - sz + sab + scd - R(2) * seg;
  const R m10 = R(-4) * sx + R(2) * (sy + sz) + sab + scd - R(2) * seg;
  const R m11 = sy - sz + sab - scd;
  const R m12 = R(2) * (sz - sy) + sab - scd;
  const R m13 = sa - sb;
  const R m14 = se - sg;
  const R m15 = sc - sd;
  const R m16 = Ad + Bd - Cd - Dd;
  const R m17 = Ed + Gd - Ad + Bd;
  const R m18 = Cd - Dd - Ed + Gd;

  // preconditioned equilibria minus the rest state (Sec. 3, D3Q19 list)
  const R jxx = jx * jx, jyy = jy * jy, jzz = jz * jz;
  const R jj = (jxx + jyy + jzz) * igr;
  const R eq1 = R(-11) * drho + R(19) * jj;
  const R eq2 = R(3) * drho - R(5.5) * jj;
  const R eq4 = R(-2.0 / 3.0) * jx;
  const R eq6 = R(-2.0 / 3.0) * jy;
  const R eq8 = R(-2.0 / 3.0) * jz;
  const R eq9 = (R(2) * jxx - jyy - jzz) * igr;
  const R eq11 = (jyy - jzz) * igr;
  const R eq13 = jx * jy * igr;
  const R eq14 = jy * jz * igr;
  const R eq15 = jx * jz * igr;

  // preconditioned moment sources P_S S^ (App. A list, Sec. 3 P_S)
  const R g1 = c.inv_gamma, g2 = c.inv_gamma2;
  const R Fu = (Fx * ux + Fy * uy + Fz * uz) * g2;
  const R Xn = (R(2) * Fx * ux - Fy * uy - Fz * uz) * g2;
  const R Yn = (Fy * uy - Fz * uz) * g2;

  // scaled changes k_k = dm_k / |T_k|^2
  const R k1 = c.B[1] * (R(38) * Fu) - c.A[1] * (m1 - eq1);
  const R k2 = c.B[2] * (R(-11) * Fu) - c.A[2] * (m2 - eq2);
  const R k4 = c.B[4] * (R(-2.0 / 3.0) * Fx * g1) - c.A[4] * (m4 - eq4);
  const R k6 = c.B[6] * (R(-2.0 / 3.0) * Fy * g1) - c.A[6] * (m6 - eq6);
  const R k8 = c.B[8] * (R(-2.0 / 3.0) * Fz * g1) - c.A[8] * (m8 - eq8);
  const R k9 = c.B[9] * (R(2) * Xn) - c.A[9] * (m9 - eq9);
  const R k10 = c.B[10] * (-Xn) - c.A[10] * (m10 + R(0.5) * eq9);
  const R k11 = c.B[11] * (R(2) * Yn) - c.A[11] * (m11 - eq11);
  const R k12 = c.B[12] * (-Yn) - c.A[12] * (m12 + R(0.5) * eq11);
  const R k13 = c.B[13] * ((Fx * uy + Fy * ux) * g2) - c.A[13] * (m13 - eq13);
  const R k14 = c.B[14] * ((Fy * uz + Fz * uy) * g2) - c.A[14] * (m14 - eq14);
  const R k15 = c.B[15] * ((Fx * uz + Fz * ux) * g2) - c.A[15] * (m15 - eq15);
  const R k16 = -c.A[16] * m16;
  const R k17 = -c.A[17] * m17;
  const R k18 = -c.A[18] * m18;
  const R bx = Fx * g1 * R(0.1);  // j change F/gamma over |T_j|^2 = 10
  const R by = Fy * g1 * R(0.1);
  const R bz = Fz * g1 * R(0.1);

  // back to velocity space: f_a += sum_k T_ka k_k
  scatter_moments<R>(f, k1, k2, k4, k6, k8, k9, k10, k11, k12, k13, k14, k15, k16, k17, k18, bx,
                     by, bz);

  return mac;
}


// Moments t = T v of a 19-vector (all rows; used by the adjoint).
template <typename R>
struct Moments19 {
  R t[Q19];
};

template <typename R>
__host__ __device__ __forceinline__ void moments_all(const R (&v)[Q19], R (&t)[Q19]) {
  const R sx = v[1] + v[2], dx = v[1] - v[2];
  const R sy = v[3] + v[4], dy = v[3] - v[4];
  const R sz = v[5] + v[6], dz = v[5] - v[6];
  const R sa = v[7] + v[8], Ad = v[7] - v[8];
  const R sb = v[9] + v[10], Bd = v[9] - v[10];
  const R sc = v[11] + v[12], Cd = v[11] - v[12];
  const R sd = v[13] + v[14], Dd = v[13] - v[14];
  const R se = v[15] + v[16], Ed = v[15] - v[16];
  const R sg = v[17] + v[18], Gd = v[17] - v[18];
  const R sax = sx + sy + sz;
  const R sab = sa + sb, scd = sc + sd, seg = se + sg;
  const R sdg = sab + scd + seg;
  const R oxd = Ad + Bd + Cd + Dd, oyd = Ad - Bd + Ed + Gd, ozd = Cd - Dd + Ed - Gd;
  t[0] = v[0] + sax + sdg;
  t[1] = R(-30) * v[0] - R(11) * sax + R(8) * sdg;
  t[2] = R(12) * v[0] - R(4) * sax + sdg;
  t[3] = dx + oxd;
  t[4] = R(-4) * dx + oxd;
  t[5] = dy + oyd;
  t[6] = R(-4) * dy + oyd;
  t[7] = dz + ozd;
  t[8] = R(-4) * dz + ozd;
  t[9] = R(2) * sx - sy - sz + sab + scd - R(2) * seg;
  t[10] = R(-4) * sx + R(2) * (sy + sz) + sab + scd - R(2) * seg;
  t[11] = sy - sz + sab - scd;
  t[12] = R(2) * (sz - sy) + sab - scd;
  t[13] = sa - sb;
  t[14] = se - sg;
  t[15] = sc - sd;
  t[16] = Ad + Bd - Cd - Dd;
  t[17] = Ed + Gd - Ad + Bd;
  t[18] = Cd - Dd - Ed + Gd;
}

// Transpose of the linearised collision at the pre-collision state f (with
// force F): given lam = dQ/df~ (the adjoint of the post-collision values),
// returns nu = (df~/df)^T lam and g = (df~/dF)^T lam.
//
// With lhat = diag(1/|T_k|^2) T lam, the collision's change is
// sum_k lhat_k dm_k with dm_k = -s_k (m_k - eq_k) + (1 - s_k/2) S*_k for the
// non-conserved k, and the conserved moments contribute F/gamma to j only.
// The m_k term transposes to -T^T (s lhat); the equilibrium and source terms
// are a scalar function Phi(drho, j, F) whose derivatives enter as
// dPhi/drho (every direction) and e_a . dPhi/dj; F enters directly and
// through j = sum f e + F/(2 gamma).
template <typename R>
__host__ __device__ __forceinline__ void collide19_adjoint(const R (&f)[Q19], R Fx, R Fy, R Fz,
                                                           const CollideArgs<R>& c,
                                                           const R (&lam)[Q19], R (&nu)[Q19],
                                                           R& gx, R& gy, R& gz) {
  // forward quantities of this node
  R drho, jx, jy, jz;
  raw_moments<R>(f, drho, jx, jy, jz);
  jx += Fx * c.half_inv_gamma;
  jy += Fy * c.half_inv_gamma;
  jz += Fz * c.half_inv_gamma;
  const R rho = c.rho0 + drho;
  const R irho = R(1) / rho;
  const R ux = jx * irho, uy = jy * irho, uz = jz * irho;
  const R G = c.inv_gamma * irho;

  R t[Q19];
  moments_all<R>(lam, t);
  // a_k = s_k lhat_k (equilibrium / moment weight), b_k = (1 - s_k/2) lhat_k (source weight)
  const R a1 = c.A[1] * t[1], a2 = c.A[2] * t[2], a4 = c.A[4] * t[4], a6 = c.A[6] * t[6];
  const R a8 = c.A[8] * t[8], a9 = c.A[9] * t[9], a10 = c.A[10] * t[10], a11 = c.A[11] * t[11];
  const R a12 = c.A[12] * t[12], a13 = c.A[13] * t[13], a14 = c.A[14] * t[14];
  const R a15 = c.A[15] * t[15], a16 = c.A[16] * t[16], a17 = c.A[17] * t[17];
  const R a18 = c.A[18] * t[18];
  const R b1 = c.B[1] * t[1], b2 = c.B[2] * t[2], b4 = c.B[4] * t[4], b6 = c.B[6] * t[6];
  const R b8 = c.B[8] * t[8], b9 = c.B[9] * t[9], b10 = c.B[10] * t[10], b11 = c.B[11] * t[11];
  const R b12 = c.B[12] * t[12], b13 = c.B[13] * t[13], b14 = c.B[14] * t[14];
  const R b15 = c.B[15] * t[15];

  // quadratic form of the equilibria: sum_k a_k eq_k(j)|_nonlinear = G j^T M j
  const R c0 = R(19) * a1 - R(5.5) * a2;
  const R A9 = a9 - R(0.5) * a10, A11 = a11 - R(0.5) * a12;
  const R Mxx = c0 + R(2) * A9, Myy = c0 - A9 + A11, Mzz = c0 - A9 - A11;
  const R Mxy = R(0.5) * a13, Myz = R(0.5) * a14, Mxz = R(0.5) * a15;
  // bilinear form of the sources: sum_k b_k S*_k|_{F u} = F^T N u / gamma^2
  const R cS = R(38) * b1 - R(11) * b2;
  const R B9 = R(2) * b9 - b10, B11 = R(2) * b11 - b12;
  const R Nxx = cS + R(2) * B9, Nyy = cS - B9 + B11, Nzz = cS - B9 - B11;
  const R Nxy = b13, Nyz = b14, Nxz = b15;

  const R Mjx = Mxx * jx + Mxy * jy + Mxz * jz;
  const R Mjy = Mxy * jx + Myy * jy + Myz * jz;
  const R Mjz = Mxz * jx + Myz * jy + Mzz * jz;
  const R jMj = jx * Mjx + jy * Mjy + jz * Mjz;
  const R NFx = Nxx * Fx + Nxy * Fy + Nxz * Fz;
  const R NFy = Nxy * Fx + Nyy * Fy + Nyz * Fz;
  const R NFz = Nxz * Fx + Nyz * Fy + Nzz * Fz;
  const R NFu = NFx * ux + NFy * uy + NFz * uz;
  const R g2 = c.inv_gamma2;

  const R a_rho = (R(-11) * a1 + R(3) * a2) - (G * jMj + g2 * NFu) * irho;
  const R ajx = R(-2.0 / 3.0) * a4 + R(2) * G * Mjx + g2 * NFx * irho;
  const R ajy = R(-2.0 / 3.0) * a6 + R(2) * G * Mjy + g2 * NFy * irho;
  const R ajz = R(-2.0 / 3.0) * a8 + R(2) * G * Mjz + g2 * NFz * irho;

#pragma unroll
  for (int a = 0; a < Q19; ++a) nu[a] = lam[a];
  scatter_moments<R>(nu, -a1, -a2, -a4, -a6, -a8, -a9, -a10, -a11, -a12, -a13, -a14, -a15, -a16,
                     -a17, -a18, R(0), R(0), R(0));
#pragma unroll
  for (int a = 0; a < Q19; ++a)
    nu[a] += a_rho + R(EX19[a]) * ajx + R(EY19[a]) * ajy + R(EZ19[a]) * ajz;

  const R Nux = Nxx * ux + Nxy * uy + Nxz * uz;
  const R Nuy = Nxy * ux + Nyy * uy + Nyz * uz;
  const R Nuz = Nxz * ux + Nyz * uy + Nzz * uz;
  const R g1 = c.inv_gamma;
  gx = g2 * Nux - R(2.0 / 3.0) * g1 * b4 + ajx * c.half_inv_gamma + g1 * R(0.1) * t[3];
  gy = g2 * Nuy - R(2.0 / 3.0) * g1 * b6 + ajy * c.half_inv_gamma + g1 * R(0.1) * t[5];
  gz = g2 * Nuz - R(2.0 / 3.0) * g1 * b8 + ajz * c.half_inv_gamma + g1 * R(0.1) * t[7];
}

}  // namespace lbm
