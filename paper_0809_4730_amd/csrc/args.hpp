// Host-side preparation of the kernels' constant arguments from lbm_params:
// rates scaled by the basis norms, the preconditioning factors of the source
// and equilibrium terms, wall-momentum terms, and the induction constants.
#pragma once

#include "../../include/lbm_capi.h"
#include "common.hpp"

namespace lbm {

template <typename R>
CollideArgs<R> collide_args(const lbm_params& p) {
  CollideArgs<R> c;
  c.rho0 = R(p.rho0);
  c.inv_gamma = R(1.0 / p.gamma);
  // the F.u source moments carry 1/gamma^2 (P_S); the naive form uses 1/gamma
  c.inv_gamma2 = R(p.source_mode == 1 ? 1.0 / p.gamma : 1.0 / (p.gamma * p.gamma));
  c.half_inv_gamma = R(0.5 / p.gamma);
  const bool d2 = p.lattice == LBM_D2Q9;
  for (int k = 0; k < 19; ++k) {
    const double norm = d2 ? (k < Q9 ? NORM9[k] : 1.0) : NORM19[k];
    const double s = (d2 && k >= Q9) ? 1.0 : p.s[k];
    c.A[k] = R(s / norm);
    c.B[k] = R((1.0 - 0.5 * s) / norm);
  }
  for (int a = 0; a < 3; ++a) c.F[a] = R(p.force_const[a]);
  // link bounce-back with wall momentum: 6 w_a rho0 (e_a . u_face); w by shell
  c.moving = 0;
  for (int a = 0; a < Q19; ++a) {
    const int e2 = EX19[a] * EX19[a] + EY19[a] * EY19[a] + EZ19[a] * EZ19[a];
    const double w = e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    for (int f = 0; f < 6; ++f) {
      const double eu = EX19[a] * p.wall_u[f][0] + EY19[a] * p.wall_u[f][1] + EZ19[a] * p.wall_u[f][2];
      c.wall[a][f] = R(6.0 * w * p.rho0 * eu);
      if (eu != 0.0) c.moving = 1;
    }
  }
  return c;
}

template <typename R>
MagArgs<R> mag_args(const lbm_params& p) {
  MagArgs<R> m{};
  if (!p.mhd) {
    m.w_rest = R(W7_REST);
    m.w_axis = R(W7_AXIS);
    return m;
  }
  // theta_m = 1/N_m and the weights: N_m = 4 (D3Q7) or 3 (D2Q5), Sec. 4
  const bool d2 = p.lattice == LBM_D2Q9;
  const double theta = d2 ? THETA_M2 : THETA_M;
  const double tau = p.eta / (p.gamma_m * theta) + 0.5;
  m.omega = R(1.0 / tau);
  m.adv = R(p.chi / (p.gamma_m * theta));
  m.a_coef = R(-1.0 / (p.mu * p.chi * tau * theta));
  m.kappa = R(2.0 / (p.mu * p.gamma_m * tau * theta));
  for (int a = 0; a < 3; ++a) m.B0[a] = R(p.B0[a]);
  m.w_rest = R(d2 ? W5_REST : W7_REST);
  m.w_axis = R(d2 ? W5_AXIS : W7_AXIS);
  return m;
}

}  // namespace lbm
