// gfx950 kernels of the two-dimensional variants: the preconditioned D2Q9
// GLBE with forcing, and its coupling to the preconditioned D2Q5 vector
// induction LKE (Sec. 2 eq. velocityd2q9, Sec. 3 D2Q9 lists, Sec. 4 eq.
// velocityd2q5).  Same structure as the 3D kernels: one thread per node of an
// nx x ny x 1 lattice, structure-of-arrays populations, pull streaming with
// halfway bounce-back, FP64 residual bookkeeping every check.
//
// In 2D the field is in-plane, B = (B_x, B_y), the current is out of plane,
// J_z, and the Lorentz force is J_z (-B_y, B_x).  Magnetic populations are held
// as deviations from W B0, field component outermost: g[j][a], j in {x, y}.
#include <type_traits>

#include "collide2d.hpp"
#include "launch.hpp"
#include "stream.hpp"

namespace lbm {

// Opposite directions are adjacent planes (pairs 1-2, 3-4, ...), as in 3D, so
// the pull offsets are taken relative to each pair's lower plane.
// KEEP0: streaming loads of the moving populations' planes, the rest
// population's plane read cacheable (with store9's KEEP0 it stays in the
// last-level cache from step to step).
template <typename S, bool WIDE, bool KEEP0 = false, int A = 0>
__device__ __forceinline__ void gather9(const S* __restrict__ fin, int64_t stride, uint32_t n,
                                        const Nbr& b, typename Storage<S>::R (&f)[Q9]) {
  if constexpr (A < Q9) {
    int32_t off;
    const bool bounce = pull_source<EX9[A], EY9[A], 0>(b, off);
    const S* base = fin + static_cast<int64_t>(pair_plane<A>()) * stride;
    f[A] = Storage<S>::template ld<KEEP0 && A != 0>(
        elem<WIDE>(base, pull_offset<A>(bounce, off, n, static_cast<uint32_t>(stride))));
    gather9<S, WIDE, KEEP0, A + 1>(fin, stride, n, b, f);
  }
}

// KEEP0: the rest population's plane keeps cacheable stores under NT, so that
// with the step's cacheable loads it stays in the last-level cache.
template <typename S, bool NT, bool WIDE, bool KEEP0 = false>
__device__ __forceinline__ void store9(S* __restrict__ fout, const GridArgs& g, uint32_t n,
                                       const typename Storage<S>::R (&f)[Q9]) {
  store_planes<S, NT, WIDE, Q9, KEEP0>(fout, g, n, f);
}

// Anti-bounce-back at a wall in deviation form: d_a = -d~_opp(a).
// NTL: streaming loads.
template <typename R, bool WIDE, bool NTL = false, int A = 0>
__device__ __forceinline__ void gather_g5(const R* __restrict__ gin, int64_t stride, uint32_t n,
                                          const Nbr& b, R (&g)[2][Q5]) {
  if constexpr (A < Q5) {
    int32_t off;
    const bool bounce = pull_source<EX5[A], EY5[A], 0>(b, off);
    const uint32_t i = pull_offset<A>(bounce, off, n, static_cast<uint32_t>(stride));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const R v = ld_pop<NTL>(elem<WIDE>(gin + static_cast<int64_t>(j * Q5 + pair_plane<A>()) * stride, i));
      g[j][A] = bounce ? -v : v;
    }
    gather_g5<R, WIDE, NTL, A + 1>(gin, stride, n, b, g);
  }
}

template <typename R, bool WIDE>
__device__ __forceinline__ void load_force2(const GridArgs& g, const CollideArgs<R>& c,
                                            const R* __restrict__ force, bool field, uint32_t n,
                                            R& Fx, R& Fy) {
  if (field) {
    Fx = *elem<WIDE>(force, n);
    Fy = *elem<WIDE>(force + g.stride, n);
  } else {
    Fx = c.F[0];
    Fy = c.F[1];
  }
}

// The node's two-component velocity snapshot of the previous check, loaded
// with the populations so that its latency hides behind theirs.
template <typename R, bool WIDE>
__device__ __forceinline__ void load_usnap2(const GridArgs& g, const R* __restrict__ usnap, uint32_t n,
                                            R (&uold)[2]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) uold[k] = *elem<WIDE>(usnap + static_cast<int64_t>(k) * g.stride, n);
}

// FP64 residual bookkeeping of one node, given its snapshot from load_usnap2.
template <typename R, bool WIDE, bool NT>
__device__ __forceinline__ void check_node2(const GridArgs& g, R* __restrict__ usnap, uint32_t n,
                                            const R (&uold)[2], const NodeMacro<R>& mac,
                                            double (&acc)[kPartials]) {
  const R ur[2] = {mac.ux, mac.uy};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    R* p = elem<WIDE>(usnap + static_cast<int64_t>(k) * g.stride, n);
    const double uk = static_cast<double>(ur[k]);
    const double d = uk - static_cast<double>(uold[k]);
    st_pop<NT>(p, ur[k]);
    acc[0] += d * d;
    acc[1] += uk * uk;
  }
  acc[2] += static_cast<double>(mac.drho);
  acc[3] += static_cast<double>(mac.jx);
  const bool fin = isfinite(static_cast<double>(mac.drho)) && isfinite(static_cast<double>(mac.jx)) &&
                   isfinite(static_cast<double>(mac.jy));
  acc[4] += fin ? 0.0 : 1.0;
}

// Self-consistent velocity, current and force at one node (2D).
// J_z = a + kappa (u_x B_y - u_y B_x), a = a_coef (Lambda_xy - Lambda_yx),
// Lambda_kj = sum_a e_{a k} g_{a j}; with p = (-B_y, B_x), J_z = a - kappa u.p and
// u = u0 - c (p.u)p, c = kappa/(2 gamma rho), so u = u0 - c (p.u0)/(1 + c|p|^2) p.
template <typename R>
struct Coupled2 {
  R Bx, By, bx, by, Fx, Fy;
};

template <typename R>
__device__ __forceinline__ Coupled2<R> lorentz_solve2(const R (&f)[Q9], const R (&g)[2][Q5], R Fex,
                                                      R Fey, const CollideArgs<R>& c,
                                                      const MagArgs<R>& m) {
  Coupled2<R> o;
  o.bx = g[0][0] + g[0][1] + g[0][2] + g[0][3] + g[0][4];
  o.by = g[1][0] + g[1][1] + g[1][2] + g[1][3] + g[1][4];
  o.Bx = m.B0[0] + o.bx;
  o.By = m.B0[1] + o.by;
  const R Lxy = g[1][1] - g[1][2];  // sum e_x g_y
  const R Lyx = g[0][3] - g[0][4];  // sum e_y g_x
  const R a = m.a_coef * (Lxy - Lyx);
  R drho, jrx, jry;
  raw_moments9<R>(f, drho, jrx, jry);
  const R irho = R(1) / (c.rho0 + drho);
  const R h = c.half_inv_gamma;
  const R px = -o.By, py = o.Bx;
  const R u0x = (jrx + (Fex + a * px) * h) * irho;
  const R u0y = (jry + (Fey + a * py) * h) * irho;
  const R cc = m.kappa * h * irho;
  const R pu = px * u0x + py * u0y;
  const R t = cc * pu / (R(1) + cc * (px * px + py * py));
  const R ux = u0x - t * px;
  const R uy = u0y - t * py;
  const R J = a + m.kappa * (ux * o.By - uy * o.Bx);
  o.Fx = Fex + J * px;
  o.Fy = Fey + J * py;
  return o;
}

// g~ = g + (g^eq* - g)/tau_m* on deviations (g^eq* - W B0 = W [b_j + adv_{a j}]).
template <typename R>
__device__ __forceinline__ void collide_g5(R (&g)[2][Q5], const Coupled2<R>& cp, R ux, R uy,
                                           const MagArgs<R>& m) {
  const R B[2] = {cp.Bx, cp.By};
  const R b[2] = {cp.bx, cp.by};
  const R u[2] = {ux, uy};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    g[j][0] += m.omega * (m.w_rest * b[j] - g[j][0]);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const R wadv = m.w_axis * m.adv * (u[k] * B[j] - B[k] * u[j]);
      const R base = m.w_axis * b[j];
      g[j][1 + 2 * k] += m.omega * (base + wadv - g[j][1 + 2 * k]);
      g[j][2 + 2 * k] += m.omega * (base - wadv - g[j][2 + 2 * k]);
    }
  }
}

// SR: 16-bit stores with stochastic rounding (store_stochastic).  KEEP0:
// streaming loads and stores except the rest population's (gather9, store9).
template <typename S, bool CHECK, bool FIELD, bool NT, bool WIDE, bool SR, bool KEEP0 = false>
__global__ __launch_bounds__(kBlock) void glbe2_step(GridArgs g, CollideArgs<typename Storage<S>::R> c,
                                                     const S* __restrict__ fin, S* __restrict__ fout,
                                                     const typename Storage<S>::R* __restrict__ force,
                                                     typename Storage<S>::R* __restrict__ usnap,
                                                     double* __restrict__ partials) {
  using R = typename Storage<S>::R;
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;
  const uint32_t n = static_cast<uint32_t>(lb) * kBlock + threadIdx.x;
  double acc[kPartials] = {};
  if (n < static_cast<uint32_t>(g.N)) {
    const Nbr b = neighbours(g, n);
    R f[Q9];
    gather9<S, WIDE, KEEP0>(fin, g.stride, n, b, f);
    R Fx, Fy;
    load_force2<R, WIDE>(g, c, force, FIELD, n, Fx, Fy);
    R uold[2];
    if constexpr (CHECK) load_usnap2<R, WIDE>(g, usnap, n, uold);
    const NodeMacro<R> mac = collide9<R>(f, Fx, Fy, c);
    if constexpr (SR)
      store_stochastic<S, NT, WIDE, Q9>(fout, g, n, f);
    else
      store9<S, NT, WIDE, KEEP0>(fout, g, n, f);
    if constexpr (CHECK) check_node2<R, WIDE, NT>(g, usnap, n, uold, mac, acc);
  }
  if constexpr (CHECK) write_partials(partials, lb, acc);
}

// KEEP0: streaming loads and stores except the rest flow population's
// (gather9, store9); the induction populations stream.
template <typename R, bool CHECK, bool FIELD, bool WIDE, bool NT, bool KEEP0 = false>
__global__ __launch_bounds__(kBlock) void mhd2_step(GridArgs g, CollideArgs<R> c, MagArgs<R> m,
                                                    const R* __restrict__ fin, R* __restrict__ fout,
                                                    const R* __restrict__ gin, R* __restrict__ gout,
                                                    const R* __restrict__ force,
                                                    R* __restrict__ usnap,
                                                    double* __restrict__ partials) {
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;
  const uint32_t n = static_cast<uint32_t>(lb) * kBlock + threadIdx.x;
  double acc[kPartials] = {};
  if (n < static_cast<uint32_t>(g.N)) {
    const Nbr b = neighbours(g, n);
    R f[Q9];
    gather9<R, WIDE, KEEP0>(fin, g.stride, n, b, f);
    R gg[2][Q5];
    gather_g5<R, WIDE, KEEP0>(gin, g.stride, n, b, gg);
    R Fx, Fy;
    load_force2<R, WIDE>(g, c, force, FIELD, n, Fx, Fy);
    R uold[2];
    if constexpr (CHECK) load_usnap2<R, WIDE>(g, usnap, n, uold);
    const Coupled2<R> cp = lorentz_solve2<R>(f, gg, Fx, Fy, c, m);
    const NodeMacro<R> mac = collide9<R>(f, cp.Fx, cp.Fy, c);
    collide_g5<R>(gg, cp, mac.ux, mac.uy, m);
    store9<R, NT, WIDE, KEEP0>(fout, g, n, f);
    R gflat[2 * Q5];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int a = 0; a < Q5; ++a) gflat[j * Q5 + a] = gg[j][a];
    store_planes<R, NT, WIDE, 2 * Q5>(gout, g, n, gflat);
    if constexpr (CHECK) check_node2<R, WIDE, NT>(g, usnap, n, uold, mac, acc);
  }
  if constexpr (CHECK) write_partials(partials, lb, acc);
}

// Fields of the streamed current state (no collision): rho, u (u_z = 0) and
// B (B_z = 0) when the pointers are non-null, and the mass / flow partials.
template <typename S, typename O, bool MHD>
__global__ __launch_bounds__(kBlock) void fields2_kernel(
    GridArgs g, CollideArgs<typename Storage<S>::R> c, MagArgs<typename Storage<S>::R> m,
    const S* __restrict__ fin, const typename Storage<S>::R* __restrict__ gin,
    const typename Storage<S>::R* __restrict__ force, int field, O* __restrict__ rho_out,
    O* __restrict__ u_out, O* __restrict__ B_out, int64_t out_stride, double* __restrict__ partials) {
  using R = typename Storage<S>::R;
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;
  const uint32_t n = static_cast<uint32_t>(lb) * kBlock + threadIdx.x;
  double acc[kPartials] = {};
  if (n < static_cast<uint32_t>(g.N)) {
    const Nbr b = neighbours(g, n);
    R f[Q9];
    gather9<S, true>(fin, g.stride, n, b, f);
    R Fx, Fy;
    load_force2<R, true>(g, c, force, field != 0, n, Fx, Fy);
    R Bx = 0, By = 0;
    if constexpr (MHD) {
      R gg[2][Q5];
      gather_g5<R, true>(gin, g.stride, n, b, gg);
      const Coupled2<R> cp = lorentz_solve2<R>(f, gg, Fx, Fy, c, m);
      Fx = cp.Fx;
      Fy = cp.Fy;
      Bx = cp.Bx;
      By = cp.By;
    }
    R drho, jx, jy;
    raw_moments9<R>(f, drho, jx, jy);
    jx += Fx * c.half_inv_gamma;
    jy += Fy * c.half_inv_gamma;
    const R rho = c.rho0 + drho;
    if (rho_out) rho_out[n] = static_cast<O>(rho);
    if (u_out) {
      u_out[n] = static_cast<O>(jx / rho);
      u_out[out_stride + n] = static_cast<O>(jy / rho);
      u_out[2 * out_stride + n] = O(0);
    }
    if (MHD && B_out) {
      B_out[n] = static_cast<O>(Bx);
      B_out[out_stride + n] = static_cast<O>(By);
      B_out[2 * out_stride + n] = O(0);
    }
    acc[2] = static_cast<double>(drho);
    acc[3] = static_cast<double>(jx);
  }
  write_partials(partials, lb, acc);
}

// ------------------------------------------------------------- launchers --
template <typename S>
hipError_t launch_glbe2_step(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                             const void* fin, void* fout, const void* force, bool field, bool check,
                             bool nt, bool stochastic, void* usnap_v, double* partials,
                             hipStream_t st) {
  using R = typename Storage<S>::R;
  R* usnap = static_cast<R*>(usnap_v);
  const S* a = static_cast<const S*>(fin);
  S* b = static_cast<S*>(fout);
  const R* F = static_cast<const R*>(force);
  return with_flag(check, [&](auto CH) {
    return with_flag(field, [&](auto FL) {
      return with_flag(nt, [&](auto NTS) {
        return with_flag(wide_offsets(g, sizeof(R)), [&](auto W) {
          constexpr bool ch = decltype(CH)::value, fl = decltype(FL)::value,
                         nts = decltype(NTS)::value, w = decltype(W)::value;
          if constexpr (sizeof(S) == 2) {
            if (stochastic) {
              launch_step(glbe2_step<S, ch, fl, nts, w, true>, step_grid(g), g.lds_reserve, st,
                        g, c, a, b, F, usnap, partials);
              return hipGetLastError();
            }
          }
          // 4-byte storage at HBM scale with no force field: the rest plane stays in
          // the last-level cache, the other planes stream (4096^2 FP32 step
          // 197.1-197.5 -> 194.1-194.5 us; 16-bit storage measured 2% slower, and
          // the FP64 rest planes do not fit)
          if (nts && !fl && sizeof(S) == 4 && g.rest_cached)
            launch_step(glbe2_step<S, ch, fl, nts, w, false, nts && !fl && sizeof(S) == 4>, step_grid(g),
                        g.lds_reserve, st, g, c, a, b, F, usnap, partials);
          else
            launch_step(glbe2_step<S, ch, fl, nts, w, false>, step_grid(g), g.lds_reserve, st,
                        g, c, a, b, F, usnap, partials);
          return hipGetLastError();
        });
      });
    });
  });
}

#define LBM_INST_STEP2(S)                                                                         \
  template hipError_t launch_glbe2_step<S>(const GridArgs&, const CollideArgs<Storage<S>::R>&,     \
                                           const void*, void*, const void*, bool, bool, bool,      \
                                           bool, void*, double*, hipStream_t);
LBM_INST_STEP2(double)
LBM_INST_STEP2(float)
LBM_INST_STEP2(bf16_t)
LBM_INST_STEP2(_Float16)
#undef LBM_INST_STEP2

template <typename R>
hipError_t launch_mhd2_step(const GridArgs& g, const CollideArgs<R>& c, const MagArgs<R>& m,
                            const void* fin, void* fout, const void* gin, void* gout,
                            const void* force, bool field, bool check, bool nt, void* usnap_v,
                            double* partials, hipStream_t st) {
  R* usnap = static_cast<R*>(usnap_v);
  const R* a = static_cast<const R*>(fin);
  R* b = static_cast<R*>(fout);
  const R* ga = static_cast<const R*>(gin);
  R* gb = static_cast<R*>(gout);
  const R* F = static_cast<const R*>(force);
  return with_flag(check, [&](auto CH) {
    return with_flag(field, [&](auto FL) {
      return with_flag(wide_offsets(g, sizeof(R)), [&](auto W) {
        return with_flag(nt, [&](auto NTF) {
          constexpr bool keep = decltype(NTF)::value && !decltype(FL)::value && sizeof(R) == 4;
          if (keep && g.rest_cached)
            launch_step(mhd2_step<R, decltype(CH)::value, decltype(FL)::value, decltype(W)::value,
                                  decltype(NTF)::value, keep>, step_grid(g), g.lds_reserve, st,
                        g, c, m, a, b, ga, gb, F, usnap, partials);
          else
            launch_step(mhd2_step<R, decltype(CH)::value, decltype(FL)::value, decltype(W)::value,
                      decltype(NTF)::value>, step_grid(g), g.lds_reserve, st,
                          g, c, m, a, b, ga, gb, F, usnap, partials);
          return hipGetLastError();
        });
      });
    });
  });
}

template hipError_t launch_mhd2_step<double>(const GridArgs&, const CollideArgs<double>&,
                                             const MagArgs<double>&, const void*, void*,
                                             const void*, void*, const void*, bool, bool, bool, void*,
                                             double*, hipStream_t);
template hipError_t launch_mhd2_step<float>(const GridArgs&, const CollideArgs<float>&,
                                            const MagArgs<float>&, const void*, void*,
                                            const void*, void*, const void*, bool, bool, bool, void*,
                                            double*, hipStream_t);

template <typename S>
hipError_t launch_fields2(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                          const MagArgs<typename Storage<S>::R>& m, bool mhd, const void* fin,
                          const void* gin, const void* force, bool field, int out_dtype, void* rho,
                          void* u, void* B, int64_t out_stride, double* partials, hipStream_t st) {
  using R = typename Storage<S>::R;
  const S* f = static_cast<const S*>(fin);
  const R* gp = static_cast<const R*>(gin);
  const R* F = static_cast<const R*>(force);
#define LBM_F2(O, M)                                                                              \
  fields2_kernel<S, O, M><<<step_grid(g), kBlock, 0, st>>>(g, c, m, f, gp, F, field ? 1 : 0,       \
                                                           static_cast<O*>(rho), static_cast<O*>(u), \
                                                           static_cast<O*>(B), out_stride, partials)
  if (out_dtype == 0) {
    if (mhd) LBM_F2(double, true); else LBM_F2(double, false);
  } else {
    if (mhd) LBM_F2(float, true); else LBM_F2(float, false);
  }
#undef LBM_F2
  return hipGetLastError();
}

#define LBM_INST_F2(S)                                                                            \
  template hipError_t launch_fields2<S>(const GridArgs&, const CollideArgs<Storage<S>::R>&,        \
                                        const MagArgs<Storage<S>::R>&, bool, const void*,          \
                                        const void*, const void*, bool, int, void*, void*, void*,  \
                                        int64_t, double*, hipStream_t);
LBM_INST_F2(double)
LBM_INST_F2(float)
LBM_INST_F2(bf16_t)
LBM_INST_F2(_Float16)
#undef LBM_INST_F2

}  // namespace lbm
