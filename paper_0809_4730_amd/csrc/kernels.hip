// gfx950 kernels of the preconditioned GLBE time step.
//
// glbe_step   fused pull-stream + preconditioned MRT collision with forcing
//             (Sec. 2 eq. streaming, Sec. 3 eqs. ppostcollision, prelax_term),
//             one thread per node, structure-of-arrays populations, A/B buffers.
// mhd_step    the same fused with the D3Q7 vector induction LKE (Sec. 4, 4.1)
//             and the Lorentz force J x B computed in registers.
// fields      hydrodynamic (and magnetic) fields of the current state plus the
//             FP64 mass / flow-rate partial sums.
// finalize    second pass of the FP64 reductions into one history record.
//
// Every population is read once and written once per step; the step is
// bandwidth-bound, so there is no LDS staging and no MFMA.  Halfway bounce-back
// needs no solid nodes: a link crossing a wall reads the opposite direction's
// post-collision value at the same node.  Loads take a scalar base and a
// 32-bit node offset; stores go through a buffer resource (store_planes).
#include <type_traits>
#include "collide.hpp"
#include "launch.hpp"
#include "stream.hpp"

namespace lbm {

// Gather of the magnetic populations, stored as deviations from the applied
// field's equilibrium, d_{a j} = g_{a j} - W_a B0_j (j outermost).  At a wall,
// anti-bounce-back g_a = -g~_opp(a) + 2 W_a B0 (insulating wall, B = B0 there)
// reads d_a = -d~_opp(a) in deviation form.
template <typename R, int A, bool WIDE, bool NTL>
__device__ __forceinline__ void gather_g_dir(const R* __restrict__ gin, int64_t stride, uint32_t n,
                                             const Nbr& b, R (&g)[3][Q7]) {
  int32_t off;
  const bool bounce = pull_source<EX7[A], EY7[A], EZ7[A]>(b, off);
  const uint32_t i = pull_offset<A>(bounce, off, n, static_cast<uint32_t>(stride));
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const R* base = gin + static_cast<int64_t>(j * Q7 + pair_plane<A>()) * stride;
    const R v = ld_pop<NTL>(elem<WIDE>(base, i));
    g[j][A] = bounce ? -v : v;
  }
}

template <typename R, bool WIDE, bool NTL = false, int A = 0>
__device__ __forceinline__ void gather_g(const R* __restrict__ gin, int64_t stride, uint32_t n,
                                         const Nbr& b, R (&g)[3][Q7]) {
  if constexpr (A < Q7) {
    gather_g_dir<R, A, WIDE, NTL>(gin, stride, n, b, g);
    gather_g<R, WIDE, NTL, A + 1>(gin, stride, n, b, g);
  }
}

// Self-consistent velocity, current and Lorentz force at one node.
// J = a + kappa (u x B) with a = a_coef * eps_ijk Lambda_jk (Lambda_jk = sum e_j g_k)
// and u = (j_raw + (F_ext + J x B)/(2 gamma))/rho; since (u x B) x B = -|B|^2 u_perp
// the linear system has the closed form u = (u0 + c (u0.B) B) / (1 + c |B|^2),
// c = kappa/(2 gamma rho), u0 = (j_raw + (F_ext + a x B)/(2 gamma))/rho.
template <typename R>
struct Coupled {
  R Bx, By, Bz;  // full field B0 + b
  R bx, by, bz;  // induced part b = sum_a d_a
  R Fx, Fy, Fz;  // total force
};

template <typename R>
__device__ __forceinline__ Coupled<R> lorentz_solve(const R (&f)[Q19], const R (&g)[3][Q7],
                                                    R Fex, R Fey, R Fez, const CollideArgs<R>& c,
                                                    const MagArgs<R>& m) {
  Coupled<R> o;
  // g holds deviations d = g - W B0: sum_a d_a = b = B - B0, and the W B0 part
  // has no first moment, so L is taken from d directly.
  R B[3], bb[3], L[3][3];  // L[k][j] = sum_a e_{a k} g_{a j}
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    bb[j] = g[j][0] + g[j][1] + g[j][2] + g[j][3] + g[j][4] + g[j][5] + g[j][6];
    B[j] = m.B0[j] + bb[j];
    L[0][j] = g[j][1] - g[j][2];
    L[1][j] = g[j][3] - g[j][4];
    L[2][j] = g[j][5] - g[j][6];
  }
  const R ax = m.a_coef * (L[1][2] - L[2][1]);
  const R ay = m.a_coef * (L[2][0] - L[0][2]);
  const R az = m.a_coef * (L[0][1] - L[1][0]);
  R drho, jrx, jry, jrz;
  raw_moments<R>(f, drho, jrx, jry, jrz);
  const R rho = c.rho0 + drho;
  const R irho = R(1) / rho;
  const R h = c.half_inv_gamma;
  const R u0x = (jrx + (Fex + (ay * B[2] - az * B[1])) * h) * irho;
  const R u0y = (jry + (Fey + (az * B[0] - ax * B[2])) * h) * irho;
  const R u0z = (jrz + (Fez + (ax * B[1] - ay * B[0])) * h) * irho;
  const R cc = m.kappa * h * irho;
  const R BB = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const R uB = u0x * B[0] + u0y * B[1] + u0z * B[2];
  const R den = R(1) / (R(1) + cc * BB);
  const R ux = (u0x + cc * uB * B[0]) * den;
  const R uy = (u0y + cc * uB * B[1]) * den;
  const R uz = (u0z + cc * uB * B[2]) * den;
  const R Jx = ax + m.kappa * (uy * B[2] - uz * B[1]);
  const R Jy = ay + m.kappa * (uz * B[0] - ux * B[2]);
  const R Jz = az + m.kappa * (ux * B[1] - uy * B[0]);
  o.Bx = B[0];
  o.By = B[1];
  o.Bz = B[2];
  o.bx = bb[0];
  o.by = bb[1];
  o.bz = bb[2];
  o.Fx = Fex + (Jy * B[2] - Jz * B[1]);
  o.Fy = Fey + (Jz * B[0] - Jx * B[2]);
  o.Fz = Fez + (Jx * B[1] - Jy * B[0]);
  return o;
}

// Outside the fluid box: the field alone (u = 0, no force).
template <typename R>
__device__ __forceinline__ Coupled<R> field_only(const R (&g)[3][Q7], const MagArgs<R>& m) {
  Coupled<R> o;
  R bb[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    bb[j] = g[j][0] + g[j][1] + g[j][2] + g[j][3] + g[j][4] + g[j][5] + g[j][6];
  o.bx = bb[0];
  o.by = bb[1];
  o.bz = bb[2];
  o.Bx = m.B0[0] + bb[0];
  o.By = m.B0[1] + bb[1];
  o.Bz = m.B0[2] + bb[2];
  o.Fx = o.Fy = o.Fz = R(0);
  return o;
}

// g~ = g + (g^eq* - g)/tau_m*, g^eq*_{a j} = W_a [B_j + (e_{a k}/theta)(chi/gamma_m)(u_k B_j - B_k u_j)],
// on deviations d = g - W B0: d~ = d + (g^eq* - W B0 - d)/tau_m*, where
// g^eq* - W B0 = W_a [b_j + (e_{a k}/theta)(chi/gamma_m)(u_k B_j - B_k u_j)].
template <typename R>
__device__ __forceinline__ void collide_g(R (&g)[3][Q7], const Coupled<R>& cp, R ux, R uy, R uz,
                                          const MagArgs<R>& m) {
  const R B[3] = {cp.Bx, cp.By, cp.Bz};
  const R b[3] = {cp.bx, cp.by, cp.bz};
  const R u[3] = {ux, uy, uz};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    g[j][0] += m.omega * (m.w_rest * b[j] - g[j][0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R adv = m.adv * (u[k] * B[j] - B[k] * u[j]);
      const R base = m.w_axis * b[j];
      const R wadv = m.w_axis * adv;
      g[j][1 + 2 * k] += m.omega * (base + wadv - g[j][1 + 2 * k]);
      g[j][2 + 2 * k] += m.omega * (base - wadv - g[j][2 + 2 * k]);
    }
  }
}

template <typename R, bool NT, bool WIDE>
__device__ __forceinline__ void store_g(R* __restrict__ gout, const GridArgs& ga, uint32_t n,
                                        const R (&g)[3][Q7]) {
  R flat[3 * Q7];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int a = 0; a < Q7; ++a) flat[j * Q7 + a] = g[j][a];
  store_planes<R, NT, WIDE, 3 * Q7>(gout, ga, n, flat);
}

template <typename R, bool WIDE, bool NTL = false>
__device__ __forceinline__ void load_force(const GridArgs& g, const CollideArgs<R>& c,
                                           const R* __restrict__ force, bool field, uint32_t n,
                                           R& Fx, R& Fy, R& Fz) {
  if (field) {
    Fx = ld_pop<NTL>(elem<WIDE>(force, n));
    Fy = ld_pop<NTL>(elem<WIDE>(force + g.stride, n));
    Fz = ld_pop<NTL>(elem<WIDE>(force + 2 * g.stride, n));
  } else {
    Fx = c.F[0];
    Fy = c.F[1];
    Fz = c.F[2];
  }
}

// ------------------------------------------------------------------ steps --
// ROWS: every wave lies in one x-row (nx a multiple of 64; neighbours_rows).
// SR: 16-bit stores with stochastic rounding (store_stochastic).  NT:
// streaming stores.  LOADS: kLoadCached, kLoadStream (streaming loads of
// populations, force and snapshot), kLoadStreamKeepForce (streaming loads
// except the force field's, which stays in the last-level cache) or
// kLoadStreamKeepRest (streaming loads and stores except the rest
// population's, whose two planes stay in that cache from step to step).
constexpr int kLoadCached = 0, kLoadStream = 1, kLoadStreamKeepForce = 2, kLoadStreamKeepRest = 3;

template <typename S, bool CHECK, bool FIELD, bool NT, int LOADS, bool MOVING, bool WIDE, bool ROWS,
          bool SR>
__global__ __launch_bounds__(kBlock) void glbe_step(GridArgs g, CollideArgs<typename Storage<S>::R> c,
                                                    const S* __restrict__ fin, S* __restrict__ fout,
                                                    const typename Storage<S>::R* __restrict__ force,
                                                    typename Storage<S>::R* __restrict__ usnap,
                                                    double* __restrict__ partials) {
  using R = typename Storage<S>::R;
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;  // padding workgroup of the XCD-balanced launch
  const uint32_t n = static_cast<uint32_t>(lb) * kBlock + threadIdx.x;
  double acc[kPartials] = {};
  if (n < static_cast<uint32_t>(g.N)) {
    const Nbr b = ROWS ? neighbours_rows(g, n) : neighbours(g, n);
    R f[Q19];
    constexpr bool NTL = LOADS != kLoadCached, KEEP0 = LOADS == kLoadStreamKeepRest;
    gather19<S, MOVING, WIDE, NTL, KEEP0>(fin, g.stride, n, b, c, f);
    R Fx, Fy, Fz;
    load_force<R, WIDE, LOADS == kLoadStream>(g, c, force, FIELD, n, Fx, Fy, Fz);
    R uold[3];
    if constexpr (CHECK) load_usnap<R, WIDE, NTL>(g, usnap, n, uold);
    const NodeMacro<R> mac = collide19<R>(f, Fx, Fy, Fz, c);
    if constexpr (SR)
      store_stochastic<S, NT, WIDE, Q19>(fout, g, n, f);
    else
      store19<S, NT, WIDE, KEEP0>(fout, g, n, f);
    if constexpr (CHECK)
      check_node<R, WIDE, NT>(g, usnap, n, uold, mac.drho, mac.jx, mac.jy, mac.jz, mac.ux, mac.uy,
                              mac.uz, acc);
  }
  if constexpr (CHECK) write_partials(partials, lb, acc);
}

// EXT: the induction lattice extends beyond the fluid box; nodes outside it
// relax g with u = 0 and leave f untouched.  NT: streaming stores; LOADS: the
// load policy, as for glbe_step.  ROWS (not with EXT): every wave lies in one
// x-row (neighbours_rows).
template <typename R, bool CHECK, bool FIELD, bool MOVING, bool EXT, bool WIDE, bool NT, int LOADS,
          bool ROWS>
__global__ __launch_bounds__(kBlock) void mhd_step(GridArgs g, CollideArgs<R> c, MagArgs<R> m,
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
    static_assert(!(ROWS && EXT), "the row-aligned form needs the fluid box to be the lattice");
    Coord q{};
    Nbr b;
    if constexpr (ROWS) {
      b = neighbours_rows(g, n);
    } else {
      q = coords(g, n);
      b = neighbours_at(g, q);
    }
    constexpr bool NTL = LOADS != kLoadCached, KEEP0 = LOADS == kLoadStreamKeepRest;
    R gg[3][Q7];
    gather_g<R, WIDE, NTL>(gin, g.stride, n, b, gg);
    bool fluid = true;
    if constexpr (EXT) fluid = in_box(g, q);
    if (fluid) {
      Nbr bf = b;
      if constexpr (EXT) bf = box_walls(g, q, b);
      R f[Q19];
      gather19<R, MOVING, WIDE, NTL, KEEP0>(fin, g.stride, n, bf, c, f);
      R Fx, Fy, Fz;
      load_force<R, WIDE, LOADS == kLoadStream>(g, c, force, FIELD, n, Fx, Fy, Fz);
      R uold[3];
      if constexpr (CHECK) load_usnap<R, WIDE, NTL>(g, usnap, n, uold);
      const Coupled<R> cp = lorentz_solve<R>(f, gg, Fx, Fy, Fz, c, m);
      const NodeMacro<R> mac = collide19<R>(f, cp.Fx, cp.Fy, cp.Fz, c);
      collide_g<R>(gg, cp, mac.ux, mac.uy, mac.uz, m);
      store19<R, NT, WIDE, KEEP0>(fout, g, n, f);
      if constexpr (CHECK)
        check_node<R, WIDE, NT>(g, usnap, n, uold, mac.drho, mac.jx, mac.jy, mac.jz, mac.ux,
                                mac.uy, mac.uz, acc);
    } else {
      const Coupled<R> cp = field_only<R>(gg, m);
      collide_g<R>(gg, cp, R(0), R(0), R(0), m);
    }
    store_g<R, NT, WIDE>(gout, g, n, gg);
  }
  if constexpr (CHECK) write_partials(partials, lb, acc);
}

// ----------------------------------------------------------------- fields --
// Fields of the streamed current state (no collision).  Writes rho, u (and B)
// when the pointers are non-null, and always the mass / flow partials.
template <typename S, typename O, bool MHD>
__global__ __launch_bounds__(kBlock) void fields_kernel(
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
    const Coord q = coords(g, n);
    const Nbr b = neighbours_at(g, q);
    if (MHD && !in_box(g, q)) {  // induction lattice outside the fluid box
      if constexpr (MHD) {
        R gg[3][Q7];
        gather_g<R, true>(gin, g.stride, n, b, gg);
        const Coupled<R> cp = field_only<R>(gg, m);
        if (rho_out) rho_out[n] = static_cast<O>(c.rho0);
        if (u_out) {
          u_out[n] = O(0);
          u_out[out_stride + n] = O(0);
          u_out[2 * out_stride + n] = O(0);
        }
        if (B_out) {
          B_out[n] = static_cast<O>(cp.Bx);
          B_out[out_stride + n] = static_cast<O>(cp.By);
          B_out[2 * out_stride + n] = static_cast<O>(cp.Bz);
        }
      }
    } else {
      const Nbr bf = box_walls(g, q, b);
      R f[Q19];
      gather19<S, true, true>(fin, g.stride, n, bf, c, f);
      R Fx, Fy, Fz;
      load_force<R, true>(g, c, force, field != 0, n, Fx, Fy, Fz);
      R Bx = 0, By = 0, Bz = 0;
      if constexpr (MHD) {
        R gg[3][Q7];
        gather_g<R, true>(gin, g.stride, n, b, gg);
        const Coupled<R> cp = lorentz_solve<R>(f, gg, Fx, Fy, Fz, c, m);
        Fx = cp.Fx;
        Fy = cp.Fy;
        Fz = cp.Fz;
        Bx = cp.Bx;
        By = cp.By;
        Bz = cp.Bz;
      }
      R drho, jx, jy, jz;
      raw_moments<R>(f, drho, jx, jy, jz);
      jx += Fx * c.half_inv_gamma;
      jy += Fy * c.half_inv_gamma;
      jz += Fz * c.half_inv_gamma;
      const R rho = c.rho0 + drho;
      if (rho_out) rho_out[n] = static_cast<O>(rho);
      if (u_out) {
        u_out[n] = static_cast<O>(jx / rho);
        u_out[out_stride + n] = static_cast<O>(jy / rho);
        u_out[2 * out_stride + n] = static_cast<O>(jz / rho);
      }
      if (MHD && B_out) {
        B_out[n] = static_cast<O>(Bx);
        B_out[out_stride + n] = static_cast<O>(By);
        B_out[2 * out_stride + n] = static_cast<O>(Bz);
      }
      acc[2] = static_cast<double>(drho);
      acc[3] = static_cast<double>(jx);
    }
  }
  write_partials(partials, lb, acc);
}

// ---------------------------------------------------------------- finalize --
// One workgroup per pending check: sum that check's per-workgroup partials in
// a fixed order and write its history record {step, residual, du2, u2, mass,
// flow, nonfinite, 0}.  Checks are check_every steps apart.  Check first + i
// takes its partials from slot (slot_first + i) mod pslots and its record to
// ring entry (first + i) mod history_len.
__global__ __launch_bounds__(kBlock) void finalize_kernel(const double* __restrict__ partials,
                                                          int nblocks, int pslots, int64_t slot_first,
                                                          int64_t first, double step0, double dstep,
                                                          double inv_nx, double* __restrict__ ring,
                                                          int history_len) {
  const int64_t k = first + blockIdx.x;
  const double* p = partials + ((slot_first + blockIdx.x) % pslots) * int64_t(nblocks) * kPartials;
  double acc[kPartials] = {};
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
    for (int q = 0; q < kPartials; ++q) acc[q] += p[static_cast<int64_t>(b) * kPartials + q];
  }
  block_sum<kPartials>(acc);
  if (threadIdx.x == 0) {
    double* record = ring + (k % history_len) * kRecordDoubles;
    const double du2 = acc[0], u2 = acc[1];
    double r;
    if (u2 > 0.0)
      r = sqrt(du2 / u2);
    else
      r = (du2 == 0.0) ? 0.0 : INFINITY;
    record[0] = step0 + dstep * double(blockIdx.x);
    record[1] = r;
    record[2] = du2;
    record[3] = u2;
    record[4] = acc[2];
    record[5] = acc[3] * inv_nx;
    record[6] = acc[4];
    record[7] = 0.0;
  }
}

// First pass of a split finalize for lattices with many workgroups: workgroup
// (g, i) sums the partials of logical blocks [g span, (g + 1) span) of check
// first + i (slot (first + i) mod pslots) in a fixed order and writes them to
// out[i][g]; finalize_kernel then reduces the `groups` sums of each check.
__global__ __launch_bounds__(kBlock) void finalize_part(const double* __restrict__ partials,
                                                        int nblocks, int pslots, int64_t first,
                                                        int span, int groups,
                                                        double* __restrict__ out) {
  const int g = blockIdx.x;
  const int64_t slot = (first + blockIdx.y) % pslots;
  const double* p = partials + slot * int64_t(nblocks) * kPartials;
  const int b0 = g * span;
  const int b1 = b0 + span < nblocks ? b0 + span : nblocks;
  double acc[kPartials] = {};
  for (int b = b0 + threadIdx.x; b < b1; b += kBlock) {
#pragma unroll
    for (int q = 0; q < kPartials; ++q) acc[q] += p[static_cast<int64_t>(b) * kPartials + q];
  }
  block_sum<kPartials>(acc);
  if (threadIdx.x == 0) {
    double* o = out + (static_cast<int64_t>(blockIdx.y) * groups + g) * kPartials;
#pragma unroll
    for (int q = 0; q < kPartials; ++q) o[q] = acc[q];
  }
}

// -------------------------------------------------------------------- init --
template <typename S>
__global__ __launch_bounds__(kBlock) void fill_zero(S* __restrict__ p, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) Storage<S>::st(p + i, typename Storage<S>::R(0));
}

__global__ __launch_bounds__(kBlock) void fill_zero_f64(double* __restrict__ p, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// ------------------------------------------------------------- convert --
// planes x N values from one storage type to another (through FP64): the state
// of one context continued in another precision.
template <typename Ss, typename Sd>
__global__ __launch_bounds__(kBlock) void convert_planes(const Ss* __restrict__ src,
                                                         Sd* __restrict__ dst, int64_t stride,
                                                         int64_t N, int planes) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
  using Rd = typename Storage<Sd>::R;
  for (int a = 0; a < planes; ++a) {
    const double v = static_cast<double>(Storage<Ss>::ld(src + a * stride + i));
    Storage<Sd>::st(dst + a * stride + i, static_cast<Rd>(v));
  }
}

template <typename Ss>
hipError_t launch_convert_to(int dst_storage, const void* src, void* dst, int64_t stride,
                             int64_t N, int planes, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((N + kBlock - 1) / kBlock));
  const Ss* s = static_cast<const Ss*>(src);
  switch (dst_storage) {
    case 0: convert_planes<Ss, double><<<grid, kBlock, 0, st>>>(s, static_cast<double*>(dst), stride, N, planes); break;
    case 1: convert_planes<Ss, float><<<grid, kBlock, 0, st>>>(s, static_cast<float*>(dst), stride, N, planes); break;
    case 2: convert_planes<Ss, bf16_t><<<grid, kBlock, 0, st>>>(s, static_cast<bf16_t*>(dst), stride, N, planes); break;
    default: convert_planes<Ss, _Float16><<<grid, kBlock, 0, st>>>(s, static_cast<_Float16*>(dst), stride, N, planes);
  }
  return hipGetLastError();
}

hipError_t launch_convert(int src_storage, int dst_storage, const void* src, void* dst,
                          int64_t stride, int64_t N, int planes, hipStream_t st) {
  if (N <= 0 || planes <= 0) return hipSuccess;
  switch (src_storage) {
    case 0: return launch_convert_to<double>(dst_storage, src, dst, stride, N, planes, st);
    case 1: return launch_convert_to<float>(dst_storage, src, dst, stride, N, planes, st);
    case 2: return launch_convert_to<bf16_t>(dst_storage, src, dst, stride, N, planes, st);
    default: return launch_convert_to<_Float16>(dst_storage, src, dst, stride, N, planes, st);
  }
}

// ------------------------------------------------------------- launchers --
template <typename S>
hipError_t launch_glbe_step(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                            const void* fin, void* fout, const void* force, bool field, bool check,
                            bool nt, bool stochastic, void* usnap_v, double* partials,
                            hipStream_t st) {
  using R = typename Storage<S>::R;
  R* usnap = static_cast<R*>(usnap_v);
  const S* a = static_cast<const S*>(fin);
  S* b = static_cast<S*>(fout);
  const R* F = static_cast<const R*>(force);
  // moving walls: small problems, regular loads and stores; streaming loads
  // only with streaming stores (lattices that stream from HBM)
  const bool ntl = nt && g.nt_load;
  return with_flag(check, [&](auto CH) {
    return with_flag(field, [&](auto FL) {
      return with_flag(wide_offsets(g, sizeof(R)), [&](auto W) {
        return with_flag(rows_per_wave(g), [&](auto RW) {
          return with_flag(stochastic && sizeof(S) == 2, [&](auto SRF) {
            constexpr bool ch = decltype(CH)::value, fl = decltype(FL)::value,
                           w = decltype(W)::value, rw = decltype(RW)::value,
                           sr = decltype(SRF)::value && sizeof(S) == 2;
            if (c.moving)
              launch_step(glbe_step<S, ch, fl, false, kLoadCached, true, w, rw, sr>, step_grid(g),
                          g.lds_reserve, st, g, c, a, b, F, usnap, partials);
            else if (ntl && fl && g.force_cached)
              launch_step(glbe_step<S, ch, fl, true, fl ? kLoadStreamKeepForce : kLoadStream, false, w, rw, sr>,
                          step_grid(g), g.lds_reserve, st, g, c, a, b, F, usnap, partials);
            else if (ntl && !fl && !sr && g.rest_cached)
              launch_step(glbe_step<S, ch, fl, true, (!fl && !sr) ? kLoadStreamKeepRest : kLoadStream, false,
                                    w, rw, sr>,
                          step_grid(g), g.lds_reserve, st, g, c, a, b, F, usnap, partials);
            else if (ntl)
              launch_step(glbe_step<S, ch, fl, true, kLoadStream, false, w, rw, sr>, step_grid(g),
                          g.lds_reserve, st, g, c, a, b, F, usnap, partials);
            else if (nt)
              launch_step(glbe_step<S, ch, fl, true, kLoadCached, false, w, rw, sr>, step_grid(g),
                          g.lds_reserve, st, g, c, a, b, F, usnap, partials);
            else
              launch_step(glbe_step<S, ch, fl, false, kLoadCached, false, w, rw, sr>, step_grid(g),
                          g.lds_reserve, st, g, c, a, b, F, usnap, partials);
            return hipGetLastError();
          });
        });
      });
    });
  });
}

#define LBM_INST_STEP(S)                                                                          \
  template hipError_t launch_glbe_step<S>(const GridArgs&, const CollideArgs<Storage<S>::R>&,      \
                                          const void*, void*, const void*, bool, bool, bool, bool, \
                                          void*, double*, hipStream_t);
LBM_INST_STEP(double)
LBM_INST_STEP(float)
LBM_INST_STEP(bf16_t)
LBM_INST_STEP(_Float16)
#undef LBM_INST_STEP

template <typename R>
hipError_t launch_mhd_step(const GridArgs& g, const CollideArgs<R>& c, const MagArgs<R>& m,
                           const void* fin, void* fout, const void* gin, void* gout,
                           const void* force, bool field, bool check, bool nt, void* usnap_v,
                           double* partials, hipStream_t st) {
  R* usnap = static_cast<R*>(usnap_v);
  const R* a = static_cast<const R*>(fin);
  R* b = static_cast<R*>(fout);
  const R* ga = static_cast<const R*>(gin);
  R* gb = static_cast<R*>(gout);
  const R* F = static_cast<const R*>(force);
  const bool ext = g.flo[0] > 0 || g.flo[1] > 0 || g.flo[2] > 0;
  const bool plain = !c.moving && !ext;
  const bool ntl = nt && g.nt_load;
  return with_flag(check, [&](auto CH) {
    return with_flag(field, [&](auto FL) {
      return with_flag(wide_offsets(g, sizeof(R)), [&](auto W) {
        constexpr bool ch = decltype(CH)::value, fl = decltype(FL)::value,
                       w = decltype(W)::value;
        if (!plain) {
          // moving walls and the extended lattice are the (cache-resident)
          // cavity: per-lane coordinates, regular loads and stores
          return with_flag(c.moving != 0, [&](auto MV) {
            return with_flag(ext, [&](auto EX) {
              launch_step(mhd_step<R, ch, fl, decltype(MV)::value, decltype(EX)::value, w, false, kLoadCached, false>, step_grid(g), g.lds_reserve, st,
                        g, c, m, a, b, ga, gb, F, usnap, partials);
              return hipGetLastError();
            });
          });
        }
        return with_flag(rows_per_wave(g), [&](auto RW) {
          constexpr bool rw = decltype(RW)::value;
          if (ntl && fl && g.force_cached)
            launch_step(mhd_step<R, ch, fl, false, false, w, true, fl ? kLoadStreamKeepForce : kLoadStream, rw>,
                        step_grid(g), g.lds_reserve, st, g, c, m, a, b, ga, gb, F, usnap, partials);
          else if (ntl && !fl && g.rest_cached)
            launch_step(mhd_step<R, ch, fl, false, false, w, true, fl ? kLoadStream : kLoadStreamKeepRest, rw>,
                        step_grid(g), g.lds_reserve, st, g, c, m, a, b, ga, gb, F, usnap, partials);
          else if (ntl)
            launch_step(mhd_step<R, ch, fl, false, false, w, true, kLoadStream, rw>, step_grid(g),
                        g.lds_reserve, st, g, c, m, a, b, ga, gb, F, usnap, partials);
          else if (nt)
            launch_step(mhd_step<R, ch, fl, false, false, w, true, kLoadCached, rw>, step_grid(g),
                        g.lds_reserve, st, g, c, m, a, b, ga, gb, F, usnap, partials);
          else
            launch_step(mhd_step<R, ch, fl, false, false, w, false, kLoadCached, rw>, step_grid(g),
                        g.lds_reserve, st, g, c, m, a, b, ga, gb, F, usnap, partials);
          return hipGetLastError();
        });
      });
    });
  });
}

template hipError_t launch_mhd_step<double>(const GridArgs&, const CollideArgs<double>&,
                                            const MagArgs<double>&, const void*, void*, const void*,
                                            void*, const void*, bool, bool, bool, void*, double*,
                                            hipStream_t);
template hipError_t launch_mhd_step<float>(const GridArgs&, const CollideArgs<float>&,
                                           const MagArgs<float>&, const void*, void*, const void*,
                                           void*, const void*, bool, bool, bool, void*, double*,
                                           hipStream_t);

template <typename S>
hipError_t launch_fields(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                         const MagArgs<typename Storage<S>::R>& m, bool mhd, const void* fin,
                         const void* gin, const void* force, bool field, int out_dtype, void* rho,
                         void* u, void* B, int64_t out_stride, double* partials, hipStream_t st) {
  using R = typename Storage<S>::R;
  const S* a = static_cast<const S*>(fin);
  const R* ga = static_cast<const R*>(gin);
  const R* F = static_cast<const R*>(force);
  const int fl = field ? 1 : 0;
  if (out_dtype == 0) {
    double *r = static_cast<double*>(rho), *uu = static_cast<double*>(u), *bb = static_cast<double*>(B);
    if (mhd)
      fields_kernel<S, double, true><<<step_grid(g), kBlock, 0, st>>>(g, c, m, a, ga, F, fl, r, uu, bb, out_stride, partials);
    else
      fields_kernel<S, double, false><<<step_grid(g), kBlock, 0, st>>>(g, c, m, a, ga, F, fl, r, uu, bb, out_stride, partials);
  } else {
    float *r = static_cast<float*>(rho), *uu = static_cast<float*>(u), *bb = static_cast<float*>(B);
    if (mhd)
      fields_kernel<S, float, true><<<step_grid(g), kBlock, 0, st>>>(g, c, m, a, ga, F, fl, r, uu, bb, out_stride, partials);
    else
      fields_kernel<S, float, false><<<step_grid(g), kBlock, 0, st>>>(g, c, m, a, ga, F, fl, r, uu, bb, out_stride, partials);
  }
  return hipGetLastError();
}

#define LBM_INST_FIELDS(S)                                                                        \
  template hipError_t launch_fields<S>(const GridArgs&, const CollideArgs<Storage<S>::R>&,       \
                                       const MagArgs<Storage<S>::R>&, bool, const void*,          \
                                       const void*, const void*, bool, int, void*, void*, void*, \
                                       int64_t, double*, hipStream_t);
LBM_INST_FIELDS(double)
LBM_INST_FIELDS(float)
LBM_INST_FIELDS(bf16_t)
LBM_INST_FIELDS(_Float16)
#undef LBM_INST_FIELDS

hipError_t launch_finalize(const double* partials, int nblocks, int pslots, int64_t first,
                           int count, double step0, double dstep, double inv_nx, double* ring,
                           int history_len, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  finalize_kernel<<<count, kBlock, 0, st>>>(partials, nblocks, pslots, first, first, step0, dstep,
                                            inv_nx, ring, history_len);
  return hipGetLastError();
}

hipError_t launch_finalize_split(const double* partials, int nblocks, int pslots, int64_t first,
                                 int count, double step0, double dstep, double inv_nx,
                                 double* ring, int history_len, double* scratch,
                                 int64_t scratch_doubles, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  constexpr int kSpan = 1024;  // logical blocks per first-pass workgroup
  const int groups = (nblocks + kSpan - 1) / kSpan;
  if (groups < 4 || count > 65535 || int64_t(count) * groups * kPartials > scratch_doubles)
    return launch_finalize(partials, nblocks, pslots, first, count, step0, dstep, inv_nx, ring,
                           history_len, st);
  finalize_part<<<dim3(groups, count), kBlock, 0, st>>>(partials, nblocks, pslots, first, kSpan,
                                                        groups, scratch);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  finalize_kernel<<<count, kBlock, 0, st>>>(scratch, groups, count, 0, first, step0, dstep, inv_nx,
                                            ring, history_len);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_fill_zero(void* p, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + kBlock - 1) / kBlock;
  fill_zero<S><<<dim3(static_cast<uint32_t>(blocks)), kBlock, 0, st>>>(static_cast<S*>(p), count);
  return hipGetLastError();
}
template hipError_t launch_fill_zero<double>(void*, int64_t, hipStream_t);
template hipError_t launch_fill_zero<float>(void*, int64_t, hipStream_t);
template hipError_t launch_fill_zero<bf16_t>(void*, int64_t, hipStream_t);
template hipError_t launch_fill_zero<_Float16>(void*, int64_t, hipStream_t);



}  // namespace lbm
