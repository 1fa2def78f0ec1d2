// Device helpers shared by the 3D and 2D step kernels: node coordinates,
// pull-streaming neighbour offsets with periodic wrap and wall flags, and the
// per-node FP64 residual / reduction bookkeeping.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"

namespace lbm {

// Launched grid of a node kernel: kXcd * blocks_per_xcd workgroups (see
// logical_block).
inline dim3 step_grid(const GridArgs& g) { return dim3(kXcd * g.blocks_per_xcd); }

// Call f with std::true_type or std::false_type: a run-time flag becomes a
// template argument of the kernel f launches.
template <typename F>
inline hipError_t with_flag(bool b, F&& f) {
  return b ? f(std::true_type{}) : f(std::false_type{});
}

// Whether a launch needs 64-bit element offsets.  The narrow form reaches
// every array through 32-bit byte offsets from one base: loads within 2 planes
// of a pair's base, stores anywhere in an array of up to 21 planes (the
// magnetic populations), so it needs 21 * stride * elem_bytes < 2^32 (FP32:
// lattices up to ~51 M nodes).  g.wide (lbm_launch.offsets = 1) forces the
// 64-bit form, so that tests can run both forms on small lattices.
inline bool wide_offsets(const GridArgs& g, size_t elem_bytes) {
  if (g.wide) return true;
  return 21.0 * static_cast<double>(g.stride) * static_cast<double>(elem_bytes) >= 4294967296.0;
}

// Per-node neighbour offsets for pull streaming.
struct Nbr {
  int32_t xm, xp, ym, yp, zm, zp;  // linear offsets to x-1, x+1, ... (periodic wrap applied)
  bool bxm, bxp, bym, byp, bzm, bzp;  // link to that neighbour crosses a wall
};

struct Coord {
  int x, y, z;
};

__device__ __forceinline__ Coord coords(const GridArgs& g, uint32_t n) {
  const uint32_t yz = fdiv(n, g.div_nx);
  const uint32_t z = fdiv(n, g.div_nxny);
  Coord q;
  q.x = static_cast<int>(n - yz * static_cast<uint32_t>(g.nx));
  q.y = static_cast<int>(yz - z * static_cast<uint32_t>(g.ny));
  q.z = static_cast<int>(z);
  return q;
}

// Offsets with periodic wrap, and the walls at the lattice faces.
__device__ __forceinline__ Nbr neighbours_at(const GridArgs& g, const Coord& q) {
  const int sx = 1, sy = g.nx, sz = g.nx * g.ny;
  Nbr b;
  b.xm = (q.x == 0) ? (g.nx - 1) * sx : -sx;
  b.xp = (q.x == g.nx - 1) ? -(g.nx - 1) * sx : sx;
  b.ym = (q.y == 0) ? (g.ny - 1) * sy : -sy;
  b.yp = (q.y == g.ny - 1) ? -(g.ny - 1) * sy : sy;
  b.zm = (q.z == 0) ? (g.nz - 1) * sz : -sz;
  b.zp = (q.z == g.nz - 1) ? -(g.nz - 1) * sz : sz;
  b.bxm = g.wall_x && q.x == 0;
  b.bxp = g.wall_x && q.x == g.nx - 1;
  b.bym = g.wall_y && q.y == 0;
  b.byp = g.wall_y && q.y == g.ny - 1;
  b.bzm = g.wall_z && q.z == 0;
  b.bzp = g.wall_z && q.z == g.nz - 1;
  return b;
}

__device__ __forceinline__ Nbr neighbours(const GridArgs& g, uint32_t n) {
  return neighbours_at(g, coords(g, n));
}

// When nx is a multiple of the wave size, the nodes of a wave lie in one
// x-row: y and z, and with them the y/z neighbour offsets and wall flags, are
// the same for every lane and are taken from one active lane's node (scalar
// registers); only the x part is per lane.
__device__ __forceinline__ Nbr neighbours_rows(const GridArgs& g, uint32_t n) {
  const uint32_t n0 = __builtin_amdgcn_readfirstlane(n);
  const uint32_t yz = fdiv(n0, g.div_nx);
  const uint32_t z = fdiv(n0, g.div_nxny);
  Coord q;
  q.x = static_cast<int>(n - yz * static_cast<uint32_t>(g.nx));
  q.y = static_cast<int>(yz - z * static_cast<uint32_t>(g.ny));
  q.z = static_cast<int>(z);
  return neighbours_at(g, q);
}

// Whether every wave of a launch lies in one x-row.
inline bool rows_per_wave(const GridArgs& g) { return g.nx % 64 == 0; }

// The same node seen by the flow: walls at the fluid box faces.
__device__ __forceinline__ Nbr box_walls(const GridArgs& g, const Coord& q, Nbr b) {
  b.bxm = g.wall_x && q.x == g.flo[0];
  b.bxp = g.wall_x && q.x == g.fhi[0] - 1;
  b.bym = g.wall_y && q.y == g.flo[1];
  b.byp = g.wall_y && q.y == g.fhi[1] - 1;
  b.bzm = g.wall_z && q.z == g.flo[2];
  b.bzp = g.wall_z && q.z == g.fhi[2] - 1;
  return b;
}

__device__ __forceinline__ bool in_box(const GridArgs& g, const Coord& q) {
  return q.x >= g.flo[0] && q.x < g.fhi[0] && q.y >= g.flo[1] && q.y < g.fhi[1] &&
         q.z >= g.flo[2] && q.z < g.fhi[2];
}

// Source of f_a(x) = f~_a(x - e_a): returns the element index to read in the
// plane of direction `plane` (a itself, or its opposite on bounce-back).
template <int EX, int EY, int EZ>
__device__ __forceinline__ bool pull_source(const Nbr& b, int32_t& off) {
  off = (EX > 0 ? b.xm : EX < 0 ? b.xp : 0) + (EY > 0 ? b.ym : EY < 0 ? b.yp : 0) +
        (EZ > 0 ? b.zm : EZ < 0 ? b.zp : 0);
  return (EX > 0 && b.bxm) || (EX < 0 && b.bxp) || (EY > 0 && b.bym) || (EY < 0 && b.byp) ||
         (EZ > 0 && b.bzm) || (EZ < 0 && b.bzp);
}

// Wall-momentum term of a bounced link of direction A at this node: mean over
// the crossed moving faces of 6 w_A rho0 (e_A . u_face).
template <typename R, int A>
__device__ __forceinline__ R wall_term(const Nbr& b, const CollideArgs<R>& c) {
  R sum = R(0);
  int cnt = 0;
  if (EX19[A] > 0 && b.bxm) { sum += c.wall[A][0]; ++cnt; }
  if (EX19[A] < 0 && b.bxp) { sum += c.wall[A][1]; ++cnt; }
  if (EY19[A] > 0 && b.bym) { sum += c.wall[A][2]; ++cnt; }
  if (EY19[A] < 0 && b.byp) { sum += c.wall[A][3]; ++cnt; }
  if (EZ19[A] > 0 && b.bzm) { sum += c.wall[A][4]; ++cnt; }
  if (EZ19[A] < 0 && b.bzp) { sum += c.wall[A][5]; ++cnt; }
  return cnt > 1 ? sum / R(cnt) : sum;
}

// Element i of an array reached from a launch-uniform base pointer.  Narrow
// form (WIDE = false): the byte offset is formed in 32 bits, which the load and
// store instructions take directly beside the scalar base; the host selects it
// when every byte offset of the launch fits (2 * stride * element size < 2^32).
template <bool WIDE, typename T>
__device__ __forceinline__ T* elem(T* base, uint32_t i) {
  if constexpr (WIDE) {
    return base + i;
  } else {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + i * static_cast<uint32_t>(sizeof(T)));
  }
}

// Where direction A of node n is pulled from, relative to the lower plane P of
// A's opposite pair (opposites are adjacent planes): the shifted neighbour in
// plane A, or node n itself in plane opp(A) when the link crosses a wall.  Both
// offsets are below 2 * stride, so the choice is a 32-bit select.
template <int A>
__device__ __forceinline__ uint32_t pull_offset(bool bounce, int32_t off, uint32_t n,
                                                uint32_t stride) {
  constexpr bool lower = (A == 0) || (A & 1);
  const uint32_t self = lower ? 0u : stride;
  const uint32_t opp = lower ? stride : 0u;
  // node-independent part first: wave-uniform when the offsets and wall flags are
  return (bounce ? opp : self + static_cast<uint32_t>(off)) + n;
}

template <int A>
constexpr int pair_plane() {
  return (A == 0 || (A & 1)) ? A : A - 1;
}

// MOVING = false compiles the wall-momentum term out (the plain step); with
// MOVING = true it is added on bounced links when c.moving is set.  NTL:
// streaming loads.
template <typename S, int A, bool MOVING, bool WIDE, bool NTL = false>
__device__ __forceinline__ typename Storage<S>::R gather_one(
    const S* __restrict__ fin, int64_t stride, uint32_t n, const Nbr& b,
    const CollideArgs<typename Storage<S>::R>& c) {
  using R = typename Storage<S>::R;
  int32_t off;
  const bool bounce = pull_source<EX19[A], EY19[A], EZ19[A]>(b, off);
  const S* base = fin + static_cast<int64_t>(pair_plane<A>()) * stride;
  R v = Storage<S>::template ld<NTL>(
      elem<WIDE>(base, pull_offset<A>(bounce, off, n, static_cast<uint32_t>(stride))));
  if constexpr (MOVING) {
    if (bounce && c.moving) v += wall_term<R, A>(b, c);
  }
  return v;
}

// KEEP0: the rest population's plane keeps cacheable loads under NTL (with
// cacheable stores, store19's KEEP0, it stays in the last-level cache).
template <typename S, bool MOVING, bool WIDE, bool NTL = false, bool KEEP0 = false, int A = 0>
__device__ __forceinline__ void gather19(const S* __restrict__ fin, int64_t stride, uint32_t n,
                                         const Nbr& b,
                                         const CollideArgs<typename Storage<S>::R>& c,
                                         typename Storage<S>::R (&f)[Q19]) {
  if constexpr (A < Q19) {
    f[A] = gather_one<S, A, MOVING, WIDE, (KEEP0 && A == 0) ? false : NTL>(fin, stride, n, b, c);
    gather19<S, MOVING, WIDE, NTL, KEEP0, A + 1>(fin, stride, n, b, c, f);
  }
}

// Narrow form: buffer stores through one resource at the array's base, the
// plane's byte offset in the scalar offset and the node's in the vector offset
// (no address arithmetic per store; wide_offsets keeps every offset below
// 2^32).
// KEEP0: plane 0 takes cacheable stores even under NT.
template <typename S, bool NT, bool WIDE, int Q, bool KEEP0 = false>
__device__ __forceinline__ void store_planes(S* __restrict__ out, const GridArgs& g, uint32_t n,
                                             const typename Storage<S>::R (&v)[Q]) {
  if constexpr (WIDE) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      if (KEEP0 && a == 0)
        Storage<S>::template st<false>(out + n, v[a]);
      else
        Storage<S>::template st<NT>(out + static_cast<int64_t>(a) * g.stride + n, v[a]);
    }
  } else {
    const __amdgpu_buffer_rsrc_t r = raw_rsrc(out);
    const uint32_t plane = static_cast<uint32_t>(g.stride) * static_cast<uint32_t>(sizeof(S));
    const uint32_t voff = n * static_cast<uint32_t>(sizeof(S));
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      if (KEEP0 && a == 0)
        Storage<S>::template st_buf<false>(r, voff, 0u, v[a]);
      else
        Storage<S>::template st_buf<NT>(r, voff, static_cast<uint32_t>(a) * plane, v[a]);
    }
  }
}

template <typename S, bool NT, bool WIDE, bool KEEP0 = false>
__device__ __forceinline__ void store19(S* __restrict__ fout, const GridArgs& g, uint32_t n,
                                        const typename Storage<S>::R (&f)[Q19]) {
  store_planes<S, NT, WIDE, Q19, KEEP0>(fout, g, n, f);
}

// 32-bit finalizer of MurmurHash3 (a bijection with full avalanche).
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// BF16 with stochastic rounding: the upper 16 bits of (FP32 bits + r), r
// uniform in [0, 2^16), round the magnitude up with probability equal to the
// fraction below; non-finite values are kept (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_stochastic(float v, uint32_t r16) {
  uint32_t bits = __float_as_uint(v);
  if ((bits & 0x7F800000u) != 0x7F800000u) bits += r16;
  else if (bits & 0x007FFFFFu) bits |= 0x00400000u;  // quiet NaN survives truncation
  return static_cast<uint16_t>(bits >> 16);
}

// FP16 with stochastic rounding, on the magnitude: 13 of the 23 FP32
// fraction bits are dropped after adding r >> 3, and the result converts
// exactly (Inf on overflow).  Below 2^-14 (FP16 subnormals, spacing 2^-24)
// the magnitude is first offset by 2^-14, which puts the subnormal grid on
// the 13-bit grid of [2^-14, 2^-13], and the offset is taken back exactly
// afterwards: one branch-free sequence for both ranges.  Inf and NaN are kept.
__device__ __forceinline__ uint16_t f16_stochastic(float v, uint32_t r16) {
  constexpr float kMinNormal = 6.103515625e-05f;  // 2^-14
  const uint32_t bits = __float_as_uint(v);
  const uint32_t a = bits & 0x7FFFFFFFu;
  if (a >= 0x7F800000u) return __builtin_bit_cast(uint16_t, static_cast<_Float16>(v));
  const bool sub = a < 0x38800000u;
  const float s = sub ? __uint_as_float(a) + kMinNormal : __uint_as_float(a);
  const float y = __uint_as_float((__float_as_uint(s) + (r16 >> 3)) & ~0x1FFFu);
  const float m = sub ? y - kMinNormal : y;
  return __builtin_bit_cast(
      uint16_t, static_cast<_Float16>(__uint_as_float(__float_as_uint(m) | (bits & 0x80000000u))));
}

template <typename S>
__device__ __forceinline__ uint16_t stochastic16(float v, uint32_t r16) {
  if constexpr (std::is_same_v<S, bf16_t>)
    return bf16_stochastic(v, r16);
  else
    return f16_stochastic(v, r16);
}

// The Q 16-bit stores of node n with stochastic rounding (the counter-based
// random bits documented with lbm_rounding in the C header).
template <typename S, bool NT, bool WIDE, int Q>
__device__ __forceinline__ void store_stochastic(S* __restrict__ fout, const GridArgs& g,
                                                 uint32_t n, const float (&f)[Q]) {
  static_assert(sizeof(S) == 2, "stochastic rounding stores 16-bit values");
  const uint32_t base = n * 0x9E3779B1u + g.step * 0x85EBCA77u + g.seed;
#pragma unroll
  for (int k = 0; k < (Q + 1) / 2; ++k) {
    const uint32_t h = fmix32(base + static_cast<uint32_t>(k) * 0xC2B2AE3Du);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int a = 2 * k + j;
      if (a < Q) {
        const uint16_t bits = stochastic16<S>(f[a], j ? (h >> 16) : (h & 0xFFFFu));
        if constexpr (WIDE) {
          S* p = fout + static_cast<int64_t>(a) * g.stride + n;
          if constexpr (std::is_same_v<S, bf16_t>)
            st_pop<NT>(&p->bits, bits);
          else
            st_pop<NT>(p, __builtin_bit_cast(S, bits));
        } else {
          __builtin_amdgcn_raw_buffer_store_b16(
              bits, raw_rsrc(fout), n * 2u,
              static_cast<uint32_t>(a) * static_cast<uint32_t>(g.stride) * 2u, buf_policy<NT>());
        }
      }
    }
  }
}

// The node's velocity snapshot of the previous check, loaded with the
// populations (before the collision) so that its latency hides behind theirs.
template <typename R, bool WIDE, bool NTL>
__device__ __forceinline__ void load_usnap(const GridArgs& g, const R* __restrict__ usnap, uint32_t n,
                                           R (&uold)[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) uold[k] = ld_pop<NTL>(elem<WIDE>(usnap + static_cast<int64_t>(k) * g.stride, n));
}

// Residual / reduction bookkeeping of one node, accumulated in FP64, given the
// snapshot `uold` from load_usnap.  The velocity snapshot is kept in the
// compute type R: u is an R value, so the FP64 difference of two snapshots is
// exact.
template <typename R, bool WIDE, bool NT>
__device__ __forceinline__ void check_node(const GridArgs& g, R* __restrict__ usnap, uint32_t n,
                                           const R (&uold)[3], R drho, R jx, R jy, R jz, R ux,
                                           R uy, R uz, double (&acc)[kPartials]) {
  const R ur[3] = {ux, uy, uz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R* p = elem<WIDE>(usnap + static_cast<int64_t>(k) * g.stride, n);
    const double uk = static_cast<double>(ur[k]);
    const double d = uk - static_cast<double>(uold[k]);
    st_pop<NT>(p, ur[k]);
    acc[0] += d * d;
    acc[1] += uk * uk;
  }
  acc[2] += static_cast<double>(drho);
  acc[3] += static_cast<double>(jx);
  const bool fin = isfinite(static_cast<double>(drho)) && isfinite(static_cast<double>(jx)) &&
                   isfinite(static_cast<double>(jy)) && isfinite(static_cast<double>(jz));
  acc[4] += fin ? 0.0 : 1.0;
}

__device__ __forceinline__ void write_partials(double* __restrict__ partials, int lb,
                                               double (&acc)[kPartials]) {
  block_sum<kPartials>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kPartials; ++k) partials[static_cast<int64_t>(lb) * kPartials + k] = acc[k];
  }
}

}  // namespace lbm
