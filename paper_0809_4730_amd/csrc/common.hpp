// Shared device/host definitions for the gfx950 kernels: kernel argument
// blocks, exact fast division, XCD-aware block numbering, storage-type
// conversion and FP64 block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.hpp"

namespace lbm {

// Streaming (non-temporal) loads and stores and the XCD block mapping are
// chosen per context at create (GridArgs::xcd_chunk, the NTL / NT template
// flags of the steps; lbm_params.launch).

// Build-time knob: LBM_BLOCK threads per workgroup (a multiple of 64).
#ifndef LBM_BLOCK
#define LBM_BLOCK 256
#endif

constexpr int kBlock = LBM_BLOCK;  // threads per workgroup (4 wave64 by default)
constexpr uint32_t kLdsPerCu = 160 * 1024;  // LDS bytes per compute unit on gfx950
static_assert(kBlock % 64 == 0 && kBlock <= 1024, "LBM_BLOCK must be a multiple of 64, at most 1024");
constexpr int kXcd = 8;       // XCDs on MI355X; workgroups are dealt round-robin
constexpr int kRecordDoubles = 8;
constexpr int kPartials = 5;  // du2, u2, mass, flow, nonfinite

// q = floor(n / d) for n < 2^32 via one 64x64 high multiply:
// M = ceil(2^64 / d) gives n*M/2^64 = n/d + e with 0 <= e < n/2^64 < 1/d.
struct FastDiv {
  uint64_t M;
  uint32_t d;
  uint32_t pad;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.pad = 0;
  f.M = (d <= 1) ? 0ull : (~0ull) / d + 1ull;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return f.d == 1 ? n : static_cast<uint32_t>(__umul64hi(static_cast<uint64_t>(n), f.M));
}

struct GridArgs {
  int32_t nx, ny, nz;
  int32_t wall_x, wall_y, wall_z;
  int32_t N;               // nodes
  int32_t nblocks;         // logical workgroups covering N
  int32_t blocks_per_xcd;  // launched grid = kXcd * blocks_per_xcd (a multiple of xcd_chunk)
  int32_t xcd_chunk;       // consecutive logical blocks an XCD takes at a time
  int64_t stride;          // elements between direction planes (N rounded up to 64)
  FastDiv div_nx, div_nxny;
  FastDiv div_chunk;       // division by xcd_chunk
  int32_t wide;            // 1: 64-bit element offsets even where 32-bit byte offsets fit
  int32_t nt_load;         // 1: streaming population and force loads (launchers: NTL flag)
  int32_t force_cached;    // 1: a force field read with streaming population loads keeps
                           // cacheable loads (it fits in the last-level cache, where the
                           // streaming traffic leaves it; launchers: the step's load policy)
  int32_t rest_cached;     // 1: without a cached force field, the rest population's two
                           // planes keep cacheable loads and stores (launchers, likewise)
  uint32_t lds_reserve;    // dynamic LDS bytes per workgroup of a 3D step launch: reserved, not
                           // used, to cap the workgroups per CU (0: no cap)
  uint32_t step;           // the step number a step launch computes (stochastic rounding)
  uint32_t seed;           // stochastic rounding seed
  // Fluid box [flo, fhi) per axis (x, y, z).  The whole lattice, unless the
  // induction lattice extends beyond the fluid; its faces are then no-slip
  // walls of the flow, while the induction lattice's walls stay at the lattice
  // faces.
  int32_t flo[3], fhi[3];
};

// Workgroup b of the launch runs on XCD (b mod 8) as that XCD's (b / 8)-th
// workgroup.  XCDs take chunks of xcd_chunk consecutive logical blocks in turn:
// chunk = blocks_per_xcd gives each XCD one contiguous slab (neighbour rows stay
// in its L2: best when the lattice lives in the caches); small chunks keep all
// XCDs on the same DRAM pages (the host picks among them for lattices that
// stream from HBM).
__device__ __forceinline__ int logical_block(const GridArgs& g) {
  const uint32_t b = blockIdx.x;
  const uint32_t xcd = b & (kXcd - 1);
  const uint32_t i = b >> 3;
  const uint32_t C = static_cast<uint32_t>(g.xcd_chunk);
  const uint32_t q = fdiv(i, g.div_chunk);  // i / C
  return static_cast<int>((q * kXcd + xcd) * C + (i - q * C));
}

// Collision constants for compute type R (host-prepared).
template <typename R>
struct CollideArgs {
  R rho0;
  R inv_gamma;     // 1/gamma: nonlinear equilibrium terms, linear source terms
  R inv_gamma2;    // 1/gamma^2: F.u source terms (1/gamma for the naive source form)
  R half_inv_gamma;  // 1/(2 gamma): half-force in j
  R A[Q19];        // s_k / |T_k|^2
  R B[Q19];        // (1 - s_k/2) / |T_k|^2
  R F[3];          // uniform force (force_mode = UNIFORM)
  R wall[Q19][6];  // 6 w_a rho0 (e_a . u_face) for link bounce-back at moving faces
  int32_t moving;  // any face moving
};

// Induction-LKE constants (Sec. 4, 4.1).
template <typename R>
struct MagArgs {
  R omega;       // 1 / tau_m*
  R adv;         // chi / (gamma_m theta_m)
  R a_coef;      // -1 / (mu chi tau_m* theta_m)
  R kappa;       // 2 / (mu gamma_m tau_m* theta_m)
  R B0[3];       // applied field: initial state and wall value
  R w_rest, w_axis;
};

// ------------------------------------------------------------- storage ----
struct bf16_t {
  uint16_t bits;
};

template <typename S>
struct Storage;

// NT: streaming load (the value is used once; do not keep its line in the caches)
template <bool NT = false, typename T>
__device__ __forceinline__ T ld_pop(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st_pop(T* p, T v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Buffer resource over an array (raw addressing, no range limit): stores
// through it take a scalar and a 32-bit vector byte offset.  Word 3 is the
// gfx9 raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, 0xffffffff, 0x00020000);
}

// cache policy of a buffer store: nt (streaming) or default
template <bool NT>
constexpr int buf_policy() {
  return NT ? 2 : 0;
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <>
struct Storage<double> {
  using R = double;
  template <bool NT = false>
  __device__ __forceinline__ static R ld(const double* p) { return ld_pop<NT>(p); }
  template <bool NT = false>
  __device__ __forceinline__ static void st(double* p, R v) { st_pop<NT>(p, v); }
  template <bool NT = false>
  __device__ __forceinline__ static void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff,
                                          buf_policy<NT>());
  }
};

template <>
struct Storage<float> {
  using R = float;
  template <bool NT = false>
  __device__ __forceinline__ static R ld(const float* p) { return ld_pop<NT>(p); }
  template <bool NT = false>
  __device__ __forceinline__ static void st(float* p, R v) { st_pop<NT>(p, v); }
  template <bool NT = false>
  __device__ __forceinline__ static void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, buf_policy<NT>());
  }
};

template <>
struct Storage<bf16_t> {
  using R = float;
  template <bool NT = false>
  __device__ __forceinline__ static R ld(const bf16_t* p) {
    return __uint_as_float(static_cast<uint32_t>(ld_pop<NT>(&p->bits)) << 16);
  }
  // round to nearest, ties to even, NaN stays NaN: one v_cvt_pk_bf16_f32 on gfx950
  template <bool NT = false>
  __device__ __forceinline__ static void st(bf16_t* p, R v) {
    st_pop<NT>(&p->bits, __builtin_bit_cast(uint16_t, static_cast<__bf16>(v)));
  }
  template <bool NT = false>
  __device__ __forceinline__ static void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, static_cast<__bf16>(v)), r,
                                          voff, soff, buf_policy<NT>());
  }
};

template <>
struct Storage<_Float16> {
  using R = float;
  template <bool NT = false>
  __device__ __forceinline__ static R ld(const _Float16* p) {
    return static_cast<float>(ld_pop<NT>(p));
  }
  template <bool NT = false>
  __device__ __forceinline__ static void st(_Float16* p, R v) {
    st_pop<NT>(p, static_cast<_Float16>(v));
  }
  template <bool NT = false>
  __device__ __forceinline__ static void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, static_cast<_Float16>(v)),
                                          r, voff, soff, buf_policy<NT>());
  }
};

// ------------------------------------------------------------ reductions --
// v from the lane CTRL selects (DPP row shift right within rows of 16 lanes);
// lanes whose source lies outside the row read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_row_shr(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                        static_cast<uint32_t>(lo));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(u), lane);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Sum over the 64 lanes of a wave (all lanes active), returned to every lane.
// Inclusive prefix sums within each row of 16 lanes by row shifts of 1, 2, 4
// and 8 (register moves, no LDS), then the four row totals from lanes 15, 31,
// 47, 63 in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_row_shr<0x111>(v);
  v += dpp_row_shr<0x112>(v);
  v += dpp_row_shr<0x114>(v);
  v += dpp_row_shr<0x118>(v);
  return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

// Sum K doubles over the workgroup; thread 0 receives the totals in v.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
  __shared__ double red[kBlock / 64][K];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) s += red[w][k];
      v[k] = s;
    }
  }
}

}  // namespace lbm
