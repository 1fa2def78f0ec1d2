// Bandwidth calibration kernels: what the HBM delivers on this GPU for a plain
// streaming copy, and for copies with the access patterns of the FP32 flow
// step (22 planes read, 19 written per node) and of the coupled step (40 and
// 40): one FP32 value per plane and node, the steps' XCD workgroup mapping,
// streaming loads and stores; first with every plane read at the node itself,
// then with every population read where the step reads it (its upstream
// neighbour, or the opposite direction at the node on a wall link), through
// the steps' own neighbour, gather and store code.  The steps' roofline
// fractions are read against these as well as against the 8 TB/s peak.
#include <hip/hip_runtime.h>

#include "../../include/lbm_capi.h"
#include "ctx.hpp"
#include "stream.hpp"

namespace {

using namespace lbm;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One 16-byte value per thread, streaming load and store.
__global__ __launch_bounds__(kBlock) void copy16(const f32x4* __restrict__ src,
                                                 f32x4* __restrict__ dst, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// The flow step's memory pattern without its arithmetic: node n reads PIN
// planes and writes POUT planes (POUT <= PIN); the planes beyond POUT are
// folded into plane 0 so that every load is used.
template <int PIN, int POUT>
__global__ __launch_bounds__(kBlock) void plane_copy(GridArgs g, const float* __restrict__ src,
                                                     float* __restrict__ dst) {
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;
  const uint32_t n = static_cast<uint32_t>(lb) * kBlock + threadIdx.x;
  if (n >= static_cast<uint32_t>(g.N)) return;
  float v[PIN];
#pragma unroll
  for (int p = 0; p < PIN; ++p) v[p] = __builtin_nontemporal_load(src + p * g.stride + n);
  float extra = 0.0f;
#pragma unroll
  for (int p = POUT; p < PIN; ++p) extra += v[p];
  v[0] += 0.0f * extra;
#pragma unroll
  for (int p = 0; p < POUT; ++p) __builtin_nontemporal_store(v[p], dst + p * g.stride + n);
}

// The coupled step's D3Q7 gather without its arithmetic: the three components
// of direction A from the upstream node, or from the opposite direction at the
// node itself on a wall link (the sign of anti-bounce-back is left out).
template <int A = 0>
__device__ __forceinline__ void gather7_raw(const float* __restrict__ gin, uint32_t stride,
                                            uint32_t n, const Nbr& b, float (&v)[3 * Q7]) {
  if constexpr (A < Q7) {
    int32_t off;
    const bool bounce = pull_source<EX7[A], EY7[A], EZ7[A]>(b, off);
    const uint32_t i = pull_offset<A>(bounce, off, n, stride);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      v[j * Q7 + A] = ld_pop<true>(elem<false>(gin + static_cast<int64_t>(j * Q7 + pair_plane<A>()) * stride, i));
    gather7_raw<A + 1>(gin, stride, n, b, v);
  }
}

// The row-aligned FP32 steps' memory traffic without their arithmetic.  Flow
// (COUPLED = false): the 19 populations gathered as the step gathers them, the
// force field's 3 planes (planes 19-21 of src) read at the node, 19 planes
// written.  Coupled: the 19 flow and 21 induction populations (planes 19-39,
// component-major as the library stores them) gathered, 40 planes written.
template <bool COUPLED>
__global__ __launch_bounds__(kBlock) void step_pattern_copy(GridArgs g, const float* __restrict__ src,
                                                            float* __restrict__ dst) {
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;
  const uint32_t n = static_cast<uint32_t>(lb) * kBlock + threadIdx.x;
  if (n >= static_cast<uint32_t>(g.N)) return;
  const Nbr b = neighbours_rows(g, n);
  const uint32_t stride = static_cast<uint32_t>(g.stride);
  const CollideArgs<float> c{};  // no moving walls: the gather does not read it
  float f[Q19];
  gather19<float, false, false, true>(src, g.stride, n, b, c, f);
  const float* __restrict__ rest = src + static_cast<int64_t>(Q19) * g.stride;
  // as in the steps, every load of a node is issued before its first store
  if constexpr (COUPLED) {
    float v[3 * Q7];
    gather7_raw(rest, stride, n, b, v);
    __builtin_amdgcn_sched_barrier(0);
    store19<float, true, false>(dst, g, n, f);
    store_planes<float, true, false, 3 * Q7>(dst + static_cast<int64_t>(Q19) * g.stride, g, n, v);
  } else {
    const float extra = ld_pop<true>(elem<false>(rest, n)) +
                        ld_pop<true>(elem<false>(rest + g.stride, n)) +
                        ld_pop<true>(elem<false>(rest + 2 * g.stride, n));
    f[0] += 0.0f * extra;
    __builtin_amdgcn_sched_barrier(0);
    store19<float, true, false>(dst, g, n, f);
  }
}

}  // namespace

extern "C" {

lbm_status lbm_bandwidth_probe(int32_t pattern, const void* src, void* dst, int32_t nx, int32_t ny,
                               int32_t nz, int32_t walls, int32_t xcd_chunk, int32_t waves,
                               void* hip_stream) {
  if (!src || !dst) return fail(nullptr, LBM_EINVAL, "src and dst must be non-null");
  if (nx < 1 || ny < 1 || nz < 1) return fail(nullptr, LBM_EINVAL, "nx, ny, nz must be >= 1");
  const int64_t nodes = int64_t(nx) * ny * nz;
  if (nodes >= (int64_t(1) << 31)) return fail(nullptr, LBM_EINVAL, "nodes out of range");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(nullptr, LBM_EINVAL, "src and dst must be 16-byte aligned");
  if (waves < 3 || waves > 8) return fail(nullptr, LBM_EINVAL, "waves must be 3..8");
  if (walls < 0 || walls > 7) return fail(nullptr, LBM_EINVAL, "walls must be a mask of bits 0..2");
  // the steps' cap on waves per SIMD: an unused LDS reservation per workgroup
  const uint32_t lds = waves < 8 ? (kLdsPerCu / uint32_t(waves)) / 512u * 512u - 512u : 0u;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (pattern == 0) {
    // 22 planes' worth of FP32 values, copied as 16-byte vectors
    const int64_t count = (22 * nodes) / 4;
    const int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks >= (int64_t(1) << 31)) return fail(nullptr, LBM_EINVAL, "too many nodes");
    copy16<<<dim3(static_cast<uint32_t>(blocks)), kBlock, lds, st>>>(
        static_cast<const f32x4*>(src), static_cast<f32x4*>(dst), count);
  } else if (pattern >= 1 && pattern <= 4) {
    if (xcd_chunk < 1) return fail(nullptr, LBM_EINVAL, "xcd_chunk must be >= 1");
    GridArgs g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.wall_x = walls & 1;
    g.wall_y = (walls >> 1) & 1;
    g.wall_z = (walls >> 2) & 1;
    g.N = static_cast<int32_t>(nodes);
    g.nblocks = static_cast<int32_t>((nodes + kBlock - 1) / kBlock);
    const int bpx0 = (g.nblocks + kXcd - 1) / kXcd;
    const int chunk = xcd_chunk < bpx0 ? xcd_chunk : bpx0;
    g.xcd_chunk = chunk;
    g.div_chunk = make_fastdiv(static_cast<uint32_t>(chunk));
    g.blocks_per_xcd = (bpx0 + chunk - 1) / chunk * chunk;
    g.stride = nodes;
    g.div_nx = make_fastdiv(static_cast<uint32_t>(nx));
    g.div_nxny = make_fastdiv(static_cast<uint32_t>(nx * ny));
    g.nt_load = 1;
    g.lds_reserve = lds;
    g.fhi[0] = nx;
    g.fhi[1] = ny;
    g.fhi[2] = nz;
    const float* s = static_cast<const float*>(src);
    float* d = static_cast<float*>(dst);
    if (pattern >= 3) {
      if (nx % 64 != 0) return fail(nullptr, LBM_EINVAL, "patterns 3 and 4 need nx a multiple of 64");
      if (wide_offsets(g, sizeof(float)))
        return fail(nullptr, LBM_EINVAL, "patterns 3 and 4 need 21 * nodes * 4 bytes below 2^32");
    }
    if (pattern == 1)
      plane_copy<22, 19><<<step_grid(g), kBlock, lds, st>>>(g, s, d);
    else if (pattern == 2)
      plane_copy<40, 40><<<step_grid(g), kBlock, lds, st>>>(g, s, d);
    else if (pattern == 3)
      step_pattern_copy<false><<<step_grid(g), kBlock, lds, st>>>(g, s, d);
    else
      step_pattern_copy<true><<<step_grid(g), kBlock, lds, st>>>(g, s, d);
  } else {
    return fail(nullptr, LBM_EINVAL, "pattern must be 0..4");
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(nullptr, e, "probe launch");
  return LBM_OK;
}

}  // extern "C"
