// Bandwidth calibration kernels: what the HBM delivers on this GPU for a plain
// streaming copy, and for copies with exactly the access patterns of the FP32
// flow step (22 planes read, 19 written per node) and of the coupled step (40
// and 40): one FP32 value per plane and node, the steps' XCD workgroup
// mapping, streaming loads and stores.  The steps' roofline fractions are
// read against these as well as against the 8 TB/s peak.
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

}  // namespace

extern "C" {

lbm_status lbm_bandwidth_probe(int32_t pattern, const void* src, void* dst, int64_t nodes,
                               int32_t xcd_chunk, int32_t waves, void* hip_stream) {
  if (!src || !dst) return fail(nullptr, LBM_EINVAL, "src and dst must be non-null");
  if (nodes < 1 || nodes >= (int64_t(1) << 31)) return fail(nullptr, LBM_EINVAL, "nodes out of range");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(nullptr, LBM_EINVAL, "src and dst must be 16-byte aligned");
  if (waves < 3 || waves > 8) return fail(nullptr, LBM_EINVAL, "waves must be 3..8");
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
  } else if (pattern == 1 || pattern == 2) {
    if (xcd_chunk < 1) return fail(nullptr, LBM_EINVAL, "xcd_chunk must be >= 1");
    GridArgs g{};
    g.N = static_cast<int32_t>(nodes);
    g.nblocks = static_cast<int32_t>((nodes + kBlock - 1) / kBlock);
    const int bpx0 = (g.nblocks + kXcd - 1) / kXcd;
    const int chunk = xcd_chunk < bpx0 ? xcd_chunk : bpx0;
    g.xcd_chunk = chunk;
    g.div_chunk = make_fastdiv(static_cast<uint32_t>(chunk));
    g.blocks_per_xcd = (bpx0 + chunk - 1) / chunk * chunk;
    g.stride = nodes;
    if (pattern == 1)
      plane_copy<22, 19><<<step_grid(g), kBlock, lds, st>>>(g, static_cast<const float*>(src),
                                                            static_cast<float*>(dst));
    else
      plane_copy<40, 40><<<step_grid(g), kBlock, lds, st>>>(g, static_cast<const float*>(src),
                                                            static_cast<float*>(dst));
  } else {
    return fail(nullptr, LBM_EINVAL, "pattern must be 0, 1 or 2");
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(nullptr, e, "probe launch");
  return LBM_OK;
}

}  // extern "C"
