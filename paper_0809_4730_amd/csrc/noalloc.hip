// lbm_reductions_noalloc: the FP64 mass and flow-rate reductions of a
// population state held by the caller, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  The same fields
// and finalize kernels as lbm_reductions; their per-workgroup partial sums and
// the reduced record live in a fixed file-scope device array instead of a
// context workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/lbm_capi.h"
#include "args.hpp"
#include "ctx.hpp"
#include "stream.hpp"

// Scratch of the no-allocation entry point: one record of kRecordDoubles FP64
// values at offset 0, then the per-workgroup partial sums (kPartials doubles
// per workgroup of kBlock nodes) from offset kPartialsAt.  Each GPU the library
// runs on holds its own copy until the process ends.
static constexpr size_t kScratchBytes = size_t(4) << 20;
static constexpr size_t kPartialsAt = 256;
static constexpr int64_t kMaxBlocks =
    static_cast<int64_t>((kScratchBytes - kPartialsAt) / (lbm::kPartials * sizeof(double)));

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

using namespace lbm;

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
char* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device
// with that device current (the array's name in host code is not a device
// address).
hipError_t scratch_ptr(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_once[dev], [dev] {
    void* p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = static_cast<char*>(p);
  });
  if (g_err[dev] != hipSuccess) return g_err[dev];
  *out = g_ptr[dev];
  return hipSuccess;
}

template <typename S>
hipError_t enqueue(const lbm_grid* grid, const lbm_params* p, const void* state, const void* force,
                   char* sc, hipStream_t st) {
  using R = typename Storage<S>::R;
  const int64_t N = int64_t(grid->n[0]) * grid->n[1] * grid->n[2];
  GridArgs g{};
  g.nx = grid->n[0];
  g.ny = grid->n[1];
  g.nz = grid->n[2];
  g.wall_x = grid->bc[0] == LBM_WALL;
  g.wall_y = grid->bc[1] == LBM_WALL;
  g.wall_z = grid->bc[2] == LBM_WALL;
  g.N = static_cast<int32_t>(N);
  g.nblocks = static_cast<int32_t>((N + kBlock - 1) / kBlock);
  g.blocks_per_xcd = (g.nblocks + kXcd - 1) / kXcd;
  g.xcd_chunk = g.blocks_per_xcd;  // one slab per XCD
  g.div_chunk = make_fastdiv(static_cast<uint32_t>(g.xcd_chunk));
  g.stride = N;  // the caller's arrays are [q][N] and [3][N], unpadded
  g.div_nx = make_fastdiv(static_cast<uint32_t>(g.nx));
  g.div_nxny = make_fastdiv(static_cast<uint32_t>(g.nx * g.ny));
  for (int a = 0; a < 3; ++a) {
    g.flo[a] = 0;
    g.fhi[a] = grid->n[a];
  }
  const CollideArgs<R> c = collide_args<R>(*p);
  const MagArgs<R> m = mag_args<R>(*p);
  const bool field = p->force_mode == LBM_FORCE_FIELD;
  double* partials = reinterpret_cast<double*>(sc + kPartialsAt);
  double* rec = reinterpret_cast<double*>(sc);
  // every workgroup below nblocks writes its partial sums and finalize writes
  // the whole record, so nothing left by an earlier call is read
  hipError_t e =
      p->lattice == LBM_D2Q9
          ? launch_fields2<S>(g, c, m, false, state, nullptr, field ? force : nullptr, field, 0,
                              nullptr, nullptr, nullptr, N, partials, st)
          : launch_fields<S>(g, c, m, false, state, nullptr, field ? force : nullptr, field, 0,
                             nullptr, nullptr, nullptr, N, partials, st);
  if (e != hipSuccess) return e;
  return launch_finalize(partials, g.nblocks, 1, 0, 1, 0.0, 0.0, 1.0 / double(grid->n[0]), rec, 1,
                         st);
}

}  // namespace

extern "C" {

lbm_status lbm_reductions_noalloc(const lbm_grid* grid, const lbm_params* params,
                                  const void* state, const void* force, void* hip_stream,
                                  double* out) {
  const std::string v = validate_params(grid, params);
  if (!v.empty()) return fail(nullptr, LBM_EINVAL, v);
  if (params->mhd) return fail(nullptr, LBM_EUNSUPPORTED, "no induction lattice (mhd = 0 only)");
  if (!state || !out) return fail(nullptr, LBM_EINVAL, "state and out must be non-null");
  if (params->force_mode == LBM_FORCE_FIELD && !force)
    return fail(nullptr, LBM_EINVAL, "force_mode = FIELD needs a force pointer");
  const int64_t N = int64_t(grid->n[0]) * grid->n[1] * grid->n[2];
  const int64_t blocks = (N + kBlock - 1) / kBlock;
  if (blocks > kMaxBlocks)
    return fail(nullptr, LBM_ENOWS,
                "lattice of " + std::to_string(N) + " nodes needs " +
                    std::to_string(kPartialsAt + blocks * kPartials * sizeof(double)) +
                    " bytes of scratch; the no-allocation reductions hold " +
                    std::to_string(kScratchBytes) + " (at most " +
                    std::to_string(kMaxBlocks * kBlock) + " nodes)");
  char* sc = nullptr;
  hipError_t e = scratch_ptr(&sc);
  if (e != hipSuccess) return hip_fail(nullptr, e, "scratch address");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  switch (params->storage) {
    case LBM_F64: e = enqueue<double>(grid, params, state, force, sc, st); break;
    case LBM_F32: e = enqueue<float>(grid, params, state, force, sc, st); break;
    case LBM_BF16: e = enqueue<bf16_t>(grid, params, state, force, sc, st); break;
    default: e = enqueue<_Float16>(grid, params, state, force, sc, st);
  }
  if (e != hipSuccess) return hip_fail(nullptr, e, "reduction launch");
  // mass (record[4]) and flow rate (record[5]) to the caller's two doubles
  e = hipMemcpyAsync(out, sc + 4 * sizeof(double), 2 * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(nullptr, e, "result copy");
  return LBM_OK;
}

}  // extern "C"
