// Host-side context of the C ABI, shared by the forward (lbm_capi.hip) and
// adjoint (adjoint.hip) entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbm_capi.h"
#include "launch.hpp"

namespace lbm {

inline size_t storage_bytes(int storage) {
  switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_BF16: return 2;
    case LBM_F16: return 2;
    default: return 0;
  }
}

inline size_t compute_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }

// Population planes of the flow (19 for D3Q19, 9 for D2Q9) and of the
// induction lattice (3 x 7 for D3Q7, 2 x 5 for D2Q5).
inline int flow_planes(const lbm_params& p) { return p.lattice == LBM_D2Q9 ? 9 : 19; }
inline int mag_planes(const lbm_params& p) { return p.lattice == LBM_D2Q9 ? 10 : 21; }

struct Layout {
  int64_t N = 0, stride = 0;
  int32_t nblocks = 0;
  size_t f[2] = {0, 0}, g[2] = {0, 0}, force = 0, usnap = 0, partials = 0, fpartials = 0, ring = 0,
         rec = 0;
  int32_t pslots = 1;  // slots of the per-check partials ring
  size_t total = 0;
};

}  // namespace lbm

using lbm::Layout;

struct lbm_ctx {
  lbm_grid grid;
  lbm_params p;
  Layout L;
  lbm::GridArgs ga;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  int cur = 0;
  bool nt_store = false;  // streaming (cache-bypassing) population stores
  bool tune_chunk = false;  // time the XCD chunk candidates at create
  int waves = 8;            // cap on waves per SIMD of the 3D step kernels (8: none)
  int64_t step = 0;
  int64_t checks = 0;            // residual checks launched since the last reset
  int64_t finalized = 0;         // checks whose history records have been written
  int64_t first_check_step = 0;  // step number of check 0
  lbm::CollideArgs<double> cd;
  lbm::CollideArgs<float> cf;
  lbm::MagArgs<double> md;
  lbm::MagArgs<float> mf;
  std::string err;
  std::vector<hipEvent_t> events;
  // pinned host staging for history reads of up to kHostRecs records (a copy
  // into pageable memory costs tens of microseconds more); null if the
  // allocation failed, and then reads go to pageable memory
  static constexpr int64_t kHostRecs = 64;
  double* host_rec = nullptr;

  lbm_ctx() = default;
  lbm_ctx(const lbm_ctx&) = delete;
  lbm_ctx& operator=(const lbm_ctx&) = delete;
  ~lbm_ctx() {
    if (host_rec) (void)hipHostFree(host_rec);
  }

  void* f(int i) const { return ws + L.f[i]; }
  void* g(int i) const { return p.mhd ? static_cast<void*>(ws + L.g[i]) : nullptr; }
  void* force() const { return p.force_mode == LBM_FORCE_FIELD ? static_cast<void*>(ws + L.force) : nullptr; }
  void* usnap() const { return ws + L.usnap; }
  double* partials() const { return reinterpret_cast<double*>(ws + L.partials); }
  double* fpartials() const { return reinterpret_cast<double*>(ws + L.fpartials); }
  double* ring() const { return reinterpret_cast<double*>(ws + L.ring); }
  double* rec() const { return reinterpret_cast<double*>(ws + L.rec); }
  bool field() const { return p.force_mode == LBM_FORCE_FIELD; }
  size_t elem() const { return lbm::storage_bytes(p.storage); }
  size_t celem() const { return lbm::compute_bytes(p.storage); }
  int qf() const { return lbm::flow_planes(p); }
  int qg() const { return lbm::mag_planes(p); }
};

namespace lbm {
// Helpers defined in lbm_capi.hip.
std::string validate_params(const lbm_grid* grid, const lbm_params* p);  // "" when valid
lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& msg);
lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* what);
lbm_status one_step(lbm_ctx* c, hipEvent_t start = nullptr, hipEvent_t stop = nullptr,
                    bool* with_start = nullptr);
void choose_launch_shape(lbm_ctx* c);
lbm_status flush_checks(lbm_ctx* c);
void reset_checks(lbm_ctx* c, int64_t step);
}  // namespace lbm

#define LBM_HIP(ctx, call, what)                          \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return ::lbm::hip_fail(ctx, e_, what); \
  } while (0)
