// Batched marches of independent lattices in one launch per step: the
// stability map of Sec. 5 classifies many (viscosity, velocity, gamma) points
// on small Poiseuille lattices, each far too small to fill the GPU alone.
//
// Every member has the same grid but its own gamma, rates and uniform force.
// Member m owns the workgroups [m B, (m+1) B) of the launch (B = its node
// count rounded up to whole workgroups), so its index, arguments and verdict
// are uniform per workgroup and its residual partial sums belong to it alone.
// A check kernel (one thread per member) turns them into a residual and a
// verdict with the single-lattice rules: non-finite values or a residual above
// 1e-2 and 1e3 times its running minimum make a member unstable, a residual
// below tol converged; decided members are not marched further.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/lbm_capi.h"
#include "args.hpp"
#include "collide.hpp"
#include "ctx.hpp"
#include "stream.hpp"

namespace lbm {
namespace {

constexpr int32_t kRunning = 0, kConverged = 1, kUnstable = 2;

struct BatchArgs {
  int32_t count;              // members
  int32_t blocks_per_member;  // workgroups per member
};

template <typename S, bool CHECK, bool WIDE>
__global__ __launch_bounds__(kBlock) void batch_step(GridArgs g, BatchArgs ba,
                                                     const CollideArgs<typename Storage<S>::R>* __restrict__ args,
                                                     const int32_t* __restrict__ verdict,
                                                     const S* __restrict__ fin, S* __restrict__ fout,
                                                     typename Storage<S>::R* __restrict__ usnap,
                                                     double* __restrict__ partials) {
  using R = typename Storage<S>::R;
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;
  const int m = lb / ba.blocks_per_member;
  if (verdict[m] != kRunning) return;  // whole workgroup: decided member
  const uint32_t base = static_cast<uint32_t>(m) * static_cast<uint32_t>(ba.blocks_per_member) * kBlock;
  const uint32_t local = static_cast<uint32_t>(lb) * kBlock + threadIdx.x - base;
  double acc[kPartials] = {};
  if (local < static_cast<uint32_t>(g.N)) {
    const CollideArgs<R>& c = args[m];
    const Nbr b = neighbours(g, local);  // offsets within the member's lattice
    const uint32_t n = base + local;
    R f[Q19];
    gather19<S, false, WIDE>(fin, g.stride, n, b, c, f);
    R uold[3];
    if constexpr (CHECK) load_usnap<R, WIDE, false>(g, usnap, n, uold);
    const NodeMacro<R> mac = collide19<R>(f, c.F[0], c.F[1], c.F[2], c);
    store19<S, false, WIDE>(fout, g, n, f);
    if constexpr (CHECK)
      check_node<R, WIDE, false>(g, usnap, n, uold, mac.drho, mac.jx, mac.jy, mac.jz, mac.ux,
                                 mac.uy, mac.uz, acc);
  }
  if constexpr (CHECK) write_partials(partials, lb, acc);
}

__global__ __launch_bounds__(kBlock) void batch_check(BatchArgs ba, const double* __restrict__ partials,
                                                      int64_t check_index, int64_t step, double tol,
                                                      int32_t* __restrict__ verdict,
                                                      int64_t* __restrict__ vstep,
                                                      double* __restrict__ rmin,
                                                      double* __restrict__ rlast) {
  const int m = blockIdx.x * kBlock + threadIdx.x;
  if (m >= ba.count || verdict[m] != kRunning) return;
  double acc[kPartials] = {};
  for (int b = 0; b < ba.blocks_per_member; ++b) {
    const double* p = partials + (static_cast<int64_t>(m) * ba.blocks_per_member + b) * kPartials;
#pragma unroll
    for (int k = 0; k < kPartials; ++k) acc[k] += p[k];
  }
  const double du2 = acc[0], u2 = acc[1];
  const double r = u2 > 0.0 ? sqrt(du2 / u2) : (du2 == 0.0 ? 0.0 : INFINITY);
  rlast[m] = r;
  if (acc[4] > 0.0 || isnan(r)) {
    verdict[m] = kUnstable;
    vstep[m] = step;
    return;
  }
  if (check_index == 0) return;  // the first check compares against zero velocity
  const double mn = fmin(rmin[m], r);
  rmin[m] = mn;
  if (r > 1e-2 && r > 1e3 * mn) {
    verdict[m] = kUnstable;
    vstep[m] = step;
  } else if (r < tol) {
    verdict[m] = kConverged;
    vstep[m] = step;
  }
}

struct BatchLayout {
  int64_t Nl = 0, stride = 0;
  int32_t bpm = 0, nblocks = 0;
  size_t f[2] = {0, 0}, usnap = 0, partials = 0, args = 0, verdict = 0, vstep = 0, rmin = 0,
         rlast = 0, total = 0;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

std::string check_grid(const lbm_grid* grid) {
  if (!grid) return "grid is NULL";
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] < 1) return "grid dimensions must be >= 1";
    if (grid->bc[a] != LBM_PERIODIC && grid->bc[a] != LBM_WALL)
      return "bc must be LBM_PERIODIC or LBM_WALL";
  }
  return "";
}

std::string make_batch_layout(const lbm_grid* grid, int32_t storage, int32_t count, BatchLayout& L) {
  const std::string e = check_grid(grid);
  if (!e.empty()) return e;
  if (storage_bytes(storage) == 0) return "storage must be LBM_F64, LBM_F32, LBM_BF16 or LBM_F16";
  if (count < 1) return "count must be >= 1";
  L.Nl = int64_t(grid->n[0]) * grid->n[1] * grid->n[2];
  const int64_t bpm = (L.Nl + kBlock - 1) / kBlock;
  const int64_t nodes = bpm * kBlock * count;
  if (nodes >= (int64_t(1) << 31)) return "count x padded member size reaches 2^31 nodes";
  L.bpm = int32_t(bpm);
  L.nblocks = int32_t(bpm * count);
  L.stride = nodes;  // a multiple of kBlock
  const size_t es = storage_bytes(storage), cs = compute_bytes(storage);
  const size_t argb = cs == 8 ? sizeof(CollideArgs<double>) : sizeof(CollideArgs<float>);
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off = align256(off + b);
    return at;
  };
  L.f[0] = take(19 * L.stride * es);
  L.f[1] = take(19 * L.stride * es);
  L.usnap = take(3 * L.stride * cs);
  L.partials = take(size_t(L.nblocks) * kPartials * sizeof(double));
  L.args = take(size_t(count) * argb);
  L.verdict = take(size_t(count) * sizeof(int32_t));
  L.vstep = take(size_t(count) * sizeof(int64_t));
  L.rmin = take(size_t(count) * sizeof(double));
  L.rlast = take(size_t(count) * sizeof(double));
  L.total = off;
  return "";
}

std::string check_member(const lbm_member& m, int i) {
  char buf[128];
  if (!(m.gamma > 0.0 && m.gamma <= 1.0)) {
    std::snprintf(buf, sizeof buf, "member %d: gamma must lie in (0, 1]", i);
    return buf;
  }
  for (int k = 0; k < 19; ++k) {
    const bool conserved = k == 0 || k == 3 || k == 5 || k == 7;
    if (!conserved && !(m.s[k] > 0.0 && m.s[k] < 2.0)) {
      std::snprintf(buf, sizeof buf, "member %d: rate s[%d] = %g outside (0, 2)", i, k, m.s[k]);
      return buf;
    }
  }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(m.force[a])) {
      std::snprintf(buf, sizeof buf, "member %d: force must be finite", i);
      return buf;
    }
  return "";
}

template <typename S>
lbm_status batch_run(const lbm_grid* grid, int32_t storage, double rho0, int32_t count,
                     const lbm_member* members, char* ws, const BatchLayout& L, hipStream_t st,
                     double tol, int64_t max_steps, int32_t check_every, int64_t poll_every,
                     int32_t wide, lbm_member_result* results) {
  using R = typename Storage<S>::R;
  GridArgs g{};
  g.nx = grid->n[0];
  g.ny = grid->n[1];
  g.nz = grid->n[2];
  g.wall_x = grid->bc[0] == LBM_WALL;
  g.wall_y = grid->bc[1] == LBM_WALL;
  g.wall_z = grid->bc[2] == LBM_WALL;
  g.N = int32_t(L.Nl);
  g.nblocks = L.nblocks;
  g.blocks_per_xcd = (L.nblocks + kXcd - 1) / kXcd;
  g.xcd_chunk = g.blocks_per_xcd;
  g.div_chunk = make_fastdiv(uint32_t(g.xcd_chunk));
  g.wide = wide;
  g.stride = L.stride;
  g.div_nx = make_fastdiv(uint32_t(g.nx));
  g.div_nxny = make_fastdiv(uint32_t(g.nx * g.ny));
  for (int a = 0; a < 3; ++a) {
    g.flo[a] = 0;
    g.fhi[a] = grid->n[a];
  }
  const BatchArgs ba{count, L.bpm};

  std::vector<CollideArgs<R>> hargs(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    lbm_params p{};
    p.storage = storage;
    p.gamma = members[i].gamma;
    for (int k = 0; k < 19; ++k) p.s[k] = members[i].s[k];
    p.rho0 = rho0;
    for (int a = 0; a < 3; ++a) p.force_const[a] = members[i].force[a];
    hargs[size_t(i)] = collide_args<R>(p);
  }
  std::vector<int32_t> hverdict(size_t(count), kRunning);
  std::vector<int64_t> hvstep(size_t(count), -1);
  std::vector<double> hrmin(size_t(count), INFINITY), hrlast(size_t(count), NAN);

  S* f[2] = {reinterpret_cast<S*>(ws + L.f[0]), reinterpret_cast<S*>(ws + L.f[1])};
  R* usnap = reinterpret_cast<R*>(ws + L.usnap);
  double* partials = reinterpret_cast<double*>(ws + L.partials);
  auto* dargs = reinterpret_cast<CollideArgs<R>*>(ws + L.args);
  auto* dverdict = reinterpret_cast<int32_t*>(ws + L.verdict);
  auto* dvstep = reinterpret_cast<int64_t*>(ws + L.vstep);
  auto* drmin = reinterpret_cast<double*>(ws + L.rmin);
  auto* drlast = reinterpret_cast<double*>(ws + L.rlast);

#define LBM_BHIP(call, what)                                  \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hip_fail(nullptr, e_, what); \
  } while (0)
  LBM_BHIP(launch_fill_zero<S>(f[0], 19 * L.stride, st), "fill");
  LBM_BHIP(launch_fill_zero<R>(usnap, 3 * L.stride, st), "fill");
  LBM_BHIP(hipMemcpyAsync(dargs, hargs.data(), hargs.size() * sizeof(CollideArgs<R>),
                          hipMemcpyHostToDevice, st), "argument copy");
  LBM_BHIP(hipMemcpyAsync(dverdict, hverdict.data(), hverdict.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st), "status copy");
  LBM_BHIP(hipMemcpyAsync(dvstep, hvstep.data(), hvstep.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, st), "status copy");
  LBM_BHIP(hipMemcpyAsync(drmin, hrmin.data(), hrmin.size() * sizeof(double),
                          hipMemcpyHostToDevice, st), "status copy");
  LBM_BHIP(hipMemcpyAsync(drlast, hrlast.data(), hrlast.size() * sizeof(double),
                          hipMemcpyHostToDevice, st), "status copy");

  const dim3 grid_dim(kXcd * g.blocks_per_xcd), check_dim((count + kBlock - 1) / kBlock);
  const bool use_wide = wide_offsets(g, sizeof(R));
  int cur = 0;
  int64_t checks = 0;
  for (int64_t step = 1; step <= max_steps; ++step) {
    const bool check = step % check_every == 0;
    LBM_BHIP(with_flag(check, [&](auto CH) {
               return with_flag(use_wide, [&](auto W) {
                 batch_step<S, decltype(CH)::value, decltype(W)::value>
                     <<<grid_dim, kBlock, 0, st>>>(g, ba, dargs, dverdict, f[cur], f[cur ^ 1], usnap,
                                                   partials);
                 return hipGetLastError();
               });
             }),
             "batch step launch");
    if (check) {
      batch_check<<<check_dim, kBlock, 0, st>>>(ba, partials, checks, step, tol, dverdict, dvstep,
                                                drmin, drlast);
      LBM_BHIP(hipGetLastError(), "batch check launch");
      ++checks;
    }
    cur ^= 1;
    if (step % poll_every == 0) {
      LBM_BHIP(hipMemcpyAsync(hverdict.data(), dverdict, hverdict.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, st), "status read");
      LBM_BHIP(hipStreamSynchronize(st), "hipStreamSynchronize");
      bool open = false;
      for (int32_t v : hverdict) open = open || v == kRunning;
      if (!open) break;
    }
  }
  LBM_BHIP(hipMemcpyAsync(hverdict.data(), dverdict, hverdict.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, st), "status read");
  LBM_BHIP(hipMemcpyAsync(hvstep.data(), dvstep, hvstep.size() * sizeof(int64_t),
                          hipMemcpyDeviceToHost, st), "status read");
  LBM_BHIP(hipMemcpyAsync(hrlast.data(), drlast, hrlast.size() * sizeof(double),
                          hipMemcpyDeviceToHost, st), "status read");
  LBM_BHIP(hipStreamSynchronize(st), "hipStreamSynchronize");
#undef LBM_BHIP
  for (int i = 0; i < count; ++i) {
    results[i].verdict = hverdict[size_t(i)];
    results[i].reserved = 0;
    results[i].step = hvstep[size_t(i)];
    results[i].residual = hrlast[size_t(i)];
  }
  return LBM_OK;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" {

lbm_status lbm_batch_workspace_bytes(const lbm_grid* grid, int32_t storage, int32_t count,
                                     size_t* bytes) {
  if (!bytes) return fail(nullptr, LBM_EINVAL, "bytes is NULL");
  BatchLayout L;
  const std::string e = make_batch_layout(grid, storage, count, L);
  if (!e.empty()) return fail(nullptr, LBM_EINVAL, e);
  *bytes = L.total;
  return LBM_OK;
}

lbm_status lbm_batch_run(const lbm_grid* grid, int32_t storage, double rho0, int32_t count,
                         const lbm_member* members, void* workspace, size_t workspace_bytes,
                         void* stream, double tol, int64_t max_steps, int32_t check_every,
                         int64_t poll_every, const lbm_launch* launch,
                         lbm_member_result* results) {
  BatchLayout L;
  std::string e = make_batch_layout(grid, storage, count, L);
  if (!e.empty()) return fail(nullptr, LBM_EINVAL, e);
  if (!members || !results) return fail(nullptr, LBM_EINVAL, "members and results must be non-null");
  if (!(rho0 > 0.0)) return fail(nullptr, LBM_EINVAL, "rho0 must be positive");
  const int32_t wide = launch ? launch->offsets : 0;
  if (wide != 0 && wide != 1) return fail(nullptr, LBM_EINVAL, "launch->offsets must be 0 or 1");
  if (!(tol > 0.0) || max_steps < 0 || check_every < 1 || poll_every < 1)
    return fail(nullptr, LBM_EINVAL, "need tol > 0, max_steps >= 0, check_every >= 1, poll_every >= 1");
  for (int i = 0; i < count; ++i) {
    e = check_member(members[i], i);
    if (!e.empty()) return fail(nullptr, LBM_EINVAL, e);
  }
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(nullptr, LBM_ENOWS, "workspace must be non-null and 256-byte aligned");
  if (workspace_bytes < L.total) return fail(nullptr, LBM_ENOWS, "workspace too small");
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (storage) {
    case LBM_F64:
      return batch_run<double>(grid, storage, rho0, count, members, ws, L, st, tol, max_steps,
                               check_every, poll_every, wide, results);
    case LBM_F32:
      return batch_run<float>(grid, storage, rho0, count, members, ws, L, st, tol, max_steps,
                              check_every, poll_every, wide, results);
    case LBM_BF16:
      return batch_run<bf16_t>(grid, storage, rho0, count, members, ws, L, st, tol, max_steps,
                               check_every, poll_every, wide, results);
    default:
      return batch_run<_Float16>(grid, storage, rho0, count, members, ws, L, st, tol, max_steps,
                                 check_every, poll_every, wide, results);
  }
}

}  // extern "C"
