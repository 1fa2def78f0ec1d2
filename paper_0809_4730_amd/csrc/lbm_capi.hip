// Host side of the C ABI declared in include/lbm_capi.h: validation, workspace
// layout inside caller-owned device memory, the time-step loop on the
// caller's stream, and the residual history.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm_capi.h"
#include "args.hpp"
#include "ctx.hpp"
#include "stream.hpp"

using namespace lbm;

namespace {

thread_local std::string g_create_error;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_conserved(int k) { return k == 0 || k == 3 || k == 5 || k == 7; }

std::string validate(const lbm_grid* grid, const lbm_params* p) {
  if (!grid || !p) return "grid and params must be non-null";
  int64_t N = 1;
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] < 1) return "grid dimensions must be >= 1";
    if (grid->bc[a] != LBM_PERIODIC && grid->bc[a] != LBM_WALL) return "bc must be LBM_PERIODIC or LBM_WALL";
    N *= grid->n[a];
  }
  if (N >= (int64_t(1) << 31)) return "grid has 2^31 or more nodes";
  if (storage_bytes(p->storage) == 0) return "storage must be LBM_F64, LBM_F32, LBM_BF16 or LBM_F16";
  if (p->lattice != LBM_D3Q19 && p->lattice != LBM_D2Q9) return "lattice must be LBM_D3Q19 or LBM_D2Q9";
  if (!(p->gamma > 0.0 && p->gamma <= 1.0)) return "gamma must lie in (0, 1]";
  const bool d2 = p->lattice == LBM_D2Q9;
  for (int k = 0; k < (d2 ? 9 : 19); ++k)
    if (!(d2 ? (k == 0 || k == 3 || k == 5) : is_conserved(k)) && !(p->s[k] > 0.0 && p->s[k] < 2.0)) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "rate s[%d] = %g outside (0, 2)", k, p->s[k]);
      return buf;
    }
  if (!(p->rho0 > 0.0)) return "rho0 must be positive";
  if (p->force_mode != LBM_FORCE_UNIFORM && p->force_mode != LBM_FORCE_FIELD)
    return "force_mode must be LBM_FORCE_UNIFORM or LBM_FORCE_FIELD";
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->force_const[a])) return "force_const must be finite";
  if (p->mhd != 0 && p->mhd != 1) return "mhd must be 0 or 1";
  if (p->mhd) {
    if (p->storage != LBM_F64 && p->storage != LBM_F32) return "mhd needs LBM_F64 or LBM_F32 storage";
    if (!(p->gamma_m > 0.0 && p->gamma_m <= 1.0)) return "gamma_m must lie in (0, 1]";
    if (!(p->chi > 0.0)) return "chi must be positive";
    if (!(p->eta > 0.0)) return "eta must be positive";
    if (!(p->mu > 0.0)) return "mu must be positive";
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->B0[a])) return "B0 must be finite";
  }
  if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC)
    return "rounding must be LBM_ROUND_NEAREST or LBM_ROUND_STOCHASTIC";
  if (p->rounding == LBM_ROUND_STOCHASTIC &&
      ((p->storage != LBM_BF16 && p->storage != LBM_F16) || p->mhd))
    return "stochastic rounding needs LBM_BF16 or LBM_F16 storage and the flow step alone (mhd = 0)";
  if (p->launch.xcd_chunk < 0) return "launch.xcd_chunk must be >= 0";
  if (p->launch.store < 0 || p->launch.store > 2) return "launch.store must be 0, 1 or 2";
  if (p->launch.offsets != 0 && p->launch.offsets != 1) return "launch.offsets must be 0 or 1";
  if (p->launch.load < 0 || p->launch.load > 2) return "launch.load must be 0, 1 or 2";
  if (p->launch.waves != 0 && (p->launch.waves < 3 || p->launch.waves > 8))
    return "launch.waves must be 0 or 3..8";
  if (p->check_every < 1) return "check_every must be >= 1";
  if (p->history_len < 1) return "history_len must be >= 1";
  if (p->source_mode != 0 && p->source_mode != 1) return "source_mode must be 0 or 1";
  for (int f = 0; f < 6; ++f)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->wall_u[f][a])) return "wall_u must be finite";
  if (p->lattice == LBM_D2Q9) {
    if (grid->n[2] != 1) return "LBM_D2Q9 needs n[2] = 1";
    if (p->force_const[2] != 0.0 || p->B0[2] != 0.0) return "LBM_D2Q9: force_const[2] and B0[2] must be 0";
    for (int f = 0; f < 6; ++f)
      for (int a = 0; a < 3; ++a)
        if (p->wall_u[f][a] != 0.0) return "LBM_D2Q9 has no moving walls";
    for (int a = 0; a < 3; ++a)
      if (p->mag_pad[a] != 0) return "LBM_D2Q9 has no extended induction lattice";
  }
  for (int a = 0; a < 3; ++a) {
    if (p->mag_pad[a] < 0) return "mag_pad must be >= 0";
    if (p->mag_pad[a] == 0) continue;
    if (!p->mhd) return "mag_pad needs mhd = 1";
    if (grid->bc[a] != LBM_WALL) return "mag_pad only on wall axes";
    if (int64_t(grid->n[a]) - 2 * int64_t(p->mag_pad[a]) < 1)
      return "mag_pad leaves no fluid nodes";
  }
  return "";
}

Layout make_layout(const lbm_grid* grid, const lbm_params* p) {
  Layout L;
  L.N = int64_t(grid->n[0]) * grid->n[1] * grid->n[2];
  L.stride = (L.N + 63) / 64 * 64;
  L.nblocks = static_cast<int32_t>((L.N + kBlock - 1) / kBlock);
  const size_t es = storage_bytes(p->storage), cs = compute_bytes(p->storage);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const int qf = flow_planes(*p), qg = mag_planes(*p);
  L.f[0] = take(qf * L.stride * es);
  L.f[1] = take(qf * L.stride * es);
  if (p->mhd) {
    L.g[0] = take(qg * L.stride * cs);
    L.g[1] = take(qg * L.stride * cs);
  }
  if (p->force_mode == LBM_FORCE_FIELD) L.force = take(3 * L.stride * cs);
  L.usnap = take(3 * L.stride * cs);
  // per-check partial sums are kept until a batched finalize: a ring of up to
  // 16 MB (at least one slot, at most history_len slots)
  const size_t slot = size_t(L.nblocks) * kPartials * sizeof(double);
  L.pslots = int32_t(std::max<size_t>(1, std::min<size_t>(size_t(p->history_len),
                                                           (size_t(16) << 20) / slot)));
  L.partials = take(size_t(L.pslots) * slot);
  L.fpartials = take(slot);
  L.ring = take(size_t(p->history_len) * kRecordDoubles * sizeof(double));
  L.rec = take(kRecordDoubles * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

namespace lbm {

StepEvents& step_events() {
  static thread_local StepEvents ev;
  return ev;
}

std::string validate_params(const lbm_grid* grid, const lbm_params* p) { return validate(grid, p); }

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return s;
}

lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, LBM_EHIP, m);
}


hipError_t launch_step_kernel(lbm_ctx* c, bool check) {
  double* partials = c->partials() + (c->checks % c->L.pslots) * int64_t(c->L.nblocks) * kPartials;
  const void* fin = c->f(c->cur);
  void* fout = c->f(c->cur ^ 1);
  const bool fld = c->field();
  c->ga.step = static_cast<uint32_t>(c->step + 1);  // the step this launch computes
  if (c->p.lattice == LBM_D2Q9) {
    if (c->p.mhd) {
      if (c->p.storage == LBM_F64)
        return launch_mhd2_step<double>(c->ga, c->cd, c->md, fin, fout, c->g(c->cur),
                                        c->g(c->cur ^ 1), c->force(), fld, check, c->nt_store,
                                        c->usnap(), partials, c->stream);
      return launch_mhd2_step<float>(c->ga, c->cf, c->mf, fin, fout, c->g(c->cur), c->g(c->cur ^ 1),
                                     c->force(), fld, check, c->nt_store, c->usnap(), partials,
                                     c->stream);
    }
    switch (c->p.storage) {
      case LBM_F64:
        return launch_glbe2_step<double>(c->ga, c->cd, fin, fout, c->force(), fld, check,
                                         c->nt_store, false, c->usnap(), partials, c->stream);
      case LBM_F32:
        return launch_glbe2_step<float>(c->ga, c->cf, fin, fout, c->force(), fld, check,
                                        c->nt_store, false, c->usnap(), partials, c->stream);
      case LBM_BF16:
        return launch_glbe2_step<bf16_t>(c->ga, c->cf, fin, fout, c->force(), fld, check,
                                         c->nt_store, c->p.rounding == LBM_ROUND_STOCHASTIC,
                                         c->usnap(), partials, c->stream);
      default:
        return launch_glbe2_step<_Float16>(c->ga, c->cf, fin, fout, c->force(), fld, check,
                                           c->nt_store, c->p.rounding == LBM_ROUND_STOCHASTIC,
                                           c->usnap(), partials, c->stream);
    }
  }
  if (c->p.mhd) {
    if (c->p.storage == LBM_F64)
      return launch_mhd_step<double>(c->ga, c->cd, c->md, fin, fout, c->g(c->cur), c->g(c->cur ^ 1),
                                     c->force(), fld, check, c->nt_store, c->usnap(), partials,
                                     c->stream);
    return launch_mhd_step<float>(c->ga, c->cf, c->mf, fin, fout, c->g(c->cur), c->g(c->cur ^ 1),
                                  c->force(), fld, check, c->nt_store, c->usnap(), partials,
                                  c->stream);
  }
  switch (c->p.storage) {
    case LBM_F64:
      return launch_glbe_step<double>(c->ga, c->cd, fin, fout, c->force(), fld, check, c->nt_store,
                                      false, c->usnap(), partials, c->stream);
    case LBM_F32:
      return launch_glbe_step<float>(c->ga, c->cf, fin, fout, c->force(), fld, check, c->nt_store,
                                     false, c->usnap(), partials, c->stream);
    case LBM_BF16:
      return launch_glbe_step<bf16_t>(c->ga, c->cf, fin, fout, c->force(), fld, check, c->nt_store,
                                      c->p.rounding == LBM_ROUND_STOCHASTIC, c->usnap(), partials,
                                      c->stream);
    default:
      return launch_glbe_step<_Float16>(c->ga, c->cf, fin, fout, c->force(), fld, check,
                                        c->nt_store, c->p.rounding == LBM_ROUND_STOCHASTIC,
                                        c->usnap(), partials, c->stream);
  }
}

// Launch shape, from the bytes of the two population buffers (measured on
// MI355X, 3D and 2D lattices from 64^3 and 2048^2 to 256^3 and 8192^2):
//  * <= 256 MB (fits the MALL): each XCD sweeps one contiguous slab, so pulled
//    neighbour rows hit its own L2; stores stay cacheable.
//  * <= 512 MB (partly MALL-resident): slabs, streaming stores.
//  * larger (streams from HBM): streaming stores, and the chunk is timed at
//    create (tune_launch_shape) among 1, 2, 4, 8 and whole slabs.  No rule of
//    the lattice shape picked the winner: chunks of 2 beat slabs by 7% for the
//    256^3 flow step, slabs beat chunks by 22% for the 2048^2 coupled 2D step,
//    chunks of 8 lead for 16-bit storage by 2-3%, and chunks of 1, 2 and 4 lie
//    within 1-2% of each other for the 256^3 steps, which of them ahead varying
//    from box to box.
// Non-zero fields of lbm_params.launch override the choice.
void set_chunk(lbm_ctx* c, int chunk) {
  const int bpx0 = (c->L.nblocks + kXcd - 1) / kXcd;
  chunk = std::max(1, std::min(chunk, bpx0));
  c->ga.xcd_chunk = chunk;
  c->ga.div_chunk = make_fastdiv(static_cast<uint32_t>(chunk));
  c->ga.blocks_per_xcd = (bpx0 + chunk - 1) / chunk * chunk;
}

double population_bytes(const lbm_ctx* c) {
  return 2.0 * double(c->L.stride) *
         (c->qf() * double(storage_bytes(c->p.storage)) +
          (c->p.mhd ? c->qg() * double(compute_bytes(c->p.storage)) : 0.0));
}

void choose_launch_shape(lbm_ctx* c) {
  constexpr double kMallBytes = 256.0 * 1024 * 1024;
  const double pop_bytes = population_bytes(c);
  const int bpx0 = (c->L.nblocks + kXcd - 1) / kXcd;
  int chunk = pop_bytes > 2.0 * kMallBytes ? 2 : bpx0;
  c->tune_chunk = pop_bytes > 2.0 * kMallBytes;
  c->nt_store = pop_bytes > kMallBytes;
  const lbm_launch& l = c->p.launch;
  if (l.xcd_chunk > 0) {
    chunk = l.xcd_chunk;
    c->tune_chunk = false;
  }
  if (l.store != 0) c->nt_store = l.store == 2;
  // streaming loads: measured 2-4% faster for the D3Q19 steps at 256^3 and
  // 2% slower for the D2Q9 step at 4096^2
  c->ga.nt_load = pop_bytes > 2.0 * kMallBytes && c->p.lattice != LBM_D2Q9;
  if (l.load != 0) c->ga.nt_load = l.load == 2;
  // the force field, read again by every step, keeps cacheable loads when it
  // fits in the last-level cache with room to spare: the streaming population
  // traffic then leaves it there (256^3: an FP32 field of 201 MB, FP32 step
  // 439-445 -> 434-438 us, BF16 249 -> 243 us); an FP64 field of 403 MB does
  // not fit, and cacheable loads of it measured 4% slower
  const double force_bytes =
      c->field() ? 3.0 * double(c->L.stride) * double(compute_bytes(c->p.storage)) : 0.0;
  c->ga.force_cached = force_bytes <= 0.8 * kMallBytes;
  // without a force field to keep, the rest population's plane in both
  // population buffers (read at the node itself, written there) takes its
  // place: read back from the cache one step later and overwritten the step
  // after, it spares HBM both its read and its write (coupled FP32 step at
  // 256^3, uniform force: 927-937 -> 907-918 us; with the FP32 flow step's
  // force field kept as well the cache overflows: 437 -> 461 us)
  const double rest_bytes = 2.0 * double(c->L.stride) * double(storage_bytes(c->p.storage));
  c->ga.rest_cached = !c->field() && rest_bytes <= 0.8 * kMallBytes;
  // waves per SIMD: fewer waves in flight stream faster from HBM (measured at
  // 256^3: FP32 flow 466 -> 446 us at 5 waves, 16-bit storage 254 -> 249 us at
  // 6; the FP64 flow step, 4 waves by its registers, 963 -> 933 us at 3, and
  // the coupled step, 5 by its registers, 967 -> 949 us at 3; D2Q9 at 4096^2:
  // FP32 207 -> 200 us at 6, FP64 456 -> 423 us at 4, the coupled D2Q9 + D2Q5
  // step 454 -> 434 us at 5, while 16-bit storage runs slower under any cap)
  c->waves = 8;
  if (pop_bytes > 2.0 * kMallBytes) {
    if (c->p.lattice != LBM_D2Q9)
      c->waves = (c->p.storage == LBM_F64 || c->p.mhd) ? 3 : c->p.storage == LBM_F32 ? 5 : 6;
    else if (c->p.storage == LBM_F32)
      c->waves = c->p.mhd ? 5 : 6;
    else if (c->p.storage == LBM_F64 && !c->p.mhd)
      c->waves = 4;
  }
  if (l.waves != 0) c->waves = l.waves;
  c->ga.lds_reserve = 0;
  if (c->waves < 8) {
    // the largest multiple of 512 B below an equal share of the CU's LDS, less
    // 512 B for the kernels' own static LDS
    c->ga.lds_reserve = (kLdsPerCu / uint32_t(c->waves)) / 512u * 512u - 512u;
  }
  c->ga.wide = l.offsets;
  set_chunk(c, chunk);
}

// Turn every pending check's partial sums into history records (one batched
// launch; records are written in check order).
lbm_status flush_checks(lbm_ctx* c) {
  const int64_t count = c->checks - c->finalized;
  if (count <= 0) return LBM_OK;
  const double step0 = double(c->first_check_step + c->finalized * c->p.check_every);
  // the reductions' partials region (nblocks x 5 doubles) is the first pass's
  // scratch: lbm_reductions uses it only between its own two stream-ordered launches
  LBM_HIP(c, launch_finalize_split(c->partials(), c->L.nblocks, c->L.pslots, c->finalized,
                                   int(count), step0, double(c->p.check_every),
                                   1.0 / (c->grid.n[0] - 2 * c->p.mag_pad[0]), c->ring(),
                                   c->p.history_len, c->fpartials(),
                                   int64_t(c->L.nblocks) * kPartials, c->stream),
          "finalize launch");
  c->finalized = c->checks;
  return LBM_OK;
}

// Reset the residual bookkeeping after (re)initialising the state at `step`.
void reset_checks(lbm_ctx* c, int64_t step) {
  c->step = step;
  c->checks = 0;
  c->finalized = 0;
  c->first_check_step = (step / c->p.check_every + 1) * c->p.check_every;
}

// Enqueue one step (its partial sums kept for a later batched finalize).
// Timed steps: `stop` rides on the step kernel's own dispatch (its end
// timestamp), and `start` too when *with_start is set on entry or this step
// first enqueued the reduction of pending checks; *with_start tells the caller
// which on return.
lbm_status one_step(lbm_ctx* c, hipEvent_t start, hipEvent_t stop, bool* with_start) {
  const int64_t next = c->step + 1;
  const bool check = (next % c->p.check_every) == 0;
  bool flushed = false;
  if (check && c->checks - c->finalized >= c->L.pslots) {
    const lbm_status s = flush_checks(c);
    if (s != LBM_OK) return s;
    flushed = true;
  }
  const bool attach_start = start && (!with_start || *with_start || flushed);
  step_events() = StepEvents{attach_start ? start : nullptr, stop};
  const hipError_t le = launch_step_kernel(c, check);
  const bool taken = step_events().start == nullptr && step_events().stop == nullptr;
  step_events() = StepEvents{};
  LBM_HIP(c, le, "step kernel launch");
  if (!taken) return fail(c, LBM_ESTATE, "step kernel launched without its timing events");
  if (with_start) *with_start = attach_start;
  c->cur ^= 1;
  c->step = next;
  if (check) ++c->checks;
  return LBM_OK;
}

template <typename S>
hipError_t fields_dispatch(lbm_ctx* c, int out_dtype, void* rho, void* u, void* B) {
  using R = typename Storage<S>::R;
  const CollideArgs<R>* ca;
  const MagArgs<R>* ma;
  if constexpr (sizeof(R) == 8) {
    ca = &c->cd;
    ma = &c->md;
  } else {
    ca = &c->cf;
    ma = &c->mf;
  }
  if (c->p.lattice == LBM_D2Q9)
    return launch_fields2<S>(c->ga, *ca, *ma, c->p.mhd != 0, c->f(c->cur), c->g(c->cur), c->force(),
                             c->field(), out_dtype, rho, u, B, c->L.N, c->fpartials(), c->stream);
  return launch_fields<S>(c->ga, *ca, *ma, c->p.mhd != 0, c->f(c->cur), c->g(c->cur), c->force(),
                          c->field(), out_dtype, rho, u, B, c->L.N, c->fpartials(), c->stream);
}

hipError_t launch_fields_any(lbm_ctx* c, int out_dtype, void* rho, void* u, void* B) {
  switch (c->p.storage) {
    case LBM_F64: return fields_dispatch<double>(c, out_dtype, rho, u, B);
    case LBM_F32: return fields_dispatch<float>(c, out_dtype, rho, u, B);
    case LBM_BF16: return fields_dispatch<bf16_t>(c, out_dtype, rho, u, B);
    default: return fields_dispatch<_Float16>(c, out_dtype, rho, u, B);
  }
}

hipError_t zero_storage(lbm_ctx* c, void* p, int64_t count) {
  switch (c->p.storage) {
    case LBM_F64: return launch_fill_zero<double>(p, count, c->stream);
    case LBM_F32: return launch_fill_zero<float>(p, count, c->stream);
    case LBM_BF16: return launch_fill_zero<bf16_t>(p, count, c->stream);
    default: return launch_fill_zero<_Float16>(p, count, c->stream);
  }
}

// The rest state: both population buffers (and both magnetic ones) zero, as
// deviations from w rho0 and W B0.
hipError_t zero_populations(lbm_ctx* c) {
  hipError_t e = zero_storage(c, c->f(0), int64_t(c->qf()) * c->L.stride);
  if (e == hipSuccess) e = zero_storage(c, c->f(1), int64_t(c->qf()) * c->L.stride);
  if (e == hipSuccess && c->p.mhd) {
    const size_t cs = compute_bytes(c->p.storage);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
      e = (cs == 8) ? launch_fill_zero<double>(c->g(i), int64_t(c->qg()) * c->L.stride, c->stream)
                    : launch_fill_zero<float>(c->g(i), int64_t(c->qg()) * c->L.stride, c->stream);
  }
  return e;
}

// Times the plain step for each chunk candidate and keeps the fastest (two
// rounds, about 2 ms of launches per candidate and round, best of the two).
// The timed steps alternate buffers as a march does (a step that rereads one
// buffer finds it in the MALL and favours other shapes); the rest state is
// restored afterwards.  The chunk only decides which workgroup updates which
// nodes, so results do not depend on it.
hipError_t tune_launch_shape(lbm_ctx* c) {
  if (!c->tune_chunk) return hipSuccess;
  const int bpx0 = (c->L.nblocks + kXcd - 1) / kXcd;
  constexpr int kCand = 5;
  const int cand[kCand] = {1, 2, 4, 8, bpx0};
  // launches per timing: ~2 ms at ~5.5 TB/s (each step moves the population bytes)
  const int reps =
      static_cast<int>(std::max(4.0, std::min(32.0, 2e-3 * 5.5e12 / population_bytes(c))));
  hipEvent_t ev[2];
  hipError_t e = hipEventCreate(&ev[0]);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return e;
  }
  float best_ms[kCand] = {};
  for (int r = 0; r < 2 && e == hipSuccess; ++r) {
    for (int i = 0; i < kCand && e == hipSuccess; ++i) {
      set_chunk(c, cand[i]);
      e = launch_step_kernel(c, false);  // warm-up
      c->cur ^= 1;
      if (e == hipSuccess) e = hipEventRecord(ev[0], c->stream);
      for (int k = 0; k < reps && e == hipSuccess; ++k) {
        e = launch_step_kernel(c, false);
        c->cur ^= 1;
      }
      if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (e == hipSuccess) best_ms[i] = (r == 0) ? ms : std::min(best_ms[i], ms);
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  int best = 0;
  if (e == hipSuccess)
    for (int i = 1; i < kCand; ++i)
      if (best_ms[i] < best_ms[best]) best = i;
  set_chunk(c, cand[best]);
  c->cur = 0;
  if (e == hipSuccess) e = zero_populations(c);
  return e;
}

lbm_status copy_force_in(lbm_ctx* c, const void* force) {
  const size_t cs = c->celem();
  LBM_HIP(c, hipMemcpy2DAsync(c->force(), c->L.stride * cs, force, c->L.N * cs, c->L.N * cs, 3,
                              hipMemcpyDeviceToDevice, c->stream),
          "force copy");
  return LBM_OK;
}

lbm_status read_records(lbm_ctx* c, int64_t first, int64_t count, std::vector<double>& out) {
  // records first .. first+count-1 (global indices), all still inside the ring
  const lbm_status fs = flush_checks(c);
  if (fs != LBM_OK) return fs;
  out.assign(size_t(count) * kRecordDoubles, 0.0);
  if (count <= 0) return LBM_OK;
  // the records occupy at most two contiguous ranges of the ring
  const int64_t len = c->p.history_len;
  const int64_t slot0 = first % len;
  const int64_t n1 = std::min(count, len - slot0);
  const size_t rec = kRecordDoubles * sizeof(double);
  // through the pinned staging buffer when the records fit in it
  double* dst = (c->host_rec && count <= lbm_ctx::kHostRecs) ? c->host_rec : out.data();
  LBM_HIP(c, hipMemcpyAsync(dst, c->ring() + slot0 * kRecordDoubles, size_t(n1) * rec,
                            hipMemcpyDeviceToHost, c->stream),
          "history copy");
  if (count > n1)
    LBM_HIP(c, hipMemcpyAsync(dst + n1 * kRecordDoubles, c->ring(), size_t(count - n1) * rec,
                              hipMemcpyDeviceToHost, c->stream),
            "history copy");
  LBM_HIP(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (dst != out.data()) std::copy(dst, dst + count * kRecordDoubles, out.begin());
  return LBM_OK;
}

}  // namespace lbm

extern "C" {

lbm_status lbm_default_rates(double nu, double gamma, int32_t mode, double Lambda, double s_out[19]) {
  if (!s_out) return fail(nullptr, LBM_EINVAL, "s_out is NULL");
  if (!(nu > 0.0)) return fail(nullptr, LBM_EINVAL, "nu must be positive");
  if (!(gamma > 0.0 && gamma <= 1.0)) return fail(nullptr, LBM_EINVAL, "gamma must lie in (0, 1]");
  if (mode != 0 && mode != 1) return fail(nullptr, LBM_EINVAL, "mode must be 0 or 1");
  if (mode == 1 && !(Lambda > 0.0)) return fail(nullptr, LBM_EINVAL, "Lambda must be positive");
  for (int k = 0; k < 19; ++k) s_out[k] = 1.0;
  const double s_nu = 1.0 / (3.0 * nu / gamma + 0.5);
  for (int k : {9, 11, 13, 14, 15}) s_out[k] = s_nu;
  s_out[1] = 1.19;
  for (int k : {2, 10, 12}) s_out[k] = 1.4;
  if (mode == 0) {
    for (int k : {4, 6, 8}) s_out[k] = 1.2;
    for (int k : {16, 17, 18}) s_out[k] = 1.98;
  } else {
    const double s_q = 1.0 / (Lambda * gamma / (3.0 * nu) + 0.5);
    for (int k : {4, 6, 8, 16, 17, 18}) s_out[k] = s_q;
  }
  return LBM_OK;
}

lbm_status lbm_default_rates_d2q9(double nu, double gamma, int32_t mode, double Lambda,
                                  double s_out[9]) {
  if (!s_out) return fail(nullptr, LBM_EINVAL, "s_out is NULL");
  if (!(nu > 0.0)) return fail(nullptr, LBM_EINVAL, "nu must be positive");
  if (!(gamma > 0.0 && gamma <= 1.0)) return fail(nullptr, LBM_EINVAL, "gamma must lie in (0, 1]");
  if (mode != 0 && mode != 1) return fail(nullptr, LBM_EINVAL, "mode must be 0 or 1");
  if (mode == 1 && !(Lambda > 0.0)) return fail(nullptr, LBM_EINVAL, "Lambda must be positive");
  for (int k = 0; k < 9; ++k) s_out[k] = 1.0;
  s_out[7] = s_out[8] = 1.0 / (3.0 * nu / gamma + 0.5);
  s_out[1] = 1.63;
  s_out[2] = 1.14;
  s_out[4] = s_out[6] = mode == 0 ? 1.92 : 1.0 / (Lambda * gamma / (3.0 * nu) + 0.5);
  return LBM_OK;
}

lbm_status lbm_lattice_velocities(int32_t q, int32_t* e_out) {
  if (!e_out) return fail(nullptr, LBM_EINVAL, "e_out is NULL");
  if (q == 19) {
    for (int a = 0; a < 19; ++a) {
      e_out[3 * a] = EX19[a];
      e_out[3 * a + 1] = EY19[a];
      e_out[3 * a + 2] = EZ19[a];
    }
    return LBM_OK;
  }
  if (q == 7) {
    for (int a = 0; a < 7; ++a) {
      e_out[3 * a] = EX7[a];
      e_out[3 * a + 1] = EY7[a];
      e_out[3 * a + 2] = EZ7[a];
    }
    return LBM_OK;
  }
  if (q == 9 || q == 5) {
    for (int a = 0; a < q; ++a) {
      e_out[3 * a] = q == 9 ? EX9[a] : EX5[a];
      e_out[3 * a + 1] = q == 9 ? EY9[a] : EY5[a];
      e_out[3 * a + 2] = 0;
    }
    return LBM_OK;
  }
  return fail(nullptr, LBM_EINVAL, "q must be 19, 7, 9 or 5");
}

lbm_status lbm_workspace_bytes(const lbm_grid* grid, const lbm_params* params, size_t* bytes) {
  if (!bytes) return fail(nullptr, LBM_EINVAL, "bytes is NULL");
  const std::string v = validate(grid, params);
  if (!v.empty()) return fail(nullptr, LBM_EINVAL, v);
  *bytes = make_layout(grid, params).total;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_grid* grid, const lbm_params* params, const void* force,
                      void* workspace, size_t workspace_bytes, void* hip_stream, lbm_ctx** out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  const std::string v = validate(grid, params);
  if (!v.empty()) return fail(nullptr, LBM_EINVAL, v);
  if (params->force_mode == LBM_FORCE_FIELD && !force)
    return fail(nullptr, LBM_EINVAL, "force_mode = FIELD needs a force pointer");
  const Layout L = make_layout(grid, params);
  if (!workspace) return fail(nullptr, LBM_ENOWS, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(nullptr, LBM_ENOWS, "workspace must be 256-byte aligned");
  if (workspace_bytes < L.total) return fail(nullptr, LBM_ENOWS, "workspace too small");

  lbm_ctx* c = new lbm_ctx();
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_rec),
                    size_t(lbm_ctx::kHostRecs) * kRecordDoubles * sizeof(double),
                    hipHostMallocDefault) != hipSuccess) {
    c->host_rec = nullptr;
    (void)hipGetLastError();  // reads fall back to pageable memory
  }
  c->grid = *grid;
  c->p = *params;
  c->L = L;
  c->ws = static_cast<char*>(workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);
  GridArgs& g = c->ga;
  g.nx = grid->n[0];
  g.ny = grid->n[1];
  g.nz = grid->n[2];
  g.wall_x = grid->bc[0] == LBM_WALL;
  g.wall_y = grid->bc[1] == LBM_WALL;
  g.wall_z = grid->bc[2] == LBM_WALL;
  g.N = static_cast<int32_t>(L.N);
  g.nblocks = L.nblocks;
  g.step = 0;
  g.seed = params->seed;
  choose_launch_shape(c);
  g.stride = L.stride;
  g.div_nx = make_fastdiv(static_cast<uint32_t>(g.nx));
  g.div_nxny = make_fastdiv(static_cast<uint32_t>(g.nx * g.ny));
  for (int a = 0; a < 3; ++a) {
    g.flo[a] = params->mag_pad[a];
    g.fhi[a] = grid->n[a] - params->mag_pad[a];
  }
  c->cd = collide_args<double>(c->p);
  c->cf = collide_args<float>(c->p);
  c->md = mag_args<double>(c->p);
  c->mf = mag_args<float>(c->p);

  hipError_t e = zero_populations(c);
  if (e == hipSuccess)
    e = (compute_bytes(params->storage) == 8)
            ? launch_fill_zero<double>(c->usnap(), 3 * L.stride, c->stream)
            : launch_fill_zero<float>(c->usnap(), 3 * L.stride, c->stream);
  reset_checks(c, 0);
  if (e == hipSuccess) e = launch_fill_zero<double>(c->ring(), int64_t(params->history_len) * kRecordDoubles, c->stream);
  if (e != hipSuccess) {
    g_create_error = std::string("initialisation: ") + hipGetErrorString(e);
    delete c;
    return LBM_EHIP;
  }
  if (c->field()) {
    if (copy_force_in(c, force) != LBM_OK) {
      g_create_error = c->err;
      delete c;
      return LBM_EHIP;
    }
  }
  e = tune_launch_shape(c);
  if (e != hipSuccess) {
    g_create_error = std::string("launch-shape timing: ") + hipGetErrorString(e);
    delete c;
    return LBM_EHIP;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_ctx* c, lbm_launch* out) {
  if (!c || !out) return fail(nullptr, LBM_EINVAL, "NULL argument");
  out->xcd_chunk = c->ga.xcd_chunk;
  out->store = c->nt_store ? 2 : 1;
  out->load = (c->nt_store && c->ga.nt_load && c->p.lattice != LBM_D2Q9) ? 2 : 1;
  out->waves = c->waves;
  out->offsets = wide_offsets(c->ga, c->celem()) ? 1 : 0;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return;
  for (hipEvent_t ev : ctx->events) (void)hipEventDestroy(ev);
  delete ctx;
}

lbm_status lbm_set_force(lbm_ctx* c, const void* force) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!c->field()) return fail(c, LBM_ESTATE, "context was created with a uniform force");
  if (!force) return fail(c, LBM_EINVAL, "force is NULL");
  return copy_force_in(c, force);
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
  for (int64_t i = 0; i < n; ++i) {
    const lbm_status s = one_step(c);
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

}  // extern "C"

namespace {

// n steps on the context's stream, each step kernel's dispatch carrying a stop
// event (its end timestamp).  Step i's duration runs from the previous step
// kernel's end to its own: the kernel plus the dispatch gap before it, which
// is what a march pays.  The first step of each chunk of kPool (after a host
// synchronization) and a step that first enqueues the reduction of pending
// checks carry a start event as well and are timed from it.  Start events on
// every dispatch would add a marker packet, several microseconds, per step.
// The pending residual checks are reduced before the call returns.  each[i]
// (if non-null) receives step i's duration in us.
lbm_status step_with_events(lbm_ctx* c, int64_t n, double* each, double* mean_kernel_us,
                            double* wall_ms) {
  constexpr int kPool = 512;
  while (c->events.size() < 2 * kPool + 2) {
    hipEvent_t ev;
    LBM_HIP(c, hipEventCreate(&ev), "hipEventCreate");
    c->events.push_back(ev);
  }
  hipEvent_t wall0 = c->events[2 * kPool], wall1 = c->events[2 * kPool + 1];
  double total_ms = 0.0;
  LBM_HIP(c, hipEventRecord(wall0, c->stream), "hipEventRecord");
  int64_t done = 0;
  while (done < n) {
    const int64_t chunk = std::min<int64_t>(kPool, n - done);
    bool started[kPool];
    for (int64_t i = 0; i < chunk; ++i) {
      started[i] = (i == 0);
      const lbm_status s = one_step(c, c->events[2 * i], c->events[2 * i + 1], &started[i]);
      if (s != LBM_OK) return s;
    }
    if (done + chunk == n) {
      // the pending residual checks reduced behind the last step on the GPU
      // (the records do not depend on when), so that reading the history
      // after the call waits for nothing but the copy
      const lbm_status s = flush_checks(c);
      if (s != LBM_OK) return s;
    }
    // a marker after the chunk (after the whole call for the last one): the
    // step events are kernel timestamps
    LBM_HIP(c, hipEventRecord(wall1, c->stream), "hipEventRecord");
    LBM_HIP(c, hipEventSynchronize(wall1), "hipEventSynchronize");
    for (int64_t i = 0; i < chunk; ++i) {
      float ms = 0.0f;
      const hipEvent_t from = started[i] ? c->events[2 * i] : c->events[2 * i - 1];
      LBM_HIP(c, hipEventElapsedTime(&ms, from, c->events[2 * i + 1]), "hipEventElapsedTime");
      total_ms += ms;
      if (each) each[done + i] = 1000.0 * double(ms);
    }
    done += chunk;
  }
  float wms = 0.0f;
  LBM_HIP(c, hipEventElapsedTime(&wms, wall0, wall1), "hipEventElapsedTime");
  *mean_kernel_us = 1000.0 * total_ms / double(n);
  *wall_ms = wms;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_step_timed(lbm_ctx* c, int64_t n, double* mean_kernel_us, double* wall_ms) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (n < 1 || !mean_kernel_us || !wall_ms) return fail(c, LBM_EINVAL, "need n >= 1 and outputs");
  return step_with_events(c, n, nullptr, mean_kernel_us, wall_ms);
}

lbm_status lbm_step_times(lbm_ctx* c, int64_t n, double* kernel_us, double* wall_ms) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (n < 1 || !kernel_us || !wall_ms) return fail(c, LBM_EINVAL, "need n >= 1 and outputs");
  double mean = 0.0;
  return step_with_events(c, n, kernel_us, &mean, wall_ms);
}

lbm_status lbm_residual(lbm_ctx* c, double* residual, int64_t* at_step) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->checks == 0) return fail(c, LBM_ESTATE, "no residual check has run yet");
  std::vector<double> r;
  const lbm_status s = read_records(c, c->checks - 1, 1, r);
  if (s != LBM_OK) return s;
  if (residual) *residual = r[1];
  if (at_step) *at_step = static_cast<int64_t>(r[0]);
  if (r[6] > 0.0) return fail(c, LBM_EUNSTABLE, "non-finite values at the last check");
  return LBM_OK;
}

lbm_status lbm_history(lbm_ctx* c, lbm_record* out, int64_t max_records, int64_t* n_out) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!out || !n_out || max_records < 0) return fail(c, LBM_EINVAL, "bad output arguments");
  const int64_t avail = std::min<int64_t>(c->checks, c->p.history_len);
  const int64_t cnt = std::min(avail, max_records);
  std::vector<double> r;
  const lbm_status s = read_records(c, c->checks - cnt, cnt, r);
  if (s != LBM_OK) return s;
  std::memcpy(out, r.data(), size_t(cnt) * sizeof(lbm_record));
  *n_out = cnt;
  return LBM_OK;
}

lbm_status lbm_run_to_residual(lbm_ctx* c, double tol, int64_t max_steps, int64_t poll_every,
                               int64_t* steps_to_tol, double* final_residual) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!(tol > 0.0) || max_steps < 0 || poll_every < 1 || !steps_to_tol || !final_residual)
    return fail(c, LBM_EINVAL, "bad arguments");
  const int64_t ce = c->p.check_every;
  const int64_t cap = int64_t(c->p.history_len) * ce;
  int64_t chunk = std::max<int64_t>(ce, poll_every / ce * ce);
  chunk = std::min(chunk, cap);
  *steps_to_tol = -1;
  *final_residual = NAN;
  double rmin = INFINITY;
  int64_t taken = 0;
  std::vector<double> r;
  while (taken < max_steps) {
    const int64_t todo = std::min(chunk, max_steps - taken);
    const int64_t first = c->checks;
    lbm_status s = lbm_step(c, todo);
    if (s != LBM_OK) return s;
    taken += todo;
    const int64_t cnt = c->checks - first;
    if (cnt == 0) continue;
    s = read_records(c, first, cnt, r);
    if (s != LBM_OK) return s;
    for (int64_t i = 0; i < cnt; ++i) {
      const double* rec = &r[size_t(i) * kRecordDoubles];
      *final_residual = rec[1];
      if (rec[6] > 0.0 || std::isnan(rec[1]))
        return fail(c, LBM_EUNSTABLE, "non-finite values during the march");
      if (first + i >= 1) {  // the first record compares against zero velocity
        rmin = std::min(rmin, rec[1]);
        if (rec[1] > 1e-2 && rec[1] > 1e3 * rmin)
          return fail(c, LBM_EUNSTABLE, "residual grew 1e3-fold over its minimum");
      }
      if (first + i >= 1 && rec[1] < tol) {
        *steps_to_tol = static_cast<int64_t>(rec[0]);
        return LBM_OK;
      }
    }
  }
  return LBM_OK;
}

lbm_status lbm_run_to_energy_change(lbm_ctx* c, double tol, int64_t max_steps, int64_t window,
                                    int64_t* step_out, double* change_out) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  const int64_t ce = c->p.check_every;
  if (!(tol > 0.0) || max_steps < 0 || !step_out || !change_out)
    return fail(c, LBM_EINVAL, "bad arguments");
  if (window < ce || window % ce != 0)
    return fail(c, LBM_EINVAL, "window must be a positive multiple of check_every");
  *step_out = -1;
  *change_out = NAN;
  std::vector<double> r;
  double e0 = 0.0;
  bool have = false;
  for (int64_t taken = 0; taken < max_steps; taken += window) {
    lbm_status s = lbm_step(c, window);
    if (s != LBM_OK) return s;
    s = read_records(c, c->checks - 1, 1, r);  // the window's last record
    if (s != LBM_OK) return s;
    if (r[6] > 0.0 || !std::isfinite(r[3]))
      return fail(c, LBM_EUNSTABLE, "non-finite values during the march");
    const double e1 = r[3];
    if (have) {
      *change_out = std::fabs(e1 - e0) / std::max(std::fabs(e1), 1e-300);
      if (*change_out < tol) {
        *step_out = static_cast<int64_t>(r[0]);
        return LBM_OK;
      }
    }
    e0 = e1;
    have = true;
  }
  return LBM_OK;
}

lbm_status lbm_reductions(lbm_ctx* c, double* mass_drift, double* flow_rate) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!mass_drift || !flow_rate) return fail(c, LBM_EINVAL, "outputs are NULL");
  LBM_HIP(c, launch_fields_any(c, 0, nullptr, nullptr, nullptr), "fields launch");
  LBM_HIP(c, launch_finalize(c->fpartials(), c->L.nblocks, 1, 0, 1, double(c->step), 0.0,
                             1.0 / (c->grid.n[0] - 2 * c->p.mag_pad[0]), c->rec(), 1, c->stream),
          "finalize launch");
  double rec[kRecordDoubles];
  LBM_HIP(c, hipMemcpyAsync(rec, c->rec(), sizeof rec, hipMemcpyDeviceToHost, c->stream), "copy");
  LBM_HIP(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  *mass_drift = rec[4];
  *flow_rate = rec[5];
  return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, int32_t out_dtype, void* rho, void* u, void* B) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (out_dtype != LBM_F64 && out_dtype != LBM_F32) return fail(c, LBM_EINVAL, "out_dtype must be F64 or F32");
  if (B && !c->p.mhd) return fail(c, LBM_EINVAL, "B requested without mhd");
  LBM_HIP(c, launch_fields_any(c, out_dtype == LBM_F64 ? 0 : 1, rho, u, B), "fields launch");
  return LBM_OK;
}

lbm_status lbm_state_bytes(const lbm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(nullptr, LBM_EINVAL, "NULL argument");
  *bytes = c->qf() * c->L.N * c->elem() + (c->p.mhd ? c->qg() * c->L.N * c->celem() : 0);
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, void* dst) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!dst) return fail(c, LBM_EINVAL, "dst is NULL");
  const size_t es = c->elem(), N = size_t(c->L.N), st = size_t(c->L.stride);
  LBM_HIP(c, hipMemcpy2DAsync(dst, N * es, c->f(c->cur), st * es, N * es, c->qf(), hipMemcpyDeviceToDevice,
                              c->stream),
          "state copy");
  if (c->p.mhd) {
    const size_t cs = c->celem();
    char* gdst = static_cast<char*>(dst) + c->qf() * N * es;
    LBM_HIP(c, hipMemcpy2DAsync(gdst, N * cs, c->g(c->cur), st * cs, N * cs, c->qg(),
                                hipMemcpyDeviceToDevice, c->stream),
            "state copy");
  }
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx* c, const void* src, int64_t step) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!src || step < 0) return fail(c, LBM_EINVAL, "src is NULL or step < 0");
  const size_t es = c->elem(), N = size_t(c->L.N), st = size_t(c->L.stride);
  LBM_HIP(c, hipMemcpy2DAsync(c->f(c->cur), st * es, src, N * es, N * es, c->qf(), hipMemcpyDeviceToDevice,
                              c->stream),
          "state copy");
  // With an extended induction lattice the step never writes f outside the
  // fluid box: give both buffers the same values there.
  if (c->p.mag_pad[0] || c->p.mag_pad[1] || c->p.mag_pad[2])
    LBM_HIP(c, hipMemcpy2DAsync(c->f(1 - c->cur), st * es, src, N * es, N * es, c->qf(),
                                hipMemcpyDeviceToDevice, c->stream),
            "state copy");
  if (c->p.mhd) {
    const size_t cs = c->celem();
    const char* gsrc = static_cast<const char*>(src) + c->qf() * N * es;
    LBM_HIP(c, hipMemcpy2DAsync(c->g(c->cur), st * cs, gsrc, N * cs, N * cs, c->qg(),
                                hipMemcpyDeviceToDevice, c->stream),
            "state copy");
  }
  LBM_HIP(c, (c->celem() == 8) ? launch_fill_zero<double>(c->usnap(), 3 * c->L.stride, c->stream)
                                : launch_fill_zero<float>(c->usnap(), 3 * c->L.stride, c->stream),
          "fill");
  reset_checks(c, step);
  return LBM_OK;
}

lbm_status lbm_convert_state(lbm_ctx* d, const lbm_ctx* s) {
  if (!d || !s) return fail(d, LBM_EINVAL, "ctx is NULL");
  for (int a = 0; a < 3; ++a)
    if (d->grid.n[a] != s->grid.n[a] || d->grid.bc[a] != s->grid.bc[a] ||
        d->p.mag_pad[a] != s->p.mag_pad[a])
      return fail(d, LBM_EINVAL, "contexts differ in grid, boundaries or mag_pad");
  if (d->p.lattice != s->p.lattice || d->p.mhd != s->p.mhd || d->p.rho0 != s->p.rho0)
    return fail(d, LBM_EINVAL, "contexts differ in lattice, mhd or rho0");
  if (d->p.mhd)
    for (int a = 0; a < 3; ++a)
      if (d->p.B0[a] != s->p.B0[a]) return fail(d, LBM_EINVAL, "contexts differ in B0");
  // dst's stream waits for the work already enqueued on src's stream
  if (s->stream != d->stream) {
    hipEvent_t ev;
    LBM_HIP(d, hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hipError_t e = hipEventRecord(ev, s->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(d->stream, ev, 0);
    const hipError_t e2 = hipEventDestroy(ev);
    LBM_HIP(d, e, "stream ordering");
    LBM_HIP(d, e2, "hipEventDestroy");
  }
  const int64_t st = d->L.stride, N = d->L.N;
  LBM_HIP(d, launch_convert(s->p.storage, d->p.storage, s->f(s->cur), d->f(d->cur), st, N, d->qf(),
                            d->stream),
          "convert launch");
  // with an extended induction lattice f outside the fluid box lives in both buffers
  if (d->p.mag_pad[0] || d->p.mag_pad[1] || d->p.mag_pad[2])
    LBM_HIP(d, launch_convert(s->p.storage, d->p.storage, s->f(s->cur), d->f(d->cur ^ 1), st, N,
                              d->qf(), d->stream),
            "convert launch");
  if (d->p.mhd) {
    const int cs_s = s->celem() == 8 ? LBM_F64 : LBM_F32, cs_d = d->celem() == 8 ? LBM_F64 : LBM_F32;
    LBM_HIP(d, launch_convert(cs_s, cs_d, s->g(s->cur), d->g(d->cur), st, N, d->qg(), d->stream),
            "convert launch");
  }
  LBM_HIP(d, (d->celem() == 8) ? launch_fill_zero<double>(d->usnap(), 3 * st, d->stream)
                               : launch_fill_zero<float>(d->usnap(), 3 * st, d->stream),
          "fill");
  reset_checks(d, s->step);
  return LBM_OK;
}

lbm_status lbm_get_step(const lbm_ctx* c, int64_t* step) {
  if (!c || !step) return fail(nullptr, LBM_EINVAL, "NULL argument");
  *step = c->step;
  return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
