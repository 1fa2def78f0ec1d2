// Discrete adjoint of the preconditioned GLBE step, for the gradient of the
// flow rate Q = (1/nx) sum_x j_x with respect to the force field.
//
// Forward step on the stored post-collision state p:  f = S p (pull
// streaming), p' = C(f; F) (collision).  Q is taken from f = S p.  The
// adjoint is carried in the pre-collision variable mu (one 19-vector per node)
// so that one kernel pass is a gather, like the forward step:
//
//   lam(x)    = (S^T mu)(x):  lam_b(x) = mu_b(x + e_b), or mu_opp(b)(x) when the
//               link x -> x + e_b crosses a wall (the transpose of halfway
//               bounce-back), periodic wrap otherwise;
//   mu'(x)    = C_f(x)^T lam(x) + q,        q_a = e_ax / nx  (dQ/df);
//   dQ/dF(x)  = C_F(x)^T lam(x) + x_hat / (2 gamma nx),
//
// with C_f, C_F the local Jacobians of the collision at f(x) = (S p*)(x),
// recomputed from the forward state in the same pass (collide19_adjoint).
//
// Steady adjoint: iterate mu' = C_f^T S^T mu + q at the converged state.  The
// step conserves mass, so 1 is an eigenvector of C_f^T S^T with eigenvalue 1
// and C_F^T 1 = 0: the mean of mu drifts linearly without changing the
// gradient.  The mean is removed every check and convergence is measured on
// the gradient field itself.  The linearised step also has undamped period-2
// (eigenvalue -1) modes; when the adjoint source excites them the iterates
// alternate between two branches whose mean is the fixed point, so the
// gradient reported at each check is the mean of the last two iterations.
//
// Unrolled adjoint over N steps from p_0: mu_{N+1} = q; for n = N..1,
// lam_n = S^T mu_{n+1}, mu_n = C_f(f_n)^T lam_n, dQ/dF += C_F(f_n)^T lam_n with
// f_n = S p_{n-1}; forward states are recomputed segment by segment from
// checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "collide.hpp"
#include "ctx.hpp"
#include "stream.hpp"

namespace lbm {

// ---------------------------------------------------------------- kernels --
// lam_a(x) = mu_a(x + e_a), or mu_opp(a)(x) if that link crosses a wall: the
// forward pull read along -e_a, with the same pair-relative offsets.  The
// adjoint populations are used once per iteration and read with the streaming
// policy, so that they do not evict the forward state, which every iteration
// reads again (a 128^3 FP32 state stays in the last-level cache: 92-96 ->
// 78-79 us per iteration).
template <typename R, bool WIDE, int A = 0>
__device__ __forceinline__ void gather_transpose(const R* __restrict__ mu, int64_t st, uint32_t n,
                                                 const Nbr& b, R shift, R (&lam)[Q19]) {
  if constexpr (A < Q19) {
    int32_t off;
    const bool bb = pull_source<-EX19[A], -EY19[A], -EZ19[A]>(b, off);
    const R* base = mu + static_cast<int64_t>(pair_plane<A>()) * st;
    lam[A] = ld_pop<true>(elem<WIDE>(base, pull_offset<A>(bb, off, n, static_cast<uint32_t>(st)))) - shift;
    gather_transpose<R, WIDE, A + 1>(mu, st, n, b, shift, lam);
  }
}

// GRAD: 0 none; 1 accumulate into grad; 3 write half the gradient (with the
// direct term) into gpre; 2 (check) grad = half the gradient + gpre, and
// accumulate the change against the previous content of grad.  NT: streaming
// stores of the adjoint populations; NTL: streaming loads of the forward state
// and the force (lattices that stream from HBM, where no cache holds them).
template <typename R, bool CHECK, int GRAD, bool FIELD, bool WIDE, bool NT, bool NTL>
__global__ __launch_bounds__(kBlock) void adjoint_step(
    GridArgs g, CollideArgs<R> c, const R* __restrict__ state, const R* __restrict__ force,
    const R* __restrict__ mu_in, R* __restrict__ mu_out, R* __restrict__ grad,
    R* __restrict__ gpre, int64_t grad_stride, const double* __restrict__ shift, R q_scale,
    R grad_direct, double* __restrict__ partials) {
  const int lb = logical_block(g);
  if (lb >= g.nblocks) return;
  const uint32_t n = static_cast<uint32_t>(lb) * kBlock + threadIdx.x;
  double acc[kPartials] = {};
  if (n < static_cast<uint32_t>(g.N)) {
    const Nbr b = neighbours(g, n);
    R f[Q19];
    // forward pull of the state; the constant wall-momentum term of moving
    // walls drops out of the transposed streaming
    gather19<R, true, WIDE, NTL>(state, g.stride, n, b, c, f);
    const R sh = shift ? R(*shift) : R(0);
    R lam[Q19];
    gather_transpose<R, WIDE>(mu_in, g.stride, n, b, sh, lam);
    R Fx, Fy, Fz;
    if (FIELD) {
      Fx = ld_pop<NTL>(elem<WIDE>(force, n));
      Fy = ld_pop<NTL>(elem<WIDE>(force + g.stride, n));
      Fz = ld_pop<NTL>(elem<WIDE>(force + 2 * g.stride, n));
    } else {
      Fx = c.F[0];
      Fy = c.F[1];
      Fz = c.F[2];
    }
    R nu[Q19], gx, gy, gz;
    collide19_adjoint<R>(f, Fx, Fy, Fz, c, lam, nu, gx, gy, gz);
    R mu[Q19];
#pragma unroll
    for (int a = 0; a < Q19; ++a) {
      mu[a] = nu[a] + q_scale * R(EX19[a]);
      if (CHECK) acc[2] += static_cast<double>(mu[a]);
    }
    store_planes<R, NT, WIDE, Q19>(mu_out, g, n, mu);
    if constexpr (GRAD == 1) {
      *elem<WIDE>(grad, n) += gx;
      *elem<WIDE>(grad + grad_stride, n) += gy;
      *elem<WIDE>(grad + 2 * grad_stride, n) += gz;
    } else if constexpr (GRAD == 3) {
      *elem<WIDE>(gpre, n) = R(0.5) * (gx + grad_direct);
      *elem<WIDE>(gpre + grad_stride, n) = R(0.5) * gy;
      *elem<WIDE>(gpre + 2 * grad_stride, n) = R(0.5) * gz;
    } else if constexpr (GRAD == 2) {
      const R gv[3] = {R(0.5) * (gx + grad_direct) + *elem<WIDE>(gpre, n),
                       R(0.5) * gy + *elem<WIDE>(gpre + grad_stride, n),
                       R(0.5) * gz + *elem<WIDE>(gpre + 2 * grad_stride, n)};
      R* gk[3] = {elem<WIDE>(grad, n), elem<WIDE>(grad + grad_stride, n),
                  elem<WIDE>(grad + 2 * grad_stride, n)};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double d = static_cast<double>(gv[k]) - static_cast<double>(*gk[k]);
        *gk[k] = gv[k];
        acc[0] += d * d;
        acc[1] += static_cast<double>(gv[k]) * static_cast<double>(gv[k]);
      }
    }
    if (CHECK) {
      const bool fin = isfinite(static_cast<double>(gx)) && isfinite(static_cast<double>(gy)) &&
                       isfinite(static_cast<double>(gz)) && isfinite(static_cast<double>(nu[0]));
      acc[4] += fin ? 0.0 : 1.0;
    }
  }
  if constexpr (CHECK) {
    block_sum<kPartials>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < kPartials; ++k) partials[int64_t(lb) * kPartials + k] = acc[k];
    }
  }
}

// record = {change = sqrt(sum dg^2 / sum g^2), sum g^2, mean(mu), nonfinite};
// shift = mean(mu), subtracted on the next read of mu.
__global__ __launch_bounds__(kBlock) void finalize_adjoint_kernel(const double* __restrict__ partials,
                                                                  int nblocks, double inv_count,
                                                                  double* __restrict__ record,
                                                                  double* __restrict__ shift) {
  double acc[kPartials] = {};
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
    for (int k = 0; k < kPartials; ++k) acc[k] += partials[int64_t(b) * kPartials + k];
  }
  block_sum<kPartials>(acc);
  if (threadIdx.x == 0) {
    record[0] = acc[1] > 0.0 ? sqrt(acc[0] / acc[1]) : (acc[0] == 0.0 ? 0.0 : INFINITY);
    record[1] = acc[1];
    record[2] = acc[2] * inv_count;
    record[3] = acc[4];
    shift[0] = acc[2] * inv_count;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void fill_q(R* __restrict__ mu, int64_t stride, int N, R q_scale) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int a = 0; a < Q19; ++a) mu[int64_t(a) * stride + i] = q_scale * R(EX19[a]);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void fill_grad(R* __restrict__ grad, int64_t stride, int N,
                                                    R gx) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
  grad[i] = gx;
  grad[stride + i] = R(0);
  grad[2 * stride + i] = R(0);
}

__global__ void fill_f64(double* __restrict__ p, int count, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

template <typename R>
hipError_t launch_adjoint(const GridArgs& g, const CollideArgs<R>& c, const void* state,
                          const void* force, bool field, const void* mu_in, void* mu_out,
                          void* grad, void* gpre, int64_t grad_stride, int grad_mode,
                          const double* shift, R q_scale, R grad_direct, bool check, bool nt,
                          double* partials, hipStream_t st) {
  const dim3 grid(kXcd * g.blocks_per_xcd);
  const R* s = static_cast<const R*>(state);
  const R* F = static_cast<const R*>(force);
  const R* mi = static_cast<const R*>(mu_in);
  R* mo = static_cast<R*>(mu_out);
  R* gr = static_cast<R*>(grad);
  R* gp = static_cast<R*>(gpre);
  // check iterations use GRAD mode 2; the others the requested mode
  const int gm = check ? 2 : grad_mode;
  // streaming state loads only where the forward steps stream from HBM too
  const bool ntl = nt && g.nt_load;
  return with_flag(field, [&](auto FL) {
    return with_flag(wide_offsets(g, sizeof(R)), [&](auto W) {
     return with_flag(nt, [&](auto NTS) {
      return with_flag(ntl, [&](auto NTL) {
       constexpr bool fl = decltype(FL)::value, w = decltype(W)::value, ns = decltype(NTS)::value,
                      nl = decltype(NTL)::value;
       switch (gm) {
         case 2:
           adjoint_step<R, true, 2, fl, w, ns, nl><<<grid, kBlock, 0, st>>>(
               g, c, s, F, mi, mo, gr, gp, grad_stride, shift, q_scale, grad_direct, partials);
           break;
         case 3:
           adjoint_step<R, false, 3, fl, w, ns, nl><<<grid, kBlock, 0, st>>>(
               g, c, s, F, mi, mo, gr, gp, grad_stride, shift, q_scale, grad_direct, partials);
           break;
         case 1:
           adjoint_step<R, false, 1, fl, w, ns, nl><<<grid, kBlock, 0, st>>>(
               g, c, s, F, mi, mo, gr, gp, grad_stride, shift, q_scale, grad_direct, partials);
           break;
         default:
           adjoint_step<R, false, 0, fl, w, ns, nl><<<grid, kBlock, 0, st>>>(
               g, c, s, F, mi, mo, gr, gp, grad_stride, shift, q_scale, grad_direct, partials);
       }
       return hipGetLastError();
      });
     });
    });
  });
}

// ------------------------------------------------------------------ host ---
namespace {

constexpr size_t kA = 256;
size_t al(size_t v) { return (v + kA - 1) / kA * kA; }

struct AdjLayout {
  size_t mu[2] = {0, 0}, gpre = 0, partials = 0, ring = 0, shift = 0, ckpt = 0, seg = 0, total = 0;
  int64_t n_ckpt = 0, seg_len = 0;
};
constexpr int kAdjRing = 64;
constexpr int kAdjRec = 4;

AdjLayout adj_layout(const lbm_ctx* c, int mode, int64_t n_steps, int64_t ckpt_every) {
  AdjLayout L;
  const size_t cs = c->celem();
  const size_t state = 19 * size_t(c->L.stride) * cs;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off = al(off + b);
    return at;
  };
  L.mu[0] = take(state);
  L.mu[1] = take(state);
  if (mode == 0) L.gpre = take(3 * size_t(c->L.N) * cs);
  L.partials = take(size_t(c->L.nblocks) * kPartials * sizeof(double));
  L.ring = take(kAdjRing * kAdjRec * sizeof(double));
  L.shift = take(2 * sizeof(double));
  if (mode == 1) {
    L.n_ckpt = (n_steps + ckpt_every - 1) / ckpt_every;
    L.seg_len = std::min<int64_t>(ckpt_every, n_steps);
    L.ckpt = take(size_t(L.n_ckpt) * state);
    L.seg = take(size_t(L.seg_len) * state);
  }
  L.total = off;
  return L;
}

lbm_status adj_common_checks(lbm_ctx* c) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->p.mhd) return fail(c, LBM_EUNSUPPORTED, "the adjoint covers the GLBE step without mhd");
  if (c->p.lattice != LBM_D3Q19) return fail(c, LBM_EUNSUPPORTED, "the adjoint covers D3Q19 only");
  if (c->p.storage != LBM_F64 && c->p.storage != LBM_F32)
    return fail(c, LBM_EUNSUPPORTED, "the adjoint needs LBM_F64 or LBM_F32 storage");
  return LBM_OK;
}

template <typename R>
const CollideArgs<R>& cargs(const lbm_ctx* c);
template <>
const CollideArgs<double>& cargs<double>(const lbm_ctx* c) { return c->cd; }
template <>
const CollideArgs<float>& cargs<float>(const lbm_ctx* c) { return c->cf; }

template <typename R>
lbm_status steady_impl(lbm_ctx* c, char* ws, double tol, int64_t max_iter, void* dQdF,
                       int64_t* iters, double* final_change) {
  const AdjLayout L = adj_layout(c, 0, 0, 1);
  const int64_t N = c->L.N, st = c->L.stride;
  const int blocks = int((N + kBlock - 1) / kBlock);
  void* mu[2] = {ws + L.mu[0], ws + L.mu[1]};
  double* partials = reinterpret_cast<double*>(ws + L.partials);
  double* ring = reinterpret_cast<double*>(ws + L.ring);
  double* shift = reinterpret_cast<double*>(ws + L.shift);
  const R q = R(1.0 / c->grid.n[0]);
  const R direct = R(0.5 / (c->p.gamma * c->grid.n[0]));
  hipLaunchKernelGGL(fill_q<R>, dim3(blocks), dim3(kBlock), 0, c->stream, static_cast<R*>(mu[0]),
                     st, int(N), q);
  hipLaunchKernelGGL(fill_grad<R>, dim3(blocks), dim3(kBlock), 0, c->stream,
                     static_cast<R*>(dQdF), N, int(N), R(0));
  hipLaunchKernelGGL(fill_f64, dim3(1), dim3(64), 0, c->stream, shift, 2, 0.0);
  LBM_HIP(c, hipGetLastError(), "adjoint initialisation");
  // a check every P >= 2 iterations; the iteration before it stores half its gradient
  const int ce = std::max(2, c->p.check_every);
  void* gpre = ws + L.gpre;
  int cur = 0;
  int64_t checks = 0, done = 0;
  bool prev_check = false;
  double change = INFINITY;
  std::vector<double> host(kAdjRing * kAdjRec);
  while (done < max_iter) {
    const int64_t it = done + 1;
    const bool check = (it % ce) == 0;
    const bool pre = ((it + 1) % ce) == 0;
    const double* sh = prev_check ? shift : nullptr;
    LBM_HIP(c, launch_adjoint<R>(c->ga, cargs<R>(c), c->f(c->cur), c->force(), c->field(),
                                 mu[cur], mu[cur ^ 1], dQdF, gpre, N, check ? 2 : (pre ? 3 : 0),
                                 sh, q, direct, check, c->nt_store, partials, c->stream),
            "adjoint launch");
    cur ^= 1;
    done = it;
    prev_check = check;
    if (check) {
      hipLaunchKernelGGL(finalize_adjoint_kernel, dim3(1), dim3(kBlock), 0, c->stream, partials,
                         c->L.nblocks, 1.0 / double(19 * N),
                         ring + (checks % kAdjRing) * kAdjRec, shift);
      LBM_HIP(c, hipGetLastError(), "adjoint finalize");
      ++checks;
      if (checks % kAdjRing == 0 || done >= max_iter) {
        LBM_HIP(c, hipMemcpyAsync(host.data(), ring, host.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream),
                "copy");
        LBM_HIP(c, hipStreamSynchronize(c->stream), "sync");
        const int64_t first = std::max<int64_t>(0, checks - kAdjRing);
        for (int64_t k = first; k < checks; ++k) {
          const double* r = &host[(k % kAdjRing) * kAdjRec];
          if (r[3] > 0.0) return fail(c, LBM_EUNSTABLE, "non-finite adjoint values");
          change = r[0];
          if (k >= 1 && change < tol) {
            *iters = done;
            *final_change = host[((checks - 1) % kAdjRing) * kAdjRec];
            return LBM_OK;
          }
        }
      }
    }
  }
  LBM_HIP(c, hipStreamSynchronize(c->stream), "sync");
  if (checks > 0) {
    LBM_HIP(c, hipMemcpy(host.data(), ring + ((checks - 1) % kAdjRing) * kAdjRec,
                         kAdjRec * sizeof(double), hipMemcpyDeviceToHost),
            "copy");
    change = host[0];
  }
  *iters = done;
  *final_change = change;
  return LBM_OK;
}

template <typename R>
lbm_status unrolled_impl(lbm_ctx* c, char* ws, int64_t n_steps, int64_t K, void* dQdF) {
  const AdjLayout L = adj_layout(c, 1, n_steps, K);
  const int64_t N = c->L.N, st = c->L.stride;
  const size_t state_bytes = 19 * size_t(st) * sizeof(R);
  const int blocks = int((N + kBlock - 1) / kBlock);
  char* ckpt = ws + L.ckpt;
  char* seg = ws + L.seg;
  void* mu[2] = {ws + L.mu[0], ws + L.mu[1]};
  // forward march with checkpoints p_0, p_K, p_2K, ...
  for (int64_t n = 0; n < n_steps; ++n) {
    if (n % K == 0)
      LBM_HIP(c, hipMemcpyAsync(ckpt + size_t(n / K) * state_bytes, c->f(c->cur), state_bytes,
                                hipMemcpyDeviceToDevice, c->stream),
              "checkpoint copy");
    const lbm_status s = one_step(c);
    if (s != LBM_OK) return s;
  }
  const R q = R(1.0 / c->grid.n[0]);
  hipLaunchKernelGGL(fill_q<R>, dim3(blocks), dim3(kBlock), 0, c->stream, static_cast<R*>(mu[0]),
                     st, int(N), q);
  hipLaunchKernelGGL(fill_grad<R>, dim3(blocks), dim3(kBlock), 0, c->stream,
                     static_cast<R*>(dQdF), N, int(N), R(0.5 / (c->p.gamma * c->grid.n[0])));
  LBM_HIP(c, hipGetLastError(), "adjoint initialisation");
  int cur = 0;
  for (int64_t sgi = L.n_ckpt - 1; sgi >= 0; --sgi) {
    const int64_t s0 = sgi * K, e = std::min(s0 + K, n_steps), len = e - s0;
    LBM_HIP(c, hipMemcpyAsync(seg, ckpt + size_t(sgi) * state_bytes, state_bytes,
                              hipMemcpyDeviceToDevice, c->stream),
            "segment copy");
    for (int64_t i = 1; i < len; ++i)
      LBM_HIP(c, launch_glbe_step<R>(c->ga, cargs<R>(c), seg + size_t(i - 1) * state_bytes,
                                     seg + size_t(i) * state_bytes, c->force(), c->field(), false,
                                     c->nt_store, false, nullptr, nullptr, c->stream),
              "segment recompute");
    for (int64_t n = e; n >= s0 + 1; --n) {
      LBM_HIP(c, launch_adjoint<R>(c->ga, cargs<R>(c), seg + size_t(n - 1 - s0) * state_bytes,
                                   c->force(), c->field(), mu[cur], mu[cur ^ 1], dQdF, nullptr, N,
                                   1, nullptr, R(0), R(0), false, c->nt_store, nullptr, c->stream),
              "adjoint launch");
      cur ^= 1;
    }
  }
  LBM_HIP(c, hipStreamSynchronize(c->stream), "sync");
  return LBM_OK;
}

}  // namespace

template hipError_t launch_adjoint<double>(const GridArgs&, const CollideArgs<double>&, const void*,
                                           const void*, bool, const void*, void*, void*, void*,
                                           int64_t, int, const double*, double, double, bool, bool,
                                           double*, hipStream_t);
template hipError_t launch_adjoint<float>(const GridArgs&, const CollideArgs<float>&, const void*,
                                          const void*, bool, const void*, void*, void*, void*,
                                          int64_t, int, const double*, float, float, bool, bool,
                                          double*, hipStream_t);

}  // namespace lbm

using namespace lbm;

extern "C" {

lbm_status lbm_adjoint_workspace_bytes(const lbm_ctx* cc, int32_t mode, int64_t n_steps,
                                       int64_t ckpt_every, size_t* bytes) {
  lbm_ctx* c = const_cast<lbm_ctx*>(cc);
  const lbm_status s = adj_common_checks(c);
  if (s != LBM_OK) return s;
  if (!bytes) return fail(c, LBM_EINVAL, "bytes is NULL");
  if (mode != 0 && mode != 1) return fail(c, LBM_EINVAL, "mode must be 0 (steady) or 1 (unrolled)");
  if (mode == 1 && (n_steps < 1 || ckpt_every < 1))
    return fail(c, LBM_EINVAL, "unrolled adjoint needs n_steps >= 1 and ckpt_every >= 1");
  *bytes = adj_layout(c, mode, n_steps, ckpt_every).total;
  return LBM_OK;
}

lbm_status lbm_adjoint_steady(lbm_ctx* c, void* adj_ws, size_t adj_ws_bytes, double tol,
                              int64_t max_iter, void* dQdF, int64_t* iters,
                              double* final_change) {
  const lbm_status s = adj_common_checks(c);
  if (s != LBM_OK) return s;
  if (!dQdF || !iters || !final_change || !(tol > 0.0) || max_iter < 1)
    return fail(c, LBM_EINVAL, "bad arguments");
  if (!adj_ws || reinterpret_cast<uintptr_t>(adj_ws) % 256 != 0 ||
      adj_ws_bytes < adj_layout(c, 0, 0, 1).total)
    return fail(c, LBM_ENOWS, "adjoint workspace missing, misaligned or too small");
  char* ws = static_cast<char*>(adj_ws);
  if (c->p.storage == LBM_F64) return steady_impl<double>(c, ws, tol, max_iter, dQdF, iters, final_change);
  return steady_impl<float>(c, ws, tol, max_iter, dQdF, iters, final_change);
}

lbm_status lbm_adjoint_unrolled(lbm_ctx* c, void* adj_ws, size_t adj_ws_bytes, int64_t n_steps,
                                int64_t ckpt_every, void* dQdF) {
  const lbm_status s = adj_common_checks(c);
  if (s != LBM_OK) return s;
  if (!dQdF || n_steps < 1 || ckpt_every < 1) return fail(c, LBM_EINVAL, "bad arguments");
  if (!adj_ws || reinterpret_cast<uintptr_t>(adj_ws) % 256 != 0 ||
      adj_ws_bytes < adj_layout(c, 1, n_steps, ckpt_every).total)
    return fail(c, LBM_ENOWS, "adjoint workspace missing, misaligned or too small");
  char* ws = static_cast<char*>(adj_ws);
  if (c->p.storage == LBM_F64) return unrolled_impl<double>(c, ws, n_steps, ckpt_every, dQdF);
  return unrolled_impl<float>(c, ws, n_steps, ckpt_every, dQdF);
}

}  // extern "C"
