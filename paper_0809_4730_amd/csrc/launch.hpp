// Host-side launchers of the gfx950 kernels (defined in kernels.hip and
// adjoint.hip); used by the C-ABI layer.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lbm {

// Start and stop events for the next step-kernel launch on this thread.  The
// timed step sets them (the start one only where the previous stream work was
// not a step kernel: a start event costs a marker packet before the dispatch,
// several microseconds per launch); launch_step attaches them to the kernel's
// own dispatch (hipExtLaunchKernelGGL) and consumes them.  Both null: an
// ordinary launch.
struct StepEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
StepEvents& step_events();

// Launch of a step kernel (kBlock threads per workgroup, `lds` bytes of
// dynamic LDS reserved): with this thread's step events attached when the
// timed step has set them, else an ordinary launch (the form that HIP graph
// capture records).  Errors are read by the caller's hipGetLastError.
template <typename F, typename... Args>
inline void launch_step(F kernel, dim3 grid, uint32_t lds, hipStream_t st, Args... args) {
  StepEvents& ev = step_events();
  if (ev.start || ev.stop) {
    hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), lds, st, ev.start, ev.stop, 0u, args...);
    ev = StepEvents{};
  } else {
    hipLaunchKernelGGL(kernel, grid, dim3(kBlock), lds, st, args...);
  }
}

template <typename S>
hipError_t launch_glbe_step(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                            const void* fin, void* fout, const void* force, bool field, bool check,
                            bool nt, bool stochastic, void* usnap, double* partials, hipStream_t st);

template <typename R>
hipError_t launch_mhd_step(const GridArgs& g, const CollideArgs<R>& c, const MagArgs<R>& m,
                           const void* fin, void* fout, const void* gin, void* gout,
                           const void* force, bool field, bool check, bool nt, void* usnap,
                           double* partials, hipStream_t st);

template <typename S>
hipError_t launch_fields(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                         const MagArgs<typename Storage<S>::R>& m, bool mhd, const void* fin,
                         const void* gin, const void* force, bool field, int out_dtype, void* rho,
                         void* u, void* B, int64_t out_stride, double* partials, hipStream_t st);

// Two-dimensional variants (kernels2d.hip): D2Q9 flow, D2Q5 induction, same
// argument conventions as above (nz = 1).
template <typename S>
hipError_t launch_glbe2_step(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                             const void* fin, void* fout, const void* force, bool field, bool check,
                             bool nt, bool stochastic, void* usnap, double* partials,
                             hipStream_t st);

template <typename R>
hipError_t launch_mhd2_step(const GridArgs& g, const CollideArgs<R>& c, const MagArgs<R>& m,
                            const void* fin, void* fout, const void* gin, void* gout,
                            const void* force, bool field, bool check, bool nt, void* usnap,
                            double* partials, hipStream_t st);

template <typename S>
hipError_t launch_fields2(const GridArgs& g, const CollideArgs<typename Storage<S>::R>& c,
                          const MagArgs<typename Storage<S>::R>& m, bool mhd, const void* fin,
                          const void* gin, const void* force, bool field, int out_dtype, void* rho,
                          void* u, void* B, int64_t out_stride, double* partials, hipStream_t st);

// Reduce `count` pending checks (global indices first .. first+count-1) from the
// partials ring (pslots slots) into the history ring.
hipError_t launch_finalize(const double* partials, int nblocks, int pslots, int64_t first,
                           int count, double step0, double dstep, double inv_nx, double* ring,
                           int history_len, hipStream_t st);

// The same result reduced in two passes (many workgroups sum spans of the
// partials into `scratch`, then one workgroup per check) for lattices with
// many workgroups; the single pass when scratch_doubles cannot hold
// count * ceil(nblocks / 1024) * 5 values or the lattice is small.
hipError_t launch_finalize_split(const double* partials, int nblocks, int pslots, int64_t first,
                                 int count, double step0, double dstep, double inv_nx,
                                 double* ring, int history_len, double* scratch,
                                 int64_t scratch_doubles, hipStream_t st);

template <typename S>
hipError_t launch_fill_zero(void* p, int64_t count, hipStream_t st);

// planes x N values (plane stride `stride`) from src to dst, converting between
// storage types (lbm_dtype codes 0..3).
hipError_t launch_convert(int src_storage, int dst_storage, const void* src, void* dst,
                          int64_t stride, int64_t N, int planes, hipStream_t st);


// ---------------------------------------------------------------- adjoint --
// One transposed step of the linearised map (adjoint.hip).
template <typename R>
hipError_t launch_adjoint(const GridArgs& g, const CollideArgs<R>& c, const void* state,
                          const void* force, bool field, const void* mu_in, void* mu_out,
                          void* grad, void* gpre, int64_t grad_stride, int grad_mode,
                          const double* shift, R q_scale, R grad_direct, bool check, bool nt,
                          double* partials, hipStream_t st);

}  // namespace lbm
