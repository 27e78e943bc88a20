// Kernel-variant selection and per-phase launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "lqr_layout.h"

namespace lqr {

// Raise the kernel's dynamic-LDS limit to at least `lds` bytes on the current
// device (the runtime call is made once per kernel, device and size increase,
// so launches under stream capture normally make none).
hipError_t ensure_dynamic_lds(const void* kernel, size_t lds);

// Call f with the kernel instantiation K<pad_rows(width), eng> (eng: product
// engine 0, 1 or 2, see pgemm_sub).
// Width 8 exists only for the vector-ALU engine: the width-8 matrix-core
// variants faulted the GPU (illegal address) on the streamed parametric sweep
// and are not compiled; asking for one returns hipErrorInvalidValue
// (kernel_width never does).
template <template <int, int> class K, typename F>
hipError_t with_variant(int width, int eng, F f) {
  switch (pad_rows(width)) {
    case 8:
      return eng == 0 ? f(K<8, 0>::fn()) : hipErrorInvalidValue;
#define LQR_CASE(W) \
  case W:           \
    return eng == 2 ? f(K<W, 2>::fn()) : eng == 1 ? f(K<W, 1>::fn()) : f(K<W, 0>::fn());
    LQR_CASE(16) LQR_CASE(24) LQR_CASE(32) LQR_CASE(48) LQR_CASE(64)
#undef LQR_CASE
  }
  return hipErrorInvalidValue;
}

// As with_variant, for kernels that only run FP64 engines (0 or 1).
template <template <int, int> class K, typename F>
hipError_t with_variant_fp64(int width, int eng, F f) {
  switch (pad_rows(width)) {
    case 8:
      return eng == 0 ? f(K<8, 0>::fn()) : hipErrorInvalidValue;
#define LQR_CASE(W) \
  case W:           \
    return eng == 1 ? f(K<W, 1>::fn()) : f(K<W, 0>::fn());
    LQR_CASE(16) LQR_CASE(24) LQR_CASE(32) LQR_CASE(48) LQR_CASE(64)
#undef LQR_CASE
  }
  return hipErrorInvalidValue;
}

// As with_variant_fp64 for the linking-solve kernels, whose width and engine
// both follow from the (largest) state dimension n: pad_rows(n) with the FP64
// matrix-core engine from kMfmaMinN states on, the vector ALUs below. Only
// those variants are compiled.
template <template <int, int> class K, typename F>
hipError_t with_link_variant(int n, F f) {
  switch (pad_rows(n)) {
    case 8: return f(K<8, 0>::fn());
    case 16: return f(K<16, 0>::fn());
    case 24: return f(K<24, 0>::fn());
    case 32: return n >= kMfmaMinN ? f(K<32, 1>::fn()) : f(K<32, 0>::fn());
    case 48: return f(K<48, 1>::fn());
    case 64: return f(K<64, 1>::fn());
  }
  return hipErrorInvalidValue;
}

// Product engine of a launch: FP32 matrix cores in the mixed-precision mode,
// else FP64 matrix cores for n >= kMfmaMinN and the vector ALUs below.
inline int launch_engine(int max_n, bool mixed) { return mixed ? 2 : max_n >= kMfmaMinN ? 1 : 0; }

// Register width (the m the kernel variant is picked for) of a launch: the
// matrix-core engines run widths of at least 16 (their width-8 variants are not
// built, see with_variant), the vector-ALU engine any width.
inline int kernel_width(int max_m, int eng) { return eng != 0 && max_m < 9 ? 9 : max_m; }

// One launcher per kernel. `single` is used when descs == nullptr; otherwise
// workgroup b runs items[b] (phases 1, 3) or descs[b] (phase 2, serial).
hipError_t launch_k_phase1(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                           unsigned grid, int width, int eng, size_t lds, hipStream_t stream);
hipError_t launch_k_phase2(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                           unsigned grid, int width, int eng, size_t lds, hipStream_t stream);
hipError_t launch_k_phase3(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                           unsigned grid, int width, int eng, size_t lds, hipStream_t stream);
hipError_t launch_k_serial(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                           unsigned grid, int width, int eng, size_t lds, hipStream_t stream);

// Persistent batched solve: clears the `sync` words, then launches one
// workgroup per resident slot (occupancy x compute units, at most ntasks),
// each draining the task queue. lds_items: LDS bytes the tasks need.
// *grid_out (if not null) receives the grid size.
hipError_t launch_persistent(const InstDesc* descs, const TaskItem* tasks, int ntasks, int ninst,
                             int32_t* sync, int max_m, int eng, size_t lds_items,
                             int* grid_out, hipStream_t stream);

// Single-instance linking solve in logarithmic depth (k_link_tree.hip):
// ceil(log2 J) scan rounds, the link maps, the forward chain of boundary
// states. lds: link_tree_lds of the instance.
hipError_t launch_link_tree(const InstDesc& d, size_t lds, hipStream_t stream);

// First launch of the logarithmic-depth linking solve: scan buffer 0 from the
// phase-1 summaries and the last segment's value (k_link_tree.hip).
hipError_t launch_link_init(const InstDesc& d, hipStream_t stream);
// Smoothed-policy seeds: the boundary values of segments 1..J-2 replaced by
// those segments' cost-to-go with their ends fixed at the link points.
hipError_t launch_smooth_seed(const InstDesc& d, size_t lds, hipStream_t stream);
// mu_j = P x + p at the J - 1 link points of a solved instance (its outputs).
hipError_t launch_link_mu(int n, int T, int J, const void* P, const void* p, const void* x, void* mu,
                          bool f32, hipStream_t stream);

// Large-state path (65..128 states, big_device.h): the sweep kernels of
// engine eng (1: FP64, 2: FP32 matrix cores) -- kind 1 phase 1, kind 3 phase 3
// (d.J workgroups), kind 0 the plain serial recursion (one workgroup) -- and
// the FP64 linking solve (any J >= 1). lds: big_sweep_lds / big_link_lds.
hipError_t launch_big_sweep(const InstDesc& d, int kind, int eng, size_t lds, hipStream_t stream);
hipError_t launch_big_link(const InstDesc& d, size_t lds, hipStream_t stream);

// FP32 mode conversions: the arrays of a device table (one block column per
// array), or a by-value list of one instance's arrays.
hipError_t launch_convert(const CvtItem* items, int nitems, hipStream_t stream);
hipError_t launch_convert_list(const CvtList& list, hipStream_t stream);

// Adjoint solve (one workgroup per instance) followed by the gradient
// outer products (one workgroup per (instance, kAdjStages stages) block).
hipError_t launch_adjoint(const AdjDesc* descs, int ninst, const int2* blocks, int nblocks,
                          size_t lds, hipStream_t stream);

}  // namespace lqr
