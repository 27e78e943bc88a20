// Host-side launchers of the solver kernels (defined in lqr_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lqr_layout.h"
#include "mi355lqr.h"

namespace lqr {

// `eng` is the product engine of the sweeps (launch_engine); the linking
// solve always runs an FP64 engine.
// Single instance, J = d.J segments: phase 1 (J workgroups), phase 2 (one),
// phase 3 (J workgroups); ldsN = dynamic LDS bytes of each launch.
hipError_t launch_parallel(const InstDesc& d, size_t lds1, size_t lds2, size_t lds3, int eng,
                           hipStream_t stream);
// One of the three launches above (phase 1, 2 or 3).
hipError_t launch_phase(const InstDesc& d, int phase, size_t lds, int eng, hipStream_t stream);
// Single instance, one plain recursion over the whole horizon.
hipError_t launch_serial(const InstDesc& d, size_t lds, int eng, hipStream_t stream);
// Batched forms: descriptors and work items live in device memory.
// max_n, max_m: largest state and input dimensions in the batch (they select
// the kernel variant; smaller instances run padded).
hipError_t launch_parallel_batched(const InstDesc* descs, const WorkItem* items, int nitems,
                                   int ninst, int max_n, int max_m, size_t lds1, size_t lds2,
                                   size_t lds3, int eng, hipStream_t stream);
hipError_t launch_serial_batched(const InstDesc* descs, int ninst, int max_m, int eng, size_t lds,
                                 hipStream_t stream);
// Plain recursion for instances with n <= 16 and m <= 16 (k_small.hip): the
// single instance `single` when descs is null, else descs[0 .. ninst).
hipError_t launch_small_serial(const InstDesc& single, const InstDesc* descs, int ninst,
                               hipStream_t stream);
constexpr int kSmallMax = 16;
// Phases 1 and 3 of a single segmented solve with n, m <= 16 (k_small.hip).
hipError_t launch_small_phase1(const InstDesc& d, hipStream_t stream);
hipError_t launch_small_phase3(const InstDesc& d, hipStream_t stream);
// Dynamic LDS of the adjoint solve for an instance with n, m <= 16 (k_adjoint.hip).
size_t adjoint_small_lds();

// lqr_solve on a caller-given device buffer of ws_bytes (lqr_api.cpp): the
// workspace of lqr_solve or the scratch array of lqr_solve_noalloc. Launches
// kernels only; allocates no device memory.
lqr_status_t solve_single(const lqr_problem_t* prob, const lqr_options_t* opts, void* ws,
                          size_t ws_bytes, void* stream);
// Device bytes solve_single needs for this problem.
lqr_status_t solve_bytes(const lqr_problem_t* prob, const lqr_options_t* opts, size_t* bytes);

}  // namespace lqr
