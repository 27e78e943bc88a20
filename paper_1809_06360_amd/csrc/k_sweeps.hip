// Launchers of the sweep kernels (k_sweeps.h): engine dispatch. The kernels
// themselves are instantiated in k_sweep_<kernel>_e<engine>.hip.
#include "k_sweeps.h"

namespace lqr {

#define LQR_DECL3(KIND) LQR_SWEEP_DECL(KIND, 0) LQR_SWEEP_DECL(KIND, 1) LQR_SWEEP_DECL(KIND, 2)
LQR_DECL3(kSweepPhase1)
LQR_DECL3(kSweepPhase3)
LQR_DECL3(kSweepSerial)
#undef LQR_DECL3

namespace {

template <int KIND>
hipError_t by_engine(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                     unsigned grid, int width, int eng, size_t lds, hipStream_t stream) {
  switch (eng) {
    case 0: return launch_sweep<KIND, 0>(single, descs, items, grid, width, lds, stream);
    case 1: return launch_sweep<KIND, 1>(single, descs, items, grid, width, lds, stream);
    case 2: return launch_sweep<KIND, 2>(single, descs, items, grid, width, lds, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_k_phase1(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                           unsigned grid, int width, int eng, size_t lds, hipStream_t stream) {
  return by_engine<kSweepPhase1>(single, descs, items, grid, width, eng, lds, stream);
}

hipError_t launch_k_phase3(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                           unsigned grid, int width, int eng, size_t lds, hipStream_t stream) {
  return by_engine<kSweepPhase3>(single, descs, items, grid, width, eng, lds, stream);
}

hipError_t launch_k_serial(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                           unsigned grid, int width, int eng, size_t lds, hipStream_t stream) {
  return by_engine<kSweepSerial>(single, descs, items, grid, width, eng, lds, stream);
}

}  // namespace lqr
