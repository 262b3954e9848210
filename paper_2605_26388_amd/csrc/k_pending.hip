// Kernel families not yet available in this build return hipErrorNotSupported.
#include "dg_internal.hpp"

namespace dg {
hipError_t launch_ns(const Ctx&, const StageParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_adjoint(const Ctx&, const void*, const void*, void*, void*, double, double, double, int,
                          hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace dg
