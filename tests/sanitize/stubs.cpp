// Device-side launchers of libjpet replaced by stubs that fail, so that the library's host code
// (validation, plans, layouts) can be built without device code and run under the sanitizers.
#include "jpet_internal.h"

namespace jpet {
hipError_t launch_sensitivity(const Geo&, float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_direct_image(const Geo&, double, const float*, int64_t, float*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_fill_u64(unsigned long long*, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fill_f32(float*, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_prepare(const Geo&, const Plan&, const float*, int64_t, const Workspace&, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_event_pass(const Geo&, const Plan&, int64_t, const Workspace&, const float*, hipStream_t, int,
                             float*) {
  return hipErrorNotSupported;
}
hipError_t launch_update(const Geo&, const float*, float*, const Workspace&, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_write_insts(const InstWrite&, BatchInst*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_batched_reset(const BatchInst*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_event_pass_batched(const BatchInst*, int, int, int, int, size_t, int64_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t set_batched_lds(int, int, int, size_t) { return hipErrorNotSupported; }
hipError_t launch_update_batched(const BatchInst*, int, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_loglik(const Geo&, const Plan&, int64_t, const Workspace&, const float*, const float*, float*,
                         float*, double*, bool, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_loglik_tiled(const Geo&, const Plan&, int64_t, const Workspace&, const float*, float*, bool,
                               hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace jpet
