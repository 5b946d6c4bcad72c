// Host-only stand-ins for the device half of libsrp, so that the plan code
// (geometry, operator fits, window selection) and the C-ABI's argument
// checks can be built with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.  Every device entry
// point fails with SRP_E_HIP; host-only plans (opts.device = -1) never reach
// them.
#include <stdexcept>

#include "../../paper_2306_08514_amd/csrc/device.hpp"

extern "C" hipError_t hipGetDevice(int* device) {
  if (device) *device = -1;
  return hipErrorNoDevice;
}
extern "C" hipError_t hipSetDevice(int) { return hipErrorNoDevice; }

namespace srp {

[[noreturn]] static void no_device() { throw Error{SRP_E_HIP, "host-only build: no device code"}; }

void device_build(HostPlan&, DevicePlan&, int64_t, size_t) { no_device(); }
void device_free(DevicePlan&) {}
void device_argmax(const void*, bool, int64_t, int64_t, int64_t, int64_t*, double*, hipStream_t) { no_device(); }
size_t workspace_bytes(const HostPlan&, const DevicePlan&, int64_t, int64_t) { no_device(); }
void device_compute(const HostPlan&, DevicePlan&, const void*, int64_t, void*, int64_t, void*, size_t, int64_t,
                    hipStream_t) {
  no_device();
}
void device_compute_static(const HostPlan&, DevicePlan&, const void*, int64_t, void*, int64_t, int64_t,
                           hipStream_t) {
  no_device();
}
void device_profile_collect(DevicePlan&, std::vector<std::pair<std::string, std::pair<double, int64_t>>>&) {
  no_device();
}
void device_crossspec(const HostPlan&, DevicePlan&, const void*, int64_t, void*, hipStream_t) { no_device(); }
void device_gcc_samples(const HostPlan&, DevicePlan&, const void*, int64_t, float*, void*, size_t, int64_t,
                        hipStream_t) {
  no_device();
}

}  // namespace srp
