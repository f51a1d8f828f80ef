// mtp_advance_to_static: mtp_advance_to on the persistent schedule for callers that cannot
// allocate device memory.  The schedule's per-slab scratch (working predecessor counts,
// ready queue, control words) lives in a file-scope device array instead of the solver's
// workspace; every GPU holds its own copy of the array, whose address is looked up once per
// device and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <string>

#include "internal.h"

static __device__ __align__(256) unsigned char scratch[MTP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];             // device address of `scratch` on each device
hipError_t g_lookup[kMaxDevices];
std::once_flag g_once[kMaxDevices];

// makes `dev` current for the call and restores the caller's device afterwards
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) throw mtp::Error(MTP_ERR_DEVICE, "hipGetDevice failed");
    if (cur != dev) {
      if (hipSetDevice(dev) != hipSuccess) throw mtp::Error(MTP_ERR_DEVICE, "hipSetDevice failed");
      prev = cur;
    }
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" mtp_status mtp_advance_to_static(mtp_solver solver, double T) {
  try {
    if (!solver) throw mtp::Error(MTP_ERR_ARG, "null solver");
    const int dev = mtp::solver_device(solver);
    if (dev < 0 || dev >= kMaxDevices) throw mtp::Error(MTP_ERR_UNSUPPORTED, "device index out of range");
    DeviceGuard guard(dev);
    // once per device, with that device current: the array's address on it
    std::call_once(g_once[dev], [dev] {
      g_lookup[dev] = hipGetSymbolAddress(&g_scratch[dev], HIP_SYMBOL(scratch));
    });
    if (g_lookup[dev] != hipSuccess || g_scratch[dev] == nullptr)
      throw mtp::Error(MTP_ERR_DEVICE, std::string("static scratch address: ") + hipGetErrorString(g_lookup[dev]));
    mtp::advance_to_dag_scratch(solver, T, static_cast<char*>(g_scratch[dev]), MTP_STATIC_SCRATCH_BYTES);
  } catch (const mtp::Error& e) {
    mtp::set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    mtp::set_last_error("host memory exhausted");
    return MTP_ERR_NOMEM;
  } catch (const std::exception& e) {
    mtp::set_last_error(e.what());
    return MTP_ERR_ARG;
  }
  return MTP_OK;
}
