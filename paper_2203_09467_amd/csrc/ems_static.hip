// ems_static.hip -- a transport context over library-owned device memory, for
// callers that cannot allocate device memory themselves.
//
// The context's workspace (track pools, interaction queues, tables, per-event
// tallies, counters) is carved from `scratch`, a file-scope device array of
// kScratchBytes that every GPU the library runs on holds until the process ends.
// Host code never passes the array's name to the device: it takes the array's
// device address once per device with hipGetSymbolAddress and uses that.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "emshower.h"
#include "ems_device.h"
#include "ems_host.h"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

extern "C" ems_status ems_create_static(const ems_config* cfg, ems_ctx** out) {
  if (!out) return ems::fail_status(EMS_E_ARG, "ems_create_static: out is null");
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return ems::fail_status(EMS_E_HIP, "ems_create_static: no current device below 64");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return ems::fail_status(EMS_E_HIP, std::string("ems_create_static: hipGetSymbolAddress: ") +
                                               hipGetErrorString(e));
      g_ptr[dev] = p;
    }
    ptr = g_ptr[dev];
  }
  const size_t need = ems_workspace_bytes(cfg);
  if (need > kScratchBytes)
    return ems::fail_status(EMS_E_CAPACITY, "ems_create_static: the configuration needs " +
                                                std::to_string(need) + " bytes of workspace; the " +
                                                "static scratch holds " + std::to_string(kScratchBytes));
  // an invalid cfg (need == 0) is reported by create_context
  return ems::create_context(cfg, ptr, kScratchBytes, false, "ems_create_static", out);
}
