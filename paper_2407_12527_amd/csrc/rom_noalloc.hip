// rom_noalloc.hip -- rom_sweep_noalloc: a single transport sweep that takes no device memory.
//
// Every buffer of the sweep (its tables, the sigma_t pool, the inflow table, the partial-flux
// slots, strip edges, progress counters and control state) is placed in `scratch`, a file-scope
// device array of kScratchBytes that each GPU holds from the library's load until the process
// ends.  Host code never passes the array's name to a kernel or a copy: on the first call on a
// device it takes the array's device address with hipGetSymbolAddress (with that device current)
// and keeps it per device.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "rom_host.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];             // device address of `scratch` on each device
uint64_t g_owner[kMaxDevices][3];     // whose plan the device's region holds

}  // namespace

extern "C" int rom_sweep_noalloc(rom_handle* h, const void* src_dev, void* phi_dev, int32_t precision, void* hip_stream)
{
    if (!h) return ROM_E_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ROM_E_DEVICE;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_ptr[dev]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ROM_E_DEVICE;
            g_ptr[dev] = p;
        }
        base = g_ptr[dev];
    }
    return rom::sweep_in_scratch(h, base, kScratchBytes, g_owner[dev], src_dev, phi_dev, precision, hip_stream);
}
