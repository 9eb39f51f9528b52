// Allocation-free forward march: bpm_propagate with its plan (status header,
// propagator table, twiddles, storage-order tables and barrier words) in a
// device array of this library instead of a caller workspace.
//
// The array is a file-scope __device__ variable; each GPU the library runs on
// holds its own copy until the process ends.  Host code never passes the
// variable's name to a kernel (in host code it is a host-side stand-in): the
// device address of each GPU's copy is looked up once per device, with that
// device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bpm.h"
#include "abi_util.hpp"
#include "internal.hpp"

namespace {

using namespace bpm::abi;

// fields up to 1024 x 1024: the plan of a 1024^2 march (8 MiB propagator
// table, 32 KiB of barrier words, small tables) with room to spare
constexpr size_t kScratchBytes = (8u << 20) + (64u << 10);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of the current device's copy of `scratch`, or null (message set)
void* scratch_ptr() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        device_status(e, "no-allocation march: current device");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        fail(BPM_ERR_DEVICE, "no-allocation march: device %d beyond the %d supported", dev,
             kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            device_status(e != hipSuccess ? e : hipErrorInvalidSymbol,
                          "no-allocation march: scratch address");
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t bpm_noalloc_scratch_bytes(void) { return kScratchBytes; }

int bpm_propagate_noalloc(const bpm_c64* field_in, const float* dn, int nx, int ny, int steps,
                          double dx, double dz, double wavelength, double n0,
                          bpm_c64* field_out, float* intensity_out, void* hip_stream) {
    // argument checks as in bpm_propagate, then the size limit of the scratch
    const size_t need = bpm_workspace_size(nx, ny, steps, BPM_WS_FORWARD);
    if (need == 0 || need > kScratchBytes) {
        if (need == 0)  // unsupported sizes get bpm_propagate's own message
            return bpm_propagate(field_in, dn, nx, ny, steps, dx, dz, wavelength, n0, field_out,
                                 intensity_out, nullptr, 0, hip_stream);
        return fail(BPM_ERR_UNSUPPORTED_SIZE,
                    "nx=%d ny=%d: the no-allocation march holds plans of at most %zu bytes "
                    "(fields up to 1024 x 1024); this size needs %zu",
                    nx, ny, kScratchBytes, need);
    }
    void* p = scratch_ptr();
    if (!p) return BPM_ERR_DEVICE;
    return bpm_propagate(field_in, dn, nx, ny, steps, dx, dz, wavelength, n0, field_out,
                         intensity_out, p, kScratchBytes, hip_stream);
}

}  // extern "C"
