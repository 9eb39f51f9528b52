// Internal interface between the C-ABI host layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace bpm {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Geometry of one march, already validated.
struct Geom {
    int nx, ny, steps;
    double dx, dz, wavelength, n0;
};

// Device plan of one geometry, carved out of the caller's workspace:
// the propagator table in the march's storage order (1 / (nx ny) folded in)
// and the two twiddle tables tw[e] = exp(-2 pi i e / n).
struct Plan {
    void* H;      // float2 [ny][nx]
    void* twx;    // float2 [nx]
    void* twy;    // float2 [ny]
    void* counter;  // grid-barrier words and time-out flag (4 KiB, zeroed by the plan)
};
size_t plan_bytes(int nx, int ny);
Plan plan_carve(void* ws, int nx, int ny);
hipError_t launch_plan(const Geom& g, const Plan& p, hipStream_t s);

// Forward march through `steps` slices; field_out doubles as working buffer.
struct MarchIO {
    const void* field_in;  // float2 [ny][nx]
    const float* dn;       // [steps][ny][nx]
    void* field_out;       // float2 [ny][nx]
    float* intensity;      // [steps][ny][nx] or nullptr
};
hipError_t launch_forward(const Geom& g, const Plan& p, const MarchIO& io, hipStream_t s);

}  // namespace bpm
