// C-ABI host layer of libbpm.so: argument validation, workspace carving,
// error reporting and dispatch to the kernel launchers.  Declarations and the
// contract of every entry point are in include/bpm.h.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/bpm.h"
#include "internal.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

bool pow2_in_range(int n) { return n >= 32 && n <= 2048 && (n & (n - 1)) == 0; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Shared validation of one march's scalar arguments.
int check_geom(int nx, int ny, int steps, double dx, double dz, double wavelength, double n0) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(BPM_ERR_UNSUPPORTED_SIZE,
                    "nx=%d ny=%d: sizes must be powers of two in [32, 2048]", nx, ny);
    if (steps < 0) return fail(BPM_ERR_INVALID_ARG, "steps=%d must be >= 0", steps);
    if (!std::isfinite(dx) || !std::isfinite(dz) || !std::isfinite(wavelength) ||
        !std::isfinite(n0))
        return fail(BPM_ERR_NOT_FINITE, "non-finite geometry (dx=%g dz=%g wavelength=%g n0=%g)",
                    dx, dz, wavelength, n0);
    if (!(dx > 0) || !(wavelength > 0) || !(n0 > 0))
        return fail(BPM_ERR_NOT_FINITE, "dx=%g, wavelength=%g and n0=%g must be > 0", dx,
                    wavelength, n0);
    return BPM_OK;
}

int check_field_ptrs(const void* in, const float* dn, int steps, const void* out) {
    if (!in || !out) return fail(BPM_ERR_INVALID_ARG, "field_in and field_out must be non-null");
    if (steps > 0 && !dn) return fail(BPM_ERR_INVALID_ARG, "dn must be non-null when steps > 0");
    if (!aligned(in, 8) || !aligned(out, 8) || (dn && !aligned(dn, 4)))
        return fail(BPM_ERR_INVALID_ARG, "fields must be 8-byte and dn 4-byte aligned");
    return BPM_OK;
}

int check_workspace(void* ws, size_t have, size_t need) {
    if (!ws || have < need)
        return fail(BPM_ERR_WORKSPACE, "workspace %p of %zu bytes; %zu bytes needed", ws, have,
                    need);
    if (!aligned(ws, bpm::kAlign))
        return fail(BPM_ERR_WORKSPACE, "workspace must be %zu-byte aligned", bpm::kAlign);
    return BPM_OK;
}

int device_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return BPM_OK;
    return fail(BPM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" {

const char* bpm_error_string(int code) {
    switch (code) {
        case BPM_OK: return "ok";
        case BPM_ERR_INVALID_ARG: return "invalid argument";
        case BPM_ERR_UNSUPPORTED_SIZE: return "unsupported size";
        case BPM_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
        case BPM_ERR_DEVICE: return "device error";
        case BPM_ERR_NOT_FINITE: return "non-finite or non-positive geometry";
        default: return "unknown error code";
    }
}

const char* bpm_last_error(void) { return g_last_error.c_str(); }

size_t bpm_workspace_size(int nx, int ny, int steps, int flags) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny) || steps < 0) return 0;
    if (flags == BPM_WS_FORWARD) return bpm::plan_bytes(nx, ny);
    if (flags == BPM_WS_ADJOINT) return bpm_adjoint_workspace_size(nx, ny, steps, 0);
    return 0;
}

int bpm_propagate(const bpm_c64* field_in, const float* dn, int nx, int ny, int steps,
                  double dx, double dz, double wavelength, double n0, bpm_c64* field_out,
                  float* intensity_out, void* workspace, size_t workspace_bytes,
                  void* hip_stream) {
    int rc = check_geom(nx, ny, steps, dx, dz, wavelength, n0);
    if (rc) return rc;
    if ((rc = check_field_ptrs(field_in, dn, steps, field_out))) return rc;
    if (intensity_out && !aligned(intensity_out, 4))
        return fail(BPM_ERR_INVALID_ARG, "intensity_out must be 4-byte aligned");
    if ((rc = check_workspace(workspace, workspace_bytes, bpm::plan_bytes(nx, ny)))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const bpm::Geom g{nx, ny, steps, dx, dz, wavelength, n0};
    const bpm::Plan p = bpm::plan_carve(workspace, nx, ny);
    if ((rc = device_status(bpm::launch_plan(g, p, s), "plan"))) return rc;
    const bpm::MarchIO io{field_in, dn, field_out, intensity_out};
    return device_status(bpm::launch_forward(g, p, io, s), "forward march");
}

size_t bpm_batch_workspace_size(const bpm_job* jobs, int n_jobs) {
    (void)jobs;
    (void)n_jobs;
    return 0;
}

int bpm_propagate_batch(const bpm_job* jobs, int n_jobs, void* workspace,
                        size_t workspace_bytes, void* hip_stream) {
    (void)jobs; (void)n_jobs; (void)workspace; (void)workspace_bytes; (void)hip_stream;
    return fail(BPM_ERR_INVALID_ARG, "bpm_propagate_batch: not built yet");
}

size_t bpm_adjoint_workspace_size(int nx, int ny, int steps, int checkpoint_every) {
    (void)nx; (void)ny; (void)steps; (void)checkpoint_every;
    return 0;
}

int bpm_adjoint(const bpm_c64* field_in, const float* dn, int nx, int ny, int steps, double dx,
                double dz, double wavelength, double n0, const bpm_c64* grad_field_out,
                const float* grad_intensity, bpm_c64* grad_field_in, bpm_c64* grad_spectrum_in,
                float* grad_dn, int checkpoint_every, void* workspace, size_t workspace_bytes,
                void* hip_stream) {
    (void)field_in; (void)dn; (void)nx; (void)ny; (void)steps; (void)dx; (void)dz;
    (void)wavelength; (void)n0; (void)grad_field_out; (void)grad_intensity;
    (void)grad_field_in; (void)grad_spectrum_in; (void)grad_dn; (void)checkpoint_every;
    (void)workspace; (void)workspace_bytes; (void)hip_stream;
    return fail(BPM_ERR_INVALID_ARG, "bpm_adjoint: not built yet");
}

int psf_surrogate_infer(const void* weights_bf16, size_t weights_bytes, const float* dn_patches,
                        const float* depth, int batch, float* psf_out, float* pred_err,
                        void* hip_stream) {
    (void)weights_bf16; (void)weights_bytes; (void)dn_patches; (void)depth; (void)batch;
    (void)psf_out; (void)pred_err; (void)hip_stream;
    return fail(BPM_ERR_INVALID_ARG, "psf_surrogate_infer: not built yet");
}

}  // extern "C"
