// C-ABI host layer of libbpm.so: argument validation, workspace carving,
// error reporting and dispatch to the kernel launchers.  Declarations and the
// contract of every entry point are in include/bpm.h.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bpm.h"
#include "abi_util.hpp"
#include "internal.hpp"

namespace {

using namespace bpm::abi;

bool pow2_in_range(int n) { return n >= 32 && n <= 2048 && (n & (n - 1)) == 0; }

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

}  // namespace

namespace bpm {

constexpr unsigned kDefaultWaitLimit = 1u << 22;
static std::atomic<unsigned> g_wait_limit{kDefaultWaitLimit};
unsigned wait_limit() { return g_wait_limit.load(std::memory_order_relaxed); }

}  // namespace bpm

extern "C" {

int bpm_set_wait_limit(unsigned long long polls) {
    if (polls > (1ull << 31))
        return fail(BPM_ERR_INVALID_ARG, "polls=%llu must be at most 2^31", polls);
    bpm::g_wait_limit.store(polls == 0 ? bpm::kDefaultWaitLimit : (unsigned)polls,
                            std::memory_order_relaxed);
    return BPM_OK;
}

int bpm_march_variant(int nx, int ny, int fields) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny) || fields < 1 || fields > bpm::kMaxFields)
        return fail(BPM_ERR_INVALID_ARG, "nx=%d ny=%d fields=%d: sizes must be powers of two in "
                    "[32, 2048] and fields in [1, %d]", nx, ny, fields, bpm::kMaxFields);
    return bpm::march_variant(nx, ny, fields);
}

int bpm_march_variant_eligible(int nx, int ny, int fields, int variant) {
    return bpm::march_variant_eligible(nx, ny, fields, variant) ? 1 : 0;
}

int bpm_set_march_variant(int nx, int ny, int fields, int variant) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny) || fields < 1 || fields > bpm::kMaxFields)
        return fail(BPM_ERR_INVALID_ARG, "nx=%d ny=%d fields=%d: sizes must be powers of two in "
                    "[32, 2048] and fields in [1, %d]", nx, ny, fields, bpm::kMaxFields);
    if (variant < BPM_MARCH_AUTO || variant > BPM_MARCH_SMALL_BLOCKS)
        return fail(BPM_ERR_INVALID_ARG, "variant=%d is not a BPM_MARCH_* value", variant);
    if (bpm::set_march_variant(nx, ny, fields, variant) != 0)
        return fail(BPM_ERR_INVALID_ARG, "variant %d cannot run %d x %d with %d field(s) on this "
                    "device", variant, nx, ny, fields);
    return BPM_OK;
}

int bpm_decode_status(unsigned status_word) {
    if (status_word == 0) return BPM_OK;
    std::string what;
    if (status_word & bpm::kStatusBarrierBit) what += " a grid-barrier wait;";
    if (status_word & bpm::kStatusQueueBit) what += " a work-queue dependency wait;";
    if (status_word & ~(bpm::kStatusBarrierBit | bpm::kStatusQueueBit))
        what += " unknown status bits;";
    what.pop_back();
    return fail(BPM_ERR_DEVICE,
                "a kernel that used this workspace gave up waiting (%s): the outputs of that "
                "call are not valid (status word 0x%x)", what.c_str() + 1, status_word);
}

int bpm_workspace_status(const void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!workspace || workspace_bytes < bpm::kStatusBytes || !aligned(workspace, bpm::kAlign))
        return fail(BPM_ERR_WORKSPACE,
                    "workspace must be non-null, %zu-byte aligned and hold at least %zu bytes",
                    bpm::kAlign, bpm::kStatusBytes);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    int rc;
    if ((rc = device_status(hipStreamIsCapturing(s, &cs), "workspace status"))) return rc;
    if (cs != hipStreamCaptureStatusNone)
        return fail(BPM_ERR_INVALID_ARG, "bpm_workspace_status must not run under stream capture");
    unsigned words[3] = {0u, 0u, 0u};
    hipError_t e = hipMemcpyAsync(words, workspace, sizeof words, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((rc = device_status(e, "workspace status"))) return rc;
    if (words[1] != bpm::kStatusMagic0 || words[2] != bpm::kStatusMagic1)
        return fail(BPM_ERR_INVALID_ARG,
                    "the workspace holds no status header: no march, batch or adjoint call has "
                    "used it");
    if (words[0] == 0) return BPM_OK;
    const unsigned zero = 0u;
    e = hipMemcpyAsync(const_cast<void*>(workspace), &zero, sizeof zero, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((rc = device_status(e, "workspace status reset"))) return rc;
    return bpm_decode_status(words[0]);
}

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
    const int var = bpm::march_variant(nx, ny, 1);
    if ((rc = device_status(bpm::launch_plan(g, p, true, s, var == bpm::kMarchTiledPair),
                            "plan")))
        return rc;
    const bpm::MarchIO io{field_in, dn, field_out, intensity_out};
    return device_status(bpm::launch_forward(g, p, &io, 1, s, nullptr, var), "forward march");
}

int bpm_slice_means(const float* dn, int nx, int ny, int steps, float* dn_ref, void* hip_stream) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(BPM_ERR_UNSUPPORTED_SIZE,
                    "nx=%d ny=%d: sizes must be powers of two in [32, 2048]", nx, ny);
    if (steps < 0) return fail(BPM_ERR_INVALID_ARG, "steps=%d must be >= 0", steps);
    if (steps > 0 && (!dn || !dn_ref || !aligned(dn, 4) || !aligned(dn_ref, 4)))
        return fail(BPM_ERR_INVALID_ARG, "dn and dn_ref must be non-null and 4-byte aligned");
    return device_status(bpm::launch_slice_means(dn, (long)nx * ny, steps, dn_ref,
                                                 static_cast<hipStream_t>(hip_stream)),
                         "slice means");
}

int bpm_propagate_adapted(const bpm_c64* field_in, const float* dn, const float* dn_ref, int nx,
                          int ny, int steps, double dx, double dz, double wavelength, double n0,
                          bpm_c64* field_out, float* intensity_out, void* workspace,
                          size_t workspace_bytes, void* hip_stream) {
    int rc = check_geom(nx, ny, steps, dx, dz, wavelength, n0);
    if (rc) return rc;
    if ((rc = check_field_ptrs(field_in, dn, steps, field_out))) return rc;
    if (steps > 0 && (!dn_ref || !aligned(dn_ref, 4)))
        return fail(BPM_ERR_INVALID_ARG, "dn_ref must be non-null and 4-byte aligned");
    if (intensity_out && !aligned(intensity_out, 4))
        return fail(BPM_ERR_INVALID_ARG, "intensity_out must be 4-byte aligned");
    if ((rc = check_workspace(workspace, workspace_bytes, bpm::plan_bytes(nx, ny)))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (steps == 0) {
        if ((const void*)field_out == (const void*)field_in) return BPM_OK;
        return device_status(hipMemcpyAsync(field_out, field_in, sizeof(bpm_c64) * (size_t)nx * ny,
                                            hipMemcpyDeviceToDevice, s),
                             "copy");
    }
    const bpm::Geom g{nx, ny, steps, dx, dz, wavelength, n0};
    const bpm::Plan p = bpm::plan_carve(workspace, nx, ny);
    if ((rc = device_status(bpm::launch_plan(g, p, false, s), "plan"))) return rc;
    return device_status(bpm::launch_adapted(g, p, field_in, dn, dn_ref, field_out, intensity_out, s),
                         "adapted march");
}

// ---------------------------------------------------------------------------
// uneven batch

}  // extern "C"

namespace {

// Host-side layout of a batch workspace: per-job plans, then the job table,
// the segment table, the queue words and the key of the uploaded tables.
struct BatchLayout {
    std::vector<size_t> plan_off;
    size_t jobs_off, segs_off, q_off, key_off, total;
    int n_segs, n_items;
};

int batch_passes(const bpm_job& j) { return j.steps > 0 ? 2 * j.steps + 1 : 0; }

// 64-bit FNV-1a over the fields of every job and the workspace address (the
// plans' addresses are carved from it); never 0, so a zeroed workspace does
// not match.  Written next to the tables at upload and passed to the batch
// kernel at launch, which does nothing when the workspace holds the tables of
// other jobs.
unsigned long long batch_key(const bpm_job* jobs, int n, const void* ws) {
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&h](const void* p, size_t bytes) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < bytes; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    mix(&n, sizeof n);
    mix(&ws, sizeof ws);
    for (int i = 0; i < n; ++i) {
        const bpm_job& j = jobs[i];
        mix(&j.field_in, sizeof j.field_in);
        mix(&j.dn, sizeof j.dn);
        mix(&j.field_out, sizeof j.field_out);
        mix(&j.intensity_out, sizeof j.intensity_out);
        mix(&j.nx, sizeof j.nx);
        mix(&j.ny, sizeof j.ny);
        mix(&j.steps, sizeof j.steps);
        mix(&j.clear_steps, sizeof j.clear_steps);
        mix(&j.dx, sizeof j.dx);
        mix(&j.dz, sizeof j.dz);
        mix(&j.wavelength, sizeof j.wavelength);
        mix(&j.n0, sizeof j.n0);
    }
    return h | 1ull;
}

BatchLayout batch_layout(const bpm_job* jobs, int n) {
    BatchLayout L;
    size_t off = 0;
    L.n_segs = 0;
    L.n_items = 0;
    for (int i = 0; i < n; ++i) {
        L.plan_off.push_back(off);
        off += bpm::align_up(bpm::plan_bytes(jobs[i].nx, jobs[i].ny));
        const int P = batch_passes(jobs[i]);
        L.n_segs += P;
        const long items = jobs[i].steps > 0
            ? (long)bpm::row_items(jobs[i].nx, jobs[i].ny) * (jobs[i].steps + 1) +
              (long)bpm::col_items(jobs[i].nx, jobs[i].ny) * jobs[i].steps
            : 0;
        L.n_items += (int)items;
    }
    L.jobs_off = off;
    off += bpm::align_up(sizeof(bpm::BatchJob) * (size_t)n);
    L.segs_off = off;
    off += bpm::align_up(sizeof(bpm::BatchSeg) * (size_t)L.n_segs);
    L.q_off = off;
    off += bpm::align_up(sizeof(unsigned) * (size_t)bpm::batch_queue_words(n));
    L.key_off = off;
    off += bpm::align_up(sizeof(unsigned long long));
    L.total = off;
    return L;
}

int check_batch(const bpm_job* jobs, int n) {
    if (!jobs || n < 1) return fail(BPM_ERR_INVALID_ARG, "jobs must be a host array of n_jobs >= 1");
    long items = 0;
    for (int i = 0; i < n; ++i) {
        const bpm_job& j = jobs[i];
        int rc = check_geom(j.nx, j.ny, j.steps, j.dx, j.dz, j.wavelength, j.n0);
        if (rc) return fail(rc, "job %d: %s", i, g_last_error.c_str());
        if ((rc = check_field_ptrs(j.field_in, j.dn, j.steps, j.field_out)))
            return fail(rc, "job %d: %s", i, g_last_error.c_str());
        if (j.intensity_out && !aligned(j.intensity_out, 4))
            return fail(BPM_ERR_INVALID_ARG, "job %d: intensity_out must be 4-byte aligned", i);
        if (j.clear_steps < 0 || j.clear_steps > j.steps)
            return fail(BPM_ERR_INVALID_ARG, "job %d: clear_steps=%d must be in [0, steps=%d]",
                        i, j.clear_steps, j.steps);
        if (j.steps > 0)
            items += (long)bpm::row_items(j.nx, j.ny) * (j.steps + 1) +
                     (long)bpm::col_items(j.nx, j.ny) * j.steps;
    }
    if (items >= (1L << 31)) return fail(BPM_ERR_INVALID_ARG, "batch has too many work items");
    return BPM_OK;
}

// Pinned staging for the job and segment tables; reused once the previous
// upload has completed.
std::mutex g_stage_mu;
void* g_stage = nullptr;
size_t g_stage_bytes = 0;
hipEvent_t g_stage_done = nullptr;

// Host half of the work-queue batch: builds the job and segment tables and
// uploads them into the workspace (stream-ordered, through pinned staging).
int batch_tables(const bpm_job* jobs, int n_jobs, char* ws, const BatchLayout& L, hipStream_t s) {
    int rc = BPM_OK;
    // job table
    std::vector<bpm::BatchJob> dj(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        const bpm_job& j = jobs[i];
        const bpm::Plan p = bpm::plan_carve(ws + L.plan_off[i], j.nx, j.ny);
        dj[i] = bpm::BatchJob{j.field_in, j.dn, j.field_out, j.intensity_out, p.H, p.twx, p.twy,
                              j.nx, j.ny, j.steps,
                              (float)(2.0 * 3.14159265358979323846 / j.wavelength * j.dz),
                              j.clear_steps, bpm::batch_tiled(j.nx, j.ny) ? 1 : 0};
    }
    // segment table: round r holds pass r of every job that has it, jobs of
    // equal pass size side by side
    std::vector<int> order(n_jobs);
    for (int i = 0; i < n_jobs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return jobs[a].nx != jobs[b].nx ? jobs[a].nx < jobs[b].nx : jobs[a].ny < jobs[b].ny;
    });
    int maxP = 0;
    for (int i = 0; i < n_jobs; ++i) maxP = std::max(maxP, batch_passes(jobs[i]));
    std::vector<bpm::BatchSeg> segs;
    segs.reserve(L.n_segs);
    int first = 0;
    for (int r = 0; r < maxP; ++r) {
        for (int i : order) {
            if (r >= batch_passes(jobs[i])) continue;
            const int R = bpm::row_items(jobs[i].nx, jobs[i].ny);
            const int C = bpm::col_items(jobs[i].nx, jobs[i].ny);
            const int count = (r % 2 == 0) ? R : C;
            const int need = r == 0 ? 0 : R + (r / 2) * C + ((r - 1) / 2) * R;
            segs.push_back(bpm::BatchSeg{i, r, first, count, need});
            first += count;
        }
    }
    // upload both tables through pinned staging
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        const size_t jb = sizeof(bpm::BatchJob) * dj.size();
        const size_t sb = sizeof(bpm::BatchSeg) * segs.size();
        const size_t kb_off = (jb + sb + 7) / 8 * 8;
        const size_t bytes = kb_off + sizeof(unsigned long long);
        const unsigned long long key = batch_key(jobs, n_jobs, ws);
        hipError_t e = hipSuccess;
        if (g_stage_done) e = hipEventSynchronize(g_stage_done);
        if (e == hipSuccess && g_stage_bytes < bytes) {
            if (g_stage) (void)hipHostFree(g_stage);
            g_stage = nullptr;
            g_stage_bytes = 0;
            e = hipHostMalloc(&g_stage, bytes, hipHostMallocDefault);
            if (e == hipSuccess) g_stage_bytes = bytes;
        }
        if (e == hipSuccess && !g_stage_done) e = hipEventCreateWithFlags(&g_stage_done, hipEventDisableTiming);
        if (e == hipSuccess) {
            std::memcpy(g_stage, dj.data(), jb);
            std::memcpy(static_cast<char*>(g_stage) + jb, segs.data(), sb);
            std::memcpy(static_cast<char*>(g_stage) + kb_off, &key, sizeof key);
            e = hipMemcpyAsync(ws + L.jobs_off, g_stage, jb, hipMemcpyHostToDevice, s);
        }
        if (e == hipSuccess && sb)
            e = hipMemcpyAsync(ws + L.segs_off, static_cast<char*>(g_stage) + jb, sb,
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + L.key_off, static_cast<char*>(g_stage) + kb_off, sizeof key,
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(g_stage_done, s);
        if ((rc = device_status(e, "batch tables"))) return rc;
    }
    return BPM_OK;
}

// Device half: plans, the copies of zero-step jobs, the queue reset and the
// batch kernel.  Only kernel launches and device-to-device copies, so it can
// be captured into a graph; it reads the tables batch_tables left in `ws`.
int batch_device(const bpm_job* jobs, int n_jobs, char* ws, const BatchLayout& L, hipStream_t s) {
    int rc = BPM_OK;
    for (int i = 0; i < n_jobs; ++i) {
        const bpm_job& j = jobs[i];
        const bpm::Plan p = bpm::plan_carve(ws + L.plan_off[i], j.nx, j.ny);
        if (j.steps > 0) {
            const bpm::Geom g{j.nx, j.ny, j.steps, j.dx, j.dz, j.wavelength, j.n0};
            if ((rc = device_status(bpm::launch_plan(g, p, true, s, bpm::batch_tiled(j.nx, j.ny)),
                                    "batch plan")))
                return rc;
        } else if ((const void*)j.field_out != (const void*)j.field_in) {
            hipError_t e = hipMemcpyAsync(j.field_out, j.field_in,
                                          sizeof(bpm_c64) * (size_t)j.nx * j.ny,
                                          hipMemcpyDeviceToDevice, s);
            if ((rc = device_status(e, "batch copy"))) return rc;
        }
    }
    // the first plan's status header opens the workspace
    unsigned* status = (unsigned*)bpm::plan_carve(ws + L.plan_off[0], jobs[0].nx, jobs[0].ny).status;
    return device_status(bpm::launch_batch((const bpm::BatchJob*)(ws + L.jobs_off),
                                           (const bpm::BatchSeg*)(ws + L.segs_off), L.n_items,
                                           (unsigned*)(ws + L.q_off), n_jobs,
                                           (const unsigned long long*)(ws + L.key_off),
                                           batch_key(jobs, n_jobs, ws), status, s),
                         "batch march");
}

}  // namespace

extern "C" {

void bpm_release(void) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (g_stage_done) {
        (void)hipEventSynchronize(g_stage_done);
        (void)hipEventDestroy(g_stage_done);
        g_stage_done = nullptr;
    }
    if (g_stage) (void)hipHostFree(g_stage);
    g_stage = nullptr;
    g_stage_bytes = 0;
}

size_t bpm_batch_workspace_size(const bpm_job* jobs, int n_jobs) {
    if (!jobs || n_jobs < 1) return 0;
    for (int i = 0; i < n_jobs; ++i)
        if (!pow2_in_range(jobs[i].nx) || !pow2_in_range(jobs[i].ny) || jobs[i].steps < 0) return 0;
    return batch_layout(jobs, n_jobs).total;
}

int bpm_propagate_batch(const bpm_job* jobs, int n_jobs, void* workspace,
                        size_t workspace_bytes, void* hip_stream) {
    int rc = check_batch(jobs, n_jobs);
    if (rc) return rc;
    const BatchLayout L = batch_layout(jobs, n_jobs);
    if ((rc = check_workspace(workspace, workspace_bytes, L.total))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(workspace);

    // jobs of one geometry march in lockstep in the cooperative march kernel
    bool same = n_jobs <= bpm::kMaxFields && jobs[0].steps > 0;
    for (int i = 1; i < n_jobs && same; ++i)
        same = jobs[i].nx == jobs[0].nx && jobs[i].ny == jobs[0].ny &&
               jobs[i].steps == jobs[0].steps && jobs[i].dx == jobs[0].dx &&
               jobs[i].dz == jobs[0].dz && jobs[i].wavelength == jobs[0].wavelength &&
               jobs[i].n0 == jobs[0].n0;
    if (same) {
        const bpm_job& j0 = jobs[0];
        const bpm::Geom g{j0.nx, j0.ny, j0.steps, j0.dx, j0.dz, j0.wavelength, j0.n0};
        const bpm::Plan p = bpm::plan_carve(ws + L.plan_off[0], j0.nx, j0.ny);
        const int var = bpm::march_variant(j0.nx, j0.ny, n_jobs);
        const bool tiled = var == bpm::kMarchTiledPair;
        if ((rc = device_status(bpm::launch_plan(g, p, true, s, tiled), "batch plan"))) return rc;
        bpm::MarchIO io[bpm::kMaxFields];
        for (int i = 0; i < n_jobs; ++i)
            io[i] = bpm::MarchIO{jobs[i].field_in, jobs[i].dn, jobs[i].field_out,
                                 jobs[i].intensity_out, jobs[i].clear_steps};
        return device_status(bpm::launch_forward(g, p, io, n_jobs, s, nullptr, var),
                             "batch march");
    }

    if ((rc = batch_tables(jobs, n_jobs, ws, L, s))) return rc;
    return batch_device(jobs, n_jobs, ws, L, s);
}

int bpm_march_phase_times(const bpm_job* jobs, int n_jobs, void* workspace,
                          size_t workspace_bytes, unsigned long long* timers, size_t timer_bytes,
                          void* hip_stream) {
    int rc = check_batch(jobs, n_jobs);
    if (rc) return rc;
    if (n_jobs > bpm::kMaxFields || jobs[0].steps < 1)
        return fail(BPM_ERR_INVALID_ARG, "phase times need 1..%d jobs with steps >= 1",
                    bpm::kMaxFields);
    for (int i = 1; i < n_jobs; ++i)
        if (jobs[i].nx != jobs[0].nx || jobs[i].ny != jobs[0].ny ||
            jobs[i].steps != jobs[0].steps || jobs[i].dx != jobs[0].dx ||
            jobs[i].dz != jobs[0].dz || jobs[i].wavelength != jobs[0].wavelength ||
            jobs[i].n0 != jobs[0].n0)
            return fail(BPM_ERR_INVALID_ARG, "phase times need jobs of one geometry (job %d)", i);
    if (!timers || !aligned(timers, 8) || timer_bytes < sizeof(unsigned long long) *
                                                          bpm::kPhaseTimerWords)
        return fail(BPM_ERR_INVALID_ARG, "timers must be 8-byte aligned, >= %zu bytes",
                    sizeof(unsigned long long) * bpm::kPhaseTimerWords);
    const BatchLayout L = batch_layout(jobs, n_jobs);
    if ((rc = check_workspace(workspace, workspace_bytes, L.total))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const bpm_job& j0 = jobs[0];
    const bpm::Geom g{j0.nx, j0.ny, j0.steps, j0.dx, j0.dz, j0.wavelength, j0.n0};
    const bpm::Plan p = bpm::plan_carve(static_cast<char*>(workspace) + L.plan_off[0], j0.nx, j0.ny);
    const int var = bpm::march_variant(j0.nx, j0.ny, n_jobs);
    const bool tiled = var == bpm::kMarchTiledPair;
    if ((rc = device_status(bpm::launch_plan(g, p, true, s, tiled), "plan"))) return rc;
    if ((rc = device_status(hipMemsetAsync(timers, 0, timer_bytes, s), "timers"))) return rc;
    bpm::MarchIO io[bpm::kMaxFields];
    for (int i = 0; i < n_jobs; ++i)
        io[i] = bpm::MarchIO{jobs[i].field_in, jobs[i].dn, jobs[i].field_out, jobs[i].intensity_out,
                             jobs[i].clear_steps};
    return device_status(bpm::launch_forward(g, p, io, n_jobs, s, timers, var), "timed march");
}

int bpm_batch_upload(const bpm_job* jobs, int n_jobs, void* workspace, size_t workspace_bytes,
                     void* hip_stream) {
    int rc = check_batch(jobs, n_jobs);
    if (rc) return rc;
    const BatchLayout L = batch_layout(jobs, n_jobs);
    if ((rc = check_workspace(workspace, workspace_bytes, L.total))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((rc = device_status(hipStreamIsCapturing(s, &cs), "batch upload"))) return rc;
    if (cs != hipStreamCaptureStatusNone)
        return fail(BPM_ERR_INVALID_ARG, "bpm_batch_upload must not run under stream capture");
    return batch_tables(jobs, n_jobs, static_cast<char*>(workspace), L, s);
}

int bpm_batch_launch(const bpm_job* jobs, int n_jobs, void* workspace, size_t workspace_bytes,
                     void* hip_stream) {
    int rc = check_batch(jobs, n_jobs);
    if (rc) return rc;
    const BatchLayout L = batch_layout(jobs, n_jobs);
    if ((rc = check_workspace(workspace, workspace_bytes, L.total))) return rc;
    return batch_device(jobs, n_jobs, static_cast<char*>(workspace), L,
                        static_cast<hipStream_t>(hip_stream));
}

static int checkpoint_interval(int steps, int checkpoint_every) {
    if (checkpoint_every > 0) return checkpoint_every;
    int k = 1;
    while (k * k < steps) ++k;
    return k;
}

size_t bpm_adjoint_workspace_size(int nx, int ny, int steps, int checkpoint_every) {
    return bpm_adjoint_batch_workspace_size(1, nx, ny, steps, checkpoint_every);
}

size_t bpm_adjoint_batch_workspace_size(int n_fields, int nx, int ny, int steps,
                                        int checkpoint_every) {
    if (n_fields < 1 || n_fields > BPM_MAX_LOCKSTEP_FIELDS) return 0;
    if (!pow2_in_range(nx) || !pow2_in_range(ny) || steps < 0 || checkpoint_every < 0) return 0;
    if (steps > 0 && checkpoint_every > steps) return 0;
    const size_t per_field =
        steps > 0 ? bpm::adjoint_field_bytes(nx, ny, steps, checkpoint_interval(steps, checkpoint_every))
                  : 0;
    return bpm::plan_bytes(nx, ny) + (size_t)n_fields * per_field;
}

// the adjoints of `n` jobs of one geometry, checked, in one lockstep launch
static_assert(BPM_MAX_LOCKSTEP_FIELDS == bpm::kMaxFields, "lockstep field limit");

static int adjoint_run(const bpm_adjoint_job* jobs, int n, int nx, int ny, int steps, double dx,
                       double dz, double wavelength, double n0, int checkpoint_every,
                       void* workspace, size_t workspace_bytes, void* hip_stream) {
    int rc = check_geom(nx, ny, steps, dx, dz, wavelength, n0);
    if (rc) return rc;
    if (checkpoint_every < 0 || (steps > 0 && checkpoint_every > steps))
        return fail(BPM_ERR_INVALID_ARG, "checkpoint_every=%d must be 0 or in [1, steps=%d]",
                    checkpoint_every, steps);
    for (int i = 0; i < n; ++i) {
        const bpm_adjoint_job& j = jobs[i];
        if (!j.field_in && (j.grad_intensity || j.grad_dn))
            return fail(BPM_ERR_INVALID_ARG,
                        "job %d: field_in must be non-null when grad_intensity or grad_dn is given",
                        i);
        if (steps > 0 && !j.dn)
            return fail(BPM_ERR_INVALID_ARG, "job %d: dn must be non-null when steps > 0", i);
        const void* ptrs8[] = {j.field_in, j.grad_field_out, j.grad_field_in, j.grad_spectrum_in};
        for (const void* q : ptrs8)
            if (q && !aligned(q, 8))
                return fail(BPM_ERR_INVALID_ARG, "job %d: complex arrays must be 8-byte aligned", i);
        const void* ptrs4[] = {j.dn, j.grad_intensity, j.grad_dn};
        for (const void* q : ptrs4)
            if (q && !aligned(q, 4))
                return fail(BPM_ERR_INVALID_ARG, "job %d: float arrays must be 4-byte aligned", i);
    }
    const size_t need = bpm_adjoint_batch_workspace_size(n, nx, ny, steps, checkpoint_every);
    if ((rc = check_workspace(workspace, workspace_bytes, need))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const bpm::Geom g{nx, ny, steps, dx, dz, wavelength, n0};
    const bpm::Plan p = bpm::plan_carve(workspace, nx, ny);
    const size_t plane = sizeof(bpm_c64) * (size_t)nx * ny;
    if (steps == 0) {
        // g_0 = dL/du_0 = dL/du_N; dL/dU_0 = DFT2(g_0) / (nx ny)
        if ((rc = device_status(bpm::launch_plan(g, p, false, s), "plan"))) return rc;
        for (int i = 0; i < n; ++i) {
            const bpm_adjoint_job& j = jobs[i];
            if (j.grad_field_in) {
                hipError_t e = j.grad_field_out
                    ? hipMemcpyAsync(j.grad_field_in, j.grad_field_out, plane,
                                     hipMemcpyDeviceToDevice, s)
                    : hipMemsetAsync(j.grad_field_in, 0, plane, s);
                if ((rc = device_status(e, "copy"))) return rc;
            }
            if (j.grad_spectrum_in) {
                hipError_t e = j.grad_field_out
                    ? bpm::launch_fft2(j.grad_field_out, j.grad_spectrum_in, nx, ny, false,
                                       (float)(1.0 / ((double)nx * ny)), p, s)
                    : hipMemsetAsync(j.grad_spectrum_in, 0, plane, s);
                if ((rc = device_status(e, "spectrum"))) return rc;
            }
        }
        return BPM_OK;
    }
    if ((rc = device_status(bpm::launch_plan(g, p, true, s), "plan"))) return rc;
    const int K = checkpoint_interval(steps, checkpoint_every);
    void* fields = static_cast<char*>(workspace) + bpm::plan_bytes(nx, ny);
    bpm::AdjointIO io[bpm::kMaxFields];
    for (int i = 0; i < n; ++i)
        io[i] = bpm::AdjointIO{jobs[i].field_in, jobs[i].dn, jobs[i].grad_field_out,
                               jobs[i].grad_intensity, jobs[i].grad_field_in,
                               jobs[i].grad_spectrum_in, jobs[i].grad_dn};
    return device_status(bpm::launch_adjoint(g, p, io, n, K, fields, s), "adjoint march");
}

int bpm_adjoint(const bpm_c64* field_in, const float* dn, int nx, int ny, int steps, double dx,
                double dz, double wavelength, double n0, const bpm_c64* grad_field_out,
                const float* grad_intensity, bpm_c64* grad_field_in, bpm_c64* grad_spectrum_in,
                float* grad_dn, int checkpoint_every, void* workspace, size_t workspace_bytes,
                void* hip_stream) {
    const bpm_adjoint_job job{field_in,      dn,           grad_field_out, grad_intensity,
                              grad_field_in, grad_spectrum_in, grad_dn};
    return adjoint_run(&job, 1, nx, ny, steps, dx, dz, wavelength, n0, checkpoint_every,
                       workspace, workspace_bytes, hip_stream);
}

int bpm_adjoint_batch(const bpm_adjoint_job* jobs, int n_fields, int nx, int ny, int steps,
                      double dx, double dz, double wavelength, double n0, int checkpoint_every,
                      void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!jobs) return fail(BPM_ERR_INVALID_ARG, "jobs must be non-null");
    if (n_fields < 1 || n_fields > BPM_MAX_LOCKSTEP_FIELDS)
        return fail(BPM_ERR_INVALID_ARG, "n_fields=%d must be in [1, %d]", n_fields,
                    BPM_MAX_LOCKSTEP_FIELDS);
    return adjoint_run(jobs, n_fields, nx, ny, steps, dx, dz, wavelength, n0, checkpoint_every,
                       workspace, workspace_bytes, hip_stream);
}

size_t bpm_fft2_workspace_size(int nx, int ny) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny)) return 0;
    return bpm::plan_bytes(nx, ny);
}

int bpm_fft2(const bpm_c64* in, bpm_c64* out, int nx, int ny, int inverse, void* workspace,
             size_t workspace_bytes, void* hip_stream) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(BPM_ERR_UNSUPPORTED_SIZE,
                    "nx=%d ny=%d: sizes must be powers of two in [32, 2048]", nx, ny);
    if (!in || !out) return fail(BPM_ERR_INVALID_ARG, "in and out must be non-null");
    if (!aligned(in, 8) || !aligned(out, 8))
        return fail(BPM_ERR_INVALID_ARG, "complex arrays must be 8-byte aligned");
    if (inverse != 0 && inverse != 1) return fail(BPM_ERR_INVALID_ARG, "inverse must be 0 or 1");
    int rc;
    if ((rc = check_workspace(workspace, workspace_bytes, bpm::plan_bytes(nx, ny)))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const bpm::Geom g{nx, ny, 0, 1.0, 0.0, 1.0, 1.0};
    const bpm::Plan p = bpm::plan_carve(workspace, nx, ny);
    if ((rc = device_status(bpm::launch_plan(g, p, false, s), "plan"))) return rc;
    const float scale = inverse ? (float)(1.0 / ((double)nx * ny)) : 1.0f;
    return device_status(bpm::launch_fft2(in, out, nx, ny, inverse != 0, scale, p, s), "fft2");
}

int bpm_pupil_spectrum(const float* amplitude, const float* phase, int nx, int ny, double dx,
                       double wavelength, double n0, double z_focus, bpm_c64* spectrum_out,
                       void* hip_stream) {
    int rc = check_geom(nx, ny, 0, dx, 0.0, wavelength, n0);
    if (rc) return rc;
    if (!std::isfinite(z_focus)) return fail(BPM_ERR_NOT_FINITE, "z_focus must be finite");
    if (!amplitude || !phase || !spectrum_out)
        return fail(BPM_ERR_INVALID_ARG, "amplitude, phase and spectrum_out must be non-null");
    if (!aligned(amplitude, 4) || !aligned(phase, 4) || !aligned(spectrum_out, 8))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    const bpm::Geom g{nx, ny, 0, dx, 0.0, wavelength, n0};
    return device_status(bpm::launch_pupil_spectrum(amplitude, phase, g, z_focus, spectrum_out,
                                                    static_cast<hipStream_t>(hip_stream)),
                         "pupil spectrum");
}

int bpm_pupil_phase_grad(const bpm_c64* grad_spectrum, const bpm_c64* spectrum, int nx, int ny,
                         float* grad_phase, void* hip_stream) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(BPM_ERR_UNSUPPORTED_SIZE,
                    "nx=%d ny=%d: sizes must be powers of two in [32, 2048]", nx, ny);
    if (!grad_spectrum || !spectrum || !grad_phase)
        return fail(BPM_ERR_INVALID_ARG, "all arrays must be non-null");
    if (!aligned(grad_spectrum, 8) || !aligned(spectrum, 8) || !aligned(grad_phase, 4))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    return device_status(bpm::launch_pupil_grad(grad_spectrum, spectrum, (long)nx * ny,
                                                grad_phase, static_cast<hipStream_t>(hip_stream)),
                         "pupil phase gradient");
}

int bpm_guide_star_phase(const bpm_c64* grad_spectrum, int nx, int ny, double dx,
                         double wavelength, double n0, double z_focus, double shift_x,
                         double shift_y, float* phase_out, void* hip_stream) {
    int rc = check_geom(nx, ny, 0, dx, 0.0, wavelength, n0);
    if (rc) return rc;
    if (!std::isfinite(z_focus) || !std::isfinite(shift_x) || !std::isfinite(shift_y))
        return fail(BPM_ERR_NOT_FINITE, "z_focus, shift_x and shift_y must be finite");
    if (!grad_spectrum || !phase_out)
        return fail(BPM_ERR_INVALID_ARG, "grad_spectrum and phase_out must be non-null");
    if (!aligned(grad_spectrum, 8) || !aligned(phase_out, 4))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    const bpm::Geom g{nx, ny, 0, dx, 0.0, wavelength, n0};
    return device_status(bpm::launch_guide_star_phase(grad_spectrum, g, z_focus, shift_x, shift_y,
                                                      phase_out,
                                                      static_cast<hipStream_t>(hip_stream)),
                         "guide-star phase");
}

int bpm_adam_step(float* params, const float* grads, float* m, float* v, long n, float lr,
                  int step, void* hip_stream) {
    if (n < 0) return fail(BPM_ERR_INVALID_ARG, "n=%ld must be >= 0", n);
    if (step < 1) return fail(BPM_ERR_INVALID_ARG, "step=%d must be >= 1", step);
    if (!std::isfinite(lr)) return fail(BPM_ERR_NOT_FINITE, "lr must be finite");
    if (n == 0) return BPM_OK;
    if (!params || !grads || !m || !v)
        return fail(BPM_ERR_INVALID_ARG, "params, grads, m and v must be non-null");
    if (!aligned(params, 4) || !aligned(grads, 4) || !aligned(m, 4) || !aligned(v, 4))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    return device_status(bpm::sg::adam_update(params, grads, m, v, n, lr, step,
                                         static_cast<hipStream_t>(hip_stream)),
                         "Adam step");
}

size_t bpm_psf_readout_workspace_size(int nx, int ny, int planes) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny) || planes < 1 || planes > 256) return 0;
    return bpm::readout_bytes(nx, ny, planes);
}

int bpm_psf_readout(const bpm_c64* exit_field, int nx, int ny, double dx, double dz,
                    double wavelength, double n0, double na, int back_steps, const int* sources,
                    int n_src, int planes, int crop, double scale, float* psf_out,
                    void* workspace, size_t workspace_bytes, void* hip_stream) {
    int rc = check_geom(nx, ny, 0, dx, dz, wavelength, n0);
    if (rc) return rc;
    if (!std::isfinite(na) || !(na > 0) || !std::isfinite(scale))
        return fail(BPM_ERR_NOT_FINITE, "na=%g must be > 0 and scale finite", na);
    if (back_steps < 0 || n_src < 0 || planes < 1 || planes > 256 || crop < 1 ||
        crop > nx || crop > ny)
        return fail(BPM_ERR_INVALID_ARG,
                    "back_steps=%d, n_src=%d, planes=%d (1..256), crop=%d (1..min(nx, ny))",
                    back_steps, n_src, planes, crop);
    if (!exit_field || (n_src > 0 && (!sources || !psf_out)))
        return fail(BPM_ERR_INVALID_ARG, "exit_field, sources and psf_out must be non-null");
    if (!aligned(exit_field, 8) || (sources && !aligned(sources, 4)) ||
        (psf_out && !aligned(psf_out, 4)))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    if ((rc = check_workspace(workspace, workspace_bytes, bpm::readout_bytes(nx, ny, planes))))
        return rc;
    const bpm::ReadoutArgs r{exit_field, nx, ny, dx, dz, wavelength, n0, na, back_steps, sources,
                             n_src, planes, crop, scale, psf_out};
    return device_status(bpm::launch_readout(r, workspace, static_cast<hipStream_t>(hip_stream)),
                         "psf readout");
}

size_t bpm_pupil_fields_workspace_size(int nx, int ny) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny)) return 0;
    return bpm::pupil_fields_bytes(nx, ny);
}

static bool zernike_crop(int crop) { return crop == 16 || crop == 32 || crop == 64; }

int bpm_pupil_fields(const bpm_c64* exit_field, int nx, int ny, double dx, double dz,
                     double wavelength, double n0, double na, int back_steps, const int* sources,
                     int n_src, int crop, bpm_c64* pupil_out, void* workspace,
                     size_t workspace_bytes, void* hip_stream) {
    int rc = check_geom(nx, ny, 0, dx, dz, wavelength, n0);
    if (rc) return rc;
    if (!std::isfinite(na) || !(na > 0)) return fail(BPM_ERR_NOT_FINITE, "na=%g must be > 0", na);
    if (!zernike_crop(crop) || crop > nx || crop > ny)
        return fail(BPM_ERR_INVALID_ARG, "crop=%d must be 16, 32 or 64 and at most min(nx, ny)",
                    crop);
    if (back_steps < 0 || n_src < 0)
        return fail(BPM_ERR_INVALID_ARG, "back_steps=%d and n_src=%d must be >= 0", back_steps,
                    n_src);
    if (!exit_field || (n_src > 0 && (!sources || !pupil_out)))
        return fail(BPM_ERR_INVALID_ARG, "exit_field, sources and pupil_out must be non-null");
    if (!aligned(exit_field, 8) || (sources && !aligned(sources, 4)) ||
        (pupil_out && !aligned(pupil_out, 8)))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    if ((rc = check_workspace(workspace, workspace_bytes, bpm::pupil_fields_bytes(nx, ny))))
        return rc;
    const bpm::PupilFieldArgs r{exit_field, nx, ny, dx, dz, wavelength, n0, na, back_steps,
                                sources, n_src, crop, pupil_out};
    return device_status(bpm::launch_pupil_fields(r, workspace,
                                                  static_cast<hipStream_t>(hip_stream)),
                         "pupil fields");
}

// points (l', m') of the crop's signed DFT grid with l'^2 + m'^2 <= R^2
static int disc_points(int crop, double R) {
    int n = 0;
    for (int l = -crop / 2; l < crop / 2; ++l)
        for (int m = -crop / 2; m < crop / 2; ++m)
            if ((double)(l * l + m * m) <= R * R) ++n;
    return n;
}

size_t bpm_zernike_workspace_size(int crop, int n_modes) {
    if (!zernike_crop(crop) || n_modes < 1 || n_modes > bpm::kMaxZernike) return 0;
    return bpm::zernike_bytes(crop, n_modes);
}

int bpm_zernike_fit(const bpm_c64* pupil, int n_src, int crop, double dx, double wavelength,
                    double na, int n_modes, float* coeffs_out, float* rms_out, void* workspace,
                    size_t workspace_bytes, void* hip_stream) {
    if (!std::isfinite(dx) || !std::isfinite(wavelength) || !std::isfinite(na) || !(dx > 0) ||
        !(wavelength > 0) || !(na > 0))
        return fail(BPM_ERR_NOT_FINITE, "dx=%g, wavelength=%g and na=%g must be finite and > 0",
                    dx, wavelength, na);
    if (!zernike_crop(crop) || n_modes < 1 || n_modes > bpm::kMaxZernike || n_src < 0)
        return fail(BPM_ERR_INVALID_ARG,
                    "crop=%d must be 16, 32 or 64, n_modes=%d in 1..%d, n_src=%d >= 0", crop,
                    n_modes, bpm::kMaxZernike, n_src);
    const double R = na * crop * dx / wavelength;
    if (!(R < crop / 2 - 1))
        return fail(BPM_ERR_INVALID_ARG,
                    "the pupil disc (radius NA crop dx / wavelength = %g samples) must lie "
                    "inside the window's band (radius < %d)", R, crop / 2 - 1);
    const int disc_n = disc_points(crop, R);
    if (disc_n < 2 * n_modes)
        return fail(BPM_ERR_INVALID_ARG,
                    "the pupil disc holds %d samples, fewer than 2 n_modes = %d", disc_n,
                    2 * n_modes);
    if (n_src > 0 && (!pupil || !coeffs_out))
        return fail(BPM_ERR_INVALID_ARG, "pupil and coeffs_out must be non-null");
    if ((pupil && !aligned(pupil, 8)) || (coeffs_out && !aligned(coeffs_out, 4)) ||
        (rms_out && !aligned(rms_out, 4)))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    int rc = check_workspace(workspace, workspace_bytes, bpm::zernike_bytes(crop, n_modes));
    if (rc) return rc;
    const bpm::ZernikeArgs a{pupil, n_src, crop, n_modes, disc_n, dx, wavelength, na, coeffs_out,
                             rms_out};
    int ok = 0;
    rc = device_status(bpm::launch_zernike_fit(a, workspace, &ok,
                                               static_cast<hipStream_t>(hip_stream)),
                       "zernike fit");
    if (rc) return rc;
    if (!ok) return fail(BPM_ERR_INVALID_ARG, "the Zernike normal matrix is not positive definite");
    return BPM_OK;
}

int bpm_camera_accumulate(const float* excitation, const float* density,
                          const float* node_psfs, int nx, int ny, int pitch, int crop,
                          float* image, void* hip_stream) {
    if (nx < 32 || ny < 32 || nx % 32 || ny % 32 || nx > (1 << 16) || ny > (1 << 16))
        return fail(BPM_ERR_UNSUPPORTED_SIZE,
                    "nx=%d ny=%d: sizes must be multiples of 32 in [32, 65536]", nx, ny);
    if ((crop != 16 && crop != 32) || pitch < 2 || nx % pitch || ny % pitch ||
        nx / pitch < 2 || ny / pitch < 2)
        return fail(BPM_ERR_INVALID_ARG,
                    "crop=%d must be 16 or 32 and pitch=%d >= 2 must divide nx and ny at "
                    "least twice", crop, pitch);
    if (!excitation || !node_psfs || !image)
        return fail(BPM_ERR_INVALID_ARG, "excitation, node_psfs and image must be non-null");
    if (!aligned(excitation, 4) || !aligned(node_psfs, 4) || !aligned(image, 4) ||
        (density && !aligned(density, 4)))
        return fail(BPM_ERR_INVALID_ARG, "misaligned array");
    if (excitation == image || density == image)
        return fail(BPM_ERR_INVALID_ARG, "image must not alias excitation or density");
    return device_status(bpm::launch_camera(excitation, density, node_psfs, nx, ny, pitch, crop,
                                            image, static_cast<hipStream_t>(hip_stream)),
                         "camera image");
}

size_t bpm_point_sources_workspace_size(int nx, int ny) {
    if (!pow2_in_range(nx) || !pow2_in_range(ny)) return 0;
    return bpm::sources_bytes(nx, ny);
}

int bpm_point_sources(const int* positions, const float* phases, int n_src, int nx, int ny,
                      double dx, double wavelength, double n0, double na, double z_d,
                      bpm_c64* field_out, void* workspace, size_t workspace_bytes,
                      void* hip_stream) {
    int rc = check_geom(nx, ny, 0, dx, 1.0, wavelength, n0);
    if (rc) return rc;
    if (!std::isfinite(na) || !std::isfinite(z_d) || !(na > 0))
        return fail(BPM_ERR_NOT_FINITE, "na=%g must be finite and > 0, z_d=%g finite", na, z_d);
    if (n_src < 0) return fail(BPM_ERR_INVALID_ARG, "n_src=%d must be >= 0", n_src);
    if (n_src > 0 && (!positions || !aligned(positions, 4)))
        return fail(BPM_ERR_INVALID_ARG, "positions must be non-null and 4-byte aligned");
    if (phases && !aligned(phases, 4))
        return fail(BPM_ERR_INVALID_ARG, "phases must be 4-byte aligned");
    if (!field_out || !aligned(field_out, 8))
        return fail(BPM_ERR_INVALID_ARG, "field_out must be non-null and 8-byte aligned");
    if ((rc = check_workspace(workspace, workspace_bytes, bpm::sources_bytes(nx, ny)))) return rc;
    const bpm::SourceArgs a{positions, phases, n_src, nx, ny, dx, wavelength, n0, na, z_d,
                            field_out};
    return device_status(
        bpm::launch_point_sources(a, workspace, static_cast<hipStream_t>(hip_stream)),
        "point sources");
}

}  // extern "C"
