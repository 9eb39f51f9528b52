// Internal interface between the C-ABI host layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace bpm {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Kernels of the forward march (values of bpm.h's BPM_MARCH_*): one
// workgroup per CU with register twiddles; two per CU with LDS twiddles; the
// tiled march of one or two fields.  march_variant gives the one a march of `fields`
// lockstep fields of this geometry takes: the override set for the shape
// (bpm_set_march_variant, e.g. from the launch-shape tuner) when eligible,
// else the built-in choice.
enum MarchVariant : int { kMarchAuto = 0, kMarchOnePerCu = 1, kMarchTwoPerCu = 2,
                          kMarchTiledPair = 3, kMarchSmallBlocks = 4 };
bool march_variant_eligible(int nx, int ny, int fields, int variant);
int march_variant(int nx, int ny, int fields);
int set_march_variant(int nx, int ny, int fields, int variant);  // 0 ok, -1 ineligible
// whether such a march takes the tiled kernel (and so needs a tiled
// propagator table)
bool march_tiled(int nx, int ny, int fields);

// Geometry of one march, already validated.
struct Geom {
    int nx, ny, steps;
    double dx, dz, wavelength, n0;
};

// Device plan of one geometry, carved out of the caller's workspace:
// the propagator table in the march's storage order (1 / (nx ny) folded in),
// the twiddle tables tw[e] = exp(-2 pi i e / n), the storage-slot ->
// frequency tables of both axes and the grid-barrier words.
struct Plan {
    void* status;   // status header (kStatusBytes): [0] sticky time-out bits, [1..2] magic
    void* H;        // float2 [ny][nx]
    void* twx;      // float2 [nx]
    void* twy;      // float2 [ny]
    void* permx;    // int [nx]
    void* permy;    // int [ny]
    void* counter;  // grid-barrier words and time-out flag (4 KiB, zeroed by the plan)
};
// Every plan, and so every march-family workspace, starts with this header;
// the plan kernel initialises it once (when its magic is absent) and never
// clears the sticky bits, which only bpm_workspace_status reads and resets.
constexpr size_t kStatusBytes = 256;
constexpr unsigned kStatusMagic0 = 0x4d50425fu, kStatusMagic1 = 0x53555441u;
// host copies of the sticky bits the kernels set (passes.hpp)
constexpr unsigned kStatusBarrierBit = 1u, kStatusQueueBit = 2u;
// polls of one grid-barrier or queue wait before a kernel gives up
unsigned wait_limit();
size_t plan_bytes(int nx, int ny);
// compute units of the current device (0 when the query fails)
int device_cus();
Plan plan_carve(void* ws, int nx, int ny);
// tiled_h: the propagator table in the tiled layout of the two-field march
hipError_t launch_plan(const Geom& g, const Plan& p, bool with_h, hipStream_t s,
                       bool tiled_h = false);


// Forward march through `steps` slices; field_out doubles as working buffer.
// Up to kMaxFields fields of one geometry (one plan) march in lockstep in one
// launch.
constexpr int kMaxFields = 8;
struct MarchIO {
    const void* field_in;  // float2 [ny][nx]
    const float* dn;       // [steps][ny][nx]
    void* field_out;       // float2 [ny][nx]
    float* intensity;      // [steps][ny][nx] or nullptr
    int clear;             // leading steps without a screen (dn not read)
};
// timers: per-workgroup phase timers (diagnostic, see PhaseTimers) or null
// variant: the kernel (MarchVariant), kMarchAuto to resolve it here; a caller
// that built the plan for a tiled march passes the variant it resolved then
hipError_t launch_forward(const Geom& g, const Plan& p, const MarchIO* io, int fields,
                          hipStream_t s, unsigned long long* timers = nullptr,
                          int variant = kMarchAuto);
// words of the phase-timer buffer: a header and one record per workgroup
constexpr size_t kPhaseTimerWords = 8 + 8 * 4096;

// Forward march of one field with a per-slice reference index n0 + dn_ref[j]
// (locally adapted expansion; the plan needs no propagator table).
hipError_t launch_adapted(const Geom& g, const Plan& p, const void* field_in, const float* dn,
                          const float* dn_ref, void* field_out, float* intensity, hipStream_t s);
// dn_ref[j] = mean of slice j of dn ([steps][plane] float32)
hipError_t launch_slice_means(const float* dn, long plane, int steps, float* out, hipStream_t s);

// Adjoint march (steps >= 1) with a checkpoint every K steps; `fields` holds
// adjoint_fields(steps, K) fields of nx * ny complex64.
struct AdjointIO {
    const void* field_in;
    const float* dn;
    const void* grad_out;     // or nullptr
    const float* grad_inten;  // or nullptr
    void* grad_in;            // or nullptr
    void* grad_spec;          // or nullptr
    float* grad_dn;           // or nullptr
};
size_t adjoint_fields(int steps, int K);
// bytes of one field's checkpoints and work fields (256-byte aligned)
size_t adjoint_field_bytes(int nx, int ny, int steps, int K);
// n (1 .. kMaxFields) adjoints of one geometry in lockstep; `fields` holds n
// consecutive blocks of adjoint_field_bytes
hipError_t launch_adjoint(const Geom& g, const Plan& p, const AdjointIO* io, int n, int K,
                          void* fields, hipStream_t s);

// Natural-order 2-D DFT (exp(-) forward, exp(+) inverse, unnormalised, times
// `scale`); needs a plan built with or without the propagator.
hipError_t launch_fft2(const void* in, void* out, int nx, int ny, bool inverse, float scale,
                       const Plan& p, hipStream_t s);

// Uneven batch (batch.hip).  Device copy of one job and one segment of the
// item list: the `count` items of pass `pass` of job `job` start at item
// `first`; they may run once the job has completed `need` items.
struct BatchJob {
    const void* field_in;
    const float* dn;
    void* work;  // the job's field_out
    float* inten;
    const void* H;
    const void* twx;
    const void* twy;
    int nx, ny, steps;
    float k0dz;
    int clear;  // leading steps without a screen
    int tiled;  // field and propagator in the tiled layout between passes
};
// whether the work queue keeps a job of this size in the tiled layout
// (columns of >= 1024, nx >= 256, nx ny <= 2^20: there a column unit covers
// less than a line of the natural layout)
bool batch_tiled(int nx, int ny);
struct BatchSeg {
    int job, pass, first, count, need;
};
int batch_queue_words(int n_jobs);
constexpr int kUnitsPerItem = 4;  // units of one pass per work item (even)
int row_units(int nx, int ny);
int col_units(int nx, int ny);
int row_items(int nx, int ny);  // work items of one row pass
int col_items(int nx, int ny);  // work items of one column pass
hipError_t launch_batch(const BatchJob* jobs_dev, const BatchSeg* segs_dev, int total,
                        unsigned* q, int n_jobs, const unsigned long long* key_dev,
                        unsigned long long key, unsigned* status, hipStream_t s);

// PSF readout of a multiplexed run (readout.hip).
struct ReadoutArgs {
    const void* exit_field;
    int nx, ny;
    double dx, dz, wavelength, n0, na;
    int back_steps;
    const int* sources;  // device [n_src][2] (y, x)
    int n_src, planes, crop;
    double scale;
    float* psf_out;  // [n_src][planes][crop][crop]
};
size_t readout_bytes(int nx, int ny, int planes);
hipError_t launch_readout(const ReadoutArgs& r, void* ws, hipStream_t s);

// Pupil fields and Zernike fits of sample-induced aberrations (readout.hip).
constexpr int kMaxZernike = 28;
struct PupilFieldArgs {
    const void* exit_field;
    int nx, ny;
    double dx, dz, wavelength, n0, na;
    int back_steps;
    const int* sources;  // device [n_src][2] (y, x)
    int n_src, crop;
    void* pupil_out;  // float2 [n_src][crop][crop]
};
size_t pupil_fields_bytes(int nx, int ny);
hipError_t launch_pupil_fields(const PupilFieldArgs& r, void* ws, hipStream_t s);
struct ZernikeArgs {
    const void* pupil;  // float2 [n_src][crop][crop]
    int n_src, crop, n_modes, disc_n;
    double dx, wavelength, na;
    float* coeffs_out;  // [n_src][n_modes]
    float* rms_out;     // [n_src] or nullptr
};
size_t zernike_bytes(int crop, int n_modes);
hipError_t launch_zernike_fit(const ZernikeArgs& a, void* ws, int* host_ok, hipStream_t s);

// Camera image through spatially varying node PSFs (camera.hip).
hipError_t launch_camera(const float* excitation, const float* density, const float* node_psfs,
                         int nx, int ny, int pitch, int crop, float* image, hipStream_t s);

// Multiplexed point-source input field (sources.hip).
struct SourceArgs {
    const int* positions;  // device [n_src][2] (y, x)
    const float* phases;   // device [n_src] or nullptr (all zero)
    int n_src, nx, ny;
    double dx, wavelength, n0, na, z_d;
    void* field_out;  // float2 [ny][nx]
};
size_t sources_bytes(int nx, int ny);
hipError_t launch_point_sources(const SourceArgs& a, void* ws, hipStream_t s);

// PSF surrogate kernels (surrogate.hip).  Activations are channels-last
// bf16; a convolution's reduction index is (tap, channel), channel fastest.
struct ConvGeo {
    int N, D, H, W, Ci;           // input [N][D][H][W][Ci]
    int Co, kd, kh, kw, sd, sh, sw, pd, ph, pw;
    int Do, Ho, Wo;               // output [N][Do][Ho][Wo][Co]
    int taps, K, Kp;              // taps = kd kh kw, K = taps Ci, Kp = K rounded up to 16
};
// forward tile of a workgroup: TY output rows x Wo columns of one (n, oz)
// plane; its input footprint kd x FY x FX voxels with channel stride CiP
struct FwdTile {
    int TY, FY, FX, CiP, tiles_y;
};
namespace sg {
constexpr size_t kMaxConvLds = 65536;  // dynamic LDS of one forward workgroup
FwdTile fwd_tile(const ConvGeo& c);
size_t fwd_lds_bytes(const ConvGeo& c);
// in_mode 0: x is bf16 channels-last; 1 (with epi 0): x is the fp32 dn patch
// [N][64][32][32] and the input channels are formed while staging (depth[N]);
// 2 (with epi 1): x is the bf16 map at half the height and width, read
// through a nearest x2 upsampling
hipError_t conv_forward(const ConvGeo& c, const void* x, const void* w, const float* bias,
                        const int4* taps, int epi, void* ybf, float* yf, float* zkeep,
                        hipStream_t s, int in_mode = 0, const float* depth = nullptr);
hipError_t conv_backward_data(const ConvGeo& c, const void* dy, const void* wt,
                              const void* xact, const int4* taps_t, void* dx, hipStream_t s);
hipError_t conv_backward_weight(const ConvGeo& c, const void* x, const void* dy,
                                const int4* taps, float* dw, float* db, hipStream_t s);
hipError_t prep_input(const float* dn, const float* depth, int B, void* x0, hipStream_t s);
hipError_t extract_patches(const float* dn, int ny, int nx, int z0, const int* src, int n,
                           float* out, hipStream_t s);
hipError_t upsample(const void* a, int N, int h, int w, int C, void* u, hipStream_t s);
hipError_t upsample_backward(const void* du, const void* a, const float* dpool, int N, int h,
                             int w, int C, void* da, hipStream_t s);
hipError_t head_forward(const void* a, int N, int hw, int C, const float* we, const float* be,
                        float* pooled, float* epre, float* err, hipStream_t s);
hipError_t loss_and_grad(const float* psf, const float* z, const float* target,
                         const float* epre, const float* err, int B, float lambda, void* dy,
                         float* derr_pre, float* loss, float* err_true, hipStream_t s);
hipError_t head_backward(const float* pooled, const float* dpre, const float* we, int B, int C,
                         float* dwe, float* dbe, float* dpool, hipStream_t s);
hipError_t adam_update(float* w, const float* g, float* m, float* v, long n, float lr, int step,
                       hipStream_t s);
hipError_t pack_weights(const float* wf, int Co, int Ci, int taps, int Kp, void* wb, void* wt,
                        hipStream_t s);
hipError_t tap_tables(const ConvGeo& c, int4* taps, int4* taps_t, hipStream_t s);
hipError_t fill_zero(float* p, long n, hipStream_t s);
}  // namespace sg

// Pupil plane of the adaptive-optics gradient.
hipError_t launch_pupil_spectrum(const float* amp, const float* phase, const Geom& g, double z_f,
                                 void* U, hipStream_t s);
hipError_t launch_pupil_grad(const void* G, const void* U, long n, float* gphi, hipStream_t s);
hipError_t launch_guide_star_phase(const void* G, const Geom& g, double z_f, double sx, double sy,
                                   float* phase, hipStream_t s);

}  // namespace bpm
