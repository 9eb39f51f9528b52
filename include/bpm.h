/*
 * bpm.h -- C ABI of the MI355X beam-propagation library (libbpm.so).
 *
 * The library marches a complex light field slice by slice through a
 * refractive-index volume with the split-step beam-propagation method using
 * the exact (non-paraxial) propagator (Weigert, Myers & Kreysing, "Biobeam",
 * arXiv 1706.02261, main text, paragraph on the beam-propagation model and
 * the multiplexed PSF calculation).  One step j = 0 .. steps-1 is
 *
 *     v       = IDFT2( H . DFT2(u_j) ),
 *     H[l][m] = exp(i dz sqrt(k^2 - kx^2 - ky^2))  where kx^2 + ky^2 <= k^2, else 0,
 *     u_{j+1} = exp(i k0 dz dn[j]) . v,
 *     I[j]    = |u_{j+1}|^2,
 *
 * with k0 = 2 pi / wavelength, k = n0 k0, kx = 2 pi m~ / (nx dx),
 * ky = 2 pi l~ / (ny dx) (m~, l~ the signed DFT indices), DFT2 unnormalised
 * with exp(-2 pi i ...), IDFT2 with exp(+...) and 1 / (nx ny).  The
 * propagating test is evaluated exactly on integers:
 * (m~ ny)^2 + (l~ nx)^2 <= (nx ny n0 dx / wavelength)^2.
 *
 * Conventions common to every entry point
 *   - Lengths in micrometres; `wavelength` is the vacuum wavelength; dn = n - n0.
 *   - Complex arrays are complex64: interleaved (re, im) float32, the memory
 *     layout of torch.complex64.  Fields are [ny][nx], volumes are
 *     [steps][ny][nx], x fastest, densely packed.
 *   - Every pointer argument is a DEVICE pointer unless stated otherwise; the
 *     caller owns all memory (inputs, outputs and the workspace).  The library
 *     keeps no pointer after the call's stream work has completed and never
 *     frees caller memory.
 *   - Calls are asynchronous on `hip_stream` (a hipStream_t; NULL = the null
 *     stream).  Argument errors are detected on the host before any launch
 *     and leave every output untouched.  A launch failure is reported as
 *     BPM_ERR_DEVICE; a fault inside a kernel surfaces at the caller's next
 *     synchronising call.
 *   - Supported lateral sizes: nx, ny powers of two in [32, 2048] (square
 *     pixels, dy = dx).  Other sizes return BPM_ERR_UNSUPPORTED_SIZE.
 *   - Return value: BPM_OK or a negative error code; bpm_last_error() gives a
 *     message for the calling thread's last failed call.
 *   - Gradients follow PyTorch's complex convention g = dL/dRe + i dL/dIm.
 */
#ifndef BPM_H
#define BPM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float re, im;
} bpm_c64;

enum {
    BPM_OK = 0,
    BPM_ERR_INVALID_ARG = -1,      /* null pointer, negative count, bad flag     */
    BPM_ERR_UNSUPPORTED_SIZE = -2, /* nx, ny not a power of two in [32, 2048]    */
    BPM_ERR_WORKSPACE = -3,        /* workspace missing, too small or misaligned */
    BPM_ERR_DEVICE = -4,           /* a HIP call or kernel launch failed         */
    BPM_ERR_NOT_FINITE = -5        /* non-finite or non-positive geometry        */
};

/* Workspace flags for bpm_workspace_size. */
enum {
    BPM_WS_FORWARD = 0, /* bpm_propagate                                       */
    BPM_WS_ADJOINT = 1  /* bpm_adjoint with the default checkpoint interval    */
};

/* Bytes of device workspace a call needs (alignment: 256 bytes).  Returns 0
 * for unsupported arguments.  The forward march needs the propagator table
 * (nx * ny complex64) and twiddle tables; the adjoint adds its checkpoints. */
size_t bpm_workspace_size(int nx, int ny, int steps, int flags);

/* Forward march (the paper's BPM with the exact propagator, main-text
 * paragraph on the method).
 *   field_in       [ny][nx] complex64, the field u_0 at the entry plane.
 *   dn             [steps][ny][nx] float32, n - n0 of each slice (may be NULL
 *                  only when steps == 0).
 *   steps          >= 0; steps == 0 copies field_in to field_out.
 *   dx, dz         lateral pixel and slice thickness (um); dx > 0, dz finite.
 *   wavelength, n0 vacuum wavelength (um) and background index, both > 0.
 *   field_out      [ny][nx] complex64, receives u_steps; may alias field_in.
 *                  Also used as the march's working buffer.
 *   intensity_out  [steps][ny][nx] float32 receiving I[j] = |u_{j+1}|^2, or
 *                  NULL to skip the intensity volume.
 *   workspace      device memory of at least
 *                  bpm_workspace_size(nx, ny, steps, BPM_WS_FORWARD) bytes,
 *                  256-byte aligned; rewritten by every call, so calls that
 *                  share a workspace must not overlap in time.
 */
int bpm_propagate(const bpm_c64* field_in, const float* dn, int nx, int ny, int steps,
                  double dx, double dz, double wavelength, double n0,
                  bpm_c64* field_out, float* intensity_out,
                  void* workspace, size_t workspace_bytes, void* hip_stream);

/* Forward march with a locally adapted expansion of the refractive index
 * (the paper's exact propagator "together with a locally adapted expansion
 * of refractive indices", main-text paragraph on the method; its details are
 * not part of the text, the reading here is a per-slice reference index).
 * Slice j is expanded about nr_j = n0 + dn_ref[j]: the step propagates with
 * the exact propagator of a homogeneous medium of index nr_j,
 *     H_j = exp(i dz sqrt((nr_j k0)^2 - kx^2 - ky^2)),  0 where kx^2 + ky^2 > (nr_j k0)^2
 * (integer test with nr_j for n0), and screens with the remainder,
 *     u_{j+1} = exp(i k0 dz (dn[j] - dn_ref[j])) . IDFT2(H_j . DFT2(u_j)),
 * so a slice homogeneous at nr_j is propagated exactly.  dn_ref = 0 gives the
 * march of bpm_propagate (to rounding: H_j is formed on the fly in FP64 and
 * turned into an FP32 phasor, not read from a table).
 *   dn_ref    device float32 [steps], reference index offsets; n0 + dn_ref[j]
 *             must be > 0 (not checked: values on the device); e.g. the slice
 *             means of bpm_slice_means.
 * Other arguments, the workspace (bpm_workspace_size(.., BPM_WS_FORWARD)) and
 * errors as in bpm_propagate.  One field, one workgroup per CU. */
int bpm_propagate_adapted(const bpm_c64* field_in, const float* dn, const float* dn_ref, int nx,
                          int ny, int steps, double dx, double dz, double wavelength, double n0,
                          bpm_c64* field_out, float* intensity_out, void* workspace,
                          size_t workspace_bytes, void* hip_stream);

/* dn_ref[j] = mean over slice j of dn ([steps][ny][nx] float32 -> [steps]
 * float32), summed in FP64 in a fixed order (deterministic). */
int bpm_slice_means(const float* dn, int nx, int ny, int steps, float* dn_ref, void* hip_stream);

/* One job of an uneven batch (host struct; its pointers are device pointers
 * with the meaning and layout of bpm_propagate's arguments). */
typedef struct {
    const bpm_c64* field_in;
    const float* dn;
    int nx, ny, steps;
    double dx, dz, wavelength, n0;
    bpm_c64* field_out;
    float* intensity_out;
    /* Steps at the start that propagate in the background medium: for
     * j < clear_steps the screen is skipped (dn[j] is taken as 0 and never
     * read).  0 .. steps.  With a source entered clear_steps slices early as
     * the clear-medium field that focuses clear_steps dz downstream, the job
     * leaves the volume exactly as the source marched from slice clear_steps
     * (free-space steps compose), so sources of different depths can march
     * in one lockstep launch of equal-length jobs. */
    int clear_steps;
} bpm_job;

/* Bytes of workspace for bpm_propagate_batch over `jobs` (host array). */
size_t bpm_batch_workspace_size(const bpm_job* jobs, int n_jobs);

/* Uneven batch: every job is an independent march (the paper's multiplexed
 * fields, light-sheet positions and volumes; main-text paragraphs on
 * multiplexing and on the light-sheet simulation), all run by ONE persistent
 * kernel launch that pulls (job, pass, tile) work items from a device queue;
 * per-job counters order each job's passes, so jobs of different size and
 * depth overlap freely.  `jobs` is a host array of n_jobs >= 1 entries, each
 * validated as in bpm_propagate; jobs must not share output buffers.
 * When every job has the same nx, ny, steps (> 0), dx, dz, wavelength and n0
 * and there are at most 8 of them, the jobs instead march in lockstep in the
 * cooperative march kernel of bpm_propagate (one plan, every pass covering the
 * units of all jobs, the two grid barriers of a step shared).
 * Results are identical, bit for bit, to n_jobs separate bpm_propagate calls. */
int bpm_propagate_batch(const bpm_job* jobs, int n_jobs,
                        void* workspace, size_t workspace_bytes, void* hip_stream);

/* The uneven batch in two halves, so that the device half can be captured
 * into a HIP graph (stream capture) and replayed.  Both always take the
 * work-queue path (never the lockstep one) and produce, bit for bit, the
 * results of bpm_propagate_batch; workspace size as for bpm_propagate_batch.
 *
 * bpm_batch_upload: builds the job and segment tables on the host and copies
 *   them into `workspace` on `hip_stream` (through library-owned pinned
 *   staging), together with a 64-bit key of the jobs and the workspace
 *   address.  Must not be called while `hip_stream` is capturing
 *   (BPM_ERR_INVALID_ARG).
 * bpm_batch_launch: kernel launches and device-to-device copies only: the
 *   per-job propagator tables, the copies of zero-step jobs, the queue reset
 *   and the persistent batch kernel.  It reads the tables that
 *   bpm_batch_upload left in `workspace` for the same `jobs` array contents;
 *   if the workspace holds no tables or those of other jobs (the key differs)
 *   the batch kernel returns at once and the outputs of jobs with steps > 0
 *   are left untouched.  The caller must not modify the workspace between
 *   upload and launch (or replays of a captured launch).
 * Arguments are validated on the host as in bpm_propagate_batch. */
int bpm_batch_upload(const bpm_job* jobs, int n_jobs,
                     void* workspace, size_t workspace_bytes, void* hip_stream);
int bpm_batch_launch(const bpm_job* jobs, int n_jobs,
                     void* workspace, size_t workspace_bytes, void* hip_stream);

/* Diagnostic: the lockstep march of bpm_propagate_batch (1 to 8 jobs of one
 * geometry, steps >= 1; other batches return BPM_ERR_INVALID_ARG) with
 * per-workgroup phase timers.  Results are those of bpm_propagate_batch.
 * timers: device buffer of at least BPM_PHASE_TIMER_WORDS 64-bit words,
 * 8-byte aligned; the call zeroes it, then writes words 0..3 = {workgroups,
 * counter ticks per second, steps, fields} and, for workgroup w, 8 words at
 * 8 (w + 1): ticks spent in {set-up, head pass, column passes, row passes,
 * draining stores before grid barriers, waiting at grid barriers, 0, 0}.
 * Workspace as for bpm_propagate_batch. */
#define BPM_PHASE_TIMER_WORDS (8 + 8 * 4096)
int bpm_march_phase_times(const bpm_job* jobs, int n_jobs, void* workspace,
                          size_t workspace_bytes, unsigned long long* timers,
                          size_t timer_bytes, void* hip_stream);

/* Bytes of workspace for bpm_adjoint with an explicit checkpoint interval
 * (0 selects ceil(sqrt(steps))). */
size_t bpm_adjoint_workspace_size(int nx, int ny, int steps, int checkpoint_every);

/* Adjoint march: gradients of a real loss L(u_steps, I) through bpm_propagate
 * (reverse-mode differentiation of the step above).  The forward fields are
 * not stored: the call re-runs the forward march keeping one field every
 * `checkpoint_every` steps, then, segment by segment from the last, recomputes
 * the segment's fields and runs the adjoint steps
 *     g_{j+1} += 2 gI[j] u_{j+1},
 *     grad_dn[j] = k0 dz Im(g_{j+1} conj(u_{j+1})),
 *     g_j = IDFT2( conj(H) . DFT2( exp(-i k0 dz dn[j]) g_{j+1} ) ).
 *   grad_field_out   [ny][nx] dL/du_steps, or NULL (zero).
 *   grad_intensity   [steps][ny][nx] float32 dL/dI, or NULL (zero).
 *   grad_field_in    [ny][nx] receives dL/du_0, or NULL.
 *   grad_spectrum_in [ny][nx] receives dL/dU_0 for u_0 = IDFT2(U_0), i.e.
 *                    DFT2(g_0) / (nx ny) in natural DFT order, or NULL; this
 *                    is the pupil-plane gradient used for adaptive optics.
 *   grad_dn          [steps][ny][nx] receives dL/ddn, or NULL.
 *   checkpoint_every 0 (= ceil(sqrt(steps))) or 1 .. steps.
 * Other arguments as in bpm_propagate.  Results do not depend on
 * checkpoint_every (bitwise).  With grad_intensity and grad_dn both NULL the
 * adjoint is the linear map M^H applied to grad_field_out (for a point at a
 * focus: the guide star's field conjugated back to the entrance plane); the
 * call then skips the forward march and field_in may be NULL; otherwise a
 * NULL field_in is BPM_ERR_INVALID_ARG. */
int bpm_adjoint(const bpm_c64* field_in, const float* dn, int nx, int ny, int steps,
                double dx, double dz, double wavelength, double n0,
                const bpm_c64* grad_field_out, const float* grad_intensity,
                bpm_c64* grad_field_in, bpm_c64* grad_spectrum_in, float* grad_dn,
                int checkpoint_every, void* workspace, size_t workspace_bytes,
                void* hip_stream);

/* Several adjoints of one geometry (the same nx, ny, steps, dx, dz,
 * wavelength, n0 and checkpoint interval) in one lockstep launch: every pass
 * covers the units of all fields, so the fields share each grid barrier
 * (throughput for several guide stars or losses; one adjoint is latency
 * bound).  One job per field, each with the pointers of bpm_adjoint and the
 * same meaning and NULL rules; the jobs' outputs must not overlap each other
 * or any input.  Results are bitwise those of separate bpm_adjoint calls.
 * When no job gives grad_intensity or grad_dn the launch takes the linear
 * path of bpm_adjoint; otherwise it runs the forward march of every job that
 * gives field_in (a job without one must be linear, as in bpm_adjoint).
 *   n_fields  1 .. BPM_MAX_LOCKSTEP_FIELDS, else BPM_ERR_INVALID_ARG.
 *   workspace bpm_adjoint_batch_workspace_size(n_fields, ...) bytes,
 *             256-byte aligned: the plan and each field's checkpoints. */
#define BPM_MAX_LOCKSTEP_FIELDS 8
typedef struct bpm_adjoint_job {
    const bpm_c64* field_in;
    const float* dn;
    const bpm_c64* grad_field_out;
    const float* grad_intensity;
    bpm_c64* grad_field_in;
    bpm_c64* grad_spectrum_in;
    float* grad_dn;
} bpm_adjoint_job;
/* 0 for n_fields outside 1 .. BPM_MAX_LOCKSTEP_FIELDS or arguments that
 * bpm_adjoint_workspace_size rejects. */
size_t bpm_adjoint_batch_workspace_size(int n_fields, int nx, int ny, int steps,
                                        int checkpoint_every);
int bpm_adjoint_batch(const bpm_adjoint_job* jobs, int n_fields, int nx, int ny, int steps,
                      double dx, double dz, double wavelength, double n0, int checkpoint_every,
                      void* workspace, size_t workspace_bytes, void* hip_stream);

/* Bytes of workspace for bpm_fft2. */
size_t bpm_fft2_workspace_size(int nx, int ny);

/* Natural-order 2-D DFT of a [ny][nx] complex64 array (helper of the pupil
 * plane; the march itself never leaves its own storage order).  inverse = 0:
 * X[l][m] = sum x[y][x] exp(-2 pi i (m x / nx + l y / ny)), unnormalised;
 * inverse = 1: exp(+...) and 1 / (nx ny).  `out` may alias `in`.  Workspace:
 * bpm_fft2_workspace_size bytes, 256-byte aligned. */
int bpm_fft2(const bpm_c64* in, bpm_c64* out, int nx, int ny, int inverse,
             void* workspace, size_t workspace_bytes, void* hip_stream);

/* Pupil-plane field of the adaptive-optics problem (the paper's guide-star
 * wavefront conjugation, main-text paragraph on adaptive optics): the angular
 * spectrum U0[l][m] = A exp(i phi) exp(-i kz z_focus), natural DFT order, with
 * kz = sqrt(k^2 - kx^2 - ky^2) (0 where evanescent) and k = 2 pi n0 /
 * wavelength.  amplitude and phase are [ny][nx] float32; the entry field of
 * the march is bpm_fft2(U0, inverse = 1). */
int bpm_pupil_spectrum(const float* amplitude, const float* phase, int nx, int ny, double dx,
                       double wavelength, double n0, double z_focus, bpm_c64* spectrum_out,
                       void* hip_stream);

/* dL/dphi = Im(dL/dU0 * conj(U0)) from bpm_adjoint's grad_spectrum_in and the
 * spectrum U0 of bpm_pupil_spectrum ([ny][nx] each; grad_phase float32). */
int bpm_pupil_phase_grad(const bpm_c64* grad_spectrum, const bpm_c64* spectrum, int nx, int ny,
                         float* grad_phase, void* hip_stream);

/* Guide-star correction (main-text paragraph on adaptive optics: conjugating
 * the wavefront of a point-like guide star at the sample surface gives a
 * diffraction-limited focus inside scattering tissue).  grad_spectrum is
 * G = dL/dU0 of bpm_adjoint with grad_field_out a point at the focus and no
 * other gradient (G = DFT2(M^H e_f) / (nx ny)).  The focus amplitude
 * u(x_f) = sum conj(G) U0 is largest over |U0| = A when every mode of
 * U0 = A exp(i phi) exp(-i kz z_focus) has the phase of G, so the call writes
 *     phase_out = arg G + kz z_focus - kx shift_x - ky shift_y   in [-pi, pi),
 * kx, ky, kz on the natural DFT grid as in bpm_pupil_spectrum.  A nonzero
 * (shift_x, shift_y) (micrometres) moves the corrected entrance field by that
 * vector (the shifted correction of a memory-effect measurement).  Arrays
 * [ny][nx]: grad_spectrum complex64, phase_out float32. */
int bpm_guide_star_phase(const bpm_c64* grad_spectrum, int nx, int ny, double dx,
                         double wavelength, double n0, double z_focus, double shift_x,
                         double shift_y, float* phase_out, void* hip_stream);

/* One Adam update (Kingma & Ba 2015, Algorithm 1: beta1 0.9, beta2 0.999,
 * eps 1e-8) of n float32 parameters in place, with the moments m and v
 * (zero before step 1) updated in place and 1-based step `step` for the bias
 * corrections:  m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
 * params -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * The optimiser of the adaptive-optics pupil phase; the same kernel updates
 * the PSF surrogate.  Device arrays, 4-byte aligned. */
int bpm_adam_step(float* params, const float* grads, float* m, float* v, long n, float lr,
                  int step, void* hip_stream);

/* Bytes of workspace for bpm_psf_readout. */
size_t bpm_psf_readout_workspace_size(int nx, int ny, int planes);

/* PSF readout of a multiplexed run through the idealised refocusing lens of
 * the detection path (main-text paragraph on the light-sheet simulation: the
 * multiplexed point sources are propagated through the sample and an
 * idealised, refocusing lens to the camera, giving the spatially varying
 * PSFs).  exit_field is the field after a march that started at the source
 * plane back_steps slices earlier.  With P the detection pupil
 * [kx^2 + ky^2 <= (2 pi NA / wavelength)^2] (integer test as for the
 * propagator):
 *   S   = DFT2(exit) . P . exp(-i kz back_steps dz)
 *   E_m = IDFT2(S . exp(i kz m dz)),  m = -planes/2 .. planes/2 - 1
 *   psf[s][m + planes/2][y][x] = scale |E_m(sy - crop/2 + y, sx - crop/2 + x)|^2
 * (periodic indices).  sources: device int32 [n_src][2] = (sy, sx) pixels;
 * psf_out: device float32 [n_src][planes][crop][crop]; planes in 1..256,
 * crop in 1..min(nx, ny).  Workspace: bpm_psf_readout_workspace_size bytes. */
int bpm_psf_readout(const bpm_c64* exit_field, int nx, int ny, double dx, double dz,
                    double wavelength, double n0, double na, int back_steps, const int* sources,
                    int n_src, int planes, int crop, double scale, float* psf_out,
                    void* workspace, size_t workspace_bytes, void* hip_stream);

/* Bytes of workspace for bpm_pupil_fields. */
size_t bpm_pupil_fields_workspace_size(int nx, int ny);

/* Pupil fields of the sources of a multiplexed run (main-text paragraph on
 * the light-sheet simulation: sample-induced aberrations extracted as
 * spatially resolved Zernike maps).  With the detection pupil P and the
 * refocusing of bpm_psf_readout, the complex source plane is
 *     E0 = IDFT2( DFT2(exit) . P . exp(-i kz back_steps dz) )
 * and source s = (sy, sx) gets the 2-D DFT of its crop x crop window, the
 * source at window index (crop/2, crop/2):
 *     pupil[s][l][m] = sum_{y,x < crop} E0(sy - crop/2 + y, sx - crop/2 + x)
 *                      exp(-2 pi i (l y + m x) / crop)      (periodic indices).
 * sources: device int32 [n_src][2]; pupil_out: device complex64
 * [n_src][crop][crop], natural DFT order; crop 16, 32 or 64 (at most
 * min(nx, ny)).  Workspace: bpm_pupil_fields_workspace_size bytes. */
int bpm_pupil_fields(const bpm_c64* exit_field, int nx, int ny, double dx, double dz,
                     double wavelength, double n0, double na, int back_steps, const int* sources,
                     int n_src, int crop, bpm_c64* pupil_out, void* workspace,
                     size_t workspace_bytes, void* hip_stream);

/* Bytes of workspace for bpm_zernike_fit (0 for unsupported arguments). */
size_t bpm_zernike_workspace_size(int crop, int n_modes);

/* Zernike coefficients of the pupil fields of bpm_pupil_fields.  On the disc
 * D = {l'^2 + m'^2 <= R^2}, R = NA crop dx / wavelength (signed frequency
 * indices l', m'; R < crop/2 - 1 and at least 2 n_modes samples, else
 * BPM_ERR_INVALID_ARG), rho = sqrt(l'^2 + m'^2) / R, theta = atan2(l', m'):
 *   Y = pupil (-1)^(l + m); t_x = arg sum Y(l, m+1) conj Y(l, m) over pairs
 *   in D, t_y likewise along l; p0 = arg sum_D Y exp(-i (t_x m' + t_y l'));
 *   T = t_x m' + t_y l' + p0; W = wrap(arg Y - T) + T  (wrap to [-pi, pi));
 *   c = P W, then twice c += P wrap(W - Z c), with Z[i][j] = Z_{j+1}(rho_i,
 *   theta_i) the Noll-normalised Zernike polynomials (Noll 1976; unit mean
 *   square on the unit disc) and P = (Z^T Z)^-1 Z^T over D;
 *   rms = sqrt(mean_D wrap(W - Z c)^2).
 * The coefficients are radians of pupil phase: c_1 piston, c_2 / c_3 tilt
 * (a lateral source shift s gives c_2 = -k0 NA s_x / 2), c_4 defocus, ...
 * coeffs_out: device float32 [n_src][n_modes] (n_modes 1..28); rms_out:
 * [n_src] or NULL.  The fit assumes the phase after tilt removal varies by
 * less than pi between neighbouring samples; rms reports what it leaves.
 * Workspace: bpm_zernike_workspace_size bytes.  The call waits for the basis
 * set-up on its stream. */
int bpm_zernike_fit(const bpm_c64* pupil, int n_src, int crop, double dx, double wavelength,
                    double na, int n_modes, float* coeffs_out, float* rms_out, void* workspace,
                    size_t workspace_bytes, void* hip_stream);

/* Camera image of a fluorescent object (Fig. 1c; main-text paragraph on the
 * light-sheet simulation: the spatially varying PSFs convolved with the
 * fluorescent object give the image seen by the camera).  Fluorescence adds
 * intensities; the slab of one depth, with emission E = excitation x density
 * (density NULL: E = excitation), adds
 *     image(x) += sum_{x'} E(x') sum_g phi_g(x') PSF_g(x - x'),
 * PSF_g the crop x crop PSF of node g in the camera's focal plane (centre
 * index crop/2 = the emitter), nodes on a pitch grid at pixel
 * (pitch/2 + pitch i, pitch/2 + pitch j), phi_g the periodic bilinear hat
 * weights max(0, 1 - |dy|/pitch) max(0, 1 - |dx|/pitch) (a partition of
 * unity), periodic indices.
 *   excitation, density [ny][nx] float32 (density may be NULL)
 *   node_psfs  [ny/pitch][nx/pitch][crop][crop] float32
 *   image      [ny][nx] float32, accumulated in place (must not alias the
 *              other arrays)
 * nx, ny multiples of 32; pitch divides both, at least twice (two nodes per
 * period keep the weights a partition of unity); crop 16 or 32.  Every output
 * pixel is summed by one thread in a fixed order (deterministic). */
int bpm_camera_accumulate(const float* excitation, const float* density,
                          const float* node_psfs, int nx, int ny, int pitch, int crop,
                          float* image, void* hip_stream);

/* Bytes of workspace for bpm_point_sources. */
size_t bpm_point_sources_workspace_size(int nx, int ny);

/* Multiplexed point-source input field (main-text paragraph on multiplexing:
 * many point sources ride in one field and one march):
 *   u0 = sum_i exp(i phase_i) shift(u_src, p_i)     (integer circular shifts)
 *   u_src = IDFT2(S) / ||IDFT2(S)||_2,
 *   S(k) = exp(-(kt / (k0 NA))^2) [kt <= k0 NA] exp(-i kz z_d),
 * a Gaussian-apodised NA-limited point source whose focus lies z_d um after
 * the input plane (z_d = 0: focused in the input plane), kz = sqrt(k^2 - kt^2),
 * k = 2 pi n0 / wavelength, pupil by the integer test of bpm_psf_readout.
 *   positions  device int32 [n_src][2] = (y, x) pixels (taken modulo ny, nx);
 *   phases     device float32 [n_src] radians, or NULL for all zero;
 *   field_out  device complex64 [ny][nx].
 * n_src = 0 gives a zero field.  Coinciding positions add (float atomics, so
 * the rounding of such sums does not depend on a fixed order). */
int bpm_point_sources(const int* positions, const float* phases, int n_src, int nx, int ny,
                      double dx, double wavelength, double n0, double na, double z_d,
                      bpm_c64* field_out, void* workspace, size_t workspace_bytes,
                      void* hip_stream);

/* Learned PSF surrogate, inference (the paper's sets of 10^5 - 10^6 spatially
 * varying PSFs, abstract and main-text paragraph on image formation; the
 * network and its training entries are in psf_surrogate.h).
 *   weights_bf16   device blob written by psf_surrogate_export (256-byte
 *                  aligned); weights_bytes must equal psf_surrogate_weights_bytes().
 *   dn_patches     [batch][64][32][32] float32 local dn patches (z, y, x).
 *   depth          [batch] float32 source depth in slices (0 .. 63).
 *   psf_out        [batch][32][32][32] float32 PSF intensity (plane, y, x).
 *   pred_err       [batch] float32 predicted relative L2 error of each PSF.
 *   workspace      psf_surrogate_workspace_size(batch, 0) bytes, 256-byte
 *                  aligned; batches are processed in chunks of 1024 samples.
 * BF16 operands, FP32 accumulation on the matrix cores.  batch = 0 is a no-op. */
int psf_surrogate_infer(const void* weights_bf16, size_t weights_bytes,
                        const float* dn_patches, const float* depth, int batch,
                        float* psf_out, float* pred_err, void* workspace,
                        size_t workspace_bytes, void* hip_stream);

/* Kernels of the forward march (bpm_propagate, and the lockstep path of
 * bpm_propagate_batch for 1-8 jobs of one geometry), chosen per shape
 * (nx, ny, number of lockstep fields):
 *   BPM_MARCH_ONE_PER_CU   one 256-thread workgroup per CU, twiddles in
 *                          registers, a workgroup's units two at a time;
 *   BPM_MARCH_TWO_PER_CU   two workgroups per CU, twiddles in LDS (nx, ny >= 512);
 *   BPM_MARCH_TILED_PAIR   one or two fields with a grid barrier each, one
 *                          workgroup per CU and field (two fields: the two
 *                          workgroups of a CU hold different fields), the
 *                          field kept in 128-byte tiles between passes (one or
 *                          two fields with nx ny = 2^20 on a device of 256 CUs);
 *   BPM_MARCH_SMALL_BLOCKS 64-thread workgroups, up to four per CU, twiddles in
 *                          registers (nx, ny <= 1024): four times as many
 *                          units per pass, for fields too small to give
 *                          every CU a 256-thread unit;
 *   BPM_MARCH_AUTO         the built-in choice (tiled pair where eligible, two
 *                          per CU for several fields of sides >= 512, small
 *                          blocks for one field of sides <= 512, else one).
 * All give bit-identical results.  A launch-shape tuner (the package's
 * tune.py) times the eligible kernels of a shape on the device and records
 * the fastest with bpm_set_march_variant. */
enum {
    BPM_MARCH_AUTO = 0,
    BPM_MARCH_ONE_PER_CU = 1,
    BPM_MARCH_TWO_PER_CU = 2,
    BPM_MARCH_TILED_PAIR = 3,
    BPM_MARCH_SMALL_BLOCKS = 4
};
/* The kernel a march of this shape takes now (BPM_MARCH_ONE_PER_CU ..), or
 * BPM_ERR_INVALID_ARG for unsupported sizes or fields outside 1 .. 8. */
int bpm_march_variant(int nx, int ny, int fields);
/* 1 if `variant` can run this shape on the current device, else 0. */
int bpm_march_variant_eligible(int nx, int ny, int fields, int variant);
/* Process-wide choice of the kernel for a shape: BPM_MARCH_AUTO clears it;
 * a variant that cannot run the shape returns BPM_ERR_INVALID_ARG.  Applies
 * to calls made after it returns; do not change a shape's choice while a
 * call of that shape is being issued on another thread. */
int bpm_set_march_variant(int nx, int ny, int fields, int variant);

/* Forward march that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results (bit for bit) and errors
 * as bpm_propagate, without the workspace: the march's plan lives in a device
 * array of the library, one per GPU, held until the process ends
 * (bpm_noalloc_scratch_bytes() bytes: fields up to 1024 x 1024; larger fields
 * return BPM_ERR_UNSUPPORTED_SIZE before any launch).  The call makes no
 * allocation of any kind.  Every call on one GPU uses that GPU's array, so
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be serialised by the caller; each call rebuilds the plan it needs
 * and clears the barrier words, so consecutive calls of different sizes are
 * independent.  Wait time-outs (see bpm_workspace_status) are recorded in the
 * array's header and cannot be queried. */
int bpm_propagate_noalloc(const bpm_c64* field_in, const float* dn, int nx, int ny, int steps,
                          double dx, double dz, double wavelength, double n0,
                          bpm_c64* field_out, float* intensity_out, void* hip_stream);
/* Size of the per-GPU device array of bpm_propagate_noalloc (bytes). */
size_t bpm_noalloc_scratch_bytes(void);

/* Wait time-outs of the persistent kernels.
 *
 * The persistent kernels of bpm_propagate, bpm_propagate_batch,
 * bpm_batch_launch and bpm_adjoint wait for each other (grid barriers between
 * the passes of a march; per-job dependency waits in the uneven batch).  Every
 * wait is bounded: a wait that has polled `polls` times gives up, the kernel
 * stops waiting from then on and runs to its end, and its outputs are NOT
 * valid.  This only happens when the workgroups of a launch cannot all run
 * (another process holding the device's compute units, a misbehaving driver);
 * the default bound (2^22 polls, tens of milliseconds per wait) is far above
 * any regular wait.
 *
 * Such a time-out is recorded in the workspace: the first 256 bytes of every
 * workspace of the calls above form a status header whose 32-bit word 0 is a
 * sticky mask (bit 0: a grid-barrier wait gave up; bit 1: a work-queue
 * dependency wait gave up), set by the kernels and never cleared by them.
 * (Words 1 and 2 mark the header as initialised; the first call on a fresh
 * workspace clears word 0.)  The calls themselves are asynchronous and
 * return before their kernels run, so they cannot report it; query it with
 * bpm_workspace_status. */

/* Synchronises hip_stream, reads the status header of `workspace` and resets
 * its mask.  Returns BPM_OK when no wait gave up since the previous query (or
 * since the workspace's first call), BPM_ERR_DEVICE with a message naming the
 * kind of wait otherwise, BPM_ERR_INVALID_ARG when no march, batch or adjoint
 * call has used the workspace or the stream is capturing, BPM_ERR_WORKSPACE
 * for a null, misaligned or short (< 256 bytes) workspace.  Must not be called
 * while a call that uses the same workspace may still be queued on another
 * stream. */
int bpm_workspace_status(const void* workspace, size_t workspace_bytes, void* hip_stream);

/* Maps a status mask (word 0 of the header, e.g. copied to the host by the
 * caller's own stream-ordered copy) to BPM_OK (0) or BPM_ERR_DEVICE with the
 * message bpm_workspace_status would give.  Host only; touches no device. */
int bpm_decode_status(unsigned status_word);

/* Process-wide bound on the polls of one wait (see above); 0 restores the
 * default 2^22, values above 2^31 return BPM_ERR_INVALID_ARG.  Applies to
 * kernels launched after the call. */
int bpm_set_wait_limit(unsigned long long polls);

/* Releases the host resources the library keeps between calls (the pinned
 * staging buffer and event of bpm_batch_upload / bpm_propagate_batch), after
 * waiting for the last upload that uses them.  Optional: call it before the
 * HIP runtime is torn down (e.g. at interpreter exit); the next call that
 * needs them allocates them again.  Not thread-safe with concurrent batch
 * uploads. */
void bpm_release(void);

/* Static text for an error code. */
const char* bpm_error_string(int code);
/* Message of the calling thread's last failed call ("" if none). */
const char* bpm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BPM_H */
