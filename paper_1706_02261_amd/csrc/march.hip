// Split-step march kernels: plan builder, fused row and column passes, the
// persistent forward march, the persistent adjoint march with checkpointing,
// a natural-order 2-D FFT and the pupil-plane helpers.
//
// One step j of the march (propagate, then phase screen) is split into two
// passes over the field, each reading and writing it once:
//
//   column pass j : forward column FFTs  ->  x H (exact propagator, evanescent
//                   modes zero, 1/(nx ny) folded in)  ->  inverse column FFTs
//   row pass j    : inverse row FFTs  ->  x exp(i k0 dz dn[j])  ->  I[j] = |u|^2
//                   ->  forward row FFTs (first half of step j+1's DFT2)
//
// plus a head row pass (forward row FFTs of u_0) and a tail row pass (no
// forward FFT; natural-order u_steps written out).  Between passes the field
// lives in a working buffer with its x axis in the FFT's storage order (see
// fft.hpp); the y axis never leaves a column pass permuted.
//
// The adjoint step (reverse-mode derivative of one step) has the same two
// passes in the same order: the row pass adds 2 dL/dI u, emits
// dL/ddn = k0 dz Im(g conj(u)) and multiplies by the conjugate screen; the
// column pass multiplies by conj(H).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "internal.hpp"
#include "march_kernels.hpp"

namespace bpm {

BPM_MARCH_EXTERN(32)
BPM_MARCH_EXTERN(64)
BPM_MARCH_EXTERN(128)
BPM_MARCH_EXTERN(256)
BPM_MARCH_EXTERN(512)
BPM_MARCH_EXTERN(1024)
BPM_MARCH_EXTERN(2048)

// ---------------------------------------------------------------------------
// plan

size_t plan_bytes(int nx, int ny) {
    return kStatusBytes + align_up(sizeof(float2) * (size_t)nx * ny) + align_up(sizeof(float2) * nx) +
           align_up(sizeof(float2) * ny) + align_up(sizeof(int) * nx) +
           align_up(sizeof(int) * ny) + sizeof(unsigned) * kBarWords;
}

Plan plan_carve(void* ws, int nx, int ny) {
    char* b = static_cast<char*>(ws);
    Plan p;
    p.status = b;
    b += kStatusBytes;
    p.H = b;
    b += align_up(sizeof(float2) * (size_t)nx * ny);
    p.twx = b;
    b += align_up(sizeof(float2) * nx);
    p.twy = b;
    b += align_up(sizeof(float2) * ny);
    p.permx = b;
    b += align_up(sizeof(int) * nx);
    p.permy = b;
    b += align_up(sizeof(int) * ny);
    p.counter = b;
    return p;
}

// Fills the propagator in storage order (when with_h), both twiddle tables,
// both storage-slot -> frequency tables, and zeroes the barrier words.
__global__ void plan_kernel(unsigned* __restrict__ status, float2* __restrict__ H,
                            float2* __restrict__ twx, float2* __restrict__ twy,
                            int* __restrict__ permx, int* __restrict__ permy,
                            unsigned* __restrict__ counter, int nx, int ny, double dx, double dz,
                            double lam, double n0, int with_h, int tiled) {
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < kBarWords; i += blockDim.x) counter[i] = 0u;
        // a workspace seen for the first time: clear its sticky status bits
        if (threadIdx.x == 0 && (status[1] != kStatusMagic0 || status[2] != kStatusMagic1)) {
            status[0] = 0u;
            status[1] = kStatusMagic0;
            status[2] = kStatusMagic1;
        }
    }
    const double kPi = 3.14159265358979323846;
    const long nh = with_h ? (long)nx * ny : 0;
    const long total = nh + 2L * (nx + ny);
    const double k0 = 2.0 * kPi / lam, k = n0 * k0;
    const double thr_sqrt = (double)nx * (double)ny * n0 * dx / lam;
    const double thr = thr_sqrt * thr_sqrt;
    const double scale = 1.0 / ((double)nx * (double)ny);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        if (e < nh) {
            const int py = (int)(e / nx), px = (int)(e % nx);
            // storage slot -> frequency index on each axis
            const int m = fft_freq_of_store(nx, kR, px);
            const int l = fft_freq_of_store(ny, kR, py);
            const long ms = m < nx / 2 ? m : m - nx, ls = l < ny / 2 ? l : l - ny;
            const long a = ms * ny, b = ls * nx;
            float2 h = make_float2(0.f, 0.f);
            if ((double)(a * a + b * b) <= thr) {
                const double kx = 2.0 * kPi * (double)ms / (nx * dx);
                const double ky = 2.0 * kPi * (double)ls / (ny * dx);
                const double kz = sqrt(fmax(k * k - kx * kx - ky * ky, 0.0));
                double sv, cv;
                sincos(dz * kz, &sv, &cv);
                h = make_float2((float)(cv * scale), (float)(sv * scale));
            }
            if (tiled) {
                // TH x W tiles of one 128-byte line (W = 4096 / ny, TH = 16 / W)
                const long W = 4096 / ny, TH = 16 / W;
                H[((py / TH) * (nx / W) + px / W) * 16 + (py % TH) * W + px % W] = h;
            } else {
                H[e] = h;
            }
        } else if (e < nh + nx + ny) {
            const long t = e - nh;
            const int n = t < nx ? nx : ny;
            const long i = t < nx ? t : t - nx;
            double sv, cv;
            sincos(-2.0 * kPi * (double)i / n, &sv, &cv);
            (t < nx ? twx : twy)[i] = make_float2((float)cv, (float)sv);
        } else {
            const long t = e - nh - nx - ny;
            if (t < nx) permx[t] = fft_freq_of_store(nx, kR, (int)t);
            else permy[t - nx] = fft_freq_of_store(ny, kR, (int)(t - nx));
        }
    }
}

bool march_variant_eligible(int nx, int ny, int fields, int variant) {
    const bool sizes = nx >= 32 && ny >= 32 && nx <= 2048 && ny <= 2048 && (nx & (nx - 1)) == 0 &&
                       (ny & (ny - 1)) == 0 && fields >= 1 && fields <= kMaxFields;
    if (!sizes) return false;
    switch (variant) {
        case kMarchOnePerCu: return true;
        case kMarchTwoPerCu: return nx >= 512 && ny >= 512;
        case kMarchSmallBlocks: return nx <= 1024 && ny <= 1024;
        case kMarchTiledPair: {
            const int cus = device_cus();
            if (cus <= 0 || 4096 % nx != 0 || 4096 % ny != 0) return false;
            const int B = 4096 / nx, W = 4096 / ny;  // rows of a row unit, columns of a column unit
            return (fields == 1 || fields == 2) && B * W == 16 && cus % 16 == 0 &&
                   ny / B == cus && nx / W == cus;
        }
        default: return false;
    }
}

namespace {
std::mutex g_variant_mu;
std::map<std::tuple<int, int, int>, int> g_variant;  // tuned kernel per (nx, ny, fields)
}  // namespace

int set_march_variant(int nx, int ny, int fields, int variant) {
    std::lock_guard<std::mutex> lk(g_variant_mu);
    if (variant == kMarchAuto) {
        g_variant.erase(std::make_tuple(nx, ny, fields));
        return 0;
    }
    if (!march_variant_eligible(nx, ny, fields, variant)) return -1;
    g_variant[std::make_tuple(nx, ny, fields)] = variant;
    return 0;
}

int march_variant(int nx, int ny, int fields) {
    {
        std::lock_guard<std::mutex> lk(g_variant_mu);
        const auto it = g_variant.find(std::make_tuple(nx, ny, fields));
        if (it != g_variant.end() && march_variant_eligible(nx, ny, fields, it->second))
            return it->second;
    }
    // built-in choice: the tiled kernel for the one- and two-field geometries
    // it serves (nx ny = 2^20; for one field measured 3 % faster than one
    // workgroup per CU at 1024^2, 32 % at 512 x 2048, even at 2048 x 512),
    // two workgroups per CU for several fields of sizes >= 512, 64-thread
    // workgroups for one field of sides <= 512 (measured 7-15 % faster from
    // 128^2 to 512^2, slower at 1024^2), else one 256-thread workgroup per CU
    if (march_variant_eligible(nx, ny, fields, kMarchTiledPair)) return kMarchTiledPair;
    if (fields >= 2 && march_variant_eligible(nx, ny, fields, kMarchTwoPerCu)) return kMarchTwoPerCu;
    if (fields == 1 && nx <= 512 && ny <= 512) return kMarchSmallBlocks;
    return kMarchOnePerCu;
}

bool march_tiled(int nx, int ny, int fields) {
    return march_variant(nx, ny, fields) == kMarchTiledPair;
}

hipError_t launch_plan(const Geom& g, const Plan& p, bool with_h, hipStream_t s, bool tiled_h) {
    const long total = (with_h ? (long)g.nx * g.ny : 0) + 2L * (g.nx + g.ny);
    const int threads = 256;
    const long blocks = (total + threads - 1) / threads;
    plan_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), threads, 0, s>>>(
        (unsigned*)p.status, (float2*)p.H, (float2*)p.twx, (float2*)p.twy, (int*)p.permx, (int*)p.permy,
        (unsigned*)p.counter, g.nx, g.ny, g.dx, g.dz, g.wavelength, g.n0, with_h ? 1 : 0,
        tiled_h ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// natural-order 2-D FFT (unnormalised; the inverse uses conj(DFT(conj x)))

template <int NY>
__global__ __launch_bounds__(kBlock) void fft2_cols_kernel(const float2* in, float2* out, int nx,
                                                           const float2* __restrict__ tw,
                                                           const int* __restrict__ permy,
                                                           int inverse, float scale) {
    constexpr int T = NY / kR, W = units_per_block<NY>();
    extern __shared__ float2 smem[];
    const int w = threadIdx.x % W, t = threadIdx.x / W;
    const int c = blockIdx.x * W + w;
    const bool on = c < nx;
    const size_t col = on ? (size_t)c : 0;
    Twiddles<NY, kR> twy;
    twy.load(tw, t);
    float2 v[kR];
    const float sg = inverse ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const float2 x = in[(size_t)(i * T + t) * nx + col];
        v[i] = make_float2(x.x, sg * x.y);
    }
    fft_forward<NY, kR, W>(v, smem + w, t, twy, BlockSync());
    __syncthreads();  // every load of an in-place call precedes every store
    if (on) {
#pragma unroll
        for (int r = 0; r < kR; ++r)
            out[(size_t)permy[r * T + t] * nx + col] =
                make_float2(scale * v[r].x, sg * scale * v[r].y);
    }
}

template <int NX>
__global__ __launch_bounds__(kBlock) void fft2_rows_kernel(float2* io, int ny,
                                                           const float2* __restrict__ tw,
                                                           const int* __restrict__ permx,
                                                           int inverse) {
    constexpr int T = NX / kR, B = units_per_block<NX>();
    extern __shared__ float2 smem[];
    const int sub = threadIdx.x / T, tau = threadIdx.x % T;
    const int row = blockIdx.x * B + sub;
    const bool on = row < ny;
    const size_t rowoff = (size_t)(on ? row : 0) * NX;
    Twiddles<NX, kR> twx;
    twx.load(tw, tau);
    float2 v[kR];
    const float sg = inverse ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const float2 x = io[rowoff + i * T + tau];
        v[i] = make_float2(x.x, sg * x.y);
    }
    fft_forward<NX, kR, 1>(v, smem + sub * lds_size<NX>(), tau, twx, BlockSync());
    __syncthreads();  // every load of the row precedes every store
    if (on) {
#pragma unroll
        for (int r = 0; r < kR; ++r) io[rowoff + permx[r * T + tau]] = make_float2(v[r].x, sg * v[r].y);
    }
}

// ---------------------------------------------------------------------------
// pupil plane: U0 = A exp(i phi) exp(-i kz z_f), and dL/dphi = Im(dL/dU0 conj(U0))

__global__ void pupil_spectrum_kernel(const float* __restrict__ amp,
                                      const float* __restrict__ phase, int nx, int ny, double dx,
                                      double k, double z_f, float2* __restrict__ U) {
    const double kPi = 3.14159265358979323846;
    const long n = (long)nx * ny;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x) {
        const int l = (int)(e / nx), m = (int)(e % nx);
        const double kx = 2.0 * kPi * (double)(m < nx / 2 ? m : m - nx) / (nx * dx);
        const double ky = 2.0 * kPi * (double)(l < ny / 2 ? l : l - ny) / (ny * dx);
        const double kz = sqrt(fmax(k * k - kx * kx - ky * ky, 0.0));
        double sv, cv;
        sincos((double)phase[e] - kz * z_f, &sv, &cv);
        U[e] = make_float2((float)(amp[e] * cv), (float)(amp[e] * sv));
    }
}

__global__ void pupil_grad_kernel(const float2* __restrict__ G, const float2* __restrict__ U,
                                  long n, float* __restrict__ gphi) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x) {
        const float2 g = G[e], u = U[e];
        gphi[e] = fmaf(g.y, u.x, -g.x * u.y);
    }
}

// Guide-star correction: the pupil phase that puts U0 = A exp(i phi) exp(-i kz z_f)
// in phase with G = dL/dU0 of a point at the focus, phi = arg G + kz z_f, with
// the lateral shift (sx, sy) of the corrected field applied as the tilt
// -(kx sx + ky sy); wrapped to [-pi, pi).
__global__ void guide_star_phase_kernel(const float2* __restrict__ G, int nx, int ny, double dx,
                                        double k, double z_f, double sx, double sy,
                                        float* __restrict__ phase) {
    const double kPi = 3.14159265358979323846;
    const long n = (long)nx * ny;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x) {
        const int l = (int)(e / nx), m = (int)(e % nx);
        const double kx = 2.0 * kPi * (double)(m < nx / 2 ? m : m - nx) / (nx * dx);
        const double ky = 2.0 * kPi * (double)(l < ny / 2 ? l : l - ny) / (ny * dx);
        const double kz = sqrt(fmax(k * k - kx * kx - ky * ky, 0.0));
        const float2 g = G[e];
        double p = atan2((double)g.y, (double)g.x) + kz * z_f - kx * sx - ky * sy;
        p -= 2.0 * kPi * floor((p + kPi) / (2.0 * kPi));
        phase[e] = (float)p;
    }
}

// ---------------------------------------------------------------------------
// launchers

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
    }
    return cus;
}

template <typename F>
static hipError_t dispatch2(int nx, int ny, F&& f) {
    auto by_y = [&](auto xc) -> hipError_t {
        constexpr int X = decltype(xc)::value;
        switch (ny) {
            case 32: return f(std::integral_constant<int, X>{}, std::integral_constant<int, 32>{});
            case 64: return f(std::integral_constant<int, X>{}, std::integral_constant<int, 64>{});
            case 128: return f(std::integral_constant<int, X>{}, std::integral_constant<int, 128>{});
            case 256: return f(std::integral_constant<int, X>{}, std::integral_constant<int, 256>{});
            case 512: return f(std::integral_constant<int, X>{}, std::integral_constant<int, 512>{});
            case 1024: return f(std::integral_constant<int, X>{}, std::integral_constant<int, 1024>{});
            case 2048: return f(std::integral_constant<int, X>{}, std::integral_constant<int, 2048>{});
            default: return hipErrorInvalidValue;
        }
    };
    switch (nx) {
        case 32: return by_y(std::integral_constant<int, 32>{});
        case 64: return by_y(std::integral_constant<int, 64>{});
        case 128: return by_y(std::integral_constant<int, 128>{});
        case 256: return by_y(std::integral_constant<int, 256>{});
        case 512: return by_y(std::integral_constant<int, 512>{});
        case 1024: return by_y(std::integral_constant<int, 1024>{});
        case 2048: return by_y(std::integral_constant<int, 2048>{});
        default: return hipErrorInvalidValue;
    }
}

static float k0dz_of(const Geom& g) {
    return (float)(2.0 * 3.14159265358979323846 / g.wavelength * g.dz);
}

// calls f(std::integral_constant<int, nx>{}) for a supported row length
template <typename F>
static hipError_t dispatch_nx(int nx, F&& f) {
    return dispatch_size(nx, f);
}

hipError_t launch_forward(const Geom& g, const Plan& p, const MarchIO* io, int fields,
                          hipStream_t s, unsigned long long* timers, int variant) {
    const size_t plane = (size_t)g.nx * g.ny;
    if (fields < 1 || fields > kMaxFields) return hipErrorInvalidValue;
    if (g.steps == 0) {
        for (int f = 0; f < fields; ++f) {
            if (io[f].field_out == io[f].field_in) continue;
            const hipError_t e = hipMemcpyAsync(io[f].field_out, io[f].field_in,
                                                plane * sizeof(float2), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (device_cus() <= 0) return hipErrorNoDevice;
    MarchArgs a{};
    for (int f = 0; f < fields; ++f) {
        a.field_in[f] = (const float2*)io[f].field_in;
        a.work[f] = (float2*)io[f].field_out;
        a.dn[f] = io[f].dn;
        a.inten[f] = io[f].intensity;
        a.clear[f] = io[f].clear;
    }
    a.H = (const float2*)p.H;
    a.twx = (const float2*)p.twx;
    a.twy = (const float2*)p.twy;
    a.counter = (unsigned*)p.counter;
    a.status = (unsigned*)p.status;
    a.limit = wait_limit();
    a.timers = timers;
    a.nx = g.nx;
    a.ny = g.ny;
    a.steps = g.steps;
    a.fields = fields;
    a.variant = variant == kMarchAuto ? march_variant(g.nx, g.ny, fields) : variant;
    if (!march_variant_eligible(g.nx, g.ny, fields, a.variant)) return hipErrorInvalidConfiguration;
    a.k0dz = k0dz_of(g);
    return dispatch_nx(g.nx, [&](auto xc) {
        constexpr int NX = decltype(xc)::value;
        return launch_forward_x<NX>(a, s);
    });
}

hipError_t launch_adapted(const Geom& g, const Plan& p, const void* field_in, const float* dn,
                          const float* dn_ref, void* field_out, float* intensity, hipStream_t s) {
    if (device_cus() <= 0) return hipErrorNoDevice;
    AdaptArgs a{};
    a.field_in = (const float2*)field_in;
    a.work = (float2*)field_out;
    a.dn = dn;
    a.dn_ref = dn_ref;
    a.inten = intensity;
    a.twx = (const float2*)p.twx;
    a.twy = (const float2*)p.twy;
    a.permx = (const int*)p.permx;
    a.permy = (const int*)p.permy;
    a.counter = (unsigned*)p.counter;
    a.status = (unsigned*)p.status;
    a.limit = wait_limit();
    a.nx = g.nx;
    a.ny = g.ny;
    a.steps = g.steps;
    a.dx = g.dx;
    a.dz = g.dz;
    a.lam = g.wavelength;
    a.n0 = g.n0;
    a.k0dz = k0dz_of(g);
    return dispatch_nx(g.nx, [&](auto xc) {
        constexpr int NX = decltype(xc)::value;
        return launch_adapted_x<NX>(a, s);
    });
}

// mean of every slice of dn: one workgroup per slice, FP64 sums in a fixed
// order (thread partial sums over a fixed stride, then a tree)
__global__ __launch_bounds__(256) void slice_mean_kernel(const float* __restrict__ dn, long plane,
                                                         int steps, float* __restrict__ out) {
    __shared__ double part[256];
    for (int j = blockIdx.x; j < steps; j += gridDim.x) {
        double acc = 0.0;
        const float* sl = dn + (size_t)j * plane;
        for (long e = threadIdx.x; e < plane; e += 256) acc += (double)sl[e];
        part[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[j] = (float)(part[0] / (double)plane);
        __syncthreads();
    }
}

hipError_t launch_slice_means(const float* dn, long plane, int steps, float* out, hipStream_t s) {
    if (steps <= 0) return hipSuccess;
    slice_mean_kernel<<<(unsigned)(steps < 4096 ? steps : 4096), 256, 0, s>>>(dn, plane, steps, out);
    return hipGetLastError();
}

size_t adjoint_fields(int steps, int K) {
    const int C = (steps + K - 1) / K;
    return (size_t)C + 2 * (size_t)K + 2;
}

size_t adjoint_field_bytes(int nx, int ny, int steps, int K) {
    return align_up(sizeof(float2) * (size_t)nx * ny * adjoint_fields(steps, K));
}

hipError_t launch_adjoint(const Geom& g, const Plan& p, const AdjointIO* io, int n, int K,
                          void* fields, hipStream_t s) {
    const size_t plane = (size_t)g.nx * g.ny;
    if (device_cus() <= 0) return hipErrorNoDevice;
    if (n < 1 || n > kMaxFields) return hipErrorInvalidValue;
    const int C = (g.steps + K - 1) / K;
    AdjointArgs a{};
    bool linear = true;
    for (int i = 0; i < n; ++i) {
        float2* f = (float2*)((char*)fields + (size_t)i * adjoint_field_bytes(g.nx, g.ny, g.steps, K));
        a.field_in[i] = (const float2*)io[i].field_in;
        a.dn[i] = io[i].dn;
        a.gout[i] = (const float2*)io[i].grad_out;
        a.gI[i] = io[i].grad_inten;
        a.gin[i] = (float2*)io[i].grad_in;
        a.gspec[i] = (float2*)io[i].grad_spec;
        a.gdn[i] = io[i].grad_dn;
        a.fwork[i] = f;
        a.gwork[i] = f + plane;
        a.ckpt[i] = f + 2 * plane;
        a.seg[i] = f + (2 + (size_t)C) * plane;
        linear = linear && !io[i].grad_inten && !io[i].grad_dn;
    }
    a.H = (const float2*)p.H;
    a.twx = (const float2*)p.twx;
    a.twy = (const float2*)p.twy;
    a.permx = (const int*)p.permx;
    a.permy = (const int*)p.permy;
    a.counter = (unsigned*)p.counter;
    a.status = (unsigned*)p.status;
    a.limit = wait_limit();
    a.nx = g.nx;
    a.ny = g.ny;
    a.steps = g.steps;
    a.K = K;
    a.fields = n;
    a.linear = linear ? 1 : 0;
    a.k0dz = k0dz_of(g);
    return dispatch_nx(g.nx, [&](auto xc) {
        constexpr int NX = decltype(xc)::value;
        return launch_adjoint_x<NX>(a, s);
    });
}

hipError_t launch_fft2(const void* in, void* out, int nx, int ny, bool inverse, float scale,
                       const Plan& p, hipStream_t s) {
    return dispatch2(nx, ny, [&](auto xc, auto yc) {
        constexpr int NX = decltype(xc)::value, NY = decltype(yc)::value;
        constexpr int W = units_per_block<NY>(), B = units_per_block<NX>();
        fft2_cols_kernel<NY><<<(nx + W - 1) / W, kBlock, sizeof(float2) * W * lds_size<NY>(), s>>>(
            (const float2*)in, (float2*)out, nx, (const float2*)p.twy, (const int*)p.permy,
            inverse ? 1 : 0, scale);
        fft2_rows_kernel<NX><<<(ny + B - 1) / B, kBlock, sizeof(float2) * B * lds_size<NX>(), s>>>(
            (float2*)out, ny, (const float2*)p.twx, (const int*)p.permx, inverse ? 1 : 0);
        return hipGetLastError();
    });
}

hipError_t launch_pupil_spectrum(const float* amp, const float* phase, const Geom& g, double z_f,
                                 void* U, hipStream_t s) {
    const long n = (long)g.nx * g.ny;
    const long blocks = (n + 255) / 256;
    const double k = 2.0 * 3.14159265358979323846 / g.wavelength * g.n0;
    pupil_spectrum_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(
        amp, phase, g.nx, g.ny, g.dx, k, z_f, (float2*)U);
    return hipGetLastError();
}

hipError_t launch_guide_star_phase(const void* G, const Geom& g, double z_f, double sx, double sy,
                                   float* phase, hipStream_t s) {
    const long n = (long)g.nx * g.ny;
    const long blocks = (n + 255) / 256;
    const double k = 2.0 * 3.14159265358979323846 / g.wavelength * g.n0;
    guide_star_phase_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(
        (const float2*)G, g.nx, g.ny, g.dx, k, z_f, sx, sy, phase);
    return hipGetLastError();
}

hipError_t launch_pupil_grad(const void* G, const void* U, long n, float* gphi, hipStream_t s) {
    const long blocks = (n + 255) / 256;
    pupil_grad_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(
        (const float2*)G, (const float2*)U, n, gphi);
    return hipGetLastError();
}

}  // namespace bpm

