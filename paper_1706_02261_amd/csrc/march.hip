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

#include <type_traits>

#include "internal.hpp"
#include "passes.hpp"

namespace bpm {

// ---------------------------------------------------------------------------
// plan

size_t plan_bytes(int nx, int ny) {
    return align_up(sizeof(float2) * (size_t)nx * ny) + align_up(sizeof(float2) * nx) +
           align_up(sizeof(float2) * ny) + align_up(sizeof(int) * nx) +
           align_up(sizeof(int) * ny) + sizeof(unsigned) * kBarWords;
}

Plan plan_carve(void* ws, int nx, int ny) {
    char* b = static_cast<char*>(ws);
    Plan p;
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
__global__ void plan_kernel(float2* __restrict__ H, float2* __restrict__ twx,
                            float2* __restrict__ twy, int* __restrict__ permx,
                            int* __restrict__ permy, unsigned* __restrict__ counter, int nx,
                            int ny, double dx, double dz, double lam, double n0, int with_h) {
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < kBarWords; i += blockDim.x) counter[i] = 0u;
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
            H[e] = h;
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

hipError_t launch_plan(const Geom& g, const Plan& p, bool with_h, hipStream_t s) {
    const long total = (with_h ? (long)g.nx * g.ny : 0) + 2L * (g.nx + g.ny);
    const int threads = 256;
    const long blocks = (total + threads - 1) / threads;
    plan_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), threads, 0, s>>>(
        (float2*)p.H, (float2*)p.twx, (float2*)p.twy, (int*)p.permx, (int*)p.permy,
        (unsigned*)p.counter, g.nx, g.ny, g.dx, g.dz, g.wavelength, g.n0, with_h ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// persistent forward march

// LDS of one workgroup's row or column unit (the larger of the two)
template <int NX, int NY>
__host__ __device__ constexpr size_t march_data_lds() {
    return sizeof(float2) * (units_per_block<NX>() * lds_size<NX>() >
                                     units_per_block<NY>() * lds_size<NY>()
                                 ? units_per_block<NX>() * lds_size<NX>()
                                 : units_per_block<NY>() * lds_size<NY>());
}

// Up to kMaxFields marches of one geometry run in lockstep: every pass covers
// the units of all fields, so the two grid barriers of a step are shared and a
// workgroup's loads and stores of one unit overlap the work on the next.
struct MarchArgs {
    const float2* field_in[kMaxFields];
    float2* work[kMaxFields];
    const float* dn[kMaxFields];
    float* inten[kMaxFields];
    const float2* H;
    const float2* twx;
    const float2* twy;
    unsigned* counter;
    int nx, ny, steps, fields;
    float k0dz;
};

// OCC = workgroups per CU.  OCC 1 keeps the twiddles in registers and walks
// a workgroup's units two at a time (the second unit's loads in flight while
// the first is transformed).  OCC 2 (several fields) reads the twiddles from
// tables in LDS instead, so that two workgroups fit one CU (two waves per
// SIMD) and one workgroup's memory waits overlap the other's arithmetic.
template <int NX, int NY, int OCC>
__global__ __launch_bounds__(kBlock, OCC) void march_kernel(MarchArgs a) {
    extern __shared__ float2 smem[];
    const int G = gridDim.x, v = virtual_block();
    const int rows_u = (a.ny + units_per_block<NX>() - 1) / units_per_block<NX>();
    const int cols_u = (a.nx + units_per_block<NY>() - 1) / units_per_block<NY>();
    const int all_r = rows_u * a.fields, all_c = cols_u * a.fields;
    const size_t plane = (size_t)a.nx * a.ny;
    unsigned nbar = 0;
    bool abort = false;
    using TwX = typename std::conditional<OCC == 1, Twiddles<NX, kR>, LdsTwiddles<NX, kR>>::type;
    using TwY = typename std::conditional<OCC == 1, Twiddles<NY, kR>, LdsTwiddles<NY, kR>>::type;
    TwX twx;
    TwY twy;
    if constexpr (OCC == 1) {
        twx.load(a.twx, threadIdx.x % (NX / kR));
        twy.load(a.twy, threadIdx.x / units_per_block<NY>());
    } else {
        float2* tabx = smem + march_data_lds<NX, NY>() / sizeof(float2);
        float2* taby = tabx + NX;
        for (int i = threadIdx.x; i < NX; i += kBlock) tabx[i] = a.twx[i];
        for (int i = threadIdx.x; i < NY; i += kBlock) taby[i] = a.twy[i];
        __syncthreads();
        twx = TwX{tabx, (int)threadIdx.x % (NX / kR)};
        twy = TwY{taby, (int)threadIdx.x / units_per_block<NY>()};
    }
    constexpr int PAIR = OCC == 1 ? 2 : 1;  // units per loop trip
    float d[kR];
    for (int i = 0; i < kR; ++i) d[i] = 0.f;
    // combined unit u is unit u / fields of field u % fields: the fields'
    // units of one column range sit next to each other, so the workgroups of
    // an XCD share that range's slice of the propagator table in its L2
    const int F = a.fields;
    for (int u = v; u < all_r; u += G) {
        const int f = u % F;
        RowArgs ra{a.field_in[f], a.work[f], nullptr, nullptr, nullptr, nullptr, nullptr, a.k0dz};
        row_unit<NX, kNaturalIn, kNoOps, kSpecOut>(u / F, a.ny, ra, d, twx, smem);
    }
    // a workgroup with a single row unit fetches its dn slice during the column pass
    const bool one_row_unit = all_r <= G;
    const int vv = v < all_r ? v : 0;
    for (int j = 0; j < a.steps; ++j) {
        if (one_row_unit) load_dn<NX>(d, vv / F, a.ny, a.dn[vv % F] + j * plane);
        grid_sync(a.counter, ++nbar, abort);
        for (int u = v; u < all_c; u += PAIR * G) {
            const int u2 = u + G;
            const bool two = PAIR == 2 && u2 < all_c;
            const int f1 = u % F, f2 = u2 % F;
            float2 va[kR], ha[kR], vb[kR], hb[kR];
            col_load<NY>(u / F, a.nx, a.work[f1], a.H, va, ha);
            if (two) col_load<NY>(u2 / F, a.nx, a.work[f2], a.H, vb, hb);
            col_body<NY, false>(u / F, a.nx, a.work[f1], twy, smem, nullptr, nullptr, nullptr, va,
                                ha);
            if (two)
                col_body<NY, false>(u2 / F, a.nx, a.work[f2], twy, smem, nullptr, nullptr,
                                    nullptr, vb, hb);
        }
        grid_sync(a.counter, ++nbar, abort);
        for (int u = v; u < all_r; u += PAIR * G) {
            const int u2 = u + G;
            const bool two = PAIR == 2 && u2 < all_r;
            const int f1 = u % F, r1 = u / F;
            const int f2 = u2 % F, r2 = two ? u2 / F : 0;
            float2 va[kR], vb[kR];
            float db[kR];
            row_load<NX, kSpecIn>(r1, a.ny, a.work[f1], va);
            if (!one_row_unit) load_dn<NX>(d, r1, a.ny, a.dn[f1] + j * plane);
            if (two) {
                row_load<NX, kSpecIn>(r2, a.ny, a.work[f2], vb);
                load_dn<NX>(db, r2, a.ny, a.dn[f2] + j * plane);
            }
            const RowArgs ra{a.work[f1], a.work[f1],
                             a.inten[f1] ? a.inten[f1] + j * plane : nullptr, nullptr, nullptr,
                             nullptr, nullptr, a.k0dz};
            if (j + 1 < a.steps)
                row_body<NX, kSpecIn, kScreen, kSpecOut>(r1, a.ny, ra, d, twx, smem, va);
            else
                row_body<NX, kSpecIn, kScreen, kNaturalOut>(r1, a.ny, ra, d, twx, smem, va);
            if (two) {
                const RowArgs rb{a.work[f2], a.work[f2],
                                 a.inten[f2] ? a.inten[f2] + j * plane : nullptr, nullptr,
                                 nullptr, nullptr, nullptr, a.k0dz};
                if (j + 1 < a.steps)
                    row_body<NX, kSpecIn, kScreen, kSpecOut>(r2, a.ny, rb, db, twx, smem, vb);
                else
                    row_body<NX, kSpecIn, kScreen, kNaturalOut>(r2, a.ny, rb, db, twx, smem, vb);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// persistent adjoint march with checkpointing
//
//   1. forward march from u_0 keeping u at every K-th slice boundary;
//   2. for each segment of K steps, last to first: recompute the segment's
//      fields from its checkpoint (kept in one of two `seg` buffers), then
//      run its adjoint steps backwards; the recompute of the segment before
//      shares the passes of these adjoint steps; the adjoint state crosses
//      segments in `gwork`;
//   3. a tail row pass brings g_0 back to natural order.
// Memory: ceil(N/K) + 2 K + 2 fields (K + 2 more than the checkpoints and
// one segment); compute: about three forward marches in about two marches'
// worth of passes.

struct AdjointArgs {
    const float2* field_in;
    const float* dn;
    const float2* gout;  // dL/du_N or null
    const float* gI;     // dL/dI or null
    float2* gin;         // dL/du_0 or null
    float2* gspec;       // dL/dU_0 or null
    float* gdn;          // dL/ddn or null
    float2* fwork;
    float2* gwork;
    float2* ckpt;  // [ceil(N/K)] fields (slot 0 unused: u_0 is field_in)
    float2* seg;   // [2 K] fields: two segment buffers
    const float2* H;
    const float2* twx;
    const float2* twy;
    const int* permx;
    const int* permy;
    unsigned* counter;
    int nx, ny, steps, K;
    float k0dz;
};

// BLK = threads per workgroup: 64 for fields of at most 512^2, so that a
// small field still spreads over many CUs (a 256^2 field has 64 units of 4
// rows instead of 16 of 16).
template <int NX, int NY, int BLK>
__global__ __launch_bounds__(BLK) void adjoint_kernel(AdjointArgs a) {
    extern __shared__ float2 smem[];
    const int G = gridDim.x, v = virtual_block();
    const int rows_u = (a.ny + units_per_block<NX, BLK>() - 1) / units_per_block<NX, BLK>();
    const int cols_u = (a.nx + units_per_block<NY, BLK>() - 1) / units_per_block<NY, BLK>();
    const size_t plane = (size_t)a.nx * a.ny;
    const int N = a.steps, K = a.K, C = (N + K - 1) / K;
    unsigned nbar = 0;
    bool abort = false;
    Twiddles<NX, kR> twx;
    Twiddles<NY, kR> twy;
    twx.load(a.twx, threadIdx.x % (NX / kR));
    twy.load(a.twy, threadIdx.x / units_per_block<NY, BLK>());
    float d[kR];
    for (int i = 0; i < kR; ++i) d[i] = 0.f;

    auto col_pass = [&](float2* work, bool conj, float2* spec_out) {
        for (int u = v; u < cols_u; u += G) {
            if (conj)
                col_unit<NY, true, BLK>(u, a.nx, work, a.H, twy, smem, spec_out, a.permx, a.permy);
            else
                col_unit<NY, false, BLK>(u, a.nx, work, a.H, twy, smem, nullptr, nullptr, nullptr);
        }
    };

    // 1. checkpoints u_K, u_2K, ..., u_(C-1)K
    if (C > 1) {
        RowArgs ra{a.field_in, a.fwork, nullptr, nullptr, nullptr, nullptr, nullptr, a.k0dz};
        for (int u = v; u < rows_u; u += G)
            row_unit<NX, kNaturalIn, kNoOps, kSpecOut, BLK>(u, a.ny, ra, d, twx, smem);
        ra.src = a.fwork;
        const int last = (C - 1) * K;
        for (int j = 0; j < last; ++j) {
            grid_sync(a.counter, ++nbar, abort);
            col_pass(a.fwork, false, nullptr);
            grid_sync(a.counter, ++nbar, abort);
            ra.keep = ((j + 1) % K == 0) ? a.ckpt + (size_t)((j + 1) / K) * plane : nullptr;
            for (int u = v; u < rows_u; u += G) {
                load_dn<NX, BLK>(d, u, a.ny, a.dn + j * plane);
                if (j + 1 < last)
                    row_unit<NX, kSpecIn, kScreen, kSpecOut, BLK>(u, a.ny, ra, d, twx, smem);
                else
                    row_unit<NX, kSpecIn, kScreen, kNoOut, BLK>(u, a.ny, ra, d, twx, smem);
            }
        }
    }

    // 2. segments, last to first.  Recomputing segment c from its checkpoint
    // takes 2 L + 1 passes (the head row pass to the spectrum, then a column
    // and a row pass per step, the row passes keeping u in segment buffer
    // c % 2); its adjoint steps take 2 L passes (a row and a column pass per
    // step, last step first) and read that buffer.  The recompute of segment
    // c - 1 runs in the same passes as the adjoint steps of segment c (the
    // other buffer, the other work field), so one grid barrier serves both.
    auto seg_of = [&](int c) { return a.seg + (size_t)(c & 1) * K * plane; };
    auto len_of = [&](int c) { return N - c * K < K ? N - c * K : K; };
    // units of pass i: recompute: 0 head row, odd column, even row;
    // adjoint: even row, odd column
    auto rec_units = [&](int i) { return i % 2 == 0 ? rows_u : cols_u; };
    auto adj_units = [&](int i) { return i % 2 == 0 ? rows_u : cols_u; };
    auto rec_unit = [&](int c, int i, int u) {
        if (i == 0) {
            RowArgs fr{c == 0 ? a.field_in : a.ckpt + (size_t)c * plane, a.fwork, nullptr,
                       nullptr, nullptr, nullptr, nullptr, a.k0dz};
            row_unit<NX, kNaturalIn, kNoOps, kSpecOut, BLK>(u, a.ny, fr, d, twx, smem);
        } else if (i % 2 == 1) {
            col_unit<NY, false, BLK>(u, a.nx, a.fwork, a.H, twy, smem, nullptr, nullptr, nullptr);
        } else {
            const int t = i / 2 - 1;
            RowArgs fr{a.fwork, a.fwork, nullptr, seg_of(c) + (size_t)t * plane, nullptr,
                       nullptr, nullptr, a.k0dz};
            load_dn<NX, BLK>(d, u, a.ny, a.dn + (size_t)(c * K + t) * plane);
            if (t + 1 < len_of(c))
                row_unit<NX, kSpecIn, kScreen, kSpecOut, BLK>(u, a.ny, fr, d, twx, smem);
            else
                row_unit<NX, kSpecIn, kScreen, kNoOut, BLK>(u, a.ny, fr, d, twx, smem);
        }
    };
    auto adj_unit = [&](int c, int i, int u) {
        const int s = len_of(c) - 1 - i / 2, j = c * K + s;
        if (i % 2 == 0) {
            RowArgs br{a.gwork, a.gwork, nullptr, nullptr, seg_of(c) + (size_t)s * plane,
                       a.gI ? a.gI + (size_t)j * plane : nullptr,
                       a.gdn ? a.gdn + (size_t)j * plane : nullptr, a.k0dz};
            load_dn<NX, BLK>(d, u, a.ny, a.dn + (size_t)j * plane);
            if (j + 1 < N) {
                row_unit<NX, kSpecIn, kAdjointOps, kSpecOut, BLK>(u, a.ny, br, d, twx, smem);
            } else if (a.gout) {
                br.src = a.gout;
                row_unit<NX, kNaturalIn, kAdjointOps, kSpecOut, BLK>(u, a.ny, br, d, twx, smem);
            } else {
                row_unit<NX, kZeroIn, kAdjointOps, kSpecOut, BLK>(u, a.ny, br, d, twx, smem);
            }
        } else {
            col_unit<NY, true, BLK>(u, a.nx, a.gwork, a.H, twy, smem, j == 0 ? a.gspec : nullptr,
                                    a.permx, a.permy);
        }
    };
    // the last segment's recompute alone, then adjoint c with recompute c - 1
    for (int i = 0; i < 2 * len_of(C - 1) + 1; ++i) {
        grid_sync(a.counter, ++nbar, abort);
        for (int u = v; u < rec_units(i); u += G) rec_unit(C - 1, i, u);
    }
    for (int c = C - 1; c >= 0; --c) {
        const int PA = 2 * len_of(c), PR = c > 0 ? 2 * len_of(c - 1) + 1 : 0;
        for (int i = 0; i < (PA > PR ? PA : PR); ++i) {
            grid_sync(a.counter, ++nbar, abort);
            const int na = i < PA ? adj_units(i) : 0, nr = i < PR ? rec_units(i) : 0;
            for (int u = v; u < na + nr; u += G) {
                if (u < na)
                    adj_unit(c, i, u);
                else
                    rec_unit(c - 1, i, u - na);
            }
        }
    }

    // 3. g_0 in natural order
    if (a.gin) {
        grid_sync(a.counter, ++nbar, abort);
        RowArgs tr{a.gwork, a.gin, nullptr, nullptr, nullptr, nullptr, nullptr, a.k0dz};
        for (int u = v; u < rows_u; u += G)
            row_unit<NX, kSpecIn, kNoOps, kNaturalOut, BLK>(u, a.ny, tr, d, twx, smem);
    }
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

// ---------------------------------------------------------------------------
// launchers

static int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
    }
    return cus;
}

template <int NX, int NY, int BLK = kBlock>
static size_t persistent_lds() {
    const size_t lds_r = sizeof(float2) * units_per_block<NX, BLK>() * lds_size<NX>();
    const size_t lds_c = sizeof(float2) * units_per_block<NY, BLK>() * lds_size<NY>();
    return lds_r > lds_c ? lds_r : lds_c;
}

template <int NX, int NY, int BLK = kBlock>
static int persistent_grid(int nx, int ny, int fields = 1, int per_cu = 1) {
    const int rows_u = (ny + units_per_block<NX, BLK>() - 1) / units_per_block<NX, BLK>();
    const int cols_u = (nx + units_per_block<NY, BLK>() - 1) / units_per_block<NY, BLK>();
    const int cus = device_cus() * per_cu;
    const int grid = (rows_u > cols_u ? rows_u : cols_u) * fields;
    return grid > cus ? cus : grid;
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

hipError_t launch_forward(const Geom& g, const Plan& p, const MarchIO* io, int fields,
                          hipStream_t s) {
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
    }
    a.H = (const float2*)p.H;
    a.twx = (const float2*)p.twx;
    a.twy = (const float2*)p.twy;
    a.counter = (unsigned*)p.counter;
    a.nx = g.nx;
    a.ny = g.ny;
    a.steps = g.steps;
    a.fields = fields;
    a.k0dz = k0dz_of(g);
    return dispatch2(g.nx, g.ny, [&](auto xc, auto yc) {
        constexpr int NX = decltype(xc)::value, NY = decltype(yc)::value;
        void* args[] = {&a};
        if constexpr (NX >= 512 && NY >= 512) {
            if (fields >= 2)
                return hipLaunchCooperativeKernel(
                    reinterpret_cast<const void*>(&march_kernel<NX, NY, 2>),
                    dim3(persistent_grid<NX, NY>(g.nx, g.ny, fields, 2)), dim3(kBlock), args,
                    (unsigned)(march_data_lds<NX, NY>() + sizeof(float2) * (NX + NY)), s);
        }
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&march_kernel<NX, NY, 1>),
                                          dim3(persistent_grid<NX, NY>(g.nx, g.ny, fields)),
                                          dim3(kBlock), args, (unsigned)persistent_lds<NX, NY>(),
                                          s);
    });
}

size_t adjoint_fields(int steps, int K) {
    const int C = (steps + K - 1) / K;
    return (size_t)C + 2 * (size_t)K + 2;
}

hipError_t launch_adjoint(const Geom& g, const Plan& p, const AdjointIO& io, int K, void* fields,
                          hipStream_t s) {
    const size_t plane = (size_t)g.nx * g.ny;
    if (device_cus() <= 0) return hipErrorNoDevice;
    float2* f = (float2*)fields;
    const int C = (g.steps + K - 1) / K;
    AdjointArgs a{(const float2*)io.field_in, io.dn, (const float2*)io.grad_out, io.grad_inten,
                  (float2*)io.grad_in, (float2*)io.grad_spec, io.grad_dn, f, f + plane,
                  f + 2 * plane, f + (2 + (size_t)C) * plane,
                  (const float2*)p.H, (const float2*)p.twx, (const float2*)p.twy,
                  (const int*)p.permx, (const int*)p.permy, (unsigned*)p.counter, g.nx, g.ny,
                  g.steps, K, k0dz_of(g)};
    return dispatch2(g.nx, g.ny, [&](auto xc, auto yc) {
        constexpr int NX = decltype(xc)::value, NY = decltype(yc)::value;
        constexpr int BLK = NX <= 512 && NY <= 512 ? 64 : kBlock;
        void* args[] = {&a};
        return hipLaunchCooperativeKernel(
            reinterpret_cast<const void*>(&adjoint_kernel<NX, NY, BLK>),
            dim3(persistent_grid<NX, NY, BLK>(g.nx, g.ny, 2)), dim3(BLK), args,
            (unsigned)persistent_lds<NX, NY, BLK>(), s);
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

hipError_t launch_pupil_grad(const void* G, const void* U, long n, float* gphi, hipStream_t s) {
    const long blocks = (n + 255) / 256;
    pupil_grad_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(
        (const float2*)G, (const float2*)U, n, gphi);
    return hipGetLastError();
}

}  // namespace bpm
