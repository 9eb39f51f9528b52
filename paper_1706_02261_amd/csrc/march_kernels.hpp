// Kernel templates of the persistent marches (forward and adjoint) and their
// launchers, instantiated once per row length NX in march_x<NX>.hip so that
// the seven lengths compile in parallel.  See march.hip for the pass
// structure of one step.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "passes.hpp"
#include "tiled.hpp"

namespace bpm {

// ---------------------------------------------------------------------------
// persistent forward march

// LDS of the per-thread twiddle tables of both axes (in float2)
template <int NX, int NY>
__host__ __device__ constexpr size_t march_twiddle_lds() {
    return sizeof(float2) * (LdsTwiddleTable<NX, kR>::size() + LdsTwiddleTable<NY, kR>::size());
}

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
    unsigned* status;  // the workspace's sticky status word
    unsigned limit;    // polls of one barrier wait before it gives up
    unsigned long long* timers;  // phase timers (diagnostic) or null
    int nx, ny, steps, fields;
    int variant;  // kernel of the march (MarchVariant), resolved on the host
    float k0dz;
    int clear[kMaxFields];  // leading steps of each field without a screen
};

// OCC = workgroups per CU.  OCC 1 keeps the twiddles in registers and walks
// a workgroup's units two at a time (the second unit's loads in flight while
// the first is transformed).  OCC 2 (several fields) reads the twiddles from
// tables in LDS instead, so that two workgroups fit one CU (two waves per
// SIMD) and one workgroup's memory waits overlap the other's arithmetic.
// BLK = threads per workgroup: 256, or 64 (OCC 1 only) for small fields,
// whose passes then have four times as many units, spread over four times
// as many CUs (one wave per SIMD, up to four workgroups per CU).
template <int NX, int NY, int OCC, int BLK = kBlock>
__global__ __launch_bounds__(BLK, OCC) void march_kernel(MarchArgs a) {
    static_assert(BLK == kBlock || OCC == 1, "small workgroups keep their twiddles in registers");
    extern __shared__ float2 smem[];
    PhaseTimers tm;
    tm.start(a.timers);
    const int G = gridDim.x, v = virtual_block();
    const int rows_u = (a.ny + units_per_block<NX, BLK>() - 1) / units_per_block<NX, BLK>();
    const int cols_u = (a.nx + units_per_block<NY, BLK>() - 1) / units_per_block<NY, BLK>();
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
        twy.load(a.twy, threadIdx.x / units_per_block<NY, BLK>());
    } else {
        float2* tabx = smem + march_data_lds<NX, NY>() / sizeof(float2);
        float2* taby = tabx + LdsTwiddleTable<NX, kR>::size();
        LdsTwiddleTable<NX, kR>::fill(tabx, a.twx, threadIdx.x, kBlock);
        LdsTwiddleTable<NY, kR>::fill(taby, a.twy, threadIdx.x, kBlock);
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
    tm.mark(kPhSetup);
    for (int u = v; u < all_r; u += G) {
        const int f = u % F;
        RowArgs ra{a.field_in[f], a.work[f], nullptr, nullptr, nullptr, nullptr, nullptr, a.k0dz};
        row_unit<NX, kNaturalIn, kNoOps, kSpecOut, BLK>(u / F, a.ny, ra, d, twx, smem);
    }
    tm.mark(kPhHead);
    // a workgroup with a single row unit fetches its dn slice during the column pass
    const bool one_row_unit = all_r <= G;
    const int vv = v < all_r ? v : 0;
    for (int j = 0; j < a.steps; ++j) {
        if (one_row_unit) {
            if (j >= a.clear[vv % F])
                load_dn<NX, BLK>(d, vv / F, a.ny, a.dn[vv % F] + j * plane);
            else
                zero_dn(d);
        }
        tm.mark(kPhRow);
        grid_sync(a.counter, ++nbar, abort, a.status, a.limit, tm);
        for (int u = v; u < all_c; u += PAIR * G) {
            const int u2 = u + G;
            const bool two = PAIR == 2 && u2 < all_c;
            const int f1 = u % F, f2 = u2 % F;
            float2 va[kR], ha[kR], vb[kR], hb[kR];
            col_load<NY, BLK>(u / F, a.nx, a.work[f1], a.H, va, ha);
            if (two) col_load<NY, BLK>(u2 / F, a.nx, a.work[f2], a.H, vb, hb);
            col_body<NY, false, BLK>(u / F, a.nx, a.work[f1], twy, smem, nullptr, nullptr, nullptr,
                                     va, ha);
            if (two)
                col_body<NY, false, BLK>(u2 / F, a.nx, a.work[f2], twy, smem, nullptr, nullptr,
                                         nullptr, vb, hb);
        }
        tm.mark(kPhCol);
        grid_sync(a.counter, ++nbar, abort, a.status, a.limit, tm);
        for (int u = v; u < all_r; u += PAIR * G) {
            const int u2 = u + G;
            const bool two = PAIR == 2 && u2 < all_r;
            const int f1 = u % F, r1 = u / F;
            const int f2 = u2 % F, r2 = two ? u2 / F : 0;
            float2 va[kR], vb[kR];
            float db[kR];
            row_load<NX, kSpecIn, BLK>(r1, a.ny, a.work[f1], va);
            if (!one_row_unit) {
                if (j >= a.clear[f1])
                    load_dn<NX, BLK>(d, r1, a.ny, a.dn[f1] + j * plane);
                else
                    zero_dn(d);
            }
            if (two) {
                row_load<NX, kSpecIn, BLK>(r2, a.ny, a.work[f2], vb);
                if (j >= a.clear[f2])
                    load_dn<NX, BLK>(db, r2, a.ny, a.dn[f2] + j * plane);
                else
                    zero_dn(db);
            }
            const RowArgs ra{a.work[f1], a.work[f1],
                             a.inten[f1] ? a.inten[f1] + j * plane : nullptr, nullptr, nullptr,
                             nullptr, nullptr, a.k0dz};
            if (j + 1 < a.steps)
                row_body<NX, kSpecIn, kScreen, kSpecOut, BLK>(r1, a.ny, ra, d, twx, smem, va);
            else
                row_body<NX, kSpecIn, kScreen, kNaturalOut, BLK>(r1, a.ny, ra, d, twx, smem, va);
            if (two) {
                const RowArgs rb{a.work[f2], a.work[f2],
                                 a.inten[f2] ? a.inten[f2] + j * plane : nullptr, nullptr,
                                 nullptr, nullptr, nullptr, a.k0dz};
                if (j + 1 < a.steps)
                    row_body<NX, kSpecIn, kScreen, kSpecOut, BLK>(r2, a.ny, rb, db, twx, smem, vb);
                else
                    row_body<NX, kSpecIn, kScreen, kNaturalOut, BLK>(r2, a.ny, rb, db, twx, smem,
                                                                     vb);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    tm.mark(kPhRow);
    tm.finish(v, a.steps, a.fields);
}

// ---------------------------------------------------------------------------
// tiled march (one or two fields): a barrier per field, tiled field layout
//
// For NF = 1 or 2 fields whose passes have one unit per CU each
// (nx ny = 2^20).  NF workgroups per CU; every workgroup works on one field
// only, one unit of each of its field's passes, and each field has a grid
// barrier of its own.
// With two fields, workgroups are laid out so that the two that share a CU (dealt 256 apart:
// virtual ids 32 apart within one XCD's range) belong to different fields,
// while an XCD's workgroups of both fields hold the same 32-unit range (one
// slice of the propagator table in its L2).  When one field's workgroups wait
// at their barrier, the other field's workgroup on the same CU has the whole
// CU.  Between the passes the field is kept in the tiled layout of tiled.hpp
// (in field_out; the head and tail passes convert in place), and the plan
// stores the propagator table in the same layout.

template <int NX, int NY, int NF>
__global__ __launch_bounds__(kBlock, NF) void march_duo_kernel(MarchArgs a) {
    extern __shared__ float2 smem[];
    PhaseTimers tm;
    tm.start(a.timers);
    const int G = gridDim.x, v = virtual_block();
    const int Gx = G / 8, half = Gx / NF;           // workgroups per XCD, per field and XCD
    const int f = (v % Gx) / half;                  // this workgroup's field
    const int unit = (v / Gx) * half + v % half;    // its unit of every pass of that field
    const size_t plane = (size_t)NX * NY;
    unsigned* bar = a.counter + f * kFieldBarWords;
    const unsigned GF = (unsigned)(G / NF);
    bool abort = false;
    float2* tabx = smem + march_data_lds<NX, NY>() / sizeof(float2);
    float2* taby = tabx + LdsTwiddleTable<NX, kR>::size();
    LdsTwiddleTable<NX, kR>::fill(tabx, a.twx, threadIdx.x, kBlock);
    LdsTwiddleTable<NY, kR>::fill(taby, a.twy, threadIdx.x, kBlock);
    __syncthreads();
    const LdsTwiddles<NX, kR> twx{tabx, (int)threadIdx.x / Tiles<NX, NY>::B};
    const LdsTwiddles<NY, kR> twy{taby, (int)threadIdx.x / Tiles<NX, NY>::W};
    float d[kR];
    for (int i = 0; i < kR; ++i) d[i] = 0.f;
    tm.mark(kPhSetup);
    {
        const RowArgs ra{a.field_in[f], a.work[f], nullptr, nullptr, nullptr, nullptr, nullptr,
                         a.k0dz};
        float2 vals[kR];
        trow_load<NX, NY, kNaturalIn>(unit, ra.src, vals);
        trow_body<NX, NY, kNaturalIn, kNoOps, kSpecOut>(unit, ra, d, twx, smem, vals);
    }
    tm.mark(kPhHead);
    unsigned gen = 0;
    // a pass's stores complete, then the arrival; read-only data of the next
    // passes is fetched between the arrival and the wait
    auto arrive = [&]() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        tm.mark(kPhDrain);
        ++gen;
        if (threadIdx.x == 0) bar_arrive(bar, gen, GF, (unsigned)unit);
    };
    auto wait = [&]() {
        bar_wait(bar, gen, abort, a.status, a.limit, (unsigned)unit);
        tm.mark(kPhWait);
    };
    for (int j = 0; j < a.steps; ++j) {
        // the unit is the same every step; hidden from the compiler, so that it
        // recomputes the passes' addresses instead of keeping them all live
        int u = unit;
        asm volatile("" : "+s"(u));
        float2 vals[kR], h[kR];
        arrive();
        if (j >= a.clear[f])
            trow_dn<NX, NY>(u, a.dn[f] + (size_t)j * plane, d);
        else
            zero_dn(d);
        tcol_h<NX, NY>(u, a.H, h);
        wait();
        tcol_load<NX, NY>(u, a.work[f], vals);
        tcol_body<NX, NY>(u, a.work[f], twy, smem, vals, h);
        tm.mark(kPhCol);
        arrive();
        wait();
        asm volatile("" : "+s"(u));
        trow_load<NX, NY, kSpecIn>(u, a.work[f], vals);
        const RowArgs ra{a.work[f], a.work[f],
                         a.inten[f] ? a.inten[f] + (size_t)j * plane : nullptr, nullptr, nullptr,
                         nullptr, nullptr, a.k0dz};
        if (j + 1 < a.steps)
            trow_body<NX, NY, kSpecIn, kScreen, kSpecOut>(u, ra, d, twx, smem, vals);
        else
            trow_body<NX, NY, kSpecIn, kScreen, kNaturalOut>(u, ra, d, twx, smem, vals);
        tm.mark(kPhRow);
    }
    tm.finish(v, a.steps, a.fields);
}

// ---------------------------------------------------------------------------
// march with a locally adapted expansion of the refractive index
//
// Slice j is expanded about its own reference index nr_j = n0 + dn_ref[j]:
// the column pass multiplies by the exact propagator of a homogeneous medium
// of index nr_j, built on the fly (evanescent cut by the integer test of the
// plan kernel with nr_j in place of n0, kz in FP64, the phase dz kz turned
// into a unit phasor in FP32), and the row pass screens with dn - dn_ref[j].
// One field, one workgroup per CU, twiddles in registers; the propagator
// values of a column unit are formed before the barrier that guards the field.

struct AdaptArgs {
    const float2* field_in;
    float2* work;
    const float* dn;
    const float* dn_ref;  // [steps]
    float* inten;
    const float2* twx;
    const float2* twy;
    const int* permx;
    const int* permy;
    unsigned* counter;
    unsigned* status;
    unsigned limit;
    int nx, ny, steps;
    double dx, dz, lam, n0;
    float k0dz;
};

template <int NX, int NY>
__global__ __launch_bounds__(kBlock, 1) void march_adapted_kernel(AdaptArgs a) {
    extern __shared__ float2 smem[];
    const int G = gridDim.x, v = virtual_block();
    constexpr int B = units_per_block<NX>(), W = units_per_block<NY>(), T = NY / kR;
    const int rows_u = (a.ny + B - 1) / B, cols_u = (a.nx + W - 1) / W;
    const size_t plane = (size_t)a.nx * a.ny;
    unsigned nbar = 0;
    bool abort = false;
    Twiddles<NX, kR> twx;
    Twiddles<NY, kR> twy;
    twx.load(a.twx, threadIdx.x % (NX / kR));
    twy.load(a.twy, threadIdx.x / W);
    float d[kR];
    for (int i = 0; i < kR; ++i) d[i] = 0.f;
    for (int u = v; u < rows_u; u += G) {
        const RowArgs ra{a.field_in, a.work, nullptr, nullptr, nullptr, nullptr, nullptr, a.k0dz};
        row_unit<NX, kNaturalIn, kNoOps, kSpecOut>(u, a.ny, ra, d, twx, smem);
    }
    const double kPi = 3.14159265358979323846;
    const double k0 = 2.0 * kPi / a.lam;
    // transverse wave numbers per frequency index (one division per kernel,
    // not one per sample and step)
    const double kxs = 2.0 * kPi / (a.nx * a.dx), kys = 2.0 * kPi / (a.ny * a.dx);
    const float scale = (float)(1.0 / ((double)a.nx * (double)a.ny));
    const int w = threadIdx.x % W, t = threadIdx.x / W;
    for (int j = 0; j < a.steps; ++j) {
        const double nr = a.n0 + (double)a.dn_ref[j];
        const double kj2 = (nr * k0) * (nr * k0);
        const double ts = (double)a.nx * (double)a.ny * nr * a.dx / a.lam;
        const double thr = ts * ts;
        // this step's propagator values of the workgroup's first column unit
        auto propagator = [&](int u, float2 (&h)[kR]) {
            const int c = u * W + w;
            const int m = a.permx[c < a.nx ? c : 0];
            const long ms = m < a.nx / 2 ? m : m - a.nx;
            const double kx = kxs * (double)ms;
            const double a2 = (double)(ms * a.ny) * (double)(ms * a.ny);
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int l = a.permy[r * T + t];
                const long ls = l < a.ny / 2 ? l : l - a.ny;
                const double ky = kys * (double)ls;
                const double b2 = (double)(ls * a.nx) * (double)(ls * a.nx);
                float2 hv = make_float2(0.f, 0.f);
                if (a2 + b2 <= thr) {
                    const double kz = sqrt(fmax(kj2 - kx * kx - ky * ky, 0.0));
                    const float2 e = expi((float)(a.dz * kz));
                    hv = make_float2(e.x * scale, e.y * scale);
                }
                h[r] = hv;
            }
        };
        float2 h[kR];
        propagator(v, h);
        grid_sync(a.counter, ++nbar, abort, a.status, a.limit);
        for (int u = v; u < cols_u; u += G) {
            if (u != v) propagator(u, h);
            float2 vals[kR];
            const int c = u * W + w;
            const size_t col = c < a.nx ? (size_t)c : 0;
#pragma unroll
            for (int i = 0; i < kR; ++i) vals[i] = ld_shared_field(a.work + (size_t)(i * T + t) * a.nx + col);
            col_body<NY, false>(u, a.nx, a.work, twy, smem, nullptr, nullptr, nullptr, vals, h);
        }
        grid_sync(a.counter, ++nbar, abort, a.status, a.limit);
        const float ref = a.dn_ref[j];
        for (int u = v; u < rows_u; u += G) {
            float2 vals[kR];
            row_load<NX, kSpecIn>(u, a.ny, a.work, vals);
            load_dn<NX>(d, u, a.ny, a.dn + (size_t)j * plane);
#pragma unroll
            for (int i = 0; i < kR; ++i) d[i] -= ref;
            const RowArgs ra{a.work, a.work, a.inten ? a.inten + (size_t)j * plane : nullptr,
                             nullptr, nullptr, nullptr, nullptr, a.k0dz};
            if (j + 1 < a.steps)
                row_body<NX, kSpecIn, kScreen, kSpecOut>(u, a.ny, ra, d, twx, smem, vals);
            else
                row_body<NX, kSpecIn, kScreen, kNaturalOut>(u, a.ny, ra, d, twx, smem, vals);
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
// Memory per field: ceil(N/K) + 2 K + 2 fields (K + 2 more than the
// checkpoints and one segment); compute: about three forward marches in
// about two marches' worth of passes.
//
// Up to kMaxFields adjoints of one geometry (one plan, one step count and
// checkpoint interval) run in lockstep: every pass covers the units of all
// fields, so they share each grid barrier.  Combined unit u is unit u / F of
// field u % F; with one field this is the single-field unit order.

struct AdjointArgs {
    const float2* field_in[kMaxFields];
    const float* dn[kMaxFields];
    const float2* gout[kMaxFields];  // dL/du_N or null
    const float* gI[kMaxFields];     // dL/dI or null
    float2* gin[kMaxFields];         // dL/du_0 or null
    float2* gspec[kMaxFields];       // dL/dU_0 or null
    float* gdn[kMaxFields];          // dL/ddn or null
    float2* fwork[kMaxFields];
    float2* gwork[kMaxFields];
    float2* ckpt[kMaxFields];  // [ceil(N/K)] fields (slot 0 unused: u_0 is field_in)
    float2* seg[kMaxFields];   // [2 K] fields: two segment buffers
    const float2* H;
    const float2* twx;
    const float2* twy;
    const int* permx;
    const int* permy;
    unsigned* counter;
    unsigned* status;
    unsigned limit;
    int nx, ny, steps, K, fields;
    int linear;  // no field takes intensity or dn gradients
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
    const int N = a.steps, K = a.K, C = (N + K - 1) / K, F = a.fields;
    unsigned nbar = 0;
    bool abort = false;
    Twiddles<NX, kR> twx;
    Twiddles<NY, kR> twy;
    twx.load(a.twx, threadIdx.x % (NX / kR));
    twy.load(a.twy, threadIdx.x / units_per_block<NY, BLK>());
    float d[kR];
    for (int i = 0; i < kR; ++i) d[i] = 0.f;

    // Without intensity and dn gradients the adjoint is the linear map M^H
    // applied to gout: the adjoint steps read no forward field, so the
    // checkpoint march and the segment recomputes are skipped.
    const bool linear = a.linear != 0;

    // 1. checkpoints u_K, u_2K, ..., u_(C-1)K.  A field without a forward
    // field (a linear job among others) has no forward units: its adjoint
    // steps read no u.
    if (C > 1 && !linear) {
        for (int u = v; u < rows_u * F; u += G) {
            const int f = u % F;
            if (!a.field_in[f]) continue;
            const RowArgs ra{a.field_in[f], a.fwork[f], nullptr, nullptr, nullptr, nullptr,
                             nullptr, a.k0dz};
            row_unit<NX, kNaturalIn, kNoOps, kSpecOut, BLK>(u / F, a.ny, ra, d, twx, smem);
        }
        const int last = (C - 1) * K;
        for (int j = 0; j < last; ++j) {
            grid_sync(a.counter, ++nbar, abort, a.status, a.limit);
            for (int u = v; u < cols_u * F; u += G)
                if (a.field_in[u % F])
                    col_unit<NY, false, BLK>(u / F, a.nx, a.fwork[u % F], a.H, twy, smem, nullptr,
                                             nullptr, nullptr);
            grid_sync(a.counter, ++nbar, abort, a.status, a.limit);
            for (int u = v; u < rows_u * F; u += G) {
                const int f = u % F;
                if (!a.field_in[f]) continue;
                const RowArgs ra{a.fwork[f], a.fwork[f], nullptr,
                                 ((j + 1) % K == 0) ? a.ckpt[f] + (size_t)((j + 1) / K) * plane
                                                    : nullptr,
                                 nullptr, nullptr, nullptr, a.k0dz};
                load_dn<NX, BLK>(d, u / F, a.ny, a.dn[f] + j * plane);
                if (j + 1 < last)
                    row_unit<NX, kSpecIn, kScreen, kSpecOut, BLK>(u / F, a.ny, ra, d, twx, smem);
                else
                    row_unit<NX, kSpecIn, kScreen, kNoOut, BLK>(u / F, a.ny, ra, d, twx, smem);
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
    auto seg_of = [&](int f, int c) { return a.seg[f] + (size_t)(c & 1) * K * plane; };
    auto len_of = [&](int c) { return N - c * K < K ? N - c * K : K; };
    // units of pass i (per field): recompute: 0 head row, odd column, even
    // row; adjoint: even row, odd column
    auto pass_units = [&](int i) { return i % 2 == 0 ? rows_u : cols_u; };
    auto rec_unit = [&](int c, int i, int f, int u) {
        if (!a.field_in[f]) return;
        if (i == 0) {
            const RowArgs fr{c == 0 ? a.field_in[f] : a.ckpt[f] + (size_t)c * plane, a.fwork[f],
                             nullptr, nullptr, nullptr, nullptr, nullptr, a.k0dz};
            row_unit<NX, kNaturalIn, kNoOps, kSpecOut, BLK>(u, a.ny, fr, d, twx, smem);
        } else if (i % 2 == 1) {
            col_unit<NY, false, BLK>(u, a.nx, a.fwork[f], a.H, twy, smem, nullptr, nullptr,
                                     nullptr);
        } else {
            const int t = i / 2 - 1;
            const RowArgs fr{a.fwork[f], a.fwork[f], nullptr, seg_of(f, c) + (size_t)t * plane,
                             nullptr, nullptr, nullptr, a.k0dz};
            load_dn<NX, BLK>(d, u, a.ny, a.dn[f] + (size_t)(c * K + t) * plane);
            if (t + 1 < len_of(c))
                row_unit<NX, kSpecIn, kScreen, kSpecOut, BLK>(u, a.ny, fr, d, twx, smem);
            else
                row_unit<NX, kSpecIn, kScreen, kNoOut, BLK>(u, a.ny, fr, d, twx, smem);
        }
    };
    auto adj_unit = [&](int c, int i, int f, int u) {
        const int s = len_of(c) - 1 - i / 2, j = c * K + s;
        if (i % 2 == 0) {
            RowArgs br{a.gwork[f], a.gwork[f], nullptr, nullptr, seg_of(f, c) + (size_t)s * plane,
                       a.gI[f] ? a.gI[f] + (size_t)j * plane : nullptr,
                       a.gdn[f] ? a.gdn[f] + (size_t)j * plane : nullptr, a.k0dz};
            load_dn<NX, BLK>(d, u, a.ny, a.dn[f] + (size_t)j * plane);
            if (j + 1 < N) {
                row_unit<NX, kSpecIn, kAdjointOps, kSpecOut, BLK>(u, a.ny, br, d, twx, smem);
            } else if (a.gout[f]) {
                br.src = a.gout[f];
                row_unit<NX, kNaturalIn, kAdjointOps, kSpecOut, BLK>(u, a.ny, br, d, twx, smem);
            } else {
                row_unit<NX, kZeroIn, kAdjointOps, kSpecOut, BLK>(u, a.ny, br, d, twx, smem);
            }
        } else {
            col_unit<NY, true, BLK>(u, a.nx, a.gwork[f], a.H, twy, smem,
                                    j == 0 ? a.gspec[f] : nullptr, a.permx, a.permy);
        }
    };
    // the last segment's recompute alone, then adjoint c with recompute c - 1
    if (!linear) {
        for (int i = 0; i < 2 * len_of(C - 1) + 1; ++i) {
            grid_sync(a.counter, ++nbar, abort, a.status, a.limit);
            for (int u = v; u < pass_units(i) * F; u += G) rec_unit(C - 1, i, u % F, u / F);
        }
    }
    for (int c = C - 1; c >= 0; --c) {
        const int PA = 2 * len_of(c), PR = c > 0 && !linear ? 2 * len_of(c - 1) + 1 : 0;
        for (int i = 0; i < (PA > PR ? PA : PR); ++i) {
            grid_sync(a.counter, ++nbar, abort, a.status, a.limit);
            const int na = i < PA ? pass_units(i) * F : 0, nr = i < PR ? pass_units(i) * F : 0;
            for (int u = v; u < na + nr; u += G) {
                if (u < na)
                    adj_unit(c, i, u % F, u / F);
                else
                    rec_unit(c - 1, i, (u - na) % F, (u - na) / F);
            }
        }
    }

    // 3. g_0 in natural order
    bool tail = false;
    for (int f = 0; f < F; ++f) tail = tail || a.gin[f] != nullptr;
    if (tail) {
        grid_sync(a.counter, ++nbar, abort, a.status, a.limit);
        for (int u = v; u < rows_u * F; u += G) {
            const int f = u % F;
            if (!a.gin[f]) continue;
            const RowArgs tr{a.gwork[f], a.gin[f], nullptr, nullptr, nullptr, nullptr, nullptr,
                             a.k0dz};
            row_unit<NX, kSpecIn, kNoOps, kNaturalOut, BLK>(u / F, a.ny, tr, d, twx, smem);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers

template <int NX, int NY, int BLK = kBlock>
inline size_t persistent_lds() {
    const size_t lds_r = sizeof(float2) * units_per_block<NX, BLK>() * lds_size<NX>();
    const size_t lds_c = sizeof(float2) * units_per_block<NY, BLK>() * lds_size<NY>();
    return lds_r > lds_c ? lds_r : lds_c;
}

template <int NX, int NY, int BLK = kBlock>
inline int persistent_grid(int nx, int ny, int fields = 1, int per_cu = 1) {
    const int rows_u = (ny + units_per_block<NX, BLK>() - 1) / units_per_block<NX, BLK>();
    const int cols_u = (nx + units_per_block<NY, BLK>() - 1) / units_per_block<NY, BLK>();
    const int cus = device_cus() * per_cu;
    const int grid = (rows_u > cols_u ? rows_u : cols_u) * fields;
    return grid > cus ? cus : grid;
}

// calls f(std::integral_constant<int, ny>{}) for a supported column length
template <typename F>
inline hipError_t dispatch_ny(int ny, F&& f) {
    return dispatch_size(ny, f);
}

template <int NX>
hipError_t launch_forward_x(const MarchArgs& a, hipStream_t s) {
    return dispatch_ny(a.ny, [&](auto yc) {
        constexpr int NY = decltype(yc)::value;
        void* args[] = {const_cast<MarchArgs*>(&a)};
        const int cus = device_cus();
        if constexpr (units_per_block<NX>() * units_per_block<NY>() == 16) {
            if (a.variant == kMarchTiledPair && a.fields == 2)
                return hipLaunchCooperativeKernel(
                    reinterpret_cast<const void*>(&march_duo_kernel<NX, NY, 2>), dim3(2 * cus),
                    dim3(kBlock), args,
                    (unsigned)(march_data_lds<NX, NY>() + march_twiddle_lds<NX, NY>()), s);
            if (a.variant == kMarchTiledPair && a.fields == 1)
                return hipLaunchCooperativeKernel(
                    reinterpret_cast<const void*>(&march_duo_kernel<NX, NY, 1>), dim3(cus),
                    dim3(kBlock), args,
                    (unsigned)(march_data_lds<NX, NY>() + march_twiddle_lds<NX, NY>()), s);
        }
        if constexpr (NX >= 512 && NY >= 512) {
            if (a.variant == kMarchTwoPerCu)
                return hipLaunchCooperativeKernel(
                    reinterpret_cast<const void*>(&march_kernel<NX, NY, 2>),
                    dim3(persistent_grid<NX, NY>(a.nx, a.ny, a.fields, 2)), dim3(kBlock), args,
                    (unsigned)(march_data_lds<NX, NY>() + march_twiddle_lds<NX, NY>()), s);
        }
        if constexpr (NX <= 1024 && NY <= 1024) {
            if (a.variant == kMarchSmallBlocks)
                return hipLaunchCooperativeKernel(
                    reinterpret_cast<const void*>(&march_kernel<NX, NY, 1, 64>),
                    dim3(persistent_grid<NX, NY, 64>(a.nx, a.ny, a.fields, 4)), dim3(64), args,
                    (unsigned)persistent_lds<NX, NY, 64>(), s);
        }
        if (a.variant != kMarchOnePerCu) return hipErrorInvalidConfiguration;
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&march_kernel<NX, NY, 1>),
                                          dim3(persistent_grid<NX, NY>(a.nx, a.ny, a.fields)),
                                          dim3(kBlock), args, (unsigned)persistent_lds<NX, NY>(),
                                          s);
    });
}
template <int NX>
hipError_t launch_adjoint_x(const AdjointArgs& a, hipStream_t s) {
    return dispatch_ny(a.ny, [&](auto yc) {
        constexpr int NY = decltype(yc)::value;
        constexpr int BLK = NX <= 512 && NY <= 512 ? 64 : kBlock;
        void* args[] = {const_cast<AdjointArgs*>(&a)};
        // A mixed pass holds two units per field, one workgroup each.  Small
        // fields take 64-thread workgroups, so that one field spreads over
        // many CUs; when several fields fill at least half the CUs with
        // 256-thread workgroups, those are faster (fewer workgroups at each
        // barrier: 8 x 256^2 x 512 in 15.9 ms against 18.3 ms with four
        // 64-thread workgroups per CU, 4 x 256^2 x 512 in 13.1 against
        // 13.9 ms, 2 x 512^2 x 256 in 10.6 ms against 13.1 ms).
        if constexpr (BLK == 64 && NX * NY >= 65536) {
            if (a.fields > 1 &&
                persistent_grid<NX, NY, kBlock>(a.nx, a.ny, 2 * a.fields) >= device_cus() / 2)
                return hipLaunchCooperativeKernel(
                    reinterpret_cast<const void*>(&adjoint_kernel<NX, NY, kBlock>),
                    dim3(persistent_grid<NX, NY, kBlock>(a.nx, a.ny, 2 * a.fields)),
                    dim3(kBlock), args, (unsigned)persistent_lds<NX, NY, kBlock>(), s);
        }
        // else up to four 64-thread workgroups per CU for several small fields
        const int per_cu = BLK == 64 && a.fields > 1 ? 4 : 1;
        return hipLaunchCooperativeKernel(
            reinterpret_cast<const void*>(&adjoint_kernel<NX, NY, BLK>),
            dim3(persistent_grid<NX, NY, BLK>(a.nx, a.ny, 2 * a.fields, per_cu)), dim3(BLK),
            args, (unsigned)persistent_lds<NX, NY, BLK>(), s);
    });
}

static_assert(kPhaseTimerWords == kPhaseWords * (kMaxTimedGroups + 1), "timer layout");

template <int NX>
hipError_t launch_adapted_x(const AdaptArgs& a, hipStream_t s) {
    return dispatch_ny(a.ny, [&](auto yc) {
        constexpr int NY = decltype(yc)::value;
        void* args[] = {const_cast<AdaptArgs*>(&a)};
        return hipLaunchCooperativeKernel(
            reinterpret_cast<const void*>(&march_adapted_kernel<NX, NY>),
            dim3(persistent_grid<NX, NY>(a.nx, a.ny, 1)), dim3(kBlock), args,
            (unsigned)persistent_lds<NX, NY>(), s);
    });
}

// one translation unit per row length
#define BPM_MARCH_INSTANTIATE(NX)                                                  \
    template hipError_t launch_forward_x<NX>(const MarchArgs&, hipStream_t);      \
    template hipError_t launch_adjoint_x<NX>(const AdjointArgs&, hipStream_t);    \
    template hipError_t launch_adapted_x<NX>(const AdaptArgs&, hipStream_t);
#define BPM_MARCH_EXTERN(NX)                                                       \
    extern template hipError_t launch_forward_x<NX>(const MarchArgs&, hipStream_t); \
    extern template hipError_t launch_adjoint_x<NX>(const AdjointArgs&, hipStream_t); \
    extern template hipError_t launch_adapted_x<NX>(const AdaptArgs&, hipStream_t);

}  // namespace bpm
