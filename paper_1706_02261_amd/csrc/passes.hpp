// Device building blocks shared by the persistent kernels: the fused row and
// column passes of one march step (forward and adjoint), agent-coherent field
// access and the grid barrier.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft.hpp"
#include "mathx.hpp"

namespace bpm {

constexpr int kR = 16;           // complex values per thread
constexpr int kBlock = 256;      // threads per workgroup
constexpr int kFieldBarWords = 1024;  // words of one grid barrier (4 KiB)
constexpr int kBarWords = 8 * kFieldBarWords;  // one barrier per lockstep field, in the plan

// rows (or columns) of length N one workgroup of BLK threads transforms at once
template <int N, int BLK = kBlock>
constexpr int units_per_block() { return BLK / (N / kR); }

// calls f(std::integral_constant<int, n>{}) for a supported transform length n
template <typename F>
__host__ inline hipError_t dispatch_size(int n, F&& f) {
    switch (n) {
        case 32: return f(std::integral_constant<int, 32>{});
        case 64: return f(std::integral_constant<int, 64>{});
        case 128: return f(std::integral_constant<int, 128>{});
        case 256: return f(std::integral_constant<int, 256>{});
        case 512: return f(std::integral_constant<int, 512>{});
        case 1024: return f(std::integral_constant<int, 1024>{});
        case 2048: return f(std::integral_constant<int, 2048>{});
        default: return hipErrorInvalidValue;
    }
}

// The field travels between the passes of a persistent march through global
// memory while the kernel runs.  The L2 caches of the eight XCDs are not
// coherent with each other, so every access to a buffer written inside the
// kernel is an agent-scope relaxed atomic (a load that does not hit a stale
// L2 line, a store that writes through to the device coherence point).
// Read-only data (propagator, twiddles, dn, dL/dI) keeps ordinary cached
// loads.
__device__ __forceinline__ float2 ld_shared_field(const float2* p) {
    const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, v);
}
__device__ __forceinline__ void st_shared_field(float2* p, float2 v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                       __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// pass bodies
//
// Every workgroup has 256 threads.  A row unit is B = 256 / (nx/16) rows, a
// column unit W = 256 / (ny/16) columns; units past the field's edge compute
// on row / column 0, store nothing and still take part in the barriers.

// workgroup-wide and wavefront-wide LDS ordering points
struct BlockSync {
    __device__ __forceinline__ void operator()() const { __syncthreads(); }
};
struct WaveSync {
    __device__ __forceinline__ void operator()() const {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// row FFTs of at most one wavefront only need wavefront-wide LDS ordering
template <int N>
using RowSync = typename std::conditional<(N / kR <= 64), WaveSync, BlockSync>::type;

// screen: v[i] *= exp(i ph[i]); when every phase of the wavefront lies in
// [-pi/4, pi/4] (the usual case: k0 dz dn is a fraction of a radian) the
// range reduction is skipped.
__device__ __forceinline__ void apply_screen(float2 (&v)[kR], const float (&ph)[kR]) {
    bool small = true;
#pragma unroll
    for (int i = 0; i < kR; ++i) small &= fabsf(ph[i]) <= kQuarterPi;
    if (__all(small)) {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = c_mul(v[i], cos_sin_quarter(ph[i]));
    } else {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = c_mul(v[i], expi(ph[i]));
    }
}

// dn of this thread's row unit, fetched ahead of the row pass
// dn of a step without a screen (the background medium)
__device__ __forceinline__ void zero_dn(float (&d)[kR]) {
#pragma unroll
    for (int i = 0; i < kR; ++i) d[i] = 0.f;
}

template <int NX, int BLK = kBlock>
__device__ __forceinline__ void load_dn(float (&d)[kR], int unit, int ny,
                                        const float* __restrict__ dn) {
    constexpr int T = NX / kR, B = units_per_block<NX, BLK>();
    const int row = unit * B + threadIdx.x / T, tau = threadIdx.x % T;
    const size_t rowoff = (size_t)(row < ny ? row : 0) * NX;
#pragma unroll
    for (int i = 0; i < kR; ++i) d[i] = dn[rowoff + i * T + tau];
}

// What a row pass takes, does and leaves.
enum RowIn : int { kSpecIn = 0, kNaturalIn = 1, kZeroIn = 2 };
enum RowOps : int { kNoOps = 0, kScreen = 1, kAdjointOps = 2 };
enum RowOut : int { kSpecOut = 0, kNaturalOut = 1, kNoOut = 2 };

struct RowArgs {
    const float2* src;  // spectrum (working buffer) or natural field
    float2* dst;        // spectrum (working buffer) or natural field
    float* inten;       // forward: I slice, or null
    float2* keep;       // forward: copy of the natural u_{j+1}, or null
    const float2* u;    // adjoint: natural u_{j+1} (read only when gI or gdn is set)
    const float* gI;    // adjoint: dL/dI slice, or null
    float* gdn;         // adjoint: dL/ddn slice, or null
    float k0dz;
};

// A row unit's field values (kSpecIn: spectrum, kNaturalIn: natural order);
// split from the computation so that a workgroup can issue the loads of its
// next unit before it works on the current one.
template <int NX, int IN, int BLK = kBlock>
__device__ __forceinline__ void row_load(int unit, int ny, const float2* src, float2 (&v)[kR]) {
    constexpr int T = NX / kR, B = units_per_block<NX, BLK>();
    const int row = unit * B + threadIdx.x / T, tau = threadIdx.x % T;
    const size_t rowoff = (size_t)(row < ny ? row : 0) * NX;
    if constexpr (IN == kZeroIn) {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = make_float2(0.f, 0.f);
    } else {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = ld_shared_field(src + rowoff + i * T + tau);
    }
}

template <int NX, int IN, int OPS, int OUT, int BLK = kBlock, typename Tw>
__device__ __forceinline__ void row_body(int unit, int ny, const RowArgs& a,
                                         const float (&d)[kR], const Tw& twx, float2* smem,
                                         float2 (&v)[kR]) {
    constexpr int T = NX / kR, B = units_per_block<NX, BLK>();
    const int sub = threadIdx.x / T, tau = threadIdx.x % T;
    const int row = unit * B + sub;
    const bool on = row < ny;
    const size_t rowoff = (size_t)(on ? row : 0) * NX;
    float2* lds = smem + sub * lds_size<NX>();
    const RowSync<NX> sync;
    // A row of more than one wavefront: the previous unit's last LDS reads
    // (by the other wavefronts of the row) may target the slots this unit's
    // first exchange writes, whenever the two units enter or leave the
    // transforms in different layouts (natural-order head or tail passes,
    // mixed units of the adjoint).  Within one wavefront LDS operations stay
    // in program order, so only multi-wavefront rows need this fence.
    if constexpr (NX / kR > 64) __syncthreads();
    if constexpr (IN == kSpecIn) fft_inverse<NX, kR, 1>(v, lds, tau, twx, sync);
    if constexpr (OPS == kScreen) {
        float ph[kR];
#pragma unroll
        for (int i = 0; i < kR; ++i) ph[i] = a.k0dz * d[i];
        apply_screen(v, ph);
        if (a.inten && on) {
#pragma unroll
            for (int i = 0; i < kR; ++i) a.inten[rowoff + i * T + tau] = c_abs2(v[i]);
        }
        if (a.keep && on) {
#pragma unroll
            for (int i = 0; i < kR; ++i) st_shared_field(a.keep + rowoff + i * T + tau, v[i]);
        }
    } else if constexpr (OPS == kAdjointOps) {
        float2 u[kR];
        if (a.gI || a.gdn) {
#pragma unroll
            for (int i = 0; i < kR; ++i) u[i] = ld_shared_field(a.u + rowoff + i * T + tau);
        }
        if (a.gI) {
#pragma unroll
            for (int i = 0; i < kR; ++i) {
                const float w = 2.f * a.gI[rowoff + i * T + tau];
                v[i] = make_float2(fmaf(w, u[i].x, v[i].x), fmaf(w, u[i].y, v[i].y));
            }
        }
        if (a.gdn && on) {
#pragma unroll
            for (int i = 0; i < kR; ++i)
                a.gdn[rowoff + i * T + tau] = a.k0dz * fmaf(v[i].y, u[i].x, -v[i].x * u[i].y);
        }
        float ph[kR];
#pragma unroll
        for (int i = 0; i < kR; ++i) ph[i] = -a.k0dz * d[i];
        apply_screen(v, ph);
    }
    if constexpr (OUT == kSpecOut) {
        fft_forward<NX, kR, 1>(v, lds, tau, twx, sync);
        if (on) {
#pragma unroll
            for (int r = 0; r < kR; ++r) st_shared_field(a.dst + rowoff + r * T + tau, v[r]);
        }
    } else if constexpr (OUT == kNaturalOut) {
        if (on) {
#pragma unroll
            for (int i = 0; i < kR; ++i) a.dst[rowoff + i * T + tau] = v[i];
        }
    }
}

template <int NX, int IN, int OPS, int OUT, int BLK = kBlock, typename Tw>
__device__ __forceinline__ void row_unit(int unit, int ny, const RowArgs& a,
                                         const float (&d)[kR], const Tw& twx, float2* smem) {
    float2 v[kR];
    row_load<NX, IN, BLK>(unit, ny, a.src, v);
    row_body<NX, IN, OPS, OUT, BLK>(unit, ny, a, d, twx, smem, v);
}

// Column pass on a working buffer: forward column FFTs, x H (or conj(H)),
// inverse column FFTs.  With spec_out, the multiplied spectrum is also written
// to spec_out in natural DFT order (the pupil-plane gradient).
template <int NY, int BLK = kBlock>
__device__ __forceinline__ void col_load(int unit, int nx, const float2* work,
                                         const float2* __restrict__ H, float2 (&v)[kR],
                                         float2 (&h)[kR]) {
    constexpr int T = NY / kR, W = units_per_block<NY, BLK>();
    const int c = unit * W + threadIdx.x % W, t = threadIdx.x / W;
    const size_t col = c < nx ? (size_t)c : 0;
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = ld_shared_field(work + (size_t)(i * T + t) * nx + col);
#pragma unroll
    for (int r = 0; r < kR; ++r) h[r] = H[(size_t)(r * T + t) * nx + col];
}

template <int NY, bool CONJ, int BLK = kBlock, typename Tw>
__device__ __forceinline__ void col_body(int unit, int nx, float2* work, const Tw& twy,
                                         float2* smem,
                                         float2* spec_out, const int* __restrict__ permx,
                                         const int* __restrict__ permy, float2 (&v)[kR],
                                         const float2 (&h)[kR]) {
    constexpr int T = NY / kR, W = units_per_block<NY, BLK>();
    const int w = threadIdx.x % W, t = threadIdx.x / W;
    const int c = unit * W + w;
    const bool on = c < nx;
    const size_t col = on ? (size_t)c : 0;
    float2* lds = smem + w;
    const BlockSync sync;
    fft_forward<NY, kR, W>(v, lds, t, twy, sync);
#pragma unroll
    for (int r = 0; r < kR; ++r) v[r] = CONJ ? c_mulc(v[r], h[r]) : c_mul(v[r], h[r]);
    if (spec_out && on) {
        const size_t m = (size_t)permx[col];
#pragma unroll
        for (int r = 0; r < kR; ++r) spec_out[(size_t)permy[r * T + t] * nx + m] = v[r];
    }
    fft_inverse<NY, kR, W>(v, lds, t, twy, sync);
    if (on) {
#pragma unroll
        for (int i = 0; i < kR; ++i) st_shared_field(work + (size_t)(i * T + t) * nx + col, v[i]);
    }
}

template <int NY, bool CONJ, int BLK = kBlock, typename Tw>
__device__ __forceinline__ void col_unit(int unit, int nx, float2* work,
                                         const float2* __restrict__ H, const Tw& twy,
                                         float2* smem,
                                         float2* spec_out, const int* __restrict__ permx,
                                         const int* __restrict__ permy) {
    float2 v[kR], h[kR];
    col_load<NY, BLK>(unit, nx, work, H, v, h);
    col_body<NY, CONJ, BLK>(unit, nx, work, twy, smem, spec_out, permx, permy, v, h);
}

// ---------------------------------------------------------------------------
// grid barrier of the persistent marches
//
// Two levels, no cache maintenance.  Workgroup b belongs to group b % 8 (the
// XCD the hardware deals it to).  Each arrival bumps its group's counter; the
// last arrival of a group bumps the global counter; the last group's closer
// publishes the barrier's generation to eight per-group flags, which the
// groups poll.  Every counter and flag sits in its own 128-byte line.  All of
// a wave's stores are complete (s_waitcnt) before its workgroup arrives, and
// buffers written inside the kernel are only accessed with agent-coherent
// operations, so no L2 write-back or invalidation is needed.
//
// Every workgroup is resident (cooperative launch), so the wait ends; as a
// guard against a launch that is not, the spin is bounded (`limit` polls) and
// a time-out is recorded, in the barrier's own word and in the workspace's
// sticky status word (bit kStatusBarrier, never cleared by a kernel; the host
// reads it through bpm_workspace_status), and ends all further waiting, so
// the kernel always exits.
//
// Barrier words (unsigned, zeroed by the plan kernel before every march):
//   [32 * g]        arrivals of group g        (g < 8)
//   [256 + 32 * g]  released generation of g
//   [512]           closed groups
//   [544]           time-out flag

// sticky status bits of a workspace's status header (word 0)
constexpr unsigned kStatusBarrier = 1u;  // a grid-barrier wait gave up
constexpr unsigned kStatusQueue = 2u;    // a work-queue dependency wait gave up

__device__ __forceinline__ void record_timeout(unsigned* status, unsigned bit) {
    __hip_atomic_fetch_or(status, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-workgroup phase timers of the persistent marches (a diagnostic, off
// unless the launch passes a buffer): the device's constant 100 MHz real-time
// counter, read uniformly, and the time since the previous mark charged to a
// phase.  Layout of the buffer: 8 header words {workgroups, ticks per second,
// steps, fields, 0...}, then 8 words per workgroup, one per phase.
enum Phase : int { kPhSetup = 0, kPhHead = 1, kPhCol = 2, kPhRow = 3, kPhDrain = 4, kPhWait = 5 };
constexpr int kPhaseWords = 8;
constexpr int kMaxTimedGroups = 4096;
struct PhaseTimers {
    unsigned long long* out;
    unsigned long long last;
    unsigned long long acc[kPhaseWords];
    __device__ __forceinline__ void start(unsigned long long* o) {
        out = o;
        for (int k = 0; k < kPhaseWords; ++k) acc[k] = 0;
        if (out) last = __builtin_amdgcn_s_memrealtime();
    }
    __device__ __forceinline__ void mark(int phase) {
        if (out) {
            const unsigned long long t = __builtin_amdgcn_s_memrealtime();
            acc[phase] += t - last;
            last = t;
        }
    }
    __device__ __forceinline__ void finish(int slot, int steps, int fields) {
        if (out && threadIdx.x == 0 && slot < kMaxTimedGroups) {
            if (slot == 0) {
                out[0] = gridDim.x;
                out[1] = 100000000ull;
                out[2] = (unsigned long long)steps;
                out[3] = (unsigned long long)fields;
            }
            for (int k = 0; k < kPhaseWords; ++k) out[kPhaseWords * (slot + 1) + k] = acc[k];
        }
    }
};

__device__ __forceinline__ void grid_sync(unsigned* bar, unsigned gen, bool& abort,
                                          unsigned* status, unsigned limit, PhaseTimers& tm) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    tm.mark(kPhDrain);
    if (threadIdx.x == 0) {
        const unsigned G = gridDim.x, g = blockIdx.x & 7u;
        const unsigned groups = G < 8u ? G : 8u;
        const unsigned members = (G - g + 7u) / 8u;
        const unsigned old = __hip_atomic_fetch_add(bar + 32 * g, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == gen * members) {
            const unsigned o2 = __hip_atomic_fetch_add(bar + 512, 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            if (o2 + 1u == gen * groups)
                for (unsigned k = 0; k < groups; ++k)
                    __hip_atomic_store(bar + 256 + 32 * k, gen, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        unsigned spins = 0;
        while (!abort && __hip_atomic_load(bar + 256 + 32 * g, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT) < gen) {
            if (++spins > limit) {
                __hip_atomic_store(bar + 544, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                record_timeout(status, kStatusBarrier);
                abort = true;
            }
        }
    }
    __syncthreads();
    tm.mark(kPhWait);
}

// grid_sync without timers
__device__ __forceinline__ void grid_sync(unsigned* bar, unsigned gen, bool& abort,
                                          unsigned* status, unsigned limit) {
    PhaseTimers none;
    none.start(nullptr);
    grid_sync(bar, gen, abort, status, limit, none);
}

// The same barrier split into its two halves, for marches that run several
// fields with one barrier each and do other work between arriving at one and
// waiting on it.  bar_arrive: thread 0, after the workgroup's stores of the
// phase are complete (s_waitcnt and a workgroup barrier before the call).
// bar_wait: every thread; returns once `gen` phases have completed everywhere.
// G workgroups take part; `index` (0 .. G-1) is this workgroup's place among
// them, which picks its group counter.
__device__ __forceinline__ void bar_arrive(unsigned* bar, unsigned gen, unsigned G,
                                           unsigned index) {
    const unsigned g = index & 7u;
    const unsigned groups = G < 8u ? G : 8u;
    const unsigned members = (G - g + 7u) / 8u;
    const unsigned old = __hip_atomic_fetch_add(bar + 32 * g, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1u == gen * members) {
        const unsigned o2 = __hip_atomic_fetch_add(bar + 512, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (o2 + 1u == gen * groups)
            for (unsigned k = 0; k < groups; ++k)
                __hip_atomic_store(bar + 256 + 32 * k, gen, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ void bar_wait(const unsigned* bar, unsigned gen, bool& abort,
                                         unsigned* status, unsigned limit, unsigned index) {
    if (threadIdx.x == 0) {
        const unsigned g = index & 7u;
        unsigned spins = 0;
        while (!abort && __hip_atomic_load(bar + 256 + 32 * g, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT) < gen) {
            if (++spins > limit) {
                __hip_atomic_store(const_cast<unsigned*>(bar) + 544, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                record_timeout(status, kStatusBarrier);
                abort = true;
            }
        }
    }
    __syncthreads();
}

// XCD-aware unit order: workgroups are dealt round-robin over the 8 XCDs, so
// give each XCD a contiguous range of units (neighbouring columns share cache
// lines).
__device__ __forceinline__ int virtual_block() {
    const int G = gridDim.x, b = blockIdx.x;
    return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
}

}  // namespace bpm
