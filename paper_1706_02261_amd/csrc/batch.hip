// Uneven batch of independent marches in one persistent launch.
//
// The work of every job is cut into items: one item is up to two units (a few
// rows or columns each) of one pass of one job.  The passes of job j are numbered
//   0          head row pass (forward row FFTs of u_0)
//   2s + 1     column pass of step s
//   2s + 2     row pass of step s (mid, or tail for the last step)
// and items are laid out round by round (all jobs' pass 0, then all jobs'
// pass 1, ...), jobs of equal size next to each other.  Workgroups claim items
// in that order from one atomic counter; before running an item of pass p a
// workgroup waits until job j has completed every item of passes < p (one
// monotone completion counter per job).  Because every item depends only on
// items earlier in the order, and an item is only claimed by a workgroup that
// is running, the earliest unfinished item can always proceed: the scheme
// needs no co-residency and cannot deadlock.  Jobs of different size and
// depth overlap freely; no grid-wide barrier exists.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "passes.hpp"
#include "tiled.hpp"

namespace bpm {

// Register twiddles whose transforms hide the thread index from the compiler
// (see LdsTwiddles), so that their LDS addresses are recomputed per call.
template <int N, int R>
struct OpaqueTwiddles : Twiddles<N, R> {
    static constexpr bool kOpaqueIndex = true;
};

// queue words: [0] next item, [16] time-out flag, [32 * (j + 1)] completed
// items of job j
__global__ void batch_zero_kernel(unsigned* q, int words) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
        q[i] = 0u;
}

// One item covers up to kUnitsPerItem consecutive units of one pass, two at a
// time (the second unit's loads are issued before the first unit is
// transformed); the queue and completion-counter round trips are shared.
// The per-size bodies are separate functions (not inlined into the item loop):
// with every transform length inlined into one kernel the compiler keeps each
// length's loop-invariant addresses live at once and spills.  Their pointer
// parameters carry the address spaces (LDS, global) so that the bodies still
// use LDS and global instructions.
typedef __attribute__((address_space(3))) float2 lds_float2;
typedef __attribute__((address_space(1))) float2 g_float2;
typedef __attribute__((address_space(1))) float g_float;

template <int NX>
__device__ __attribute__((noinline)) void batch_row(const g_float2* field_in, g_float2* work_g,
                                                    const g_float* dn, g_float* inten,
                                                    const g_float2* twx, int nx, int ny,
                                                    int steps, float k0dz, int clear, int pass,
                                                    int item, lds_float2* lds) {
    float2* smem = (float2*)lds;
    float2* work = (float2*)work_g;
    OpaqueTwiddles<NX, kR> tw;
    tw.load((const float2*)twx, threadIdx.x % (NX / kR));
    const int units = (ny + units_per_block<NX>() - 1) / units_per_block<NX>();
    const int s = pass / 2 - 1;
    const size_t plane = (size_t)nx * ny;
    for (int u0 = item * kUnitsPerItem; u0 < units && u0 < (item + 1) * kUnitsPerItem; u0 += 2) {
        const int u1 = u0 + 1;
        const bool two = u1 < units;
        float d0[kR], d1[kR];
        float2 va[kR], vb[kR];
        if (pass == 0) {
#pragma unroll
            for (int i = 0; i < kR; ++i) d0[i] = 0.f;
            const RowArgs ra{(const float2*)field_in, work, nullptr, nullptr, nullptr, nullptr,
                             nullptr, k0dz};
            row_load<NX, kNaturalIn>(u0, ny, ra.src, va);
            if (two) row_load<NX, kNaturalIn>(u1, ny, ra.src, vb);
            row_body<NX, kNaturalIn, kNoOps, kSpecOut>(u0, ny, ra, d0, tw, smem, va);
            if (two) row_body<NX, kNaturalIn, kNoOps, kSpecOut>(u1, ny, ra, d0, tw, smem, vb);
            continue;
        }
        const float* dns = (const float*)dn + s * plane;
        const RowArgs ra{work, work, inten ? (float*)inten + s * plane : nullptr, nullptr,
                         nullptr, nullptr, nullptr, k0dz};
        row_load<NX, kSpecIn>(u0, ny, ra.src, va);
        if (s >= clear)
            load_dn<NX>(d0, u0, ny, dns);
        else
            zero_dn(d0);
        if (two) {
            row_load<NX, kSpecIn>(u1, ny, ra.src, vb);
            if (s >= clear)
                load_dn<NX>(d1, u1, ny, dns);
            else
                zero_dn(d1);
        }
        if (s + 1 < steps) {
            row_body<NX, kSpecIn, kScreen, kSpecOut>(u0, ny, ra, d0, tw, smem, va);
            if (two) row_body<NX, kSpecIn, kScreen, kSpecOut>(u1, ny, ra, d1, tw, smem, vb);
        } else {
            row_body<NX, kSpecIn, kScreen, kNaturalOut>(u0, ny, ra, d0, tw, smem, va);
            if (two) row_body<NX, kSpecIn, kScreen, kNaturalOut>(u1, ny, ra, d1, tw, smem, vb);
        }
    }
}

template <int NY>
__device__ __attribute__((noinline)) void batch_col(g_float2* work_g, const g_float2* H_g,
                                                    const g_float2* twy, int nx, int item,
                                                    lds_float2* lds) {
    float2* smem = (float2*)lds;
    float2* work = (float2*)work_g;
    const float2* H = (const float2*)H_g;
    OpaqueTwiddles<NY, kR> tw;
    tw.load((const float2*)twy, threadIdx.x / units_per_block<NY>());
    const int units = (nx + units_per_block<NY>() - 1) / units_per_block<NY>();
    for (int u0 = item * kUnitsPerItem; u0 < units && u0 < (item + 1) * kUnitsPerItem; u0 += 2) {
        const int u1 = u0 + 1;
        const bool two = u1 < units;
        float2 va[kR], ha[kR], vb[kR], hb[kR];
        col_load<NY>(u0, nx, work, H, va, ha);
        if (two) col_load<NY>(u1, nx, work, H, vb, hb);
        col_body<NY, false>(u0, nx, work, tw, smem, nullptr, nullptr, nullptr, va, ha);
        if (two) col_body<NY, false>(u1, nx, work, tw, smem, nullptr, nullptr, nullptr, vb, hb);
    }
}

// The same row and column items for a job kept in the tiled layout of
// tiled.hpp between its passes (batch_tiled): the column pass of a
// 1024-long column then reads and writes whole lines instead of a quarter
// of each.  The head row pass converts natural -> tiled and the last row pass
// tiled -> natural in place, as in the tiled march.  In the tiled mapping a
// row or column spans every wavefront of the workgroup, so a workgroup
// barrier precedes each unit's transforms: the previous unit's last LDS
// reads (other wavefronts, possibly another layout of the slots) are done
// before this unit's first LDS writes.
template <int NX, int NY>
__device__ __attribute__((noinline)) void batch_trow(const g_float2* field_in, g_float2* work_g,
                                                     const g_float* dn, g_float* inten,
                                                     const g_float2* twx, int steps, float k0dz,
                                                     int clear, int pass, int item,
                                                     lds_float2* lds) {
    using TL = Tiles<NX, NY>;
    float2* smem = (float2*)lds;
    float2* work = (float2*)work_g;
    OpaqueTwiddles<NX, kR> tw;
    tw.load((const float2*)twx, threadIdx.x / TL::B);
    constexpr int units = NY / TL::B;
    constexpr size_t plane = (size_t)NX * NY;
    const int s = pass / 2 - 1;
    for (int u0 = item * kUnitsPerItem; u0 < units && u0 < (item + 1) * kUnitsPerItem; u0 += 2) {
        const int u1 = u0 + 1;
        const bool two = u1 < units;
        float d0[kR], d1[kR];
        float2 va[kR], vb[kR];
        if (pass == 0) {
#pragma unroll
            for (int i = 0; i < kR; ++i) d0[i] = 0.f;
            const RowArgs ra{(const float2*)field_in, work, nullptr, nullptr, nullptr, nullptr,
                             nullptr, k0dz};
            trow_load<NX, NY, kNaturalIn>(u0, ra.src, va);
            if (two) trow_load<NX, NY, kNaturalIn>(u1, ra.src, vb);
            __syncthreads();
            trow_body<NX, NY, kNaturalIn, kNoOps, kSpecOut>(u0, ra, d0, tw, smem, va);
            if (two) {
                __syncthreads();
                trow_body<NX, NY, kNaturalIn, kNoOps, kSpecOut>(u1, ra, d0, tw, smem, vb);
            }
            continue;
        }
        const float* dns = (const float*)dn + s * plane;
        const RowArgs ra{work, work, inten ? (float*)inten + s * plane : nullptr, nullptr,
                         nullptr, nullptr, nullptr, k0dz};
        trow_load<NX, NY, kSpecIn>(u0, ra.src, va);
        if (s >= clear)
            trow_dn<NX, NY>(u0, dns, d0);
        else
            zero_dn(d0);
        if (two) {
            trow_load<NX, NY, kSpecIn>(u1, ra.src, vb);
            if (s >= clear)
                trow_dn<NX, NY>(u1, dns, d1);
            else
                zero_dn(d1);
        }
        __syncthreads();
        if (s + 1 < steps)
            trow_body<NX, NY, kSpecIn, kScreen, kSpecOut>(u0, ra, d0, tw, smem, va);
        else
            trow_body<NX, NY, kSpecIn, kScreen, kNaturalOut>(u0, ra, d0, tw, smem, va);
        if (two) {
            __syncthreads();
            if (s + 1 < steps)
                trow_body<NX, NY, kSpecIn, kScreen, kSpecOut>(u1, ra, d1, tw, smem, vb);
            else
                trow_body<NX, NY, kSpecIn, kScreen, kNaturalOut>(u1, ra, d1, tw, smem, vb);
        }
    }
}

template <int NX, int NY>
__device__ __attribute__((noinline)) void batch_tcol(g_float2* work_g, const g_float2* H_g,
                                                     const g_float2* twy, int item,
                                                     lds_float2* lds) {
    using TL = Tiles<NX, NY>;
    float2* smem = (float2*)lds;
    float2* work = (float2*)work_g;
    const float2* H = (const float2*)H_g;
    OpaqueTwiddles<NY, kR> tw;
    tw.load((const float2*)twy, threadIdx.x / TL::W);
    constexpr int units = NX / TL::W;
    for (int u0 = item * kUnitsPerItem; u0 < units && u0 < (item + 1) * kUnitsPerItem; u0 += 2) {
        const int u1 = u0 + 1;
        const bool two = u1 < units;
        float2 va[kR], ha[kR], vb[kR], hb[kR];
        tcol_load<NX, NY>(u0, work, va);
        tcol_h<NX, NY>(u0, H, ha);
        if (two) {
            tcol_load<NX, NY>(u1, work, vb);
            tcol_h<NX, NY>(u1, H, hb);
        }
        __syncthreads();
        tcol_body<NX, NY>(u0, work, tw, smem, va, ha);
        if (two) {
            __syncthreads();
            tcol_body<NX, NY>(u1, work, tw, smem, vb, hb);
        }
    }
}

bool batch_tiled(int nx, int ny) { return ny >= 1024 && nx >= 256 && (long)nx * ny <= (1L << 20); }

// (nx, ny) of the tiled jobs, as one switch key
constexpr int tkey(int nx, int ny) { return nx * 4096 + ny; }

__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchJob* __restrict__ jobs,
                                                       const BatchSeg* __restrict__ segs,
                                                       int total, unsigned* q,
                                                       const unsigned long long* key_dev,
                                                       unsigned long long key, unsigned* status,
                                                       unsigned limit) {
    // the tables in the workspace belong to other jobs (or were never
    // written): take no item, touch nothing
    if (*key_dev != key) return;
    extern __shared__ float2 smem[];
    lds_float2* lds = (lds_float2*)smem;
    __shared__ int s_item;
    int cursor = 0;
    bool abort = false;
    if (threadIdx.x == 0) s_item = (int)__hip_atomic_fetch_add(q, 1u, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    int item = s_item;
    while (item < total) {
        // claim the next item now; its number is only needed at the end
        unsigned next = 0;
        if (threadIdx.x == 0)
            next = __hip_atomic_fetch_add(q, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (segs[cursor].first + segs[cursor].count <= item) ++cursor;
        const BatchSeg sg = segs[cursor];
        const BatchJob jb = jobs[sg.job];
        const int tile = item - sg.first;
        unsigned* done = q + 32 * (sg.job + 1);
        if (threadIdx.x == 0 && !abort) {
            unsigned spins = 0;
            while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                   (unsigned)sg.need) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > limit) {
                    __hip_atomic_store(q + 16, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    record_timeout(status, kStatusQueue);
                    abort = true;
                    break;
                }
            }
        }
        __syncthreads();
        if (jb.tiled) {
#define BPM_TILED_CASE(X, Y)                                                                   \
    case tkey(X, Y):                                                                           \
        if (sg.pass % 2 == 0)                                                                  \
            batch_trow<X, Y>((const g_float2*)jb.field_in, (g_float2*)jb.work,                 \
                             (const g_float*)jb.dn, (g_float*)jb.inten, (const g_float2*)jb.twx, \
                             jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds);                 \
        else                                                                                   \
            batch_tcol<X, Y>((g_float2*)jb.work, (const g_float2*)jb.H,                        \
                             (const g_float2*)jb.twy, tile, lds);                              \
        break;
            switch (tkey(jb.nx, jb.ny)) {
                BPM_TILED_CASE(256, 1024)
                BPM_TILED_CASE(512, 1024)
                BPM_TILED_CASE(1024, 1024)
                BPM_TILED_CASE(256, 2048)
                BPM_TILED_CASE(512, 2048)
                default: break;
            }
#undef BPM_TILED_CASE
        } else if (sg.pass % 2 == 0) {
            switch (jb.nx) {
                case 32: batch_row<32>((const g_float2*)jb.field_in, (g_float2*)jb.work, (const g_float*)jb.dn,
                                                  (g_float*)jb.inten, (const g_float2*)jb.twx, jb.nx,
                                                  jb.ny, jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds); break;
                case 64: batch_row<64>((const g_float2*)jb.field_in, (g_float2*)jb.work, (const g_float*)jb.dn,
                                                  (g_float*)jb.inten, (const g_float2*)jb.twx, jb.nx,
                                                  jb.ny, jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds); break;
                case 128: batch_row<128>((const g_float2*)jb.field_in, (g_float2*)jb.work, (const g_float*)jb.dn,
                                                  (g_float*)jb.inten, (const g_float2*)jb.twx, jb.nx,
                                                  jb.ny, jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds); break;
                case 256: batch_row<256>((const g_float2*)jb.field_in, (g_float2*)jb.work, (const g_float*)jb.dn,
                                                  (g_float*)jb.inten, (const g_float2*)jb.twx, jb.nx,
                                                  jb.ny, jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds); break;
                case 512: batch_row<512>((const g_float2*)jb.field_in, (g_float2*)jb.work, (const g_float*)jb.dn,
                                                  (g_float*)jb.inten, (const g_float2*)jb.twx, jb.nx,
                                                  jb.ny, jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds); break;
                case 1024: batch_row<1024>((const g_float2*)jb.field_in, (g_float2*)jb.work, (const g_float*)jb.dn,
                                                  (g_float*)jb.inten, (const g_float2*)jb.twx, jb.nx,
                                                  jb.ny, jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds); break;
                case 2048: batch_row<2048>((const g_float2*)jb.field_in, (g_float2*)jb.work, (const g_float*)jb.dn,
                                                  (g_float*)jb.inten, (const g_float2*)jb.twx, jb.nx,
                                                  jb.ny, jb.steps, jb.k0dz, jb.clear, sg.pass, tile, lds); break;
                default: break;
            }
        } else {
            switch (jb.ny) {
                case 32: batch_col<32>((g_float2*)jb.work, (const g_float2*)jb.H,
                                                  (const g_float2*)jb.twy, jb.nx, tile, lds); break;
                case 64: batch_col<64>((g_float2*)jb.work, (const g_float2*)jb.H,
                                                  (const g_float2*)jb.twy, jb.nx, tile, lds); break;
                case 128: batch_col<128>((g_float2*)jb.work, (const g_float2*)jb.H,
                                                  (const g_float2*)jb.twy, jb.nx, tile, lds); break;
                case 256: batch_col<256>((g_float2*)jb.work, (const g_float2*)jb.H,
                                                  (const g_float2*)jb.twy, jb.nx, tile, lds); break;
                case 512: batch_col<512>((g_float2*)jb.work, (const g_float2*)jb.H,
                                                  (const g_float2*)jb.twy, jb.nx, tile, lds); break;
                case 1024: batch_col<1024>((g_float2*)jb.work, (const g_float2*)jb.H,
                                                  (const g_float2*)jb.twy, jb.nx, tile, lds); break;
                case 2048: batch_col<2048>((g_float2*)jb.work, (const g_float2*)jb.H,
                                                  (const g_float2*)jb.twy, jb.nx, tile, lds); break;
                default: break;
            }
        }
        // every store of the item is complete before it is counted
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_item = (int)next;
        }
        __syncthreads();
        item = s_item;
    }
}

int batch_queue_words(int n_jobs) { return 32 * (n_jobs + 1); }


hipError_t launch_batch(const BatchJob* jobs_dev, const BatchSeg* segs_dev, int total,
                        unsigned* q, int n_jobs, const unsigned long long* key_dev,
                        unsigned long long key, unsigned* status, hipStream_t s) {
    const int words = batch_queue_words(n_jobs);
    batch_zero_kernel<<<(words + 255) / 256, 256, 0, s>>>(q, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || total == 0) return e;
    const int cus = device_cus();
    if (cus <= 0) return hipErrorNoDevice;
    // every size needs the same LDS: units_per_block * lds_size = 17 * 256 float2
    const size_t lds = sizeof(float2) * units_per_block<1024>() * lds_size<1024>();
    batch_kernel<<<cus, kBlock, lds, s>>>(jobs_dev, segs_dev, total, q, key_dev, key, status,
                                          wait_limit());
    return hipGetLastError();
}

int row_units(int nx, int ny) {
    const int b = kBlock / (nx / kR);
    return (ny + b - 1) / b;
}
int col_units(int nx, int ny) {
    const int w = kBlock / (ny / kR);
    return (nx + w - 1) / w;
}
int row_items(int nx, int ny) { return (row_units(nx, ny) + kUnitsPerItem - 1) / kUnitsPerItem; }
int col_items(int nx, int ny) { return (col_units(nx, ny) + kUnitsPerItem - 1) / kUnitsPerItem; }

}  // namespace bpm
