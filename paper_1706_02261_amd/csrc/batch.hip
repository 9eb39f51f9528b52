// Uneven batch of independent marches in one persistent launch.
//
// The work of every job is cut into items: one item is one unit (a few rows
// or columns) of one pass of one job.  The passes of job j are numbered
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

namespace bpm {

// queue words: [0] next item, [16] time-out flag, [32 * (j + 1)] completed
// items of job j
__global__ void batch_zero_kernel(unsigned* q, int words) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
        q[i] = 0u;
}

template <int NX>
__device__ __forceinline__ void batch_row(const BatchJob& jb, int pass, int tile, float2* smem) {
    Twiddles<NX, kR> tw;
    tw.load((const float2*)jb.twx, threadIdx.x % (NX / kR));
    float d[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) d[i] = 0.f;
    if (pass == 0) {
        RowArgs ra{(const float2*)jb.field_in, (float2*)jb.work, nullptr, nullptr, nullptr, nullptr, nullptr, jb.k0dz};
        row_unit<NX, kNaturalIn, kNoOps, kSpecOut>(tile, jb.ny, ra, d, tw, smem);
        return;
    }
    const int s = pass / 2 - 1;
    const size_t plane = (size_t)jb.nx * jb.ny;
    load_dn<NX>(d, tile, jb.ny, jb.dn + s * plane);
    RowArgs ra{(const float2*)jb.work, (float2*)jb.work, jb.inten ? jb.inten + s * plane : nullptr, nullptr, nullptr,
               nullptr, nullptr, jb.k0dz};
    if (s + 1 < jb.steps)
        row_unit<NX, kSpecIn, kScreen, kSpecOut>(tile, jb.ny, ra, d, tw, smem);
    else
        row_unit<NX, kSpecIn, kScreen, kNaturalOut>(tile, jb.ny, ra, d, tw, smem);
}

template <int NY>
__device__ __forceinline__ void batch_col(const BatchJob& jb, int tile, float2* smem) {
    Twiddles<NY, kR> tw;
    tw.load((const float2*)jb.twy, threadIdx.x / units_per_block<NY>());
    col_unit<NY, false>(tile, jb.nx, (float2*)jb.work, (const float2*)jb.H, tw, smem, nullptr,
                        nullptr, nullptr);
}

__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchJob* __restrict__ jobs,
                                                       const BatchSeg* __restrict__ segs,
                                                       int total, unsigned* q) {
    extern __shared__ float2 smem[];
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
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(q + 16, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort = true;
                    break;
                }
            }
        }
        __syncthreads();
        if (sg.pass % 2 == 0) {
            switch (jb.nx) {
                case 32: batch_row<32>(jb, sg.pass, tile, smem); break;
                case 64: batch_row<64>(jb, sg.pass, tile, smem); break;
                case 128: batch_row<128>(jb, sg.pass, tile, smem); break;
                case 256: batch_row<256>(jb, sg.pass, tile, smem); break;
                case 512: batch_row<512>(jb, sg.pass, tile, smem); break;
                case 1024: batch_row<1024>(jb, sg.pass, tile, smem); break;
                case 2048: batch_row<2048>(jb, sg.pass, tile, smem); break;
                default: break;
            }
        } else {
            switch (jb.ny) {
                case 32: batch_col<32>(jb, tile, smem); break;
                case 64: batch_col<64>(jb, tile, smem); break;
                case 128: batch_col<128>(jb, tile, smem); break;
                case 256: batch_col<256>(jb, tile, smem); break;
                case 512: batch_col<512>(jb, tile, smem); break;
                case 1024: batch_col<1024>(jb, tile, smem); break;
                case 2048: batch_col<2048>(jb, tile, smem); break;
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

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

hipError_t launch_batch(const BatchJob* jobs_dev, const BatchSeg* segs_dev, int total,
                        unsigned* q, int n_jobs, hipStream_t s) {
    const int words = batch_queue_words(n_jobs);
    batch_zero_kernel<<<(words + 255) / 256, 256, 0, s>>>(q, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || total == 0) return e;
    const int cus = device_cus();
    if (cus <= 0) return hipErrorNoDevice;
    // every size needs the same LDS: units_per_block * lds_size = 17 * 256 float2
    const size_t lds = sizeof(float2) * units_per_block<1024>() * lds_size<1024>();
    batch_kernel<<<cus, kBlock, lds, s>>>(jobs_dev, segs_dev, total, q);
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

}  // namespace bpm
