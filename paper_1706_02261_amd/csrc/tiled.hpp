// Tiled field layout between the passes of the tiled march and of the work
// queue's tall jobs, and the row and column passes that read and write it.
//
// A column unit is W columns (W = 4096 / ny) and a row unit B rows
// (B = 4096 / nx).  A tile is TH = 16 / W rows x W columns of complex64: one
// 128-byte line.  The field between passes is stored tile by tile (tiles
// row-major, each tile row-major), and both passes give each thread a
// sequence of one unit (a row, or a column) interleaved with the unit's other
// B (or W) sequences across consecutive lanes: consecutive lanes then cover
// whole tiles, and every wavefront load or store touches whole lines, in the
// row pass and in the column pass alike.  (In the natural [y][x] layout a
// column pass of a 1024-long column reaches only 32 bytes of each line.)
// The layout needs W <= 16 and nx ny <= 2^20, so that a row unit is a whole
// number of tile rows (B = TH when nx ny = 2^20: 1024^2, 2048 x 512,
// 512 x 2048).  The B rows of a row unit then hold exactly the bytes of its B
// natural rows, so the head pass (natural in, tiled out) and the tail pass
// (tiled in, natural out) convert in place.
#pragma once

#include "passes.hpp"

namespace bpm {

template <int NX, int NY>
struct Tiles {
    static constexpr int B = units_per_block<NX>();  // rows of a row unit
    static constexpr int W = units_per_block<NY>();  // columns of a column unit: tile width
    static constexpr int TH = 16 / W;                // tile height
    static_assert(W <= 16 && TH * W == 16, "a tile is one 128-byte line of complex64");
    static_assert(B % TH == 0, "a row unit is a whole number of tile rows");
    __device__ static __forceinline__ size_t off(int y, int x) {
        return ((size_t)(y / TH) * (NX / W) + x / W) * 16 + (y % TH) * W + x % W;
    }
};

// Row unit `unit` (rows unit*B .. unit*B + B-1): thread (w, t) = (tid % B,
// tid / B) holds row unit*B + w at slots i T + t.  IN: kNaturalIn reads the
// natural field, kSpecIn the tiled spectrum.
template <int NX, int NY, int IN>
__device__ __forceinline__ void trow_load(int unit, const float2* src, float2 (&v)[kR]) {
    using TL = Tiles<NX, NY>;
    constexpr int T = NX / kR;
    const int w = threadIdx.x % TL::B, t = threadIdx.x / TL::B, y = unit * TL::B + w;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const int x = i * T + t;
        v[i] = ld_shared_field(src + (IN == kNaturalIn ? (size_t)y * NX + x : TL::off(y, x)));
    }
}

template <int NX, int NY>
__device__ __forceinline__ void trow_dn(int unit, const float* __restrict__ dn, float (&d)[kR]) {
    using TL = Tiles<NX, NY>;
    constexpr int T = NX / kR;
    const int w = threadIdx.x % TL::B, t = threadIdx.x / TL::B, y = unit * TL::B + w;
#pragma unroll
    for (int i = 0; i < kR; ++i) d[i] = dn[(size_t)y * NX + i * T + t];
}

// OPS: kNoOps or kScreen (screen, intensity).  OUT: kSpecOut (forward row
// FFTs, tiled) or kNaturalOut (natural u_{j+1} to a.dst).
template <int NX, int NY, int IN, int OPS, int OUT, typename Tw>
__device__ __forceinline__ void trow_body(int unit, const RowArgs& a, const float (&d)[kR],
                                          const Tw& twx, float2* smem, float2 (&v)[kR]) {
    using TL = Tiles<NX, NY>;
    constexpr int T = NX / kR;
    const int w = threadIdx.x % TL::B, t = threadIdx.x / TL::B, y = unit * TL::B + w;
    float2* lds = smem + w;
    const BlockSync sync;
    if constexpr (IN == kSpecIn) fft_inverse<NX, kR, TL::B>(v, lds, t, twx, sync);
    if constexpr (OPS == kScreen) {
        float ph[kR];
#pragma unroll
        for (int i = 0; i < kR; ++i) ph[i] = a.k0dz * d[i];
        apply_screen(v, ph);
        if (a.inten) {
#pragma unroll
            for (int i = 0; i < kR; ++i) a.inten[(size_t)y * NX + i * T + t] = c_abs2(v[i]);
        }
    }
    if constexpr (OUT == kSpecOut) {
        fft_forward<NX, kR, TL::B>(v, lds, t, twx, sync);
#pragma unroll
        for (int r = 0; r < kR; ++r) st_shared_field(a.dst + TL::off(y, r * T + t), v[r]);
    } else {
#pragma unroll
        for (int i = 0; i < kR; ++i) a.dst[(size_t)y * NX + i * T + t] = v[i];
    }
}

// Column unit `unit` (slots unit*W .. unit*W + W-1): thread (w, t) = (tid % W,
// tid / W) holds column unit*W + w at rows i T + t.
template <int NX, int NY>
__device__ __forceinline__ void tcol_load(int unit, const float2* work, float2 (&v)[kR]) {
    using TL = Tiles<NX, NY>;
    constexpr int T = NY / kR;
    const int w = threadIdx.x % TL::W, t = threadIdx.x / TL::W, x = unit * TL::W + w;
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = ld_shared_field(work + TL::off(i * T + t, x));
}

// the unit's propagator values, from a table stored in the same tiled layout
// (read-only: fetched before the grid barrier that guards the field)
template <int NX, int NY>
__device__ __forceinline__ void tcol_h(int unit, const float2* __restrict__ H,
                                       float2 (&h)[kR]) {
    using TL = Tiles<NX, NY>;
    constexpr int T = NY / kR;
    const int w = threadIdx.x % TL::W, t = threadIdx.x / TL::W, x = unit * TL::W + w;
#pragma unroll
    for (int r = 0; r < kR; ++r) h[r] = H[TL::off(r * T + t, x)];
}

template <int NX, int NY, typename Tw>
__device__ __forceinline__ void tcol_body(int unit, float2* work, const Tw& twy, float2* smem,
                                          float2 (&v)[kR], const float2 (&h)[kR]) {
    using TL = Tiles<NX, NY>;
    constexpr int T = NY / kR;
    const int w = threadIdx.x % TL::W, t = threadIdx.x / TL::W, x = unit * TL::W + w;
    float2* lds = smem + w;
    const BlockSync sync;
    fft_forward<NY, kR, TL::W>(v, lds, t, twy, sync);
#pragma unroll
    for (int r = 0; r < kR; ++r) v[r] = c_mul(v[r], h[r]);
    fft_inverse<NY, kR, TL::W>(v, lds, t, twy, sync);
#pragma unroll
    for (int i = 0; i < kR; ++i) st_shared_field(work + TL::off(i * T + t, x), v[i]);
}

}  // namespace bpm
