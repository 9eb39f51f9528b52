// Camera image of a fluorescent object through spatially varying PSFs
// (Fig. 1c): fluorescence adds intensities, so an emission slab E (the
// excitation times the fluorophore density at one depth, multiplied here) adds
//
//   image(x) += sum_{x'} E(x') sum_g phi_g(x') PSF_g(x - x')
//
// where PSF_g is the C x C detection PSF (centre C/2 = the emitter) of node g
// of a pitch-P grid (node (i, j) at pixel (P/2 + P i, P/2 + P j)) in the
// camera's focal plane, and phi_g the periodic bilinear hat weights of the
// nodes (a partition of unity).  Indices are periodic.
//
// One workgroup per 32 x 32 output tile (a deterministic gather: every output
// pixel is summed by one thread in a fixed order).  For each node within
// reach of the tile the workgroup stages the hat-weighted emission patch
// (32 + C - 1 square) and the node's PSF in LDS; a thread owns a column of
// four output pixels and walks the PSF rows with a sliding window of four
// emission values, so one LDS read of the patch serves four products.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace bpm {

namespace {

constexpr int kTile = 32;
constexpr int kCamBlock = 256;

__device__ inline int pmod(int a, int n) { return ((a % n) + n) % n; }

// hat weight of the node at g (pixels) for pixel y, periodic over n
__device__ inline float hat(int y, int g, int n, int pitch) {
    int d = pmod(y - g + n / 2, n) - n / 2;
    d = d < 0 ? -d : d;
    return d >= pitch ? 0.f : 1.f - (float)d / (float)pitch;
}

template <int C>
__global__ __launch_bounds__(kCamBlock) void camera_kernel(const float* __restrict__ E,
                                                           const float* __restrict__ D,
                                                           const float* __restrict__ psf,
                                                           int nx, int ny, int pitch,
                                                           float* __restrict__ image) {
    constexpr int H = kTile + C - 1;  // emitter rows / columns that reach the tile
    constexpr int LD = H + 2;         // odd-ish stride: rows 4 apart fall in other banks
    __shared__ float raw[H * LD];
    __shared__ float eg[H * LD];
    __shared__ float pg[C * C];
    __shared__ float wy[H], wx[H];
    const int ty0 = blockIdx.y * kTile, tx0 = blockIdx.x * kTile;
    const int py0 = ty0 + C / 2 - (C - 1), px0 = tx0 + C / 2 - (C - 1);
    const int gy = ny / pitch, gx = nx / pitch;
    for (int e = threadIdx.x; e < H * H; e += kCamBlock) {
        const int r = e / H, c = e % H;
        const size_t o = (size_t)pmod(py0 + r, ny) * nx + pmod(px0 + c, nx);
        raw[r * LD + c] = D ? E[o] * D[o] : E[o];
    }
    // candidate nodes along an axis: the consecutive nodes whose support
    // (g - pitch, g + pitch) meets the patch, at most all of them once
    auto first_node = [&](int p0) {
        // smallest i with pitch/2 + pitch i > p0 - pitch
        const int t = p0 - pitch - pitch / 2;
        return (t >= 0 ? t / pitch : -((-t + pitch - 1) / pitch)) + 1;
    };
    const int iy0 = first_node(py0), ix0 = first_node(px0);
    int ky = 0, kx = 0;
    while (ky < gy && pitch / 2 + pitch * (iy0 + ky) < py0 + H - 1 + pitch) ++ky;
    while (kx < gx && pitch / 2 + pitch * (ix0 + kx) < px0 + H - 1 + pitch) ++kx;

    const int x = threadIdx.x % kTile, y0 = (threadIdx.x / kTile) * 4;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < ky; ++a) {
        const int iy = pmod(iy0 + a, gy);
        for (int b = 0; b < kx; ++b) {
            const int ix = pmod(ix0 + b, gx);
            __syncthreads();  // the previous node's patch and PSF are consumed
            for (int r = threadIdx.x; r < H; r += kCamBlock) {
                wy[r] = hat(pmod(py0 + r, ny), pitch / 2 + pitch * iy, ny, pitch);
                wx[r] = hat(pmod(px0 + r, nx), pitch / 2 + pitch * ix, nx, pitch);
            }
            const float* pn = psf + ((size_t)iy * gx + ix) * C * C;
            for (int e = threadIdx.x; e < C * C; e += kCamBlock) pg[e] = pn[e];
            __syncthreads();
            for (int e = threadIdx.x; e < H * H; e += kCamBlock) {
                const int r = e / H, c = e % H;
                eg[r * LD + c] = raw[r * LD + c] * wy[r] * wx[c];
            }
            __syncthreads();
            // out(y, x) += sum_{r,c} eg[y + C-1 - r][x + C-1 - c] pg[r][c]
            for (int c = 0; c < C; ++c) {
                const float* col = eg + (x + C - 1 - c);
                // window rows for r = 0: y0 + C-1 .. y0 + C+2
                float w0 = col[(y0 + C - 1) * LD], w1 = col[(y0 + C) * LD];
                float w2 = col[(y0 + C + 1) * LD], w3 = col[(y0 + C + 2) * LD];
#pragma unroll 8
                for (int r = 0; r < C; ++r) {
                    const float p = pg[r * C + c];
                    acc[0] = fmaf(w0, p, acc[0]);
                    acc[1] = fmaf(w1, p, acc[1]);
                    acc[2] = fmaf(w2, p, acc[2]);
                    acc[3] = fmaf(w3, p, acc[3]);
                    // next r: rows shift down by one
                    w3 = w2;
                    w2 = w1;
                    w1 = w0;
                    if (r + 1 < C) w0 = col[(y0 + C - 2 - r) * LD];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t o = (size_t)(ty0 + y0 + k) * nx + tx0 + x;
        image[o] += acc[k];
    }
}

}  // namespace

hipError_t launch_camera(const float* excitation, const float* density, const float* node_psfs,
                         int nx, int ny, int pitch, int crop, float* image, hipStream_t s) {
    const dim3 grid(nx / kTile, ny / kTile);
    switch (crop) {
        case 16:
            camera_kernel<16><<<grid, kCamBlock, 0, s>>>(excitation, density, node_psfs, nx, ny,
                                                         pitch, image);
            break;
        case 32:
            camera_kernel<32><<<grid, kCamBlock, 0, s>>>(excitation, density, node_psfs, nx, ny,
                                                         pitch, image);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bpm
