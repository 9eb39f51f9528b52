// Learned PSF surrogate: BF16 matrix-core kernels (FP32 accumulation).
//
// Activations are channels-last (N, D, H, W, C) bf16 and the reduction index
// of every convolution is ordered (tap, channel) with channels fastest, so the
// 8 consecutive K values a lane feeds to v_mfma_f32_32x32x16_bf16 are 8
// consecutive channels of one input voxel: one 16-byte load.  Weights are
// [Co][Kp] bf16 (K = taps * Ci zero-padded to a multiple of 16).
//
// Operand layout of v_mfma_f32_32x32x16_bf16 (checked on the device against a
// host matmul): lane l supplies A[l % 32][8 (l / 32) + j] and
// B[8 (l / 32) + j][l % 32], j < 8; accumulator i of lane l is
// D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"

namespace bpm {
namespace sg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16;

__device__ __forceinline__ u16 f2bf(float f) {  // round to nearest even
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ float softplus(float z) { return z > 20.f ? z : log1pf(expf(z)); }
__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + expf(-z)); }

// ---------------------------------------------------------------------------
// convolution forward: y = act(conv(x) + bias)
//   EPI 0: ReLU, bf16 channels-last output
//   EPI 1: softplus, fp32 output [N][Co][Ho][Wo] (Do == 1) and the
//          pre-activation kept in the same layout
//
// A workgroup computes 32 output channels of an output tile of TY rows x Wo
// columns of one (n, oz) plane (TY = min(Ho, 128 / Wo)); wave w takes the
// flattened tile positions [32 w, 32 w + 32).  The tile's input footprint,
// kd x FY x FX voxels with FY = (TY - 1) sh + kh and FX = (Wo - 1) sw + kw, is
// staged in LDS once (zero outside the input; channel stride CiP = Ci, plus 8
// when Ci >= 32 against bank conflicts), so each input voxel crosses the
// memory system once per tile instead of once per tap.

// The network's input channels of voxel (z, y, x) of a [64][32][32] patch:
// dn / 0.05, the mask [z >= depth], (y - 15.5) / 16, (x - 15.5) / 16, their
// squared norm, zeros.
__device__ __forceinline__ uint4 input_channels(float dn, float depth, int z, int y, int x) {
    const float m = (float)z >= depth ? 1.f : 0.f;
    const float cy = ((float)y - 15.5f) * 0.0625f, cx = ((float)x - 15.5f) * 0.0625f;
    const float r2 = cy * cy + cx * cx;
    return make_uint4(f2bf(dn * 20.f) | ((unsigned)f2bf(m) << 16),
                      f2bf(cy) | ((unsigned)f2bf(cx) << 16), f2bf(r2), 0);
}

// Where the staged input comes from:
//   kInBf16   x is the bf16 activation [N][D][H][W][Ci];
//   kInPatch  x is the fp32 dn patch [N][64][32][32] (Ci = 8): the network's
//             input channels are formed while staging (depth[] per sample);
//   kInUp2    x is the bf16 map [N][D][H/2][W/2][Ci] read through a nearest
//             x2 upsampling in y and x.
enum ConvIn : int { kInBf16 = 0, kInPatch = 1, kInUp2 = 2 };

template <int EPI, int IN>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const void* __restrict__ xin,
                                                       const float* __restrict__ depth,
                                                       const u16* __restrict__ w,
                                                       const float* __restrict__ bias, ConvGeo c,
                                                       FwdTile t, const int4* __restrict__ taps,
                                                       u16* ybf, float* yf, float* zkeep) {
    extern __shared__ uint4 lds_raw[];
    u16* xs = reinterpret_cast<u16*>(lds_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
    int b = blockIdx.x;
    const int ty = b % t.tiles_y;
    b /= t.tiles_y;
    const int oz = b % c.Do, n = b / c.Do;
    const int oy0 = ty * t.TY;
    const int iz0 = oz * c.sd - c.pd, iy0 = oy0 * c.sh - c.ph, ix0 = -c.pw;
    const int cch = c.Ci / 8;
    const int total = c.kd * t.FY * t.FX * cch;
    // staging: each thread issues the loads of up to kStageBatch chunks before
    // it writes any of them to LDS, so their memory latencies overlap
    constexpr int kStageBatch = 8;
    using Raw = typename std::conditional<IN == kInPatch, float, uint4>::type;
    auto voxel = [&](int e, int& c8, int& iz, int& iy, int& ix, int& slot) {
        int q = e;
        c8 = q % cch;
        q /= cch;
        const int fx = q % t.FX;
        q /= t.FX;
        const int fy = q % t.FY, fz = q / t.FY;
        iz = iz0 + fz;
        iy = iy0 + fy;
        ix = ix0 + fx;
        slot = ((fz * t.FY + fy) * t.FX + fx) * t.CiP + c8 * 8;
        return (unsigned)iz < (unsigned)c.D && (unsigned)iy < (unsigned)c.H &&
               (unsigned)ix < (unsigned)c.W;
    };
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * kStageBatch) {
        Raw raw[kStageBatch];
        bool inb[kStageBatch];
#pragma unroll
        for (int i = 0; i < kStageBatch; ++i) {
            const int e = e0 + 256 * i;
            int c8, iz, iy, ix, slot;
            inb[i] = e < total && voxel(e, c8, iz, iy, ix, slot);
            if constexpr (IN == kInPatch) {
                raw[i] = 0.f;
                if (inb[i]) {
                    const float* dn =
                        static_cast<const float*>(xin) + (size_t)n * c.D * c.H * c.W;
                    raw[i] = dn[((size_t)iz * c.H + iy) * c.W + ix];
                }
            } else if constexpr (IN == kInBf16) {
                raw[i] = make_uint4(0, 0, 0, 0);
                if (inb[i]) {
                    const u16* xn =
                        static_cast<const u16*>(xin) + (size_t)n * c.D * c.H * c.W * c.Ci;
                    raw[i] = *reinterpret_cast<const uint4*>(
                        xn + (((size_t)iz * c.H + iy) * c.W + ix) * c.Ci + c8 * 8);
                }
            } else {
                raw[i] = make_uint4(0, 0, 0, 0);
                if (inb[i]) {
                    const int h2 = c.H / 2, w2 = c.W / 2;
                    const u16* xn =
                        static_cast<const u16*>(xin) + (size_t)n * c.D * h2 * w2 * c.Ci;
                    raw[i] = *reinterpret_cast<const uint4*>(
                        xn + (((size_t)iz * h2 + iy / 2) * w2 + ix / 2) * c.Ci + c8 * 8);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kStageBatch; ++i) {
            const int e = e0 + 256 * i;
            if (e >= total) break;
            int c8, iz, iy, ix, slot;
            voxel(e, c8, iz, iy, ix, slot);
            uint4 v;
            if constexpr (IN == kInPatch)
                v = inb[i] ? input_channels(raw[i], depth[n], iz, iy, ix) : make_uint4(0, 0, 0, 0);
            else
                v = raw[i];
            *reinterpret_cast<uint4*>(xs + slot) = v;
        }
    }
    // after the tile: the LDS offset of every 8-channel chunk of the reduction
    // index relative to a position's tap (0, 0, 0) voxel (-1: zero padding of
    // K), then one chunk of zeros
    const int tile = c.kd * t.FY * t.FX * t.CiP;
    int* offs = reinterpret_cast<int*>(xs + tile);
    const int nchunk = c.Kp / 8;
    u16* zero = xs + tile + 2 * nchunk;
    for (int j = threadIdx.x; j < nchunk; j += 256) {
        int o = -1;
        if (8 * j < c.K) {
            const int4 tp = taps[j];  // (a, b, cc, ci) of this chunk
            o = ((tp.x * t.FY + tp.y) * t.FX + tp.z) * t.CiP + tp.w;
        }
        offs[j] = o;
    }
    if (threadIdx.x == 0) *reinterpret_cast<uint4*>(zero) = make_uint4(0, 0, 0, 0);
    __syncthreads();
    const int pl = wave * 32 + (lane & 31);
    const int oyl = pl / c.Wo, ox = pl % c.Wo;
    const int oy = oy0 + oyl;
    const bool pon = oyl < t.TY && oy < c.Ho;
    // positions past the tile read valid LDS; their outputs are not stored
    const u16* xb = xs + (pon ? (oyl * c.sh * t.FX + ox * c.sw) * t.CiP : 0);
    const int co0 = blockIdx.y * 32;
    const u16* wrow = w + (size_t)(co0 + (lane & 31)) * c.Kp + half * 8;
    f32x16 acc = {};
    // four reduction steps per trip, all loads issued before the first MFMA
    auto b_of = [&](int k0) {
        const int o = offs[k0 / 8 + half];
        return *reinterpret_cast<const uint4*>(o >= 0 ? xb + o : zero);
    };
    int k0 = 0;
    for (; k0 + 64 <= c.Kp; k0 += 64) {
        const uint4 a0 = *reinterpret_cast<const uint4*>(wrow + k0);
        const uint4 a1 = *reinterpret_cast<const uint4*>(wrow + k0 + 16);
        const uint4 a2 = *reinterpret_cast<const uint4*>(wrow + k0 + 32);
        const uint4 a3 = *reinterpret_cast<const uint4*>(wrow + k0 + 48);
        const uint4 b0 = b_of(k0), b1 = b_of(k0 + 16), b2 = b_of(k0 + 32), b3 = b_of(k0 + 48);
        acc = mfma(a0, b0, acc);
        acc = mfma(a1, b1, acc);
        acc = mfma(a2, b2, acc);
        acc = mfma(a3, b3, acc);
    }
    for (; k0 < c.Kp; k0 += 16)
        acc = mfma(*reinterpret_cast<const uint4*>(wrow + k0), b_of(k0), acc);
    if (!pon) return;
    const size_t p = (((size_t)n * c.Do + oz) * c.Ho + oy) * c.Wo + ox;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int cob = co0 + 8 * g + 4 * half;
        if constexpr (EPI == 0) {
            u16 o[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) o[i] = f2bf(fmaxf(acc[4 * g + i] + bias[cob + i], 0.f));
            *reinterpret_cast<uint2*>(ybf + p * c.Co + cob) =
                make_uint2(o[0] | ((unsigned)o[1] << 16), o[2] | ((unsigned)o[3] << 16));
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[4 * g + i] + bias[cob + i];
                const size_t idx = (((size_t)n * c.Co + cob + i) * c.Ho + oy) * c.Wo + ox;
                if (zkeep) zkeep[idx] = z;
                yf[idx] = softplus(z);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// convolution backward, data: dx = (conv^T dy) * [xact > 0]  (mask optional)
// wt: [Ci][taps * Co] bf16, the transposed weights; K ordered (tap, co).
// One wave computes 32 input channels x 32 input positions.

__global__ __launch_bounds__(256) void conv_bwd_data_kernel(const u16* __restrict__ dy,
                                                            const u16* __restrict__ wt,
                                                            const u16* __restrict__ xact,
                                                            ConvGeo c,
                                                            const int4* __restrict__ taps_t,
                                                            u16* __restrict__ dx) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
    const long P = (long)c.N * c.D * c.H * c.W;
    const long p = ((long)blockIdx.x * 4 + wave) * 32 + (lane & 31);
    const bool pon = p < P;
    long q = pon ? p : 0;
    const int ix = (int)(q % c.W);
    q /= c.W;
    const int iy = (int)(q % c.H);
    q /= c.H;
    const int iz = (int)(q % c.D);
    const int n = (int)(q / c.D);
    const u16* dyn = dy + (size_t)n * c.Do * c.Ho * c.Wo * c.Co;
    const int ci0 = blockIdx.y * 32;
    const int Kt = c.taps * c.Co;
    const u16* wrow = wt + (size_t)(ci0 + (lane & 31)) * Kt;
    f32x16 acc = {};
    for (int k0 = 0; k0 < Kt; k0 += 16) {
        const int kk = k0 + half * 8;
        const uint4 av = *reinterpret_cast<const uint4*>(wrow + kk);
        uint4 bv = make_uint4(0, 0, 0, 0);
        if (pon) {
            const int4 t = taps_t[kk / 8];  // (a, b, cc, co)
            const int zz = iz + c.pd - t.x, yy = iy + c.ph - t.y, xx = ix + c.pw - t.z;
            if (zz >= 0 && yy >= 0 && xx >= 0 && zz % c.sd == 0 && yy % c.sh == 0 &&
                xx % c.sw == 0) {
                const int oz = zz / c.sd, oy = yy / c.sh, ox = xx / c.sw;
                if (oz < c.Do && oy < c.Ho && ox < c.Wo)
                    bv = *reinterpret_cast<const uint4*>(
                        dyn + (((size_t)oz * c.Ho + oy) * c.Wo + ox) * c.Co + t.w);
            }
        }
        acc = mfma(av, bv, acc);
    }
    if (!pon) return;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int cib = ci0 + 8 * g + 4 * half;
        u16 o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = acc[4 * g + i];
            if (xact && !(bf2f(xact[(size_t)p * c.Ci + cib + i]) > 0.f)) v = 0.f;
            o[i] = f2bf(v);
        }
        *reinterpret_cast<uint2*>(dx + (size_t)p * c.Ci + cib) =
            make_uint2(o[0] | ((unsigned)o[1] << 16), o[2] | ((unsigned)o[3] << 16));
    }
}

// ---------------------------------------------------------------------------
// convolution backward, weights: dw[co][k] += sum over positions of dy[pos][co] x[pos, k]
// The reduction runs over output positions, which are the slow index of the
// channels-last tensors, so each wave stages 16 positions x 32 channels of dy
// and of the gathered input (16-byte loads, one per lane and operand) in LDS
// and reads them back transposed (8 positions of one channel per lane) for
// the MFMA.  Each wave reduces a contiguous chunk of positions for a 32 (co)
// x 32 (k) tile; the four waves of a block add their tiles in LDS, then one
// atomic add per element into the fp32 gradient.

__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const u16* __restrict__ x,
                                                              const u16* __restrict__ dy,
                                                              ConvGeo c,
                                                              const int4* __restrict__ taps,
                                                              int chunk, float* __restrict__ dw) {
    __shared__ float red[4][32][33];
    __shared__ u16 stage[4][2][16 * 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
    const long P = (long)c.N * c.Do * c.Ho * c.Wo;
    const int k0 = blockIdx.x * 32, co0 = blockIdx.y * 32;
    // this lane's loads: position pp of the 16, channel chunk c4 of the 4
    const int pp = lane >> 2, c4 = lane & 3;
    const int kc = k0 / 8 + c4;  // 8-wide chunk of the reduction index
    const bool kon = 8 * kc < c.K;
    const int4 t = taps[kon ? kc : 0];
    u16* sd = stage[wave][0];
    u16* sx = stage[wave][1];
    const long pbeg = ((long)blockIdx.z * 4 + wave) * chunk;
    const long pend = pbeg + chunk < P ? pbeg + chunk : P;
    f32x16 acc = {};
    for (long p0 = pbeg; p0 < pend; p0 += 16) {
        const long p = p0 + pp;
        uint4 dv = make_uint4(0, 0, 0, 0), xv = make_uint4(0, 0, 0, 0);
        if (p < pend) {
            dv = *reinterpret_cast<const uint4*>(dy + (size_t)p * c.Co + co0 + c4 * 8);
            if (kon) {
                long q = p;
                const int ox = (int)(q % c.Wo);
                q /= c.Wo;
                const int oy = (int)(q % c.Ho);
                q /= c.Ho;
                const int oz = (int)(q % c.Do);
                const int n = (int)(q / c.Do);
                const int iz = oz * c.sd - c.pd + t.x, iy = oy * c.sh - c.ph + t.y,
                          ix = ox * c.sw - c.pw + t.z;
                if ((unsigned)iz < (unsigned)c.D && (unsigned)iy < (unsigned)c.H &&
                    (unsigned)ix < (unsigned)c.W)
                    xv = *reinterpret_cast<const uint4*>(
                        x + ((((size_t)n * c.D + iz) * c.H + iy) * c.W + ix) * c.Ci + t.w);
            }
        }
        *reinterpret_cast<uint4*>(sd + pp * 32 + c4 * 8) = dv;
        *reinterpret_cast<uint4*>(sx + pp * 32 + c4 * 8) = xv;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // lane: channel (co or k) lane % 32, positions 8 half .. 8 half + 7
        unsigned short av[8], bv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            av[j] = sd[(8 * half + j) * 32 + (lane & 31)];
            bv[j] = sx[(8 * half + j) * 32 + (lane & 31)];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint4 av4, bv4;
        av4.x = av[0] | ((unsigned)av[1] << 16);
        av4.y = av[2] | ((unsigned)av[3] << 16);
        av4.z = av[4] | ((unsigned)av[5] << 16);
        av4.w = av[6] | ((unsigned)av[7] << 16);
        bv4.x = bv[0] | ((unsigned)bv[1] << 16);
        bv4.y = bv[2] | ((unsigned)bv[3] << 16);
        bv4.z = bv[4] | ((unsigned)bv[5] << 16);
        bv4.w = bv[6] | ((unsigned)bv[7] << 16);
        acc = mfma(av4, bv4, acc);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) red[wave][8 * (i / 4) + 4 * half + i % 4][lane & 31] = acc[i];
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
        const int r = e / 32, col = e % 32;
        const float v = red[0][r][col] + red[1][r][col] + red[2][r][col] + red[3][r][col];
        if (k0 + col < c.K && v != 0.f)
            atomicAdd(dw + (size_t)(co0 + r) * c.Kp + k0 + col, v);
    }
}

// bias gradient: db[co] += sum over positions of dy[pos][co].  blockDim.x = 256;
// a thread adds 8 channels (one 16-byte load) of every G-th position, G =
// 256 / (Co / 8); the block then adds its G partial sums per channel.
__global__ void bias_grad_kernel(const u16* __restrict__ dy, long P, int Co,
                                 float* __restrict__ db) {
    __shared__ float part[256 * 8];
    const int cch = Co / 8, c8 = threadIdx.x % cch, grp = threadIdx.x / cch;
    const int G = blockDim.x / cch;
    float s[8] = {};
    for (long p = (long)blockIdx.x * G + grp; p < P; p += (long)gridDim.x * G) {
        const uint4 v = *reinterpret_cast<const uint4*>(dy + (size_t)p * Co + c8 * 8);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            s[2 * i] += bf2f((u16)(w[i] & 0xffffu));
            s[2 * i + 1] += bf2f((u16)(w[i] >> 16));
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) part[threadIdx.x * 8 + i] = s[i];
    __syncthreads();
    if (threadIdx.x < Co) {
        const int ch = threadIdx.x, cc = ch / 8, i = ch % 8;
        float t = 0.f;
        for (int g = 0; g < G; ++g) t += part[(g * cch + cc) * 8 + i];
        atomicAdd(db + ch, t);
    }
}

// (a, b, c, base) of every 8-wide chunk of the reduction index: forward
// K = (tap, ci), transposed K = (tap, co); tap = (a kh + b) kw + c
__global__ void tap_table_kernel(ConvGeo g, int4* __restrict__ taps, int4* __restrict__ taps_t) {
    const int nf = g.K / 8, nt = taps_t ? g.taps * g.Co / 8 : 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nf + nt; j += gridDim.x * blockDim.x) {
        const bool fw = j < nf;
        const int k = 8 * (fw ? j : j - nf), C = fw ? g.Ci : g.Co;
        const int tap = k / C, ch = k % C;
        const int4 v = make_int4(tap / (g.kh * g.kw), tap / g.kw % g.kh, tap % g.kw, ch);
        if (fw)
            taps[j] = v;
        else
            taps_t[j - nf] = v;
    }
}

// ---------------------------------------------------------------------------
// element-wise and small kernels

// x0[n][z][y][x][8]: channel 0 = dn / 0.05, channel 1 = [z >= depth], channels
// 2, 3 = (y - 15.5) / 16, (x - 15.5) / 16 and channel 4 = their squared norm
// (where the source sits in the patch: a convolution cannot see it otherwise),
// channels 5..7 = 0
__global__ void prep_input_kernel(const float* __restrict__ dn, const float* __restrict__ depth,
                                  long n_vox, u16* __restrict__ x0) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n_vox;
         e += (long)gridDim.x * blockDim.x) {
        const long n = e / (64 * 32 * 32);
        const int z = (int)(e / (32 * 32) % 64), y = (int)(e / 32 % 32), x = (int)(e % 32);
        *reinterpret_cast<uint4*>(x0 + e * 8) = input_channels(dn[e], depth[n], z, y, x);
    }
}

// patches[s][z][y][x] = dn[z0 + z][(sy - 16 + y) mod ny][(sx - 16 + x) mod nx]
// grid (64, sources): 64 blocks of 256 threads per patch, four consecutive x
// per thread (one 16-byte store)
__global__ void extract_kernel(const float* __restrict__ dn, int ny, int nx, int z0,
                               const int* __restrict__ src, int s0, float* __restrict__ out) {
    const int s = s0 + blockIdx.y;
    const int sy = ((src[2 * s] % ny) + ny) % ny, sx = ((src[2 * s + 1] % nx) + nx) % nx;
    const int e = (blockIdx.x * blockDim.x + threadIdx.x) * 4;  // < 64 * 32 * 32
    const int z = e >> 10, y = (e >> 5) & 31, x = e & 31;
    int gy = sy - 16 + y;
    gy += gy < 0 ? ny : (gy >= ny ? -ny : 0);
    const float* row = dn + ((size_t)(z0 + z) * ny + gy) * nx;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int gx = sx - 16 + x + i;
        gx += gx < 0 ? nx : (gx >= nx ? -nx : 0);
        v[i] = row[gx];
    }
    *reinterpret_cast<float4*>(out + (size_t)s * (64 * 32 * 32) + e) =
        make_float4(v[0], v[1], v[2], v[3]);
}

// nearest-neighbour x2 upsampling of [N][h][w][C] (bf16)
__global__ void upsample_kernel(const u16* __restrict__ a, int N, int h, int w, int C,
                                u16* __restrict__ u) {
    const long total = (long)N * 2 * h * 2 * w * C;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(e % C);
        long q = e / C;
        const int x = (int)(q % (2 * w));
        q /= 2 * w;
        const int y = (int)(q % (2 * h));
        const long n = q / (2 * h);
        u[e] = a[(((size_t)n * h + y / 2) * w + x / 2) * C + ch];
    }
}

// da[n][y][x][c] = (sum of the 2x2 du block + dpool[n][c] / (h w)) * [a > 0]
__global__ void upsample_bwd_kernel(const u16* __restrict__ du, const u16* __restrict__ a,
                                    const float* __restrict__ dpool, int N, int h, int w, int C,
                                    u16* __restrict__ da) {
    const long total = (long)N * h * w * C;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(e % C);
        long q = e / C;
        const int x = (int)(q % w);
        q /= w;
        const int y = (int)(q % h);
        const long n = q / h;
        float s = dpool ? dpool[n * C + ch] / (float)(h * w) : 0.f;
#pragma unroll
        for (int dyy = 0; dyy < 2; ++dyy)
#pragma unroll
            for (int dxx = 0; dxx < 2; ++dxx)
                s += bf2f(du[(((size_t)n * 2 * h + 2 * y + dyy) * 2 * w + 2 * x + dxx) * C + ch]);
        da[e] = bf2f(a[e]) > 0.f ? f2bf(s) : (u16)0;
    }
}

// error head forward: pooled[n][c] = mean a[n][.][.][c]; e[n] = softplus(we . pooled + be)
__global__ void head_fwd_kernel(const u16* __restrict__ a, int hw, int C,
                                const float* __restrict__ we, const float* __restrict__ be,
                                float* __restrict__ pooled, float* __restrict__ epre,
                                float* __restrict__ err) {
    // blockDim.x = 256, C divides 256: 256 / C groups of C threads sum
    // interleaved positions (consecutive threads read consecutive channels)
    __shared__ float part[256];
    const int n = blockIdx.x, ch = threadIdx.x % C, grp = threadIdx.x / C;
    const int groups = blockDim.x / C;
    float s = 0.f;
    for (int i = grp; i < hw; i += groups) s += bf2f(a[((size_t)n * hw + i) * C + ch]);
    part[threadIdx.x] = s;
    __syncthreads();
    float dot = 0.f;
    if (threadIdx.x < C) {
        float t = 0.f;
        for (int g = 0; g < groups; ++g) t += part[g * C + ch];
        t /= (float)hw;
        pooled[(size_t)n * C + ch] = t;
        dot = we[ch] * t;
    }
    __syncthreads();
    part[threadIdx.x] = dot;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float z = part[0] + be[0];
        if (epre) epre[n] = z;
        err[n] = softplus(z);
    }
}

// loss of one batch.  Per sample: r2 = |psf - t|^2 / |t|^2, err_true = sqrt(r2).
// loss = mean(r2) + lambda mean((err_pred - err_true)^2)
// Writes dy of the last layer (d softplus, bf16 channels-last [n][y][x][plane]),
// derr_pre[n] and adds the sample's terms to loss[0], loss[1].
__global__ void loss_kernel(const float* __restrict__ psf, const float* __restrict__ z,
                            const float* __restrict__ target, const float* __restrict__ epre,
                            const float* __restrict__ err, int B, float lambda,
                            u16* __restrict__ dy, float* __restrict__ derr_pre,
                            float* __restrict__ loss, float* __restrict__ err_true) {
    constexpr int V = 32 * 32 * 32;
    __shared__ float sd[256], st[256];
    const int n = blockIdx.x;
    const float* p = psf + (size_t)n * V;
    const float* t = target + (size_t)n * V;
    float a = 0.f, b = 0.f;
    for (int i = threadIdx.x; i < V; i += blockDim.x) {
        const float d = p[i] - t[i];
        a += d * d;
        b += t[i] * t[i];
    }
    sd[threadIdx.x] = a;
    st[threadIdx.x] = b;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sd[threadIdx.x] += sd[threadIdx.x + s];
            st[threadIdx.x] += st[threadIdx.x + s];
        }
        __syncthreads();
    }
    const float tt = fmaxf(st[0], 1e-30f);
    const float r2 = sd[0] / tt, et = sqrtf(r2);
    const float g = 2.f / ((float)B * tt);
    for (int i = threadIdx.x; i < V; i += blockDim.x) {
        const int plane = i / 1024, yx = i % 1024;
        const float gz = g * (p[i] - t[i]) * sigmoid(z[(size_t)n * V + i]);
        dy[((size_t)n * 1024 + yx) * 32 + plane] = f2bf(gz);
    }
    if (threadIdx.x == 0) {
        const float de = err[n] - et;
        derr_pre[n] = 2.f * lambda * de / (float)B * sigmoid(epre[n]);
        atomicAdd(loss, r2 / (float)B);
        atomicAdd(loss + 1, lambda * de * de / (float)B);
        if (err_true) err_true[n] = et;
    }
}

// head backward: dwe[c] += sum_n dpre[n] pooled[n][c]; dbe += sum dpre; dpool = dpre we
__global__ void head_bwd_kernel(const float* __restrict__ pooled, const float* __restrict__ dpre,
                                const float* __restrict__ we, int B, int C,
                                float* __restrict__ dwe, float* __restrict__ dbe,
                                float* __restrict__ dpool) {
    const int ch = threadIdx.x;
    if (ch >= C) return;
    float s = 0.f;
    for (int n = 0; n < B; ++n) {
        s += dpre[n] * pooled[(size_t)n * C + ch];
        dpool[(size_t)n * C + ch] = dpre[n] * we[ch];
    }
    dwe[ch] += s;
    if (ch == 0) {
        float t = 0.f;
        for (int n = 0; n < B; ++n) t += dpre[n];
        dbe[0] += t;
    }
}

// Adam on the fp32 master parameters; bf16 copies of the conv weights
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, long n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x) {
        const float gi = g[e];
        const float mi = b1 * m[e] + (1.f - b1) * gi;
        const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
        m[e] = mi;
        v[e] = vi;
        w[e] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// bf16 weights [Co][Kp] and transposed weights [Ci][taps * Co] from fp32 [Co][Kp]
__global__ void pack_weights_kernel(const float* __restrict__ wf, int Co, int Ci, int taps, int Kp,
                                    u16* __restrict__ wb, u16* __restrict__ wt) {
    const long total = (long)Co * Kp;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int co = (int)(e / Kp), k = (int)(e % Kp);
        const u16 h = f2bf(wf[e]);
        wb[e] = h;
        if (wt && k < taps * Ci) {
            const int tap = k / Ci, ci = k % Ci;
            wt[((size_t)ci * taps + tap) * Co + co] = h;
        }
    }
}

__global__ void fill_zero_kernel(float* p, long n) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x)
        p[e] = 0.f;
}

// ---------------------------------------------------------------------------
// launchers

static unsigned grid_for(long n, int per = 256) {
    long b = (n + per - 1) / per;
    return (unsigned)(b < 65535 ? (b > 0 ? b : 1) : 65535);
}

FwdTile fwd_tile(const ConvGeo& c) {
    FwdTile t{};
    const int rows = 128 / c.Wo > 0 ? 128 / c.Wo : 1;
    t.TY = c.Ho < rows ? c.Ho : rows;
    t.FY = (t.TY - 1) * c.sh + c.kh;
    t.FX = (c.Wo - 1) * c.sw + c.kw;
    t.CiP = c.Ci + (c.Ci >= 32 ? 8 : 0);
    t.tiles_y = (c.Ho + t.TY - 1) / t.TY;
    return t;
}

size_t fwd_lds_bytes(const ConvGeo& c) {
    const FwdTile t = fwd_tile(c);
    // input tile, chunk offsets (Kp / 8 ints), one zero chunk (16 bytes)
    return sizeof(u16) * (size_t)c.kd * t.FY * t.FX * t.CiP + sizeof(int) * (size_t)(c.Kp / 8) +
           16;
}

hipError_t conv_forward(const ConvGeo& c, const void* x, const void* w, const float* bias,
                        const int4* taps, int epi, void* ybf, float* yf, float* zkeep,
                        hipStream_t s, int in_mode, const float* depth) {
    const FwdTile t = fwd_tile(c);
    const size_t lds = fwd_lds_bytes(c);
    dim3 grid((unsigned)((long)c.N * c.Do * t.tiles_y), c.Co / 32);
    const u16* wb = (const u16*)w;
    if (in_mode == kInPatch && epi == 0)
        conv_fwd_kernel<0, kInPatch><<<grid, 256, lds, s>>>(x, depth, wb, bias, c, t, taps,
                                                            (u16*)ybf, yf, zkeep);
    else if (in_mode == kInUp2 && epi == 1)
        conv_fwd_kernel<1, kInUp2><<<grid, 256, lds, s>>>(x, depth, wb, bias, c, t, taps,
                                                          (u16*)ybf, yf, zkeep);
    else if (in_mode != kInBf16)
        return hipErrorInvalidValue;
    else if (epi == 0)
        conv_fwd_kernel<0, kInBf16><<<grid, 256, lds, s>>>(x, depth, wb, bias, c, t, taps,
                                                           (u16*)ybf, yf, zkeep);
    else
        conv_fwd_kernel<1, kInBf16><<<grid, 256, lds, s>>>(x, depth, wb, bias, c, t, taps,
                                                           (u16*)ybf, yf, zkeep);
    return hipGetLastError();
}

hipError_t conv_backward_data(const ConvGeo& c, const void* dy, const void* wt,
                              const void* xact, const int4* taps_t, void* dx, hipStream_t s) {
    const long P = (long)c.N * c.D * c.H * c.W;
    dim3 grid((unsigned)((P + 127) / 128), c.Ci / 32);
    conv_bwd_data_kernel<<<grid, 256, 0, s>>>((const u16*)dy, (const u16*)wt, (const u16*)xact,
                                               c, taps_t, (u16*)dx);
    return hipGetLastError();
}

hipError_t conv_backward_weight(const ConvGeo& c, const void* x, const void* dy,
                                const int4* taps, float* dw, float* db, hipStream_t s) {
    const long P = (long)c.N * c.Do * c.Ho * c.Wo;
    if (dw) {
        const int chunk = 512;
        const long zs = (P + 4L * chunk - 1) / (4L * chunk);
        dim3 grid((unsigned)((c.K + 31) / 32), c.Co / 32, (unsigned)zs);
        conv_bwd_weight_kernel<<<grid, 256, 0, s>>>((const u16*)x, (const u16*)dy, c, taps,
                                                     chunk, dw);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !db) return e;
    const long per_block = 256L / (c.Co / 8) * 64;  // positions per block, 64 rounds
    const long blocks = (P + per_block - 1) / per_block;
    bias_grad_kernel<<<(unsigned)(blocks < 65535 ? blocks : 65535), 256, 0, s>>>(
        (const u16*)dy, P, c.Co, db);
    return hipGetLastError();
}

hipError_t prep_input(const float* dn, const float* depth, int B, void* x0, hipStream_t s) {
    const long n = (long)B * 64 * 32 * 32;
    prep_input_kernel<<<grid_for(n), 256, 0, s>>>(dn, depth, n, (u16*)x0);
    return hipGetLastError();
}

hipError_t extract_patches(const float* dn, int ny, int nx, int z0, const int* src, int n,
                           float* out, hipStream_t s) {
    for (int s0 = 0; s0 < n; s0 += 65535) {
        const int m = n - s0 < 65535 ? n - s0 : 65535;
        extract_kernel<<<dim3(64, m), 256, 0, s>>>(dn, ny, nx, z0, src, s0, out);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t upsample(const void* a, int N, int h, int w, int C, void* u, hipStream_t s) {
    upsample_kernel<<<grid_for((long)N * 4 * h * w * C), 256, 0, s>>>((const u16*)a, N, h, w, C,
                                                                      (u16*)u);
    return hipGetLastError();
}

hipError_t upsample_backward(const void* du, const void* a, const float* dpool, int N, int h,
                             int w, int C, void* da, hipStream_t s) {
    upsample_bwd_kernel<<<grid_for((long)N * h * w * C), 256, 0, s>>>(
        (const u16*)du, (const u16*)a, dpool, N, h, w, C, (u16*)da);
    return hipGetLastError();
}

hipError_t head_forward(const void* a, int N, int hw, int C, const float* we, const float* be,
                        float* pooled, float* epre, float* err, hipStream_t s) {
    head_fwd_kernel<<<N, 256, 0, s>>>((const u16*)a, hw, C, we, be, pooled, epre, err);
    return hipGetLastError();
}

hipError_t loss_and_grad(const float* psf, const float* z, const float* target,
                         const float* epre, const float* err, int B, float lambda, void* dy,
                         float* derr_pre, float* loss, float* err_true, hipStream_t s) {
    loss_kernel<<<B, 256, 0, s>>>(psf, z, target, epre, err, B, lambda, (u16*)dy, derr_pre, loss,
                                  err_true);
    return hipGetLastError();
}

hipError_t head_backward(const float* pooled, const float* dpre, const float* we, int B, int C,
                         float* dwe, float* dbe, float* dpool, hipStream_t s) {
    head_bwd_kernel<<<1, 256, 0, s>>>(pooled, dpre, we, B, C, dwe, dbe, dpool);
    return hipGetLastError();
}

hipError_t adam_update(float* w, const float* g, float* m, float* v, long n, float lr, int step,
                       hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    adam_kernel<<<grid_for(n), 256, 0, s>>>(w, g, m, v, n, lr, b1, b2, 1e-8f, bc1, bc2);
    return hipGetLastError();
}

hipError_t pack_weights(const float* wf, int Co, int Ci, int taps, int Kp, void* wb, void* wt,
                        hipStream_t s) {
    pack_weights_kernel<<<grid_for((long)Co * Kp), 256, 0, s>>>(wf, Co, Ci, taps, Kp, (u16*)wb,
                                                               (u16*)wt);
    return hipGetLastError();
}

hipError_t tap_tables(const ConvGeo& c, int4* taps, int4* taps_t, hipStream_t s) {
    tap_table_kernel<<<grid_for(c.K / 8 + c.taps * c.Co / 8), 256, 0, s>>>(c, taps, taps_t);
    return hipGetLastError();
}

hipError_t fill_zero(float* p, long n, hipStream_t s) {
    fill_zero_kernel<<<grid_for(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace sg
}  // namespace bpm
