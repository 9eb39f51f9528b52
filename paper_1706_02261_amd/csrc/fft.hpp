// Register/LDS FFT building blocks for gfx950 (wave64).
//
// A length-N transform is held by T = N / R threads, R complex values per
// thread.  Stage 0 is a radix-R DFT inside each thread's registers over the
// "strided" index (thread t holds x[i*T + t], i < R, so global loads and
// stores of rows are coalesced).  The remaining T-point DFTs are done in
// further stages of radix r_s = min(R, T_{s-1}); between stages the values are
// exchanged through LDS.  Each stage is a decimation-in-frequency split
//
//     X[k0 + r0 * k']  =  sum_t W_N^{t k0} (sum_i x[i T + t] W_r0^{i k0}) W_T^{t k'}
//
// applied recursively, and every stage writes its outputs to the LDS slots it
// read its inputs from (in-place Gentleman-Sande).  The spectrum therefore
// ends up digit-reversed in registers; the march never needs it in natural
// order, because the propagator table is stored in exactly that permuted order
// (see FftLayout::freq_of_store) and the inverse transform consumes the same
// layout and returns natural order.
//
// The index arithmetic is constexpr and host-callable so that the plan
// builder derives the permutation from the very same functions.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace bpm {

// ---------------------------------------------------------------------------
// complex helpers (float2 = interleaved re, im; bit-identical to complex64)

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float c_abs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// ---------------------------------------------------------------------------
// compile-time roots of unity of order 16: cos(2 pi p / 16), p = 0..3 quarter

__host__ __device__ constexpr double cos16(int p) {
    // cos(2 pi p / 16) for p in [0, 16)
    constexpr double c[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                             0.38268343236508977173, 0.0};
    p &= 15;
    return p <= 4 ? c[p] : p <= 8 ? -c[8 - p] : p <= 12 ? -c[p - 8] : c[16 - p];
}
__host__ __device__ constexpr double sin16(int p) { return cos16(p - 4); }

// a * exp(DIR * 2 pi i P / 16), with the cheap forms for multiples of pi/4
template <int P, int DIR>
__device__ __forceinline__ float2 mul_w16(float2 a) {
    constexpr int p = ((P * DIR) % 16 + 16) % 16;
    if constexpr (p == 0) {
        return a;
    } else if constexpr (p == 4) {   // * i
        return make_float2(-a.y, a.x);
    } else if constexpr (p == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (p == 12) {  // * -i
        return make_float2(a.y, -a.x);
    } else if constexpr (p % 2 == 0) {  // (+-1 +-i) / sqrt 2
        constexpr float c = (float)cos16(p), s = (float)sin16(p);
        constexpr float h = 0.70710678118654752440f;
        if constexpr (c > 0 && s > 0) return make_float2((a.x - a.y) * h, (a.x + a.y) * h);
        else if constexpr (c < 0 && s > 0) return make_float2(-(a.x + a.y) * h, (a.x - a.y) * h);
        else if constexpr (c < 0 && s < 0) return make_float2((a.y - a.x) * h, -(a.x + a.y) * h);
        else return make_float2((a.x + a.y) * h, (a.y - a.x) * h);
    } else {
        constexpr float c = (float)cos16(p), s = (float)sin16(p);
        return make_float2(fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c));
    }
}

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }
__host__ __device__ constexpr int bitrev(int v, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
    return r;
}

// In-register DFT of size RAD (power of two <= 16) over v[OFF + j*STR], natural
// order in and out: out[m] = sum_j in[j] exp(DIR 2 pi i j m / RAD).
// Radix-2 decimation in frequency, outputs renamed from bit-reversed order.
template <int RAD, int DIR, int N_REG, int OFF = 0, int STR = 1>
__device__ __forceinline__ void dft_reg(float2 (&v)[N_REG]) {
    static_assert(RAD >= 1 && RAD <= 16 && (RAD & (RAD - 1)) == 0, "radix");
    if constexpr (RAD == 1) {
        return;
    } else {
        float2 a[RAD];
#pragma unroll
        for (int j = 0; j < RAD; ++j) a[j] = v[OFF + j * STR];
#pragma unroll
        for (int h = RAD / 2; h >= 1; h >>= 1) {
#pragma unroll
            for (int s = 0; s < RAD; s += 2 * h) {
#pragma unroll
                for (int k = 0; k < h; ++k) {
                    float2 x = a[s + k], y = a[s + k + h];
                    a[s + k] = c_add(x, y);
                    float2 d = c_sub(x, y);
                    // twiddle W_{2h}^k = W_16^{k * 16 / (2h)}
                    switch (k * (16 / (2 * h))) {
                        case 0: a[s + k + h] = d; break;
                        case 1: a[s + k + h] = mul_w16<1, DIR>(d); break;
                        case 2: a[s + k + h] = mul_w16<2, DIR>(d); break;
                        case 3: a[s + k + h] = mul_w16<3, DIR>(d); break;
                        case 4: a[s + k + h] = mul_w16<4, DIR>(d); break;
                        case 5: a[s + k + h] = mul_w16<5, DIR>(d); break;
                        case 6: a[s + k + h] = mul_w16<6, DIR>(d); break;
                        case 7: a[s + k + h] = mul_w16<7, DIR>(d); break;
                        default: break;
                    }
                }
            }
        }
        constexpr int bits = ilog2(RAD);
#pragma unroll
        for (int m = 0; m < RAD; ++m) v[OFF + m * STR] = a[bitrev(m, bits)];
    }
}

// ---------------------------------------------------------------------------
// stage structure of a length-n transform with r values per thread
//
// Free constexpr functions of (n, r) so that kernels use them with template
// arguments and the plan builder with runtime sizes: one implementation.

__host__ __device__ constexpr int fft_radix(int n, int r, int s) {
    int t = n;
    for (int i = 0; i < s; ++i) t /= (i == 0 ? r : (t < r ? t : r));
    return s == 0 ? r : (t < r ? t : r);
}
// size still to be transformed after stage s
__host__ __device__ constexpr int fft_t_after(int n, int r, int s) {
    int t = n;
    for (int i = 0; i <= s; ++i) t /= fft_radix(n, r, i);
    return t;
}
__host__ __device__ constexpr int fft_num_stages(int n, int r) {
    int s = 1;
    while (fft_t_after(n, r, s - 1) > 1) ++s;
    return s;
}
// digit-reversed slot -> frequency index
__host__ __device__ constexpr int fft_freq_of_pos(int n, int r, int pos) {
    const int S = fft_num_stages(n, r);
    int digits[16] = {};
    for (int s = S - 1; s >= 0; --s) {
        digits[s] = pos % fft_radix(n, r, s);
        pos /= fft_radix(n, r, s);
    }
    int k = 0, w = 1;
    for (int s = 0; s < S; ++s) {
        k += digits[s] * w;
        w *= fft_radix(n, r, s);
    }
    return k;
}
// after the forward transform, register reg of thread tau holds this slot
__host__ __device__ constexpr int fft_pos_of_reg(int n, int r, int tau, int reg) {
    const int rl = fft_radix(n, r, fft_num_stages(n, r) - 1);
    return (tau + (n / r) * (reg / rl)) * rl + reg % rl;
}
// the march stores register reg of thread tau at memory slot reg * (n / r) + tau;
// this is the frequency index found at memory slot `slot`
__host__ __device__ constexpr int fft_freq_of_store(int n, int r, int slot) {
    return fft_freq_of_pos(n, r, fft_pos_of_reg(n, r, slot % (n / r), slot / (n / r)));
}

template <int N, int R>
struct FftLayout {
    static_assert((N & (N - 1)) == 0 && (R & (R - 1)) == 0 && R <= N, "sizes");
    static constexpr int T = N / R;  // threads per transform
    __host__ __device__ static constexpr int radix(int s) { return fft_radix(N, R, s); }
    __host__ __device__ static constexpr int t_after(int s) { return fft_t_after(N, R, s); }
    static constexpr int S = fft_num_stages(N, R);
    __host__ __device__ static constexpr int freq_of_store(int slot) { return fft_freq_of_store(N, R, slot); }
};

// LDS slot of position p (one pad slot every 16 against bank conflicts)
__host__ __device__ constexpr int lds_pad(int p) { return p + (p >> 4); }
template <int N>
__host__ __device__ constexpr int lds_size() { return N + N / 16; }

// ---------------------------------------------------------------------------
// compile-time loop

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(f);
    }
}

// radix-RAD DFTs over the R / RAD consecutive groups of v
template <int RAD, int DIR, int R>
__device__ __forceinline__ void dft_groups(float2 (&v)[R]) {
    static_for<0, R / RAD>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        dft_reg<RAD, DIR, R, q * RAD, 1>(v);
    });
}

// ---------------------------------------------------------------------------
// per-thread twiddles
//
// Stage s < S-1 multiplies output m of its group by W^(tp m) with tp fixed per
// thread (tp = tau for stage 0; every intermediate stage has one group per
// thread).  A thread's twiddles therefore never change: they are fetched once
// from the fp32 table tw[e] = exp(-2 pi i e / N) (rounded from fp64) and kept
// in registers.

template <int N, int R>
struct Twiddles {
    static constexpr int S = fft_num_stages(N, R);
    static constexpr int NS = S > 1 ? S - 1 : 1;  // stages that apply twiddles
    float2 w[NS][R];                              // w[s][m]; m = 0 is 1 and unused

    __device__ __forceinline__ void load(const float2* __restrict__ tw, int tau) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int ta = fft_t_after(N, R, s);
            const int tp = s == 0 ? tau : tau % ta;
            const int step = N / (fft_radix(N, R, s) * ta);
#pragma unroll
            for (int m = 0; m < R; ++m) w[s][m] = m ? tw[(tp * m * step) & (N - 1)] : make_float2(1.f, 0.f);
        }
    }
    __device__ __forceinline__ float2 get(int s, int m) const { return w[s][m]; }
    static constexpr bool kOpaqueIndex = false;
};

// The same twiddles read on use from a table in LDS (shared by the
// workgroup): no registers held across the passes, one LDS read per twiddle.
// The table holds, for every twiddled stage s and every value tp the thread
// parameter takes in that stage, the row W^(tp m step_s), m = 0 .. R-1, in
// rows of R + 1 entries (the pad puts the rows of consecutive tp in different
// banks), so a thread reads its twiddles at a per-stage base plus the
// compile-time offset m.
template <int N, int R>
struct LdsTwiddleTable {
    static constexpr int S = fft_num_stages(N, R);
    static constexpr int NS = S > 1 ? S - 1 : 0;  // stages that apply twiddles
    static constexpr int kRow = R + 1;
    __host__ __device__ static constexpr int rows(int s) {
        return s == 0 ? N / R : fft_t_after(N, R, s);
    }
    __host__ __device__ static constexpr int offset(int s) {
        int o = 0;
        for (int i = 0; i < s; ++i) o += rows(i) * kRow;
        return o;
    }
    __host__ __device__ static constexpr int size() { return offset(NS) > 0 ? offset(NS) : 1; }
    // fills the table from tw[e] = exp(-2 pi i e / N); threads tid of nthreads
    __device__ static void fill(float2* tab, const float2* __restrict__ tw, int tid,
                                int nthreads) {
        for (int e = tid; e < offset(NS); e += nthreads) {
            int st = 0;
            while (e >= offset(st + 1)) ++st;
            const int row = (e - offset(st)) / kRow, m = (e - offset(st)) % kRow;
            const int ta = fft_t_after(N, R, st);
            const int step = N / (fft_radix(N, R, st) * ta);
            tab[e] = m < R ? tw[(row * m * step) & (N - 1)] : make_float2(0.f, 0.f);
        }
    }
};

template <int N, int R>
struct LdsTwiddles {
    // used where registers are short: the transforms then hide the thread
    // index from the compiler, so that it recomputes their LDS addresses on
    // every call instead of keeping them all live across the caller's loop
    static constexpr bool kOpaqueIndex = true;
    using Table = LdsTwiddleTable<N, R>;
    const float2* tab;
    int tau;
    __device__ __forceinline__ float2 get(int s, int m) const {
        const int ta = fft_t_after(N, R, s);
        const int tp = s == 0 ? tau : tau % ta;
        return tab[Table::offset(s) + tp * Table::kRow + m];
    }
};

// ---------------------------------------------------------------------------
// block transforms
//
// lds: this transform's region; position p lives at lds[lds_pad(p) * LSTRIDE].
// sync(): ordering point over every thread that shares the LDS region.  Within
// one stage every slot is read and rewritten by the same thread, so a sync is
// only needed after each LDS write phase.
//
// Every LDS access of a stage is p = B + j ta for a per-thread base B and
// j < r, and B, ta and r are powers of two laid out so that the j ta never
// carry B's low four bits past a 16-slot boundary: lds_pad(B + j ta) =
// lds_pad(B) + j ta + (j ta) / 16 (pad_off below).  The transforms therefore
// compute one base address per stage and reach the slots at compile-time
// offsets (immediate fields of the LDS instructions), with no per-access
// index arithmetic.  (The same holds for the stage-0 positions k T + tau.)

__host__ __device__ constexpr int pad_off(int d) { return d + d / 16; }

// Forward transform (exp(-...)).  In: v[i] = x[i*T + tau], natural order.
// Out: v[reg] = X[fft_freq_of_pos(pos_of_reg(tau, reg))].
template <int N, int R, int LSTRIDE, typename Tw, typename Sync>
__device__ __forceinline__ void fft_forward(float2 (&v)[R], float2* lds, int tau, const Tw& tw,
                                            Sync sync) {
    using L = FftLayout<N, R>;
    constexpr int T = L::T;
    if constexpr (Tw::kOpaqueIndex) asm volatile("" : "+v"(tau));
    dft_reg<R, -1>(v);
    if constexpr (L::S > 1) {
#pragma unroll
        for (int k = 1; k < R; ++k) v[k] = c_mul(v[k], tw.get(0, k));
        float2* const w0 = lds + lds_pad(tau) * LSTRIDE;
#pragma unroll
        for (int k = 0; k < R; ++k) w0[pad_off(k * T) * LSTRIDE] = v[k];
        sync();
        static_for<1, L::S>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            constexpr int r = L::radix(s), ta = L::t_after(s), groups = R / r;
#pragma unroll
            for (int q = 0; q < groups; ++q) {
                const int g = tau + T * q;
                const float2* b = lds + lds_pad((g / ta) * r * ta + g % ta) * LSTRIDE;
#pragma unroll
                for (int j = 0; j < r; ++j) v[q * r + j] = b[pad_off(j * ta) * LSTRIDE];
            }
            dft_groups<r, -1>(v);
            if constexpr (s < L::S - 1) {
                // one group per thread
                float2* b = lds + lds_pad((tau / ta) * r * ta + tau % ta) * LSTRIDE;
#pragma unroll
                for (int m = 0; m < r; ++m) {
                    const float2 z = m ? c_mul(v[m], tw.get(s, m)) : v[m];
                    b[pad_off(m * ta) * LSTRIDE] = z;
                }
                sync();
            }
        });
    }
}

// Inverse transform (exp(+...), unnormalised): exact mirror of fft_forward.
// In: the forward's output layout.  Out: v[i] = N * x[i*T + tau].
template <int N, int R, int LSTRIDE, typename Tw, typename Sync>
__device__ __forceinline__ void fft_inverse(float2 (&v)[R], float2* lds, int tau, const Tw& tw,
                                            Sync sync) {
    using L = FftLayout<N, R>;
    constexpr int T = L::T;
    if constexpr (Tw::kOpaqueIndex) asm volatile("" : "+v"(tau));
    if constexpr (L::S > 1) {
        static_for<1, L::S>([&](auto ic) {
            constexpr int s = L::S - decltype(ic)::value;  // S-1 down to 1
            constexpr int r = L::radix(s), ta = L::t_after(s), groups = R / r;
            if constexpr (s < L::S - 1) {
                // one group per thread
                const float2* b = lds + lds_pad((tau / ta) * r * ta + tau % ta) * LSTRIDE;
#pragma unroll
                for (int m = 0; m < r; ++m) {
                    const float2 z = b[pad_off(m * ta) * LSTRIDE];
                    v[m] = m ? c_mulc(z, tw.get(s, m)) : z;
                }
            }
            dft_groups<r, +1>(v);
#pragma unroll
            for (int q = 0; q < groups; ++q) {
                const int g = tau + T * q;
                float2* b = lds + lds_pad((g / ta) * r * ta + g % ta) * LSTRIDE;
#pragma unroll
                for (int j = 0; j < r; ++j) b[pad_off(j * ta) * LSTRIDE] = v[q * r + j];
            }
            sync();
        });
        const float2* const w0 = lds + lds_pad(tau) * LSTRIDE;
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = w0[pad_off(k * T) * LSTRIDE];
#pragma unroll
        for (int k = 1; k < R; ++k) v[k] = c_mulc(v[k], tw.get(0, k));
    }
    dft_reg<R, +1>(v);
}

}  // namespace bpm
