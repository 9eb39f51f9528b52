// CPU emulation of the GPU block FFT (paper_1706_02261_amd/csrc/fft.hpp).
//
// One std::thread stands for each GPU thread of a transform and a
// std::barrier for the LDS ordering point, so the very same device functions
// (fft_forward / fft_inverse, register radix DFTs, LDS slot arithmetic and the
// storage-slot -> frequency permutation) run on the host.  Each forward
// transform is compared with the O(N^2) definition at the frequency that
// fft_freq_of_store assigns to its storage slot; the inverse must return N x.
// Test infrastructure only.
#include <hip/hip_runtime.h>
#include <barrier>
#include <thread>
#include <vector>
#include <complex>
#include <cstdio>
#include <cmath>
#include <random>
#include "fft.hpp"
using namespace bpm;

// LS: LDS stride (1: rows; 4: four interleaved columns, this one at slot 0);
// LDSTW: twiddles read from the per-thread LDS table instead of registers
template <int N, int R, int LS = 1, bool LDSTW = false>
int run() {
  using L = FftLayout<N, R>;
  constexpr int T = L::T;
  std::vector<float2> tw(N);
  for (int e = 0; e < N; ++e) { double a = -2 * M_PI * e / N; tw[e] = make_float2((float)cos(a), (float)sin(a)); }
  std::vector<float2> tab(LdsTwiddleTable<N, R>::size());
  LdsTwiddleTable<N, R>::fill(tab.data(), tw.data(), 0, 1);
  std::vector<std::complex<double>> x(N);
  std::mt19937 g(N * 31 + R);
  std::normal_distribution<double> nd;
  for (auto& v : x) v = {nd(g), nd(g)};
  std::vector<float2> lds((lds_size<N>() + 16) * LS);
  std::vector<float2> spec(N), back(N);
  std::barrier bar(T);
  std::vector<std::thread> th;
  for (int tau = 0; tau < T; ++tau) th.emplace_back([&, tau] {
    float2 v[R];
    for (int i = 0; i < R; ++i) v[i] = make_float2((float)x[i * T + tau].real(), (float)x[i * T + tau].imag());
    auto sync = [&] { bar.arrive_and_wait(); };
    auto body = [&](const auto& twr) {
      fft_forward<N, R, LS>(v, lds.data(), tau, twr, sync);
      for (int reg = 0; reg < R; ++reg) spec[reg * T + tau] = v[reg];
      bar.arrive_and_wait();
      fft_inverse<N, R, LS>(v, lds.data(), tau, twr, sync);
    };
    if constexpr (LDSTW) {
      LdsTwiddles<N, R> twl{tab.data(), tau};
      body(twl);
    } else {
      Twiddles<N, R> twr; twr.load(tw.data(), tau);
      body(twr);
    }
    for (int i = 0; i < R; ++i) back[i * T + tau] = v[i];
  });
  for (auto& t : th) t.join();
  double err = 0, nrm = 0, err2 = 0;
  for (int slot = 0; slot < N; ++slot) {
    int k = L::freq_of_store(slot);
    std::complex<double> ref = 0;
    for (int n = 0; n < N; ++n) ref += x[n] * std::polar(1.0, -2 * M_PI * (double)n * k / N);
    err = std::max(err, std::abs(std::complex<double>(spec[slot].x, spec[slot].y) - ref));
    nrm = std::max(nrm, std::abs(ref));
  }
  for (int n = 0; n < N; ++n) err2 = std::max(err2, std::abs(std::complex<double>(back[n].x, back[n].y) / (double)N - x[n]));
  // permutation check
  std::vector<int> seen(N, 0);
  for (int s = 0; s < N; ++s) seen[L::freq_of_store(s)]++;
  int bad = 0; for (int k = 0; k < N; ++k) bad += seen[k] != 1;
  // every LDS access of a stage at base + compile-time offset: the padded
  // slot of B + j ta equals lds_pad(B) + pad_off(j ta) (and so for k T + tau)
  int split_bad = 0;
  for (int tau = 0; tau < T; ++tau) {
    for (int k = 0; k < R; ++k) split_bad += lds_pad(k * T + tau) != lds_pad(tau) + pad_off(k * T);
    for (int s = 1; s < L::S; ++s) {
      const int r = L::radix(s), ta = L::t_after(s);
      for (int q = 0; q < R / r; ++q) {
        const int gq = tau + T * q, B = (gq / ta) * r * ta + gq % ta;
        for (int j = 0; j < r; ++j) split_bad += lds_pad(B + j * ta) != lds_pad(B) + pad_off(j * ta);
      }
    }
  }
  printf("N=%5d R=%2d T=%4d S=%d LS=%d lds-tw=%d: fwd rel err %.2e  inv err %.2e  perm bad %d  split bad %d\n",
         N, R, T, L::S, LS, (int)LDSTW, err / nrm, err2, bad, split_bad);
  return (err / nrm < 1e-5 && err2 < 1e-5 && !bad && !split_bad) ? 0 : 1;
}
int main() {
  int f = 0;
  f |= run<16, 16>(); f |= run<32, 16>(); f |= run<64, 16>(); f |= run<128, 16>(); f |= run<256, 16>();
  f |= run<512, 16>(); f |= run<1024, 16>(); f |= run<2048, 16>(); f |= run<1024, 8>(); f |= run<64, 4>();
  f |= run<1024, 16, 4>(); f |= run<256, 16, 4>(); f |= run<2048, 16, 2>();
  f |= run<32, 16, 1, true>(); f |= run<128, 16, 1, true>(); f |= run<512, 16, 1, true>();
  f |= run<1024, 16, 1, true>(); f |= run<1024, 16, 4, true>(); f |= run<2048, 16, 1, true>();
  printf(f ? "FAIL\n" : "ALL OK\n");
  return f;
}
