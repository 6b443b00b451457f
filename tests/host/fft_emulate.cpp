// CPU check of the in-LDS FFT stages of csrc/fft_core.h (lds_fft, lds_fft_rows,
// lds_fft_pair): NT std::threads play the threads of one block and a
// std::barrier their __syncthreads(), so the stage code runs unchanged on
// the host.  One case per stdin line; the buffer after the transform is
// printed (%.17g, re im pairs) for test_fft_emulation.py to compare with
// numpy.  Built with the address sanitizer, which also checks that no stage
// touches memory outside the buffer it is given.
//
//   fft  prec N inv nlines lstride estride buflen buf[2*buflen]
//   rows prec N inv nlines lstride estride lmap[nlines] buflen buf[2*buflen]
//   pair prec N lstride estride scale[MAXL*N] buflen buf[2*buflen]
//
// prec 0: double, 1: float (lengths 48, 60, 108).  Lines are MAXL = 12 (fft, rows) or MAXL = 10
// (pair) lines of N elements at buf[l * lstride + e * estride].
#include <barrier>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "fft_core.h"

thread_local EmuDim3 threadIdx;
static std::barrier<>* g_bar = nullptr;
void __syncthreads() { g_bar->arrive_and_wait(); }

namespace {

constexpr int NT = 128;
constexpr int MAXL_FFT = 12;
constexpr int MAXL_PAIR = 10;

template <typename F> void run_block(F&& body) {
  std::barrier<> bar(NT);
  g_bar = &bar;
  std::vector<std::thread> th;
  th.reserve(NT);
  for (int t = 0; t < NT; ++t)
    th.emplace_back([&body, t] {
      threadIdx.x = (unsigned)t;
      body();
    });
  for (auto& x : th) x.join();
  g_bar = nullptr;
}

double num(std::istream& in) {
  std::string t;
  in >> t;
  return std::strtod(t.c_str(), nullptr);
}

struct Case {
  std::string kind;
  int prec = 0, N = 0, inv = 0, nlines = 0, lstride = 0, estride = 0;
  std::vector<int> lmap;
  std::vector<double> scale;
  std::vector<double> buf;   // re, im interleaved
};

template <typename R> std::vector<ikr::cplx<R>> twiddles(int N) {
  std::vector<ikr::cplx<R>> tw(N);
  const double PI = 3.14159265358979323846;
  for (int m = 0; m < N; ++m)
    tw[m] = ikr::mk<R>((R)std::cos(2 * PI * m / N), (R)-std::sin(2 * PI * m / N));
  return tw;
}

template <typename R, int N> void run_typed(const Case& c) {
  std::vector<ikr::cplx<R>> b(c.buf.size() / 2);
  for (size_t i = 0; i < b.size(); ++i) b[i] = ikr::mk<R>((R)c.buf[2 * i], (R)c.buf[2 * i + 1]);
  const std::vector<ikr::cplx<R>> tw = twiddles<R>(N);
  ikr::cplx<R>* p = b.data();
  const ikr::cplx<R>* t = tw.data();
  if (c.kind == "fft") {
    if (c.inv)
      run_block([&] { ikr::lds_fft<R, N, NT, MAXL_FFT, true>(p, c.nlines, c.lstride, c.estride, t); });
    else
      run_block([&] { ikr::lds_fft<R, N, NT, MAXL_FFT, false>(p, c.nlines, c.lstride, c.estride, t); });
  } else if (c.kind == "rows") {
    const int* lm = c.lmap.data();
    if (c.inv)
      run_block([&] {
        ikr::lds_fft_rows<R, N, NT, MAXL_FFT, true>(p, c.nlines, c.lstride, c.estride, t, lm);
      });
    else
      run_block([&] {
        ikr::lds_fft_rows<R, N, NT, MAXL_FFT, false>(p, c.nlines, c.lstride, c.estride, t, lm);
      });
  } else {
    if constexpr (ikr::PairOrd<N>::S <= 2) {
      std::vector<R> s(c.scale.begin(), c.scale.end());
      const R* sp = s.data();
      run_block([&] {
        ikr::lds_fft_pair<R, N, NT, MAXL_PAIR>(p, c.lstride, c.estride, t,
                                               [&](int l, int e) { return sp[l * N + e]; });
      });
    } else {
      std::fprintf(stderr, "pair: length %d has three stages\n", N);
      std::exit(2);
    }
  }
  for (size_t i = 0; i < b.size(); ++i)
    std::printf(i ? " %.17g %.17g" : "%.17g %.17g", (double)b[i].x, (double)b[i].y);
  std::printf("\n");
}

// FP32 for the lengths of the FP32 planes of the test cells only (compile time)
template <int N> void run_n(const Case& c) {
  if (c.prec == 0) {
    run_typed<double, N>(c);
  } else {
    if constexpr (N == 48 || N == 60 || N == 108) {
      run_typed<float, N>(c);
    } else {
      std::fprintf(stderr, "no FP32 build for length %d\n", N);
      std::exit(2);
    }
  }
}

void dispatch(const Case& c) {
  switch (c.N) {
#define IKR_LEN(n) \
  case n: run_n<n>(c); return;
    IKR_LEN(8) IKR_LEN(12) IKR_LEN(16) IKR_LEN(18) IKR_LEN(20) IKR_LEN(24) IKR_LEN(30)
    IKR_LEN(32) IKR_LEN(36) IKR_LEN(40) IKR_LEN(48) IKR_LEN(60) IKR_LEN(64) IKR_LEN(72)
    IKR_LEN(80) IKR_LEN(90) IKR_LEN(96) IKR_LEN(100) IKR_LEN(108) IKR_LEN(120) IKR_LEN(128)
#undef IKR_LEN
    default:
      std::fprintf(stderr, "unsupported length %d\n", c.N);
      std::exit(2);
  }
}

}  // namespace

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    Case c;
    if (!(in >> c.kind)) continue;
    in >> c.prec >> c.N;
    if (c.kind == "pair") {
      in >> c.lstride >> c.estride;
      c.scale.resize((size_t)MAXL_PAIR * c.N);
      for (double& v : c.scale) v = num(in);
    } else if (c.kind == "fft" || c.kind == "rows") {
      in >> c.inv >> c.nlines >> c.lstride >> c.estride;
      if (c.kind == "rows") {
        c.lmap.resize(c.nlines);
        for (int& v : c.lmap) in >> v;
      }
    } else {
      std::fprintf(stderr, "unknown case %s\n", c.kind.c_str());
      return 2;
    }
    size_t n = 0;
    in >> n;
    c.buf.resize(2 * n);
    for (double& v : c.buf) v = num(in);
    if (in.fail()) {
      std::fprintf(stderr, "short input for %s\n", c.kind.c_str());
      return 2;
    }
    dispatch(c);
  }
  return 0;
}
