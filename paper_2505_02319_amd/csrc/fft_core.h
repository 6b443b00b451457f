// In-LDS batched 1D FFTs for gfx950: mixed-radix Stockham autosort stages
// (butterflies of 2, 3, 4, 5 points and their composites 6, 8, 9, 12, 16,
// so that the common lengths take two stages), each thread holding its butterflies in registers for the
// duration of a stage, so that a stage reads every element of the line,
// synchronises, then writes every element back in place (no ping-pong
// buffer: a 60 x 108 FP64 plane already takes 101 KiB of the 160 KiB LDS).
//
// Transforms are unnormalised.  FWD: X_k = sum_j x_j e^{-2 pi i jk/N};
// INV uses e^{+...}.  Twiddle table tw[m] = e^{-2 pi i m/N}, m < N.
#pragma once

#include "common.h"

namespace ikr {

// ------------------------------------------------------------ factorisation
// Radix order per supported length (first stage has no twiddles).
template <int N> struct Rad;
#define IKR_RAD(N, ...)                                                        \
  template <> struct Rad<N> {                                                  \
    static constexpr int r[] = {__VA_ARGS__};                                  \
    static constexpr int S = sizeof(r) / sizeof(int);                          \
  };
IKR_RAD(8, 8)
IKR_RAD(12, 12)
IKR_RAD(16, 16)
IKR_RAD(18, 6, 3)
IKR_RAD(20, 4, 5)
IKR_RAD(24, 8, 3)
IKR_RAD(30, 6, 5)
IKR_RAD(32, 16, 2)
IKR_RAD(36, 6, 6)
IKR_RAD(40, 8, 5)
IKR_RAD(48, 16, 3)
IKR_RAD(60, 12, 5)
IKR_RAD(64, 16, 4)
IKR_RAD(72, 8, 9)
IKR_RAD(80, 16, 5)
IKR_RAD(90, 6, 5, 3)
IKR_RAD(96, 16, 6)
IKR_RAD(100, 4, 5, 5)
IKR_RAD(108, 12, 9)
IKR_RAD(120, 8, 5, 3)
IKR_RAD(128, 16, 8)
#undef IKR_RAD

// A radix order of one or two stages reversed: a transform in this order
// starts with the butterflies the original order ends with, on the same
// elements (lds_fft_pair).
template <typename ORD> struct RevOrd {
  static constexpr int S = ORD::S;
  static constexpr int r[2] = {ORD::r[S - 1], ORD::r[0]};
};

// The radix order of the inverse transform of lds_fft_pair (the forward one
// runs in reverse).  By default that of Rad<N>; 48 takes 12 * 4, whose stages
// deal 4 and 12 butterflies per line, whole wavefronts over 48 lines, where
// 16 * 3 deals 3 per line (144 per 48 lines: the third wavefront of 256
// threads a quarter full) for about the same arithmetic.
template <int N> struct PairOrd : Rad<N> {};
template <> struct PairOrd<48> {
  static constexpr int r[] = {12, 4};
  static constexpr int S = 2;
};

// ------------------------------------------------------------ small DFTs
template <typename R, bool INV>
__host__ __device__ __forceinline__ cplx<R> mul_mi(cplx<R> a) {  // a * (-i) forward, a * (+i) inverse
  return INV ? mk<R>(-a.y, a.x) : mk<R>(a.y, -a.x);
}

template <typename R, int RAD, bool INV> struct Dft;

template <typename R, bool INV> struct Dft<R, 2, INV> {
  __host__ __device__ __forceinline__ static void run(cplx<R>* v) {
    cplx<R> a = v[0], b = v[1];
    v[0] = cadd<R>(a, b);
    v[1] = csub<R>(a, b);
  }
};

template <typename R, bool INV> struct Dft<R, 3, INV> {
  __host__ __device__ __forceinline__ static void run(cplx<R>* v) {
    const R s = R(0.86602540378443864676372317075294);   // sqrt(3)/2
    cplx<R> a = v[0], b = v[1], c = v[2];
    cplx<R> t1 = cadd<R>(b, c);
    cplx<R> t2 = mk<R>(a.x - R(0.5) * t1.x, a.y - R(0.5) * t1.y);
    cplx<R> t3 = mul_mi<R, INV>(cscale<R>(csub<R>(b, c), s));
    v[0] = cadd<R>(a, t1);
    v[1] = cadd<R>(t2, t3);
    v[2] = csub<R>(t2, t3);
  }
};

template <typename R, bool INV> struct Dft<R, 4, INV> {
  __host__ __device__ __forceinline__ static void run(cplx<R>* v) {
    cplx<R> a = v[0], b = v[1], c = v[2], d = v[3];
    cplx<R> t0 = cadd<R>(a, c), t1 = csub<R>(a, c);
    cplx<R> t2 = cadd<R>(b, d), t3 = mul_mi<R, INV>(csub<R>(b, d));
    v[0] = cadd<R>(t0, t2);
    v[2] = csub<R>(t0, t2);
    v[1] = cadd<R>(t1, t3);
    v[3] = csub<R>(t1, t3);
  }
};

template <typename R, bool INV> struct Dft<R, 5, INV> {
  __host__ __device__ __forceinline__ static void run(cplx<R>* v) {
    // c1 = cos(2pi/5), c2 = cos(4pi/5), s1 = sin(2pi/5), s2 = sin(4pi/5)
    const R c1 = R(0.30901699437494742410229341718282);
    const R c2 = R(-0.80901699437494742410229341718282);
    const R s1 = R(0.95105651629515357211643933337938);
    const R s2 = R(0.58778525229247312916870595463907);
    cplx<R> a = v[0];
    cplx<R> t1 = cadd<R>(v[1], v[4]), t2 = cadd<R>(v[2], v[3]);
    cplx<R> t3 = csub<R>(v[1], v[4]), t4 = csub<R>(v[2], v[3]);
    cplx<R> u1 = mk<R>(a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y);
    cplx<R> u2 = mk<R>(a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y);
    cplx<R> w1 = mul_mi<R, INV>(mk<R>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
    cplx<R> w2 = mul_mi<R, INV>(mk<R>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
    v[0] = mk<R>(a.x + t1.x + t2.x, a.y + t1.y + t2.y);
    v[1] = cadd<R>(u1, w1);
    v[4] = csub<R>(u1, w1);
    v[2] = cadd<R>(u2, w2);
    v[3] = csub<R>(u2, w2);
  }
};

// ------------------------------------------------------------ composite DFTs
// e^{-2 pi i m / N} = c[m] - i s[m] for the composite radices (correctly
// rounded values of the cosines and sines of 2 pi m / N).
template <int N> struct TwConst;
template <> struct TwConst<6> {
  static constexpr double c[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
  static constexpr double s[6] = {0.0, 0.8660254037844386, 0.8660254037844386, 0.0, -0.8660254037844386, -0.8660254037844386};
};
template <> struct TwConst<8> {
  static constexpr double c[8] = {1.0, 0.7071067811865476, 0.0, -0.7071067811865476, -1.0, -0.7071067811865476, 0.0, 0.7071067811865476};
  static constexpr double s[8] = {0.0, 0.7071067811865476, 1.0, 0.7071067811865476, 0.0, -0.7071067811865476, -1.0, -0.7071067811865476};
};
template <> struct TwConst<9> {
  static constexpr double c[9] = {1.0, 0.766044443118978, 0.17364817766693036, -0.5, -0.9396926207859084, -0.9396926207859084, -0.5, 0.17364817766693036, 0.766044443118978};
  static constexpr double s[9] = {0.0, 0.6427876096865394, 0.984807753012208, 0.8660254037844386, 0.3420201433256687, -0.3420201433256687, -0.8660254037844386, -0.984807753012208, -0.6427876096865394};
};
template <> struct TwConst<12> {
  static constexpr double c[12] = {1.0, 0.8660254037844386, 0.5, 0.0, -0.5, -0.8660254037844386, -1.0, -0.8660254037844386, -0.5, 0.0, 0.5, 0.8660254037844386};
  static constexpr double s[12] = {0.0, 0.5, 0.8660254037844386, 1.0, 0.8660254037844386, 0.5, 0.0, -0.5, -0.8660254037844386, -1.0, -0.8660254037844386, -0.5};
};
template <> struct TwConst<16> {
  static constexpr double c[16] = {1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898, 0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867};
  static constexpr double s[16] = {0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867, 1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898};
};

// N = A * B point DFT: A-point DFTs over the B interleaved subsequences,
// twiddles W_N^{j2 k1}, then B-point DFTs (output index k1 + A k2).
template <typename R, int A, int B, bool INV> struct DftComp {
  __host__ __host__ __device__ __forceinline__ static void run(cplx<R>* v) {
    constexpr int N = A * B;
    cplx<R> y[B][A];
#pragma unroll
    for (int j2 = 0; j2 < B; ++j2) {
      cplx<R> t[A];
#pragma unroll
      for (int j1 = 0; j1 < A; ++j1) t[j1] = v[B * j1 + j2];
      Dft<R, A, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        const int m = (j2 * k1) % N;
        if (m == 0) {
          y[j2][k1] = t[k1];
        } else if (4 * m == N) {         // -i forward, +i inverse
          y[j2][k1] = mul_mi<R, INV>(t[k1]);
        } else if (2 * m == N) {         // -1
          y[j2][k1] = mk<R>(-t[k1].x, -t[k1].y);
        } else if (4 * m == 3 * N) {     // +i forward, -i inverse
          y[j2][k1] = mul_mi<R, !INV>(t[k1]);
        } else {
          const R c = R(TwConst<N>::c[m]);
          const R sn = INV ? R(TwConst<N>::s[m]) : R(-TwConst<N>::s[m]);
          y[j2][k1] = mk<R>(t[k1].x * c - t[k1].y * sn, t[k1].x * sn + t[k1].y * c);
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cplx<R> t[B];
#pragma unroll
      for (int j2 = 0; j2 < B; ++j2) t[j2] = y[j2][k1];
      Dft<R, B, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = t[k2];
    }
  }
};

template <typename R, bool INV> struct Dft<R, 6, INV> : DftComp<R, 3, 2, INV> {};
template <typename R, bool INV> struct Dft<R, 8, INV> : DftComp<R, 4, 2, INV> {};
template <typename R, bool INV> struct Dft<R, 9, INV> : DftComp<R, 3, 3, INV> {};
template <typename R, bool INV> struct Dft<R, 12, INV> : DftComp<R, 4, 3, INV> {};
template <typename R, bool INV> struct Dft<R, 16, INV> : DftComp<R, 4, 4, INV> {};

// ------------------------------------------------------------ stage driver
// Lines live in LDS at buf[l * lstride + e * estride], l < nlines <= MAXL.
// The (line, butterfly) pairs of a stage are dealt out flat over the NT
// threads with the line fastest (pair i -> line i % MAXL, butterfly
// i / MAXL; lines past nlines idle), so every thread has at most
// ceil(MAXL * NB / NT) butterflies, neighbouring lanes take the same
// butterfly of neighbouring lines (an LDS stride of lstride, which is 1 or
// an odd pitch: no bank conflicts) and read the same twiddle (a broadcast).
// With lmap, line l is the buffer line lmap[l] (a subset of the lines); PK
// deals the pairs over the nlines listed lines instead of MAXL.
template <typename R, int N, int NT, int MAXL, bool INV, int STAGE, int NS,
          typename ORD = Rad<N>, bool PK = false>
struct Stages {
  // this stage alone
  __device__ __forceinline__ static void one(cplx<R>* buf, int nlines,
                                             int lstride, int estride,
                                             const cplx<R>* __restrict__ tw,
                                             const int* lmap = nullptr) {
    constexpr int RAD = ORD::r[STAGE];
    constexpr int NB = N / RAD;                   // butterflies per line
    constexpr int NV = (MAXL * NB + NT - 1) / NT; // butterflies per thread
    const int tid = threadIdx.x;
    // PK (packed; lmap required): the pairs are dealt over the nlines listed
    // lines only (pair i -> line i % nlines, butterfly i / nlines), so no
    // lane idles on an unlisted line and whole wavefronts drop out past
    // nlines * NB.  i / n is (i * M) >> 31 with M = floor(2^31 / n) + 1:
    // with e = M n - 2^31 in (0, n], i M / 2^31 = i / n + i e / (n 2^31), and
    // the added term stays below 1 / n (the least distance from i / n up to
    // the next integer) while i e < 2^31, true for i < MAXL * NB <= 128 * 64.
    // Otherwise: line i % MAXL, lines past nlines idle.
    const int tot = PK ? nlines * NB : MAXL * NB;
    unsigned magic = 0;
    if constexpr (PK) magic = 0x80000000u / (unsigned)(nlines > 0 ? nlines : 1) + 1u;
    auto pair = [&](int i, int& l, int& b) {
      if constexpr (PK) {
        b = (int)(((unsigned long long)(unsigned)i * magic) >> 31);
        l = i - b * nlines;
      } else {
        l = i % MAXL;
        b = i / MAXL;
      }
    };
    cplx<R> v[NV][RAD];
#pragma unroll
    for (int vi = 0; vi < NV; ++vi) {
      const int i = tid + NT * vi;
      int l, b;
      pair(i, l, b);
      if (i < tot && l < nlines) {
        cplx<R>* line = buf + (PK ? lmap[l] : (lmap ? lmap[l] : l)) * lstride;
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
          cplx<R> x = line[(b + r * NB) * estride];
          if (NS > 1 && r > 0) {
            cplx<R> w = tw[(r * (b % NS)) * (N / (NS * RAD))];
            if (INV) w.y = -w.y;
            x = cmul<R>(x, w);
          }
          v[vi][r] = x;
        }
        Dft<R, RAD, INV>::run(v[vi]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int vi = 0; vi < NV; ++vi) {
      const int i = tid + NT * vi;
      int l, b;
      pair(i, l, b);
      if (i < tot && l < nlines) {
        cplx<R>* line = buf + (PK ? lmap[l] : (lmap ? lmap[l] : l)) * lstride;
        const int d = (b / NS) * NS * RAD + (b % NS);
#pragma unroll
        for (int r = 0; r < RAD; ++r) line[(d + r * NS) * estride] = v[vi][r];
      }
    }
    __syncthreads();
  }
  // this stage and the ones after it
  __device__ __forceinline__ static void run(cplx<R>* buf, int nlines,
                                             int lstride, int estride,
                                             const cplx<R>* __restrict__ tw,
                                             const int* lmap = nullptr) {
    one(buf, nlines, lstride, estride, tw, lmap);
    if constexpr (STAGE + 1 < ORD::S)
      Stages<R, N, NT, MAXL, INV, STAGE + 1, NS * ORD::r[STAGE], ORD, PK>::run(
          buf, nlines, lstride, estride, tw, lmap);
  }
};

// Entry point: all lines transformed (or the nlines lines lmap lists);
// caller must __syncthreads() before (data written) -- the first stage's
// reads happen without a barrier.
template <typename R, int N, int NT, int MAXL, bool INV>
__device__ __forceinline__ void lds_fft(cplx<R>* buf, int nlines, int lstride,
                                        int estride, const cplx<R>* tw,
                                        const int* lmap = nullptr) {
  Stages<R, N, NT, MAXL, INV, 0, 1>::run(buf, nlines, lstride, estride, tw, lmap);
}

// The nlines lines that lmap lists (non-null), their (line, butterfly)
// pairs dealt over those lines only.
template <typename R, int N, int NT, int MAXL, bool INV>
__device__ __forceinline__ void lds_fft_rows(cplx<R>* buf, int nlines, int lstride,
                                             int estride, const cplx<R>* tw, const int* lmap) {
  Stages<R, N, NT, MAXL, INV, 0, 1, Rad<N>, true>::run(buf, nlines, lstride, estride, tw, lmap);
}

// An inverse transform of all MAXL lines, a pointwise multiply by
// scale(line, element), and the forward transform, for lengths of one or two
// stages.  The inverse runs in the order of PairOrd<N>, the forward one in the
// reverse order: the last inverse stage (radix A, stride NS = N / A) reads
// and writes elements b + r N/A of a line, and a forward transform that
// starts with radix A (stride 1) reads exactly those, so the two stages and
// the multiply between them run on the butterfly's registers, with one LDS
// read and one write where separate passes take three of each.
template <typename R, int N, int NT, int MAXL, typename F>
__device__ __forceinline__ void lds_fft_pair(cplx<R>* buf, int lstride, int estride,
                                             const cplx<R>* __restrict__ tw, F&& scale) {
  using ORD = PairOrd<N>;
  static_assert(ORD::S <= 2, "lds_fft_pair: one or two stages");
  constexpr int S = ORD::S;
  constexpr int RAD = ORD::r[S - 1];         // radix of the last inverse stage
  constexpr int NB = N / RAD;                // its butterflies per line = its stride
  constexpr int NV = (MAXL * NB + NT - 1) / NT;
  constexpr int tot = MAXL * NB;
  const int tid = threadIdx.x;
  // the multipliers of this thread's elements, requested before the first stage
  R sv[NV][RAD];
#pragma unroll
  for (int vi = 0; vi < NV; ++vi) {
    const int i = tid + NT * vi;
    const int l = i % MAXL, b = i / MAXL;
#pragma unroll
    for (int r = 0; r < RAD; ++r) sv[vi][r] = i < tot ? scale(l, b + r * NB) : R(0);
  }
  if constexpr (S == 2)
    Stages<R, N, NT, MAXL, true, 0, 1, ORD>::one(buf, MAXL, lstride, estride, tw);
  cplx<R> v[NV][RAD];
#pragma unroll
  for (int vi = 0; vi < NV; ++vi) {
    const int i = tid + NT * vi;
    const int l = i % MAXL, b = i / MAXL;
    if (i < tot) {
      cplx<R>* line = buf + l * lstride;
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        cplx<R> x = line[(b + r * NB) * estride];
        if (NB > 1 && r > 0) {   // inverse twiddles of the last stage
          cplx<R> w = tw[r * b];
          w.y = -w.y;
          x = cmul<R>(x, w);
        }
        v[vi][r] = x;
      }
      Dft<R, RAD, true>::run(v[vi]);
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[vi][r] = cscale<R>(v[vi][r], sv[vi][r]);
      Dft<R, RAD, false>::run(v[vi]);   // the first forward stage (stride 1: no twiddles)
    }
  }
  __syncthreads();
#pragma unroll
  for (int vi = 0; vi < NV; ++vi) {
    const int i = tid + NT * vi;
    const int l = i % MAXL, b = i / MAXL;
    if (i < tot) {
      cplx<R>* line = buf + l * lstride;
#pragma unroll
      for (int r = 0; r < RAD; ++r) line[(b * RAD + r) * estride] = v[vi][r];
    }
  }
  __syncthreads();
  if constexpr (S == 2)
    Stages<R, N, NT, MAXL, false, 1, RAD, RevOrd<ORD>>::run(buf, MAXL, lstride, estride, tw);
}

}  // namespace ikr
