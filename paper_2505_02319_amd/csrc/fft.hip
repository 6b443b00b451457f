// Pruned batched 3D FFT kernels for the plane-wave Hamiltonian on gfx950.
//
// F^-1 and F of paper eq. fft_ifft are applied as three sweeps over HBM:
//   column sweep  (sphere <-> column buffer, 1D FFT along the column axis C,
//                  only the footprint columns of the sphere on the (P,Q) plane)
//   plane sweep   (2D FFT of a whole (P,Q) plane in LDS; the local-potential
//                  multiply of H psi, or the density accumulation, is fused
//                  between the inverse and forward plane transforms)
// The footprint columns of each k-point are listed at setup; the basis is
// ordered column by column so that each column's coefficients are contiguous.
#include "fft_core.h"

namespace ikr {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ int fold(int i, int n) { return i < 0 ? i + n : i; }

// Column of basis element e within the block's columns [0, ncb): binary
// search over the block-local prefix offsets held in LDS.
__device__ __forceinline__ int find_col(const int* s, int ncb, int e) {
  int lo = 0, hi = ncb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (s[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Twiddle table of length N copied into LDS (read by every butterfly stage).
template <typename R, int N, int BT_ = NT>
__device__ __forceinline__ void load_tw(cplx<R>* dst, const cplx<R>* __restrict__ src) {
  for (int i = threadIdx.x; i < N; i += BT_) dst[i] = src[i];
}

template <int C> constexpr int ncb_for() { return C <= 24 ? 32 : (C <= 64 ? 32 : 16); }

// ---------------------------------------------------------------- columns
// MODE 0: sphere -> T (inverse along C); optional fused p = z + beta * x.
// MODE 1: T -> sphere (forward along C) with epilogue
//         y = scale * fft + (kin - shift[slot]) * x   (x may be null).
// MODE 2: full grid columns, T -> T: forward, * khat, inverse.
template <typename R, int C, int MODE>
__global__ __launch_bounds__(NT) void col_kernel(
    Geom g, const cplx<R>* __restrict__ tw, Slots s,
    const cplx<R>* __restrict__ xin, int x_stride, cplx<R>* __restrict__ T,
    const cplx<R>* __restrict__ z, const R* __restrict__ beta,
    cplx<R>* __restrict__ pout, cplx<R>* __restrict__ yout, int y_stride,
    const R* __restrict__ shift, R scale, const R* __restrict__ khat) {
  constexpr int NCB = ncb_for<C>();
  constexpr int LS = C + 1;                      // padded line stride
  __shared__ cplx<R> buf[NCB * LS];
  __shared__ int sstart[NCB + 1];
  __shared__ int sclo[NCB];
  __shared__ cplx<R> stw[C];

  if (!row_live(s, blockIdx.y)) return;
  const int slot = slot_of(s, blockIdx.y);
  if (s.active && !s.active[slot]) return;
  const int k = (MODE == 2) ? 0 : s.k[slot];
  const int ncol = (MODE == 2) ? g.P * g.Q : g.ncol[k];
  const int col0 = blockIdx.x * NCB;
  if (col0 >= ncol) return;
  const int ncb = min(NCB, ncol - col0);
  const int tid = threadIdx.x;
  const size_t tbase = (size_t)slot * C * g.ncol_max;
  load_tw<R, C>(stw, tw);

  if (MODE == 0) {
    for (int i = tid; i < NCB * LS; i += NT) buf[i] = mk<R>(0, 0);
    const int* cs = g.col_start + (size_t)k * (g.ncol_max + 1) + col0;
    const int* cl = g.col_clo + (size_t)k * g.ncol_max + col0;
    for (int i = tid; i <= ncb; i += NT) sstart[i] = cs[i];
    for (int i = tid; i < ncb; i += NT) sclo[i] = cl[i];
    __syncthreads();
    const int e0 = sstart[0], e1 = sstart[ncb];
    const cplx<R>* xs = xin + (size_t)slot * x_stride;
    const R b = z ? beta[slot] : R(0);
    // U elements per thread and round: loads first, so their latencies overlap
    constexpr int U = 4;
    for (int e00 = e0 + tid; e00 < e1; e00 += U * NT) {
      cplx<R> v[U], zz[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e00 + u * NT;
        if (e < e1) {
          v[u] = xs[e];
          if (z) zz[u] = z[(size_t)slot * x_stride + e];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e00 + u * NT;
        if (e < e1) {
          const int l = find_col(sstart, ncb, e);
          const int c = fold(sclo[l] + (e - sstart[l]), C);
          cplx<R> w = v[u];
          if (z) {
            w = mk<R>(zz[u].x + b * w.x, zz[u].y + b * w.y);
            pout[(size_t)slot * x_stride + e] = w;
          }
          buf[l * LS + c] = w;
        }
      }
    }
    __syncthreads();
    lds_fft<R, C, NT, NCB, true>(buf, ncb, LS, 1, stw);
    for (int i = tid; i < C * NCB; i += NT) {
      const int c = i / NCB, l = i % NCB;
      if (l < ncb) T[tbase + (size_t)c * g.ncol_max + col0 + l] = buf[l * LS + c];
    }
  } else {
#pragma unroll
    for (int u = 0; u < (C * NCB + NT - 1) / NT; ++u) {
      const int i = tid + u * NT;
      const int c = i / NCB, l = i % NCB;
      if (i < C * NCB && l < ncb) buf[l * LS + c] = T[tbase + (size_t)c * g.ncol_max + col0 + l];
    }
    if (MODE == 1) {
      const int* cs = g.col_start + (size_t)k * (g.ncol_max + 1) + col0;
      const int* cl = g.col_clo + (size_t)k * g.ncol_max + col0;
      for (int i = tid; i <= ncb; i += NT) sstart[i] = cs[i];
      for (int i = tid; i < ncb; i += NT) sclo[i] = cl[i];
    }
    __syncthreads();
    lds_fft<R, C, NT, NCB, false>(buf, ncb, LS, 1, stw);
    if (MODE == 1) {
      const int e0 = sstart[0], e1 = sstart[ncb];
      const double* kin = g.kin + (size_t)k * g.nb_max;
      const R sh = shift ? shift[slot] : R(0);
      constexpr int U = 4;
      for (int e00 = e0 + tid; e00 < e1; e00 += U * NT) {
        cplx<R> xx[U];
        R kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e00 + u * NT;
          if (xin && e < e1) {
            xx[u] = xin[(size_t)slot * x_stride + e];
            kv[u] = R(kin[e]);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e00 + u * NT;
          if (e < e1) {
            const int l = find_col(sstart, ncb, e);
            const int c = fold(sclo[l] + (e - sstart[l]), C);
            cplx<R> v = cscale<R>(buf[l * LS + c], scale);
            if (xin) {
              const R d = kv[u] - sh;
              v = mk<R>(v.x + d * xx[u].x, v.y + d * xx[u].y);
            }
            yout[(size_t)slot * y_stride + e] = v;
          }
        }
      }
    } else {
      // MODE 2: multiply by khat (internal layout [c][pq]) and transform back
      for (int i = tid; i < C * NCB; i += NT) {
        const int c = i / NCB, l = i % NCB;
        if (l < ncb) {
          const R kh = khat[(size_t)c * g.P * g.Q + col0 + l];
          buf[l * LS + c] = cscale<R>(buf[l * LS + c], kh);
        }
      }
      __syncthreads();
      lds_fft<R, C, NT, NCB, true>(buf, ncb, LS, 1, stw);
      for (int i = tid; i < C * NCB; i += NT) {
        const int c = i / NCB, l = i % NCB;
        if (l < ncb) T[tbase + (size_t)c * g.ncol_max + col0 + l] = buf[l * LS + c];
      }
    }
  }
}

// ---------------------------------------------------------------- planes
// rows (nullable): the nrows rows p that hold sphere columns.  The inverse
// transform along q then skips the other rows (zero on input) and the
// forward one along q skips them too (not read afterwards).
template <typename R, int P, int Q, bool INV, int BT_ = NT>
__device__ __forceinline__ void fft2d(cplx<R>* pl, const cplx<R>* twP,
                                      const cplx<R>* twQ, const int* rows = nullptr,
                                      int nrows = P) {
  constexpr int LQ = Q + 1;
  if (INV) {
    if (rows)
      lds_fft_rows<R, Q, BT_, P, true>(pl, nrows, LQ, 1, twQ, rows);
    else
      lds_fft<R, Q, BT_, P, true>(pl, P, LQ, 1, twQ);
    lds_fft<R, P, BT_, Q, true>(pl, Q, 1, LQ, twP);
  } else {
    lds_fft<R, P, BT_, Q, false>(pl, Q, 1, LQ, twP);
    if (rows)
      lds_fft_rows<R, Q, BT_, P, false>(pl, nrows, LQ, 1, twQ, rows);
    else
      lds_fft<R, Q, BT_, P, false>(pl, P, LQ, 1, twQ);
  }
}

// The footprint rows of k-point k in LDS (rows[P]); returns their number.
// A geometry without row lists gives all P rows.
template <int P, int BT_ = NT>
__device__ __forceinline__ int load_rows(const Geom& g, int k, int* rows) {
  for (int i = threadIdx.x; i < P; i += BT_) rows[i] = g.prow ? g.prow[(size_t)k * P + i] : i;
  return g.prow ? g.nprow[k] : P;
}

// Threads per plane block: the 60 x 108 FP64 plane (105 KiB of LDS, one
// block per CU) takes 512 so that two wavefronts per SIMD share the barriers.
template <typename R, int P, int Q> constexpr int plane_threads() {
  return (sizeof(R) == 8 && P * Q > 4096) ? 512 : NT;
}

// The plane transform pair with the multiply by V as a pass of its own
// (lengths of three stages along p).
template <typename R, int P, int Q, int PT>
__device__ __forceinline__ void plane_hv_mul(cplx<R>* pl, const cplx<R>* sP, const cplx<R>* sQ,
                                             const int* rows, int nrows,
                                             const R* __restrict__ vp) {
  constexpr int LQ = Q + 1;
  const int tid = threadIdx.x;
  fft2d<R, P, Q, true, PT>(pl, sP, sQ, rows, nrows);
  constexpr int NV = (P * Q + PT - 1) / PT;
  R vv[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int i = tid + u * PT;
    if (i < P * Q) vv[u] = vp[i];
  }
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int i = tid + u * PT;
    if (i < P * Q) {
      const int p = i / Q, q = i % Q;
      pl[p * LQ + q] = cscale<R>(pl[p * LQ + q], vv[u]);
    }
  }
  __syncthreads();
  fft2d<R, P, Q, false, PT>(pl, sP, sQ, rows, nrows);
}

// H psi local part: T -> inverse 2D -> * V -> forward 2D -> T.
template <typename R, int P, int Q, int PT = plane_threads<R, P, Q>()>
__global__ __launch_bounds__(PT) void plane_hv_kernel(
    Geom g, const cplx<R>* __restrict__ twP, const cplx<R>* __restrict__ twQ,
    Slots s, const cplx<R>* __restrict__ Tin, cplx<R>* __restrict__ Tout,
    const R* __restrict__ V, int v_per_slot) {
  constexpr int LQ = Q + 1;
  __shared__ cplx<R> pl[P * LQ];
  __shared__ cplx<R> sP[P], sQ[Q];
  __shared__ int rows[P];
  load_tw<R, P, PT>(sP, twP);
  load_tw<R, Q, PT>(sQ, twQ);
  if (!row_live(s, blockIdx.y)) return;
  const int slot = slot_of(s, blockIdx.y);
  if (s.active && !s.active[slot]) return;
  const int c = blockIdx.x;
  const int k = s.k[slot];
  const int ncol = g.ncol[k];
  const int tid = threadIdx.x;
  const int nrows = load_rows<P, PT>(g, k, rows);
  for (int i = tid; i < P * LQ; i += PT) pl[i] = mk<R>(0, 0);
  __syncthreads();
  const int* pq = g.col_pq + (size_t)k * g.ncol_max;
  const size_t tb = ((size_t)slot * g.C + c) * g.ncol_max;
  constexpr int U = 4;   // columns per thread and round, loads first
  for (int c00 = tid; c00 < ncol; c00 += U * PT) {
    cplx<R> tv[U];
    int pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = c00 + u * PT;
      const bool in = col < ncol;
      pv[u] = in ? pq[col] : -1;
      tv[u] = in ? Tin[tb + col] : mk<R>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (pv[u] >= 0) pl[(pv[u] / Q) * LQ + (pv[u] % Q)] = tv[u];
  }
  __syncthreads();
  const R* vp = V + (v_per_slot ? (size_t)slot * g.C * P * Q : 0) + (size_t)c * P * Q;
  if constexpr (PairOrd<P>::S <= 2) {
    // inverse along q, then along p with the multiply by V and the forward
    // transform along p fused into the middle stage, then forward along q
    lds_fft_rows<R, Q, PT, P, true>(pl, nrows, LQ, 1, sQ, rows);
    lds_fft_pair<R, P, PT, Q>(pl, 1, LQ, sP, [&](int q, int p) { return vp[p * Q + q]; });
    lds_fft_rows<R, Q, PT, P, false>(pl, nrows, LQ, 1, sQ, rows);
  } else {
    plane_hv_mul<R, P, Q, PT>(pl, sP, sQ, rows, nrows, vp);
  }
  for (int col = tid; col < ncol; col += PT) {
    const int v = pq[col];
    Tout[tb + col] = pl[(v / Q) * LQ + (v % Q)];
  }
}



// Density terms: for the slots of a group, a = IFFT2(Ta), b = IFFT2(Tb),
// acc += wa Re(conj a b) + wb |a|^2, per plane element; written per group.
template <int P, int Q>
__global__ __launch_bounds__(NT) void plane_rho_kernel(
    Geom g, const double2* __restrict__ twP, const double2* __restrict__ twQ,
    int nslots, const int* __restrict__ slot_k, const double2* __restrict__ Ta,
    const double2* __restrict__ Tb, const double* __restrict__ wa,
    const double* __restrict__ wb, int gsize, double* __restrict__ part) {
  constexpr int LQ = Q + 1;
  constexpr int OWN = (P * Q + NT - 1) / NT;
  __shared__ double2 pl[P * LQ];
  __shared__ double2 sP[P], sQ[Q];
  load_tw<double, P>(sP, twP);
  load_tw<double, Q>(sQ, twQ);
  const int c = blockIdx.x;
  const int grp = blockIdx.y;
  const int tid = threadIdx.x;
  double acc[OWN];
  double2 av[OWN];
#pragma unroll
  for (int o = 0; o < OWN; ++o) acc[o] = 0.0;
  const int s0 = grp * gsize, s1 = min(nslots, s0 + gsize);
  for (int slot = s0; slot < s1; ++slot) {
    const int k = slot_k[slot];
    const int ncol = g.ncol[k];
    const int* pq = g.col_pq + (size_t)k * g.ncol_max;
    const size_t tb = ((size_t)slot * g.C + c) * g.ncol_max;
    for (int pass = 0; pass < 2; ++pass) {
      const double2* T = pass == 0 ? Ta : Tb;
      for (int i = tid; i < P * LQ; i += NT) pl[i] = mk<double>(0, 0);
      __syncthreads();
      constexpr int U = 4;   // columns per thread and round, loads first
      for (int c00 = tid; c00 < ncol; c00 += U * NT) {
        double2 tv[U];
        int pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int col = c00 + u * NT;
          const bool in = col < ncol;
          pv[u] = in ? pq[col] : -1;
          tv[u] = in ? T[tb + col] : mk<double>(0, 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (pv[u] >= 0) pl[(pv[u] / Q) * LQ + (pv[u] % Q)] = tv[u];
      }
      __syncthreads();
      fft2d<double, P, Q, true>(pl, sP, sQ);
      const double ka = wa[slot], kb = wb[slot];
#pragma unroll
      for (int o = 0; o < OWN; ++o) {
        const int i = tid + o * NT;
        if (i < P * Q) {
          const double2 v = pl[(i / Q) * LQ + (i % Q)];
          if (pass == 0) {
            av[o] = v;
          } else {
            acc[o] += ka * (av[o].x * v.x + av[o].y * v.y) +
                      kb * (av[o].x * av[o].x + av[o].y * av[o].y);
          }
        }
      }
      __syncthreads();
    }
  }
  double* out = part + ((size_t)grp * g.C + c) * P * Q;
#pragma unroll
  for (int o = 0; o < OWN; ++o) {
    const int i = tid + o * NT;
    if (i < P * Q) out[i] = acc[o];
  }
}

// Complex grid values (unnormalised inverse) of each slot.
template <int P, int Q>
__global__ __launch_bounds__(NT) void plane_grid_kernel(
    Geom g, const double2* __restrict__ twP, const double2* __restrict__ twQ,
    const int* __restrict__ slot_k, const double2* __restrict__ T,
    double2* __restrict__ grid) {
  constexpr int LQ = Q + 1;
  __shared__ double2 pl[P * LQ];
  __shared__ double2 sP[P], sQ[Q];
  load_tw<double, P>(sP, twP);
  load_tw<double, Q>(sQ, twQ);
  const int c = blockIdx.x, slot = blockIdx.y, tid = threadIdx.x;
  const int k = slot_k[slot];
  const int ncol = g.ncol[k];
  const int* pq = g.col_pq + (size_t)k * g.ncol_max;
  const size_t tb = ((size_t)slot * g.C + c) * g.ncol_max;
  for (int i = tid; i < P * LQ; i += NT) pl[i] = mk<double>(0, 0);
  __syncthreads();
  for (int col = tid; col < ncol; col += NT) {
    const int v = pq[col];
    pl[(v / Q) * LQ + (v % Q)] = T[tb + col];
  }
  __syncthreads();
  fft2d<double, P, Q, true>(pl, sP, sQ);
  double2* out = grid + ((size_t)slot * g.C + c) * P * Q;
  for (int i = tid; i < P * Q; i += NT) out[i] = pl[(i / Q) * LQ + (i % Q)];
}

// Full real grid -> forward 2D per plane -> T (layout [c][p*Q+q]).
template <int P, int Q>
__global__ __launch_bounds__(NT) void plane_fwd_kernel(
    Geom g, const double2* __restrict__ twP, const double2* __restrict__ twQ,
    const double* __restrict__ v, double2* __restrict__ T) {
  constexpr int LQ = Q + 1;
  __shared__ double2 pl[P * LQ];
  __shared__ double2 sP[P], sQ[Q];
  load_tw<double, P>(sP, twP);
  load_tw<double, Q>(sQ, twQ);
  const int c = blockIdx.x, tid = threadIdx.x;
  const double* vp = v + (size_t)c * P * Q;
  for (int i = tid; i < P * Q; i += NT) pl[(i / Q) * LQ + (i % Q)] = mk<double>(vp[i], 0.0);
  __syncthreads();
  fft2d<double, P, Q, false>(pl, sP, sQ);
  double2* out = T + (size_t)c * P * Q;
  for (int i = tid; i < P * Q; i += NT) out[i] = pl[(i / Q) * LQ + (i % Q)];
}

// T (full) -> inverse 2D -> out = Re/N_g + fx * v; partial[c] = sum out^2.
template <int P, int Q>
__global__ __launch_bounds__(NT) void plane_inv_kernel(
    Geom g, const double2* __restrict__ twP, const double2* __restrict__ twQ,
    const double2* __restrict__ T, const double* __restrict__ v,
    const double* __restrict__ fx, double* __restrict__ out,
    double* __restrict__ partial) {
  constexpr int LQ = Q + 1;
  __shared__ double2 pl[P * LQ];
  __shared__ double2 sP[P], sQ[Q];
  load_tw<double, P>(sP, twP);
  load_tw<double, Q>(sQ, twQ);
  __shared__ double red[NT];
  const int c = blockIdx.x, tid = threadIdx.x;
  const double2* tp = T + (size_t)c * P * Q;
  for (int i = tid; i < P * Q; i += NT) pl[(i / Q) * LQ + (i % Q)] = tp[i];
  __syncthreads();
  fft2d<double, P, Q, true>(pl, sP, sQ);
  const double inv_ng = 1.0 / ((double)g.C * P * Q);
  const size_t base = (size_t)c * P * Q;
  double ss = 0.0;
  for (int i = tid; i < P * Q; i += NT) {
    double o = pl[(i / Q) * LQ + (i % Q)].x * inv_ng;
    if (fx) o += fx[base + i] * v[base + i];
    out[base + i] = o;
    ss += o * o;
  }
  red[tid] = ss;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) partial[c] = red[0];
}

}  // namespace

// ---------------------------------------------------------------- dispatch
bool fft_length_supported(int n) {
  switch (n) {
    case 8: case 12: case 16: case 18: case 20: case 24: case 30: case 32:
    case 36: case 40: case 48: case 60: case 64: case 72: case 80: case 90:
    case 96: case 100: case 108: case 120: case 128:
      return true;
    default:
      return false;
  }
}

#define IKR_COL_LENGTHS(X) X(8) X(12) X(16) X(18) X(20) X(24) X(30) X(32) X(36) \
  X(40) X(48) X(60) X(64) X(72) X(80) X(90) X(96) X(100) X(108) X(120) X(128)
// Plane shapes (P, Q) compiled in; the column axis takes the remaining length.
#define IKR_PLANES(X) X(8, 8) X(12, 12) X(16, 16) X(20, 20) X(24, 24) X(32, 32) \
  X(36, 36) X(40, 40) X(48, 48) X(60, 108) X(64, 64)

bool plane_supported(int P, int Q) {
#define X(a, b) if (P == a && Q == b) return true;
  IKR_PLANES(X)
#undef X
  return false;
}

template <typename R>
static const cplx<R>* twp(const FftTables& t, int off);
template <> const double2* twp<double>(const FftTables& t, int off) { return t.tw64 + off; }
template <> const float2* twp<float>(const FftTables& t, int off) { return t.tw32 + off; }

template <typename R, int MODE>
static void col_dispatch(const Geom& g, const FftTables& t, const Slots& s,
                         const cplx<R>* xin, int x_stride, cplx<R>* T,
                         const cplx<R>* z, const R* beta, cplx<R>* pout,
                         cplx<R>* yout, int y_stride, const R* shift, R scale,
                         const R* khat, int ncols, hipStream_t st) {
  const cplx<R>* tw = twp<R>(t, t.offC);
#define X(LEN)                                                                 \
  if (g.C == LEN) {                                                            \
    constexpr int NCB = ncb_for<LEN>();                                        \
    dim3 grid((ncols + NCB - 1) / NCB, s.n);                                   \
    hipLaunchKernelGGL((col_kernel<R, LEN, MODE>), grid, dim3(NT), 0, st, g, tw, \
                       s, xin, x_stride, T, z, beta, pout, yout, y_stride,     \
                       shift, scale, khat);                                    \
    IKR_HIP(hipGetLastError());                                                \
    return;                                                                    \
  }
  IKR_COL_LENGTHS(X)
#undef X
  throw Error(1, "unsupported FFT column length " + std::to_string(g.C));
}

template <typename R>
void launch_col_inv(const Geom& g, const FftTables& t, const Slots& s,
                    const cplx<R>* x, int x_stride, cplx<R>* T,
                    const cplx<R>* z, const R* beta, cplx<R>* pout,
                    hipStream_t st) {
  col_dispatch<R, 0>(g, t, s, x, x_stride, T, z, beta, pout, nullptr, 0,
                     nullptr, R(1), nullptr, g.ncol_max, st);
}

template <typename R>
void launch_col_fwd(const Geom& g, const FftTables& t, const Slots& s,
                    const cplx<R>* T, cplx<R>* y, int y_stride,
                    const cplx<R>* x, const R* shift, R scale, hipStream_t st) {
  col_dispatch<R, 1>(g, t, s, x, y_stride, const_cast<cplx<R>*>(T), nullptr,
                     nullptr, nullptr, y, y_stride, shift, scale, nullptr,
                     g.ncol_max, st);
}

// Both 256 and 512 threads per block are built for planes of 48 x 48 points
// and more; smaller planes take 256.
template <int P, int Q> constexpr bool plane_pt_choice() { return P * Q >= 2304; }

template <typename R, int P, int Q>
static int plane_pt_pick(int pt) {
  if constexpr (plane_pt_choice<P, Q>())
    if (pt == NT || pt == 512) return pt;
  return plane_threads<R, P, Q>();
}

int plane_hv_threads(const Geom& g, int pt, bool fp64) {
#define X(a, b) \
  if (g.P == a && g.Q == b) return fp64 ? plane_pt_pick<double, a, b>(pt) : plane_pt_pick<float, a, b>(pt);
  IKR_PLANES(X)
#undef X
  return 0;
}

template <typename R, int P, int Q, int PT>
static void plane_hv_go(const Geom& g, const cplx<R>* tP, const cplx<R>* tQ, const Slots& s,
                        const cplx<R>* Tin, cplx<R>* Tout, const R* V, int v_per_slot,
                        hipStream_t st) {
  hipLaunchKernelGGL((plane_hv_kernel<R, P, Q, PT>), dim3(g.C, s.n), dim3(PT), 0, st, g, tP,
                     tQ, s, Tin, Tout, V, v_per_slot);
  IKR_HIP(hipGetLastError());
}

template <typename R>
void launch_plane_hv(const Geom& g, const FftTables& t, const Slots& s,
                     const cplx<R>* Tin, cplx<R>* Tout, const R* V,
                     int v_per_slot, hipStream_t st, int pt) {
  const cplx<R>* tP = twp<R>(t, t.offP);
  const cplx<R>* tQ = twp<R>(t, t.offQ);
#define X(a, b)                                                                      \
  if (g.P == a && g.Q == b) {                                                        \
    if constexpr (plane_pt_choice<a, b>()) {                                         \
      if (plane_pt_pick<R, a, b>(pt) == 512)                                         \
        return plane_hv_go<R, a, b, 512>(g, tP, tQ, s, Tin, Tout, V, v_per_slot, st); \
      return plane_hv_go<R, a, b, NT>(g, tP, tQ, s, Tin, Tout, V, v_per_slot, st);   \
    }                                                                                \
    return plane_hv_go<R, a, b, plane_threads<R, a, b>()>(g, tP, tQ, s, Tin, Tout, V, \
                                                          v_per_slot, st);           \
  }
  IKR_PLANES(X)
#undef X
  throw Error(1, "unsupported FFT plane shape");
}

void launch_plane_rho(const Geom& g, const FftTables& t, int nslots,
                      const int* slot_k, const double2* Ta, const double2* Tb,
                      const double* wa, const double* wb, int gsize,
                      double* part, hipStream_t st) {
  const double2* tP = t.tw64 + t.offP;
  const double2* tQ = t.tw64 + t.offQ;
  const int ng = (nslots + gsize - 1) / gsize;
#define X(a, b)                                                                \
  if (g.P == a && g.Q == b) {                                                  \
    hipLaunchKernelGGL((plane_rho_kernel<a, b>), dim3(g.C, ng), dim3(NT), 0,   \
                       st, g, tP, tQ, nslots, slot_k, Ta, Tb, wa, wb, gsize,   \
                       part);                                                  \
    IKR_HIP(hipGetLastError());                                                \
    return;                                                                    \
  }
  IKR_PLANES(X)
#undef X
  throw Error(1, "unsupported FFT plane shape");
}

void launch_plane_grid(const Geom& g, const FftTables& t, int nslots,
                       const int* slot_k, const double2* T, double2* grid,
                       hipStream_t st) {
  const double2* tP = t.tw64 + t.offP;
  const double2* tQ = t.tw64 + t.offQ;
#define X(a, b)                                                                \
  if (g.P == a && g.Q == b) {                                                  \
    hipLaunchKernelGGL((plane_grid_kernel<a, b>), dim3(g.C, nslots), dim3(NT), \
                       0, st, g, tP, tQ, slot_k, T, grid);                     \
    IKR_HIP(hipGetLastError());                                                \
    return;                                                                    \
  }
  IKR_PLANES(X)
#undef X
  throw Error(1, "unsupported FFT plane shape");
}

void launch_kernel_apply(const Geom& g, const FftTables& t, const double* v,
                         const double* khat, const double* fx, double* out,
                         double2* work1, double2* work2, double* partial,
                         hipStream_t st) {
  const double2* tP = t.tw64 + t.offP;
  const double2* tQ = t.tw64 + t.offQ;
  // Column pass treats the whole plane as footprint: T layout [c][P*Q].
  Geom gf = g;
  gf.ncol_max = g.P * g.Q;
  Slots one{1, nullptr, nullptr};
  bool done = false;
#define X(a, b)                                                                \
  if (!done && g.P == a && g.Q == b) {                                         \
    hipLaunchKernelGGL((plane_fwd_kernel<a, b>), dim3(g.C), dim3(NT), 0, st,   \
                       gf, tP, tQ, v, work1);                                  \
    IKR_HIP(hipGetLastError());                                                \
    col_dispatch<double, 2>(gf, t, one, nullptr, 0, work1, nullptr, nullptr,   \
                            nullptr, nullptr, 0, nullptr, 1.0, khat, a * b,    \
                            st);                                               \
    hipLaunchKernelGGL((plane_inv_kernel<a, b>), dim3(g.C), dim3(NT), 0, st,   \
                       gf, tP, tQ, work1, v, fx, out, partial);                \
    IKR_HIP(hipGetLastError());                                                \
    done = true;                                                               \
  }
  IKR_PLANES(X)
#undef X
  (void)work2;
  if (!done) throw Error(1, "unsupported FFT plane shape");
}

template void launch_col_inv<double>(const Geom&, const FftTables&, const Slots&,
                                     const double2*, int, double2*, const double2*,
                                     const double*, double2*, hipStream_t);
template void launch_col_inv<float>(const Geom&, const FftTables&, const Slots&,
                                    const float2*, int, float2*, const float2*,
                                    const float*, float2*, hipStream_t);
template void launch_col_fwd<double>(const Geom&, const FftTables&, const Slots&,
                                     const double2*, double2*, int, const double2*,
                                     const double*, double, hipStream_t);
template void launch_col_fwd<float>(const Geom&, const FftTables&, const Slots&,
                                    const float2*, float2*, int, const float2*,
                                    const float*, float, hipStream_t);
template void launch_plane_hv<double>(const Geom&, const FftTables&, const Slots&,
                                      const double2*, double2*, const double*, int,
                                      hipStream_t, int);
template void launch_plane_hv<float>(const Geom&, const FftTables&, const Slots&,
                                     const float2*, float2*, const float*, int,
                                     hipStream_t, int);

}  // namespace ikr
