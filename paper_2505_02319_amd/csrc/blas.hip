// Batched vector kernels for the Sternheimer CG and the response assembly.
//
// Bands are grouped in tiles of up to BT slots sharing one k-point, so that
// a projection against the occupied orbitals Phi_k (paper: P = Phi Phi^H,
// Q = I - P) or the nonlocal projectors reads each column of Phi_k / P_k
// once per tile rather than once per band: the projections are the tall
// skinny products W^H X (gram) and X + W C (update).  Every reduction is
// two-stage (per-block partials, then a fixed-order sum), so results are
// bitwise reproducible run to run.
#include "blas.h"
#include "mfma.h"

#include <algorithm>
#include <atomic>

namespace ikr {
namespace {

constexpr int NT = 256;
constexpr int CH = 64;        // elements per inner chunk of the gram kernel
// gram blocks aimed for over ntiles tiles: few, long blocks amortise the
// per-block reduction and partial writes (measured on 48^3 and 48^2 x 96
// cells with up to 16 tiles: FP64 fastest near 256, FP32 near 512); with
// many tiles every block is long anyway, and about 2048 blocks keep the
// last round of blocks from leaving most CUs idle (60 x 108^2 cell, 135
// tiles: 270 blocks were 10% slower than 2160).  The matrix-core kernel
// prefers twice the floor (48^3 cell: FP64 gram 33.5 against 36.4 ms per
// solve, FP32 11.7 against 12.2).
constexpr int GRAM_BLOCKS_MAX = 2048;
template <typename R> int gram_blocks(int ntiles, bool mfma) {
  const int floor = (sizeof(R) == 8 ? 256 : 512) * (mfma ? 2 : 1);
  return std::max(floor, std::min(GRAM_BLOCKS_MAX, 16 * ntiles));
}
constexpr int UPD_BLOCKS = 1024;    // update blocks below which tiles are split

// True when some slot of tile t takes part (active == null: all do).
__device__ __forceinline__ bool tile_live(const Tiles& tl, int t, const int* active) {
  if (tl.dn && t >= *tl.dn) return false;
  if (!active) return true;
  const int nbt = tl.nb[t];
  bool any = false;
  for (int b = 0; b < nbt; ++b) any |= active[tslot(tl, t, b)] != 0;
  return any;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// part[((t * nsc + sc) * Mmax + m) * BT + b] = sum_{g in super-chunk}
//                                 conj(W[k][m][g]) X[slot0 + b][g]
//
// Chunks of CH coefficients of the tile's BT bands and of MT = RB * SBM
// projector rows are staged in LDS.  Each thread owns an RB x 4 block of the
// MT x BT output (rows RB*mi.., bands 4bi..) over one of KS interleaved
// slices of the chunk, so every LDS value it reads feeds four (or RB)
// complex multiply-adds; the slices are summed by shuffles inside a
// wavefront, then across the wavefronts.
template <typename R, int RB, int SBM>
__global__ __launch_bounds__(NT) void gram_kernel(
    Tiles tl, const int* __restrict__ nb, const int* __restrict__ Mk, int Mmax,
    const cplx<R>* __restrict__ W, size_t wk_stride, int w_stride,
    const cplx<R>* __restrict__ X, int x_stride, int nsc, int sc_len,
    cplx<R>* __restrict__ part, const int* __restrict__ active) {
  constexpr int MT = RB * SBM;            // rows per pass
  constexpr int SB = SBM * (BT / 4);      // threads covering one slice
  constexpr int KS = NT / SB;             // slices per chunk
  static_assert(64 % SB == 0 && CH % KS == 0, "gram tiling");
  constexpr int LW = CH + 1;
  constexpr int NWAVE = NT / 64;
  constexpr int STAGE = (BT + MT) * LW, RED = NWAVE * MT * BT;
  __shared__ cplx<R> smem[STAGE > RED ? STAGE : RED];
  __shared__ int ss[BT];
  cplx<R>* Xs = smem;                     // [BT][LW]
  cplx<R>* Ws = smem + BT * LW;           // [MT][LW]
  cplx<R>* red = smem;                    // [NWAVE][MT * BT], after the chunks
  // items (super-chunk, tile) with the tile fastest: the tiles of one k-point
  // read the same W_k chunk back to back on one XCD
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nsc * tl.n) return;
  const int t = item % tl.n, sc = item / tl.n, tid = threadIdx.x;
  if (!tile_live(tl, t, active)) return;
  const int k = tl.k[t], nbt = tl.nb[t];
  const int M = Mk[k], n = nb[k];
  if (tid < BT) ss[tid] = tid < nbt ? tslot(tl, t, tid) : 0;
  __syncthreads();
  const int sb = tid % SB, mi = sb >> 2, bi = sb & 3, ks = tid / SB;
  const int wave = tid >> 6, lane = tid & 63;
  const cplx<R>* Wk = W + (size_t)k * wk_stride;
  const int gbeg = sc * sc_len, gend = min(n, gbeg + sc_len);
  // chunks are fetched into registers one chunk ahead of their use
  constexpr int XL = BT * CH / NT;
  constexpr int WL = (MT * CH + NT - 1) / NT;
  static_assert(BT * CH % NT == 0, "gram staging");
  cplx<R> xr[XL], wr[WL];
  auto fetch = [&](int g0, int m0) {
#pragma unroll
    for (int l = 0; l < XL; ++l) {
      const int i = tid + l * NT, b = i / CH, e = i % CH, gg = g0 + e;
      xr[l] = (b < nbt && gg < gend) ? X[(size_t)ss[b] * x_stride + gg] : mk<R>(0, 0);
    }
#pragma unroll
    for (int l = 0; l < WL; ++l) {
      const int i = tid + l * NT, m = i / CH, e = i % CH, gg = g0 + e;
      wr[l] = (i < MT * CH && m0 + m < M && gg < gend) ? Wk[(size_t)(m0 + m) * w_stride + gg]
                                                        : mk<R>(0, 0);
    }
  };
  for (int m0 = 0; m0 < M; m0 += MT) {
    R ar[RB][4], ai[RB][4];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) ar[i][j] = ai[i][j] = R(0);
    if (gbeg < gend) fetch(gbeg, m0);
    for (int g0 = gbeg; g0 < gend; g0 += CH) {
#pragma unroll
      for (int l = 0; l < XL; ++l) {
        const int i = tid + l * NT;
        Xs[(i / CH) * LW + i % CH] = xr[l];
      }
#pragma unroll
      for (int l = 0; l < WL; ++l) {
        const int i = tid + l * NT;
        if (i < MT * CH) Ws[(i / CH) * LW + i % CH] = wr[l];
      }
      __syncthreads();
      if (g0 + CH < gend) fetch(g0 + CH, m0);
#pragma unroll
      for (int u = 0; u < CH / KS; ++u) {
        const int e = ks + KS * u;
        cplx<R> w[RB], x[4];
#pragma unroll
        for (int i = 0; i < RB; ++i) w[i] = Ws[(RB * mi + i) * LW + e];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = Xs[(4 * bi + j) * LW + e];
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            ar[i][j] += w[i].x * x[j].x + w[i].y * x[j].y;
            ai[i][j] += w[i].x * x[j].y - w[i].y * x[j].x;
          }
      }
      __syncthreads();
    }
    // the slices held by one wavefront sit in lanes sb, sb + SB, ...
#pragma unroll
    for (int o = SB; o < 64; o <<= 1)
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ar[i][j] += __shfl_xor(ar[i][j], o, 64);
          ai[i][j] += __shfl_xor(ai[i][j], o, 64);
        }
    if (lane < SB)
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          red[wave * MT * BT + (RB * mi + i) * BT + 4 * bi + j] = mk<R>(ar[i][j], ai[i][j]);
    __syncthreads();
    for (int o = tid; o < MT * BT; o += NT) {
      const int m = o / BT, b = o % BT;
      cplx<R> v = red[o];
#pragma unroll
      for (int w = 1; w < NWAVE; ++w) v = cadd<R>(v, red[w * MT * BT + o]);
      if (m0 + m < M) part[(((size_t)t * nsc + sc) * Mmax + m0 + m) * BT + b] = v;
    }
    __syncthreads();
  }
}

// The same partials on the matrix cores: C = conj(W) X as four real 16x16x4
// MFMA products per 16-row tile (Re += Wr Xr + Wi Xi, Im += Wr Xi - Wi Xr).
// Wavefront w of the four takes the row tiles w, w + 4, ... over the whole
// super-chunk, so no reduction across wavefronts is needed (all four stage
// the chunks).  Chunks of MCH
// coefficients of W (rows up to 16 * RTMAX) and of the tile's BT bands are
// staged in LDS ([rows][MCH + 1]); RTM row tiles at most, CHM coefficients
// per chunk.


template <typename R, int RTM, int CHM>
__global__ __launch_bounds__(NT) void gram_mfma_kernel(
    Tiles tl, const int* __restrict__ nb, const int* __restrict__ Mk, int Mmax,
    const cplx<R>* __restrict__ W, size_t wk_stride, int w_stride,
    const cplx<R>* __restrict__ X, int x_stride, int nsc, int sc_len,
    cplx<R>* __restrict__ part, const int* __restrict__ active) {
  using M = Mfma<R>;
  constexpr int MCH = CHM, RTMAX = RTM;
  constexpr int LC = MCH + 1;
  extern __shared__ __align__(16) unsigned char gm_smem[];
  cplx<R>* Xs = reinterpret_cast<cplx<R>*>(gm_smem);   // [BT][LC]
  cplx<R>* Ws = Xs + BT * LC;                          // [16 RT][LC]
  __shared__ int ss[BT];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nsc * tl.n) return;
  const int t = item % tl.n, sc = item / tl.n, tid = threadIdx.x;
  if (!tile_live(tl, t, active)) return;
  const int k = tl.k[t], nbt = tl.nb[t];
  const int Mr = Mk[k], n = nb[k];
  const int RT = (Mr + 15) / 16, nw = blockDim.x >> 6;
  const int wave = tid >> 6, lane = tid & 63;
  if (tid < BT) ss[tid] = tid < nbt ? tslot(tl, t, tid) : 0;
  __syncthreads();
  const cplx<R>* Wk = W + (size_t)k * wk_stride;
  const int gbeg = sc * sc_len, gend = min(n, gbeg + sc_len);
  // row tiles per wavefront (NT / 64 = 4 wavefronts)
  constexpr int PW = (RTMAX + 3) / 4;
  typename M::acc cre[PW], cim[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) cre[q][v] = cim[q][v] = R(0);
  // the next chunk is fetched into registers while the current one is used
  constexpr int XL = BT * MCH / NT, WLM = 16 * RTMAX * MCH / NT;
  const int wl = 16 * RT * MCH / NT;
  cplx<R> xr[XL], wr[WLM];
  auto fetch = [&](int g0) {
#pragma unroll
    for (int u = 0; u < XL; ++u) {
      const int i = tid + u * NT, b = i / MCH, g = g0 + i % MCH;
      xr[u] = (b < nbt && g < gend) ? X[(size_t)ss[b] * x_stride + g] : mk<R>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < WLM; ++u) {
      const int i = tid + u * NT, m = i / MCH, g = g0 + i % MCH;
      if (u < wl) wr[u] = (m < Mr && g < gend) ? Wk[(size_t)m * w_stride + g] : mk<R>(0, 0);
    }
  };
  if (gbeg < gend) fetch(gbeg);
  for (int g0 = gbeg; g0 < gend; g0 += MCH) {
#pragma unroll
    for (int u = 0; u < XL; ++u) {
      const int i = tid + u * NT;
      Xs[(i / MCH) * LC + i % MCH] = xr[u];
    }
#pragma unroll
    for (int u = 0; u < WLM; ++u) {
      const int i = tid + u * NT;
      if (u < wl) Ws[(i / MCH) * LC + i % MCH] = wr[u];
    }
    __syncthreads();
    if (g0 + MCH < gend) fetch(g0 + MCH);
#pragma unroll 2
    for (int ks = 0; ks < MCH / 4; ++ks) {
      const int e = 4 * ks + (lane >> 4);
      const cplx<R> xb = Xs[(lane & 15) * LC + e];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int rt = wave + q * nw;
        if (rt < RT) {
          const cplx<R> wa = Ws[(16 * rt + (lane & 15)) * LC + e];
          cre[q] = M::mac(wa.x, xb.x, cre[q]);
          cre[q] = M::mac(wa.y, xb.y, cre[q]);
          cim[q] = M::mac(wa.x, xb.y, cim[q]);
          cim[q] = M::mac(-wa.y, xb.x, cim[q]);
        }
      }
    }
    __syncthreads();
  }
  const int j = lane & 15;
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    const int rt = wave + q * nw;
    if (rt >= RT) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = 16 * rt + M::row(lane, v);
      if (m < Mr) part[(((size_t)t * nsc + sc) * Mmax + m) * BT + j] = mk<R>(cre[q][v], cim[q][v]);
    }
  }
}

// The same partials for all bands of a k-point at once, on the matrix cores.
// A block takes one (k, super-chunk) item and the up to KT tiles of k
// (t0[k] .. t0[k+1]); it stages chunks of KCH coefficients of all Mr rows of
// W_k and of the k's bands in LDS, so W_k is read once per iteration
// whatever the number of bands, and its wavefronts deal the (row tile,
// band tile) pairs of the output round-robin (pair = wave + NWV q).  Each pair
// is four real 16x16x4 MFMA products per 4 coefficients (Re += Wr Xr + Wi Xi,
// Im += Wr Xi - Wi Xr).  The next chunk is fetched into registers while the
// current one is used.
constexpr int KW_NT = 512;

template <typename R, int KT, int RTM, int KCH, int NTH>
__global__ __launch_bounds__(NTH) void gram_kw_kernel(
    Tiles tl, KTileRange kr, const int* __restrict__ nb, const int* __restrict__ Mk, int Mmax,
    const cplx<R>* __restrict__ W, size_t wk_stride, int w_stride,
    const cplx<R>* __restrict__ X, int x_stride, int nsc, int sc_len,
    cplx<R>* __restrict__ part, const int* __restrict__ active) {
  using M = Mfma<R>;
  constexpr int LC = KCH + 1;
  constexpr int NBT = KT * 16;                       // band rows staged
  constexpr int NWV = NTH / 64;                      // wavefronts
  constexpr int PW = (KT * RTM + NWV - 1) / NWV;     // pairs per wavefront
  __shared__ cplx<R> Xs[NBT * LC];
  __shared__ cplx<R> Ws[RTM * 16 * LC];
  __shared__ int ss[NBT];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nsc * kr.nk) return;
  const int k = item / nsc, sc = item % nsc, tid = threadIdx.x;
  int t0 = kr.t0[k], nt = kr.t0[k + 1] - t0;
  if (tl.dn) nt = min(nt, *tl.dn - t0);
  if (nt <= 0) return;
  nt = min(nt, KT);
  const int Mr = Mk[k], n = nb[k];
  const int RT = (Mr + 15) / 16;
  const int wave = tid >> 6, lane = tid & 63;
  if (tid < NBT) {
    const int t = tid / 16, b = tid % 16;
    int slot = -1;
    if (t < nt && b < tl.nb[t0 + t]) {
      slot = tslot(tl, t0 + t, b);
      if (active && !active[slot]) slot = -1;
    }
    ss[tid] = slot;
  }
  __syncthreads();
  const cplx<R>* Wk = W + (size_t)k * wk_stride;
  const int gbeg = sc * sc_len, gend = min(n, gbeg + sc_len);
  const int npair = RT * nt;
  typename M::acc cre[PW], cim[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) cre[q][v] = cim[q][v] = R(0);
  constexpr int XL = NBT * KCH / NTH, WLM = RTM * 16 * KCH / NTH;
  // 16 KCH is a multiple of NTH, so whole band and row tiles fill the
  // fetch registers exactly
  static_assert(16 * KCH % NTH == 0, "k-wide gram staging");
  const int xl = nt * 16 * KCH / NTH, wl = RT * 16 * KCH / NTH;
  cplx<R> xr[XL], wr[WLM];
  auto fetch = [&](int g0) {
#pragma unroll
    for (int u = 0; u < XL; ++u) {
      if (u < xl) {
        const int i = tid + u * NTH, b = i / KCH, g = g0 + i % KCH;
        const int slot = b < NBT ? ss[b] : -1;
        xr[u] = (slot >= 0 && g < gend) ? X[(size_t)slot * x_stride + g] : mk<R>(0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < WLM; ++u) {
      if (u < wl) {
        const int i = tid + u * NTH, m = i / KCH, g = g0 + i % KCH;
        wr[u] = (m < Mr && g < gend) ? Wk[(size_t)m * w_stride + g] : mk<R>(0, 0);
      }
    }
  };
  if (gbeg < gend) fetch(gbeg);
  for (int g0 = gbeg; g0 < gend; g0 += KCH) {
#pragma unroll
    for (int u = 0; u < XL; ++u) {
      const int i = tid + u * NTH;
      if (i < nt * 16 * KCH) Xs[(i / KCH) * LC + i % KCH] = xr[u];
    }
#pragma unroll
    for (int u = 0; u < WLM; ++u) {
      const int i = tid + u * NTH;
      if (i < RT * 16 * KCH) Ws[(i / KCH) * LC + i % KCH] = wr[u];
    }
    __syncthreads();
    if (g0 + KCH < gend) fetch(g0 + KCH);
#pragma unroll 2
    for (int ks = 0; ks < KCH / 4; ++ks) {
      const int e = 4 * ks + (lane >> 4);
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int pr = wave + NWV * q;
        if (pr < npair) {
          const int rt = pr / nt, bt = pr - rt * nt;
          const cplx<R> wa = Ws[(16 * rt + (lane & 15)) * LC + e];
          const cplx<R> xb = Xs[(16 * bt + (lane & 15)) * LC + e];
          cre[q] = M::mac(wa.x, xb.x, cre[q]);
          cre[q] = M::mac(wa.y, xb.y, cre[q]);
          cim[q] = M::mac(wa.x, xb.y, cim[q]);
          cim[q] = M::mac(-wa.y, xb.x, cim[q]);
        }
      }
    }
    __syncthreads();
  }
  const int j = lane & 15;
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    const int pr = wave + NWV * q;
    if (pr >= npair) continue;
    const int rt = pr / nt, bt = pr - rt * nt, t = t0 + bt;
    if (j >= tl.nb[t]) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = 16 * rt + M::row(lane, v);
      if (m < Mr) part[(((size_t)t * nsc + sc) * Mmax + m) * BT + j] = mk<R>(cre[q][v], cim[q][v]);
    }
  }
}

// coef[(slot0 + b) * cstride + m] = sum_sc part[...]: one wavefront per
// output, lanes take super-chunks lane, lane + 64, ... (fixed order), then
// a fixed shuffle tree.
template <typename R>
__global__ __launch_bounds__(NT) void gram_reduce_kernel(
    Tiles tl, const int* __restrict__ Mk, int Mmax, int nsc,
    const cplx<R>* __restrict__ part, cplx<R>* __restrict__ coef, int cstride,
    const int* __restrict__ active) {
  const int t = blockIdx.x;
  if (!tile_live(tl, t, active)) return;
  const int k = tl.k[t], nbt = tl.nb[t], M = Mk[k];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int o = blockIdx.y * (NT / 64) + wave;
  const int m = o / BT, b = o % BT;
  if (m >= M || b >= nbt) return;
  R sx = 0, sy = 0;
  for (int sc = lane; sc < nsc; sc += 64) {
    const cplx<R> v = part[(((size_t)t * nsc + sc) * Mmax + m) * BT + b];
    sx += v.x;
    sy += v.y;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  if (lane == 0) coef[(size_t)tslot(tl, t, b) * cstride + m] = mk<R>(sx, sy);
}

// acc[b] += sum_{m < M} Wt[m * ws] c[b * Mmax + m]; rows are loaded U at a
// time before use, so that their latencies overlap.
template <typename R, int BPT, int U>
__device__ __forceinline__ void add_term(cplx<R> (&acc)[BPT], const cplx<R>* __restrict__ Wt,
                                         int ws, int M, const cplx<R>* c, int Mmax) {
  int m = 0;
  for (; m + U <= M; m += U) {
    cplx<R> w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) w[u] = Wt[(size_t)(m + u) * ws];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int b = 0; b < BPT; ++b) acc[b] = cadd<R>(acc[b], cmul<R>(w[u], c[b * Mmax + m + u]));
  }
  for (; m < M; ++m) {
    const cplx<R> w = Wt[(size_t)m * ws];
#pragma unroll
    for (int b = 0; b < BPT; ++b) acc[b] = cadd<R>(acc[b], cmul<R>(w, c[b * Mmax + m]));
  }
}

// Y[slot][g] = a * Y[slot][g] + sum_j alpha_j sum_m W_j[k][m][g] coef_j[slot][m]
// for up to two (W, coef) sets; optional per-slot mask; optional partial
// dot <D, Y_new> (real part) per (slot, block) into dpart[slot * nparts + gb].
// A block takes NT coefficients g of BPT bands of its tile: BT / BPT band
// groups split a tile when there are few tiles.  Blocks that share a range
// of g (and so the rows of W they read) are launched 8 apart, which puts
// them on the same XCD and its L2.  The coefficients sit in dynamic LDS,
// BPT * (M1max + M2max) entries.
template <typename R, int BPT>
__global__ __launch_bounds__(NT) void update_kernel(
    Tiles tl, const int* __restrict__ nb, const int* __restrict__ active,
    cplx<R>* __restrict__ Y, int y_stride, R a,
    const cplx<R>* __restrict__ W1, size_t w1k, int w1s, const int* __restrict__ M1k,
    const cplx<R>* __restrict__ C1, int c1s, R alpha1, int M1max,
    const cplx<R>* __restrict__ W2, size_t w2k, int w2s, const int* __restrict__ M2k,
    const cplx<R>* __restrict__ C2, int c2s, R alpha2, int M2max,
    const cplx<R>* __restrict__ D, R* __restrict__ dpart, int nparts) {
  constexpr int G = BT / BPT;
  extern __shared__ __align__(16) unsigned char upd_smem[];
  cplx<R>* c1 = reinterpret_cast<cplx<R>*>(upd_smem);   // [BPT][M1max]
  cplx<R>* c2 = c1 + BPT * M1max;                          // [BPT][M2max]
  __shared__ R red[(NT / 64) * BPT];
  __shared__ int ss[BPT];
  const int t = blockIdx.y, tid = threadIdx.x;
  const int grp = (blockIdx.x >> 3) % G;
  const int gb = (blockIdx.x / (8 * G)) * 8 + (blockIdx.x & 7);
  if (!tile_live(tl, t, active)) return;
  const int k = tl.k[t];
  const int nbg = min(BPT, tl.nb[t] - grp * BPT);     // bands of this group
  if (nbg <= 0) return;
  const int n = nb[k];
  const int M1 = W1 ? min(M1k[k], M1max) : 0, M2 = W2 ? min(M2k[k], M2max) : 0;
  if (tid < BPT) ss[tid] = tid < nbg ? tslot(tl, t, grp * BPT + tid) : 0;
  __syncthreads();
  for (int i = tid; i < BPT * M1max; i += NT) {
    const int b = i / M1max, m = i % M1max;
    c1[i] = (b < nbg && m < M1) ? cscale<R>(C1[(size_t)ss[b] * c1s + m], alpha1) : mk<R>(0, 0);
  }
  for (int i = tid; i < BPT * M2max; i += NT) {
    const int b = i / M2max, m = i % M2max;
    c2[i] = (b < nbg && m < M2) ? cscale<R>(C2[(size_t)ss[b] * c2s + m], alpha2) : mk<R>(0, 0);
  }
  __syncthreads();
  const int g = gb * NT + tid;
  cplx<R> acc[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) acc[b] = mk<R>(0, 0);
  constexpr int U = 4;
  if (g < n) {
    if (W1) add_term<R, BPT, U>(acc, W1 + (size_t)k * w1k + g, w1s, M1, c1, M1max);
    if (W2) add_term<R, BPT, U>(acc, W2 + (size_t)k * w2k + g, w2s, M2, c2, M2max);
  }
  // outputs U bands at a time: loads first, then the stores
#pragma unroll
  for (int b0 = 0; b0 < BPT; b0 += U) {
    cplx<R> yv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      yv[u] = dv[u] = mk<R>(0, 0);
      const int slot = ss[b0 + u];
      if (b0 + u < nbg && (!active || active[slot]) && g < n) {
        if (a != R(0)) yv[u] = Y[(size_t)slot * y_stride + g];   // a = 0: Y is write-only
        if (D) dv[u] = D[(size_t)slot * y_stride + g];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u;
      const int slot = ss[b];
      R d = 0;
      if (b < nbg && (!active || active[slot]) && g < n) {
        const cplx<R> y = mk<R>(a * yv[u].x + acc[b].x, a * yv[u].y + acc[b].y);
        Y[(size_t)slot * y_stride + g] = y;
        d = dv[u].x * y.x + dv[u].y * y.y;
      }
      if (dpart) {
        d = wave_sum(d);
        if ((tid & 63) == 0) red[(tid >> 6) * BPT + b] = d;
      }
    }
  }
  if (dpart) {
    __syncthreads();
    if (tid < nbg) {
      R v = red[tid];
#pragma unroll
      for (int w = 1; w < NT / 64; ++w) v += red[w * BPT + tid];
      dpart[(size_t)ss[tid] * nparts + gb] = v;
    }
  }
}


// out[i] = sum_g part[g][i] (fixed order), optional scale
__global__ void sum_groups_kernel(int n, int ngroups, const double* __restrict__ part,
                                  double scale, double* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n) return;
  double s = 0;
  for (int g = 0; g < ngroups; ++g) s += part[(size_t)g * n + i];
  out[i] = s * scale;
}

// Layout permutes between external C order [N0][N1][N2] and internal
// [C][P][Q]: st_c, st_p, st_q are the external strides of the internal axes.
__global__ void to_internal_kernel(int C, int P, int Q, int st_c, int st_p, int st_q,
                                   const double* __restrict__ ext, double* __restrict__ in) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)C * P * Q) return;
  const int q = i % Q, p = (i / Q) % P, c = i / ((size_t)P * Q);
  in[i] = ext[(size_t)c * st_c + (size_t)p * st_p + (size_t)q * st_q];
}
__global__ void to_external_kernel(int C, int P, int Q, int st_c, int st_p, int st_q,
                                   const double* __restrict__ in, double* __restrict__ ext,
                                   double a, const double* __restrict__ base, double bscale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)C * P * Q) return;
  const int q = i % Q, p = (i / Q) % P, c = i / ((size_t)P * Q);
  const size_t e = (size_t)c * st_c + (size_t)p * st_p + (size_t)q * st_q;
  double v = a * in[i];
  if (base) v += bscale * base[e];
  ext[e] = v;
}

// partial[j * nblk + b] = sum over block b of V[j] . w   (j < nv)
__global__ __launch_bounds__(NT) void multidot_kernel(int n, int nv, const double* __restrict__ V,
                                                      size_t vstride, const double* __restrict__ w,
                                                      double* __restrict__ partial) {
  __shared__ double red[NT];
  const int tid = threadIdx.x;
  for (int j = 0; j < nv; ++j) {
    double s = 0;
    for (size_t i = (size_t)blockIdx.x * NT + tid; i < (size_t)n; i += (size_t)gridDim.x * NT)
      s += V[j * vstride + i] * w[i];
    red[tid] = s;
    __syncthreads();
    for (int q = NT / 2; q > 0; q >>= 1) {
      if (tid < q) red[tid] += red[tid + q];
      __syncthreads();
    }
    if (tid == 0) partial[(size_t)j * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// y = a*y + sum_j c[j] V[j]   (c in device memory, nv <= 64)
__global__ __launch_bounds__(NT) void multiaxpy_kernel(int n, int nv, const double* __restrict__ V,
                                                       size_t vstride, const double* __restrict__ c,
                                                       double a, double* __restrict__ y) {
  __shared__ double cs[64];
  if (threadIdx.x < nv) cs[threadIdx.x] = c[threadIdx.x];
  __syncthreads();
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i >= (size_t)n) return;
  double s = a * y[i];
  for (int j = 0; j < nv; ++j) s += cs[j] * V[j * vstride + i];
  y[i] = s;
}

__global__ void scale_copy_kernel(size_t n, const double* __restrict__ x, double a,
                                  double* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// X = alpha[slot] * Z + beta[slot] * X  over the sphere of each slot
__global__ __launch_bounds__(NT) void cheb_combine_kernel(
    int nb_max, const int* __restrict__ slot_k, const int* __restrict__ nb,
    const double2* __restrict__ Z, double2* __restrict__ X, const double* __restrict__ alpha,
    const double* __restrict__ beta) {
  const int slot = blockIdx.y;
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= nb[slot_k[slot]]) return;
  const size_t o = (size_t)slot * nb_max + g;
  const double a = alpha[slot], b = beta[slot];
  const double2 z = Z[o], x = X[o];
  X[o] = mk<double>(a * z.x + b * x.x, a * z.y + b * x.y);
}

// Per-slot dots against stored vectors (warm starts of the Sternheimer CG):
// part[(slot * nv + l) * gridDim.x + b] = sum over block b's coefficients of
// conj(V[l][slot][g]) x[slot][g], l < nv, V with a stride vstride per l.
constexpr int SD_PER = 4;   // coefficients per thread
__global__ __launch_bounds__(NT) void slot_dots_kernel(
    int nb_max, const int* __restrict__ slot_k, const int* __restrict__ nb, int nv,
    const double2* __restrict__ V, size_t vstride, const double2* __restrict__ x,
    double2* __restrict__ part) {
  __shared__ double rx[NT / 64], ry[NT / 64];
  const int slot = blockIdx.y, tid = threadIdx.x;
  const int n = nb[slot_k[slot]];
  const size_t o = (size_t)slot * nb_max;
  double2 xv[SD_PER];
#pragma unroll
  for (int u = 0; u < SD_PER; ++u) {
    const int g = (blockIdx.x * SD_PER + u) * NT + tid;
    xv[u] = g < n ? x[o + g] : mk<double>(0, 0);
  }
  for (int l = 0; l < nv; ++l) {
    double sx = 0, sy = 0;
#pragma unroll
    for (int u = 0; u < SD_PER; ++u) {
      const int g = (blockIdx.x * SD_PER + u) * NT + tid;
      if (g < n) {
        const double2 v = V[l * vstride + o + g];
        sx += v.x * xv[u].x + v.y * xv[u].y;
        sy += v.x * xv[u].y - v.y * xv[u].x;
      }
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if ((tid & 63) == 0) {
      rx[tid >> 6] = sx;
      ry[tid >> 6] = sy;
    }
    __syncthreads();
    if (tid == 0) {
      double ax = rx[0], ay = ry[0];
      for (int w = 1; w < NT / 64; ++w) {
        ax += rx[w];
        ay += ry[w];
      }
      part[((size_t)slot * nv + l) * gridDim.x + blockIdx.x] = mk<double>(ax, ay);
    }
    __syncthreads();
  }
}

// out[slot][i] = sum_b part[(slot * nv + i) * nb + b] (fixed order)
__global__ void slot_dots_reduce_kernel(int total, int nblk, const double2* __restrict__ part,
                                        double2* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double sx = 0, sy = 0;
  for (int b = 0; b < nblk; ++b) {
    const double2 v = part[(size_t)i * nblk + b];
    sx += v.x;
    sy += v.y;
  }
  out[i] = mk<double>(sx, sy);
}

// y[slot][g] = sum_l c[slot * nv + l] V[l][slot][g] for the listed slots
// (others untouched), over each slot's sphere.
__global__ __launch_bounds__(NT) void slot_combine_kernel(
    int nb_max, const int* __restrict__ list, const int* __restrict__ slot_k,
    const int* __restrict__ nb, int nv, const double2* __restrict__ V, size_t vstride,
    const double2* __restrict__ c, double2* __restrict__ y) {
  const int slot = list[blockIdx.y];
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= nb[slot_k[slot]]) return;
  const size_t o = (size_t)slot * nb_max + g;
  double ax = 0, ay = 0;
  for (int l = 0; l < nv; ++l) {
    const double2 v = V[l * vstride + o], w = c[(size_t)slot * nv + l];
    ax += w.x * v.x - w.y * v.y;
    ay += w.x * v.y + w.y * v.x;
  }
  y[o] = mk<double>(ax, ay);
}

// partial |HX - lam X|^2 per (slot, block)
__global__ __launch_bounds__(NT) void resid_kernel(
    int nb_max, const int* __restrict__ slot_k, const int* __restrict__ nb,
    const double2* __restrict__ HX, const double2* __restrict__ X,
    const double* __restrict__ lam, double* __restrict__ part) {
  __shared__ double red[NT];
  const int slot = blockIdx.y, tid = threadIdx.x;
  const int g = blockIdx.x * NT + tid;
  double s = 0;
  if (g < nb[slot_k[slot]]) {
    const size_t o = (size_t)slot * nb_max + g;
    const double l = lam[slot];
    const double2 h = HX[o], x = X[o];
    const double rx = h.x - l * x.x, ry = h.y - l * x.y;
    s = rx * rx + ry * ry;
  }
  red[tid] = s;
  __syncthreads();
  for (int q = NT / 2; q > 0; q >>= 1) {
    if (tid < q) red[tid] += red[tid + q];
    __syncthreads();
  }
  if (tid == 0) part[(size_t)slot * gridDim.x + blockIdx.x] = red[0];
}

// full[i] = sum_n |G[n][i]|^2 and re[i] = sum_n (Re(ph[n] G[n][i]))^2 over the
// nv rows (ph[n] = (cos, sin) of a phase; null: no phase)
__global__ void grid_row_norms_kernel(size_t ng, int nv, const double2* __restrict__ G,
                                      const double2* __restrict__ ph,
                                      double* __restrict__ full, double* __restrict__ re) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  double f = 0, r = 0;
  for (int n = 0; n < nv; ++n) {
    const double2 v = G[(size_t)n * ng + i];
    const double x = ph ? v.x * ph[n].x - v.y * ph[n].y : v.x;
    f += v.x * v.x + v.y * v.y;
    r += x * x;
  }
  full[i] = f;
  re[i] = r;
}

// part[n * gridDim.x + b] = sum over block b's points of G[n][i]^2 (complex)
__global__ __launch_bounds__(NT) void grid_square_sums_kernel(size_t ng, const double2* __restrict__ G,
                                                             double2* __restrict__ part) {
  __shared__ double rx[NT / 64], ry[NT / 64];
  const int n = blockIdx.y;
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  double sx = 0, sy = 0;
  if (i < ng) {
    const double2 v = G[(size_t)n * ng + i];
    sx = v.x * v.x - v.y * v.y;
    sy = 2 * v.x * v.y;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  if ((threadIdx.x & 63) == 0) {
    rx[threadIdx.x >> 6] = sx;
    ry[threadIdx.x >> 6] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) {
      rx[0] += rx[w];
      ry[0] += ry[w];
    }
    part[(size_t)n * gridDim.x + blockIdx.x] = make_double2(rx[0], ry[0]);
  }
}

// out[slot] = in[slot] over the sphere of the listed slots (precision change)
template <typename A, typename B>
__global__ __launch_bounds__(NT) void cvt_slots_kernel(
    const int* __restrict__ list, const int* __restrict__ slot_k, const int* __restrict__ nb,
    int nb_max, const A* __restrict__ in, B* __restrict__ out) {
  const int slot = list[blockIdx.y];
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= nb[slot_k[slot]]) return;
  const size_t o = (size_t)slot * nb_max + g;
  const A v = in[o];
  B w;
  w.x = v.x;
  w.y = v.y;
  out[o] = w;
}

template <typename A, typename B>
__global__ void cvt_array_kernel(size_t n, const A* __restrict__ in, B* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (B)in[i];
}

template <typename A, typename B>
__global__ void cvt_carray_kernel(size_t n, const A* __restrict__ in, B* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  B w;
  w.x = in[i].x;
  w.y = in[i].y;
  out[i] = w;
}

template <typename R>
__global__ void cscale_kernel(size_t n, cplx<R>* __restrict__ x, R a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = cscale<R>(x[i], a);
}

}  // namespace

// ------------------------------------------------------------ launchers
static std::atomic<int> g_kernel_paths{0};
void set_kernel_paths(int mask) { g_kernel_paths.store(mask); }
int kernel_paths() { return g_kernel_paths.load(); }

// Super-chunks per tile: about `target` blocks over all tiles, each at
// least one chunk long.
static int nsc_for(int nb_max, int ntiles, int target, int& sc_len) {
  const int nch = (nb_max + CH - 1) / CH;
  const int want = (target + ntiles - 1) / (ntiles > 0 ? ntiles : 1);
  int nsc = std::max(1, std::min(nch, want));
  const int per = (nch + nsc - 1) / nsc;
  sc_len = per * CH;
  nsc = (nb_max + sc_len - 1) / sc_len;
  return nsc;
}

// Super-chunks per k-point of the k-wide gram: about KW_BLOCKS blocks over
// the nk k-points (four rounds of one block per CU), each at least one chunk.
constexpr int KW_BLOCKS = 1024;
template <typename R> constexpr int kw_chunk() { return sizeof(R) == 8 ? 32 : 64; }
constexpr int KW_NT_THIN = 256;
template <typename R> constexpr int kw_chunk_thin() { return sizeof(R) == 8 ? 16 : 32; }
static int kw_nsc(int nb_max, int nk, int kch, int& sc_len, double scale = 1.0) {
  const int nch = (nb_max + kch - 1) / kch;
  int nsc = std::max(1, std::min(nch, (int)(scale * KW_BLOCKS) / std::max(nk, 1)));
  const int per = (nch + nsc - 1) / nsc;
  sc_len = per * kch;
  return (nb_max + sc_len - 1) / sc_len;
}

size_t gram_part_elems(int ntiles, int nb_max, int Mmax, int nk, double max_scale) {
  const double sc = std::min(2.0, std::max(1.0, max_scale));
  size_t most = 0;
  for (int t = 1; t <= ntiles; ++t) {
    int sc_len;
    most = std::max(most, (size_t)t * nsc_for(nb_max, t,
                                                 (int)(sc * std::max(gram_blocks<double>(t, true),
                                                                     gram_blocks<float>(t, true))),
                                                 sc_len));
  }
  if (nk > 0) {
    int sc_len;
    const int nsc = std::max(kw_nsc(nb_max, nk, kw_chunk<double>(), sc_len, sc),
                             kw_nsc(nb_max, nk, kw_chunk<float>(), sc_len, sc));
    most = std::max(most, (size_t)ntiles * nsc);
    // the one-tile-per-k instance: at most nk tiles
    const int nsc1 = std::max(kw_nsc(nb_max, nk, kw_chunk_thin<double>(), sc_len, 2 * sc),
                              kw_nsc(nb_max, nk, kw_chunk_thin<float>(), sc_len, 2 * sc));
    most = std::max(most, (size_t)std::min(ntiles, nk) * nsc1);
  }
  return most * Mmax * BT;
}

int gram_variant(int Mmax, const KTileRange& kr, const KernelTune* kt) {
  const int paths = kernel_paths();
  // (k-wide instances: up to 6 tiles of 96 rows, or 5 tiles of 176 rows)
  const bool kw_ok = kr.t0 && kr.nk > 0 &&
                     ((kr.ktmax <= 6 && Mmax <= 96) || (kr.ktmax <= 5 && Mmax <= 176));
  if (paths & PATH_VECTOR_GRAM) return 3;
  if (paths & PATH_KWIDE) return kw_ok ? 2 : (Mmax <= 64 ? 1 : 3);
  if (kt && kt->gram == 1 && Mmax <= 64) return 1;
  if (kt && kt->gram == 2 && kw_ok) return 2;
  if (kt && kt->gram == 3) return 3;
  // by size: matrix cores per tile up to 64 rows, k-wide above when it fits
  if (Mmax <= 64) return 1;
  return kw_ok ? 2 : 3;
}

template <typename R>
int gram_partials(const Tiles& tl, const int* nb, int nb_max, const int* Mk, int Mmax,
                  const cplx<R>* W, size_t wk_stride, int w_stride, const cplx<R>* X,
                  int x_stride, cplx<R>* part, hipStream_t st, const int* active,
                  const KTileRange& kr, const KernelTune* kt) {
  IKR_CHECK(tl.k && tl.slot0 && tl.nb && nb && Mk && W && X && part, 8,
            "gram: null device pointer");
  if (tl.n <= 0) return 0;
  const int variant = gram_variant(Mmax, kr, kt);
  const double scale = kt ? std::min(2.0, std::max(0.5, (double)kt->gram_scale)) : 1.0;
  if (variant == 2) {
    int sc_len;
    if (kr.ktmax <= 1) {
      // at most one band tile per k-point (the late iterations of a CG run):
      // a 4-wavefront block with one band tile and half the chunk, three
      // blocks per CU, twice the blocks
      constexpr int kch = kw_chunk_thin<R>();
      const int nsc = kw_nsc(nb_max, kr.nk, kch, sc_len, 2 * scale);
      const dim3 grid(round8(nsc * kr.nk));
#define IKR_GRAMKW1(RTM)                                                                         \
  hipLaunchKernelGGL((gram_kw_kernel<R, 1, RTM, kch, KW_NT_THIN>), grid, dim3(KW_NT_THIN), 0, st, \
                     tl, kr, nb, Mk, Mmax, W, wk_stride, w_stride, X, x_stride, nsc, sc_len, part,  \
                     active)
      if (Mmax <= 96) IKR_GRAMKW1(6);
      else IKR_GRAMKW1(11);
#undef IKR_GRAMKW1
      IKR_HIP(hipGetLastError());
      return nsc;
    }
    constexpr int kch = kw_chunk<R>();
    const int nsc = kw_nsc(nb_max, kr.nk, kch, sc_len, scale);
    const dim3 grid(round8(nsc * kr.nk));
#define IKR_GRAMKW(KT, RTM)                                                                   \
  hipLaunchKernelGGL((gram_kw_kernel<R, KT, RTM, kch, KW_NT>), grid, dim3(KW_NT), 0, st, tl,  \
                     kr, nb, Mk, Mmax, W, wk_stride, w_stride, X, x_stride, nsc, sc_len, part, \
                     active)
    if (Mmax <= 96) IKR_GRAMKW(6, 6);
    else IKR_GRAMKW(5, 11);
#undef IKR_GRAMKW
    IKR_HIP(hipGetLastError());
    return nsc;
  }
  int sc_len;
  const bool mfma = variant == 1;
  const int nsc = nsc_for(nb_max, tl.n, (int)(scale * gram_blocks<R>(tl.n, mfma)), sc_len);
  // matrix cores up to 64 rows (faster than the vector kernel on the 48^3
  // cell; with more rows the accumulators and prefetch registers leave one or
  // two wavefronts per SIMD)
  if (mfma) {
    const int rt = (Mmax + 15) / 16;
    const int chm = 64;
    const size_t lds = (size_t)(BT + 16 * rt) * (chm + 1) * sizeof(cplx<R>);
    (void)rt;
    IKR_CHECK(sc_len % chm == 0, 8, "gram: super-chunk not a multiple of the MFMA chunk");
#define IKR_GRAMM(RTM, CHM)                                                                   \
  hipLaunchKernelGGL((gram_mfma_kernel<R, RTM, CHM>), dim3(round8(nsc * tl.n)), dim3(NT), lds, \
                     st, tl, nb, Mk, Mmax, W, wk_stride, w_stride, X, x_stride, nsc, sc_len,   \
                     part, active)
    IKR_GRAMM(4, 64);
#undef IKR_GRAMM
    IKR_HIP(hipGetLastError());
    return nsc;
  }
  // rows per pass: 16, 32 or 48 (the smallest that holds Mmax, else 48)
#define IKR_GRAM(RB, SBM)                                                              \
  hipLaunchKernelGGL((gram_kernel<R, RB, SBM>), dim3(round8(nsc * tl.n)), dim3(NT), 0, st, \
                     tl, nb,                                                              \
                     Mk, Mmax, W, wk_stride, w_stride, X, x_stride, nsc, sc_len, part,   \
                     active)
  if (Mmax <= 16) IKR_GRAM(4, 4);
  else if (Mmax <= 32) IKR_GRAM(4, 8);
  else IKR_GRAM(6, 8);
#undef IKR_GRAM
  IKR_HIP(hipGetLastError());
  return nsc;
}

template <typename R>
void gram(const Tiles& tl, const int* nb, int nb_max, const int* Mk, int Mmax,
          const cplx<R>* W, size_t wk_stride, int w_stride, const cplx<R>* X,
          int x_stride, cplx<R>* part, cplx<R>* coef, int cstride, hipStream_t st,
          const int* active, const KTileRange& kr) {
  IKR_CHECK(coef, 8, "gram: null device pointer");
  IKR_CHECK(Mmax <= cstride, 1, "gram: coefficient stride below the row count");
  const int nsc = gram_partials<R>(tl, nb, nb_max, Mk, Mmax, W, wk_stride, w_stride, X,
                                   x_stride, part, st, active, kr);
  gram_reduce<R>(tl, Mk, Mmax, nsc, part, coef, cstride, st, active);
}

template <typename R>
void gram_reduce(const Tiles& tl, const int* Mk, int Mmax, int nsc, const cplx<R>* part,
                 cplx<R>* coef, int cstride, hipStream_t st, const int* active) {
  if (tl.n <= 0 || nsc <= 0) return;
  IKR_CHECK(coef && part, 8, "gram_reduce: null device pointer");
  IKR_CHECK(Mmax <= cstride, 1, "gram_reduce: coefficient stride below the row count");
  const int outs_per_block = NT / 64;
  hipLaunchKernelGGL((gram_reduce_kernel<R>),
                     dim3(tl.n, (Mmax * BT + outs_per_block - 1) / outs_per_block), dim3(NT),
                     0, st, tl, Mk, Mmax, nsc, part, coef, cstride, active);
  IKR_HIP(hipGetLastError());
}

// Partials per slot of the update's dot: NT-wide blocks of g, padded to a
// multiple of 8 (the XCD interleave of the launch).
int update_nblocks(int nb_max) { return ((nb_max + NT - 1) / NT + 7) / 8 * 8; }

template <typename R>
void update(const Tiles& tl, const int* nb, int nb_max, const int* active,
            cplx<R>* Y, int y_stride, R a, const UpdTerm<R>& t1,
            const UpdTerm<R>& t2, const cplx<R>* D, R* dpart, hipStream_t st) {
  IKR_CHECK(tl.k && tl.slot0 && tl.nb && nb && Y, 8, "update: null device pointer");
  IKR_CHECK((!t1.W || (t1.Mk && t1.C)) && (!t2.W || (t2.Mk && t2.C)), 8,
            "update: null coefficient pointer");
  const int M1max = t1.W ? t1.Mmax : 0, M2max = t2.W ? t2.Mmax : 0;
  IKR_CHECK((size_t)BT * (M1max + M2max) * sizeof(cplx<R>) <= 65536, 1,
            "update: too many projector rows");
  if (tl.n <= 0) return;
  const int ngb = update_nblocks(nb_max);
  const int blocks = ngb * tl.n;
  const int bpt = blocks >= UPD_BLOCKS ? 16 : (2 * blocks >= UPD_BLOCKS ? 8 : 4);
  const size_t lds = (size_t)bpt * (M1max + M2max) * sizeof(cplx<R>);
  const dim3 grid(ngb * (BT / bpt), tl.n);
#define IKR_UPD(B)                                                                    \
  hipLaunchKernelGGL((update_kernel<R, B>), grid, dim3(NT), lds, st, tl, nb, active, Y,  \
                     y_stride, a, t1.W, t1.wk, t1.ws, t1.Mk, t1.C, t1.cs, t1.alpha, M1max, \
                     t2.W, t2.wk, t2.ws, t2.Mk, t2.C, t2.cs, t2.alpha, M2max, D, dpart, ngb)
  if (bpt == 16) IKR_UPD(16);
  else if (bpt == 8) IKR_UPD(8);
  else IKR_UPD(4);
#undef IKR_UPD
  IKR_HIP(hipGetLastError());
}

int vec_nblocks(int nb_max) { return (nb_max + NT - 1) / NT; }

void sum_groups(int n, int ngroups, const double* part, double scale, double* out,
                hipStream_t st) {
  hipLaunchKernelGGL(sum_groups_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, ngroups,
                     part, scale, out);
  IKR_HIP(hipGetLastError());
}

void to_internal(const Layout& L, const double* ext, double* in, hipStream_t st) {
  const size_t n = (size_t)L.C * L.P * L.Q;
  hipLaunchKernelGGL(to_internal_kernel, dim3((n + 255) / 256), dim3(256), 0, st, L.C, L.P,
                     L.Q, L.st_c, L.st_p, L.st_q, ext, in);
  IKR_HIP(hipGetLastError());
}

void to_external(const Layout& L, const double* in, double* ext, double a,
                 const double* base, double bscale, hipStream_t st) {
  const size_t n = (size_t)L.C * L.P * L.Q;
  hipLaunchKernelGGL(to_external_kernel, dim3((n + 255) / 256), dim3(256), 0, st, L.C, L.P,
                     L.Q, L.st_c, L.st_p, L.st_q, in, ext, a, base, bscale);
  IKR_HIP(hipGetLastError());
}

int multidot_nblocks(int n) {
  int b = (n + NT * 4 - 1) / (NT * 4);
  return b < 256 ? b : 256;
}

void multidot(int n, int nv, const double* V, size_t vstride, const double* w,
              double* partial, hipStream_t st) {
  hipLaunchKernelGGL(multidot_kernel, dim3(multidot_nblocks(n)), dim3(NT), 0, st, n, nv, V,
                     vstride, w, partial);
  IKR_HIP(hipGetLastError());
}

void multiaxpy(int n, int nv, const double* V, size_t vstride, const double* c, double a,
               double* y, hipStream_t st) {
  IKR_CHECK(nv <= 64, 1, "too many vectors in multiaxpy");
  hipLaunchKernelGGL(multiaxpy_kernel, dim3((n + NT - 1) / NT), dim3(NT), 0, st, n, nv, V,
                     vstride, c, a, y);
  IKR_HIP(hipGetLastError());
}

void grid_row_norms(size_t ng, int nv, const double2* G, const double2* phase, double* full,
                    double* re, hipStream_t st) {
  hipLaunchKernelGGL(grid_row_norms_kernel, dim3((ng + 255) / 256), dim3(256), 0, st, ng, nv, G,
                     phase, full, re);
  IKR_HIP(hipGetLastError());
}

int grid_square_nblocks(size_t ng) { return (int)((ng + NT - 1) / NT); }

void grid_square_sums(size_t ng, int nv, const double2* G, double2* part, hipStream_t st) {
  if (nv <= 0) return;
  hipLaunchKernelGGL(grid_square_sums_kernel, dim3(grid_square_nblocks(ng), nv), dim3(NT), 0, st,
                     ng, G, part);
  IKR_HIP(hipGetLastError());
}

void scale_copy(size_t n, const double* x, double a, double* y, hipStream_t st) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, x, a, y);
  IKR_HIP(hipGetLastError());
}

void convert_slots(int n, const int* list, const int* slot_k, const int* nb, int nb_max,
                   const double2* in, float2* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((cvt_slots_kernel<double2, float2>), dim3(vec_nblocks(nb_max), n),
                     dim3(NT), 0, st, list, slot_k, nb, nb_max, in, out);
  IKR_HIP(hipGetLastError());
}

void convert_slots(int n, const int* list, const int* slot_k, const int* nb, int nb_max,
                   const float2* in, double2* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((cvt_slots_kernel<float2, double2>), dim3(vec_nblocks(nb_max), n),
                     dim3(NT), 0, st, list, slot_k, nb, nb_max, in, out);
  IKR_HIP(hipGetLastError());
}

void convert_array(size_t n, const double* in, float* out, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL((cvt_array_kernel<double, float>), dim3((n + 255) / 256), dim3(256), 0, st,
                     n, in, out);
  IKR_HIP(hipGetLastError());
}

void convert_array(size_t n, const double2* in, float2* out, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL((cvt_carray_kernel<double2, float2>), dim3((n + 255) / 256), dim3(256), 0,
                     st, n, in, out);
  IKR_HIP(hipGetLastError());
}

void cheb_combine(int nslots, int nb_max, const int* slot_k, const int* nb, const double2* Z,
                  double2* X, const double* alpha, const double* beta, hipStream_t st) {
  hipLaunchKernelGGL(cheb_combine_kernel, dim3(vec_nblocks(nb_max), nslots), dim3(NT), 0, st,
                     nb_max, slot_k, nb, Z, X, alpha, beta);
  IKR_HIP(hipGetLastError());
}

void slot_dots(int nslots, int nb_max, const int* slot_k, const int* nb, int nv,
               const double2* V, size_t vstride, const double2* x, double2* part,
               double2* out, hipStream_t st) {
  if (nslots <= 0 || nv <= 0) return;
  const int nblk = (nb_max + SD_PER * NT - 1) / (SD_PER * NT);
  hipLaunchKernelGGL(slot_dots_kernel, dim3(nblk, nslots), dim3(NT), 0, st, nb_max, slot_k, nb,
                     nv, V, vstride, x, part);
  IKR_HIP(hipGetLastError());
  const int total = nslots * nv;
  hipLaunchKernelGGL(slot_dots_reduce_kernel, dim3((total + 255) / 256), dim3(256), 0, st, total,
                     nblk, part, out);
  IKR_HIP(hipGetLastError());
}

size_t slot_dots_part_elems(int nslots, int nb_max, int nv) {
  return (size_t)nslots * nv * ((nb_max + SD_PER * NT - 1) / (SD_PER * NT));
}

void slot_combine(int nlist, const int* list, int nb_max, const int* slot_k, const int* nb,
                  int nv, const double2* V, size_t vstride, const double2* c, double2* y,
                  hipStream_t st) {
  if (nlist <= 0) return;
  hipLaunchKernelGGL(slot_combine_kernel, dim3(vec_nblocks(nb_max), nlist), dim3(NT), 0, st,
                     nb_max, list, slot_k, nb, nv, V, vstride, c, y);
  IKR_HIP(hipGetLastError());
}

void resid_norms(int nslots, int nb_max, const int* slot_k, const int* nb, const double2* HX,
                 const double2* X, const double* lam, double* part, hipStream_t st) {
  hipLaunchKernelGGL(resid_kernel, dim3(vec_nblocks(nb_max), nslots), dim3(NT), 0, st, nb_max,
                     slot_k, nb, HX, X, lam, part);
  IKR_HIP(hipGetLastError());
}

template <typename R>
void cscale_vec(size_t n, cplx<R>* x, R a, hipStream_t st) {
  hipLaunchKernelGGL((cscale_kernel<R>), dim3((n + 255) / 256), dim3(256), 0, st, n, x, a);
  IKR_HIP(hipGetLastError());
}

#define IKR_INST(R)                                                                       \
  template void gram<R>(const Tiles&, const int*, int, const int*, int, const cplx<R>*,   \
                        size_t, int, const cplx<R>*, int, cplx<R>*, cplx<R>*, int,        \
                        hipStream_t, const int*, const KTileRange&);                      \
  template int gram_partials<R>(const Tiles&, const int*, int, const int*, int,           \
                                const cplx<R>*, size_t, int, const cplx<R>*, int,         \
                                cplx<R>*, hipStream_t, const int*, const KTileRange&,     \
                                const KernelTune*);                                       \
  template void gram_reduce<R>(const Tiles&, const int*, int, int, const cplx<R>*,        \
                               cplx<R>*, int, hipStream_t, const int*);                   \
  template void update<R>(const Tiles&, const int*, int, const int*, cplx<R>*, int, R,    \
                          const UpdTerm<R>&, const UpdTerm<R>&, const cplx<R>*, R*,       \
                          hipStream_t);                                                   \
  template void cscale_vec<R>(size_t, cplx<R>*, R, hipStream_t);
IKR_INST(double)
IKR_INST(float)
#undef IKR_INST

}  // namespace ikr
