// Fused Sternheimer CG kernels: one projection gram and one two-output
// update per iteration, the vector step with both dots, per-slot scalars,
// and the on-device active-set compaction (no host round trip per
// iteration).  Reductions are two-stage with fixed orders, so results are
// bitwise reproducible run to run.
#include "cg.h"
#include "mfma.h"

namespace ikr {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;
constexpr int CT = 1024;     // threads of the compaction block

template <typename T> __device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block sums of two values (result in thread 0): shuffles, then the waves
// in order.
template <typename R> __device__ __forceinline__ void block_sum2(R& a, R& b, R* red) {
  a = wsum(a);
  b = wsum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = a;
    red[NW + w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = red[0];
    b = red[NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
      a += red[i];
      b += red[NW + i];
    }
  }
}

template <typename R>
__global__ __launch_bounds__(NT) void cg_start_kernel(
    Slots s, const int* __restrict__ nb, const double* __restrict__ kin, int nb_max,
    const R* __restrict__ pshift, const cplx<R>* __restrict__ r, cplx<R>* __restrict__ z,
    R* __restrict__ rpart, R* __restrict__ zpart) {
  __shared__ R red[2 * NW];
  if (!row_live(s, blockIdx.y)) return;
  const int slot = slot_of(s, blockIdx.y);
  const int k = s.k[slot];
  const int g = blockIdx.x * NT + threadIdx.x;
  R rr = 0, rz = 0;
  if (g < nb[k]) {
    const size_t o = (size_t)slot * nb_max + g;
    const R m = R(1) / (R(kin[(size_t)k * nb_max + g]) + pshift[slot]);
    const cplx<R> rv = r[o];
    z[o] = cscale<R>(rv, m);
    rr = rv.x * rv.x + rv.y * rv.y;
    rz = m * rr;
  }
  block_sum2(rr, rz, red);
  if (threadIdx.x == 0) {
    rpart[(size_t)slot * gridDim.x + blockIdx.x] = rr;
    zpart[(size_t)slot * gridDim.x + blockIdx.x] = rz;
  }
}

// One block per listed slot.  The slot's raw coefficients (q, then a_m,
// h_m interleaved) are staged in LDS; the j-sum of c is split over the
// wavefronts (j = wave, wave + NW, ...) and the partials are added in wave
// order.  LDS: c [Mr], wave partials [NW][Mq_max].
template <typename R>
__global__ __launch_bounds__(NT) void cg_combine_kernel(
    Slots s, int Na, const int* __restrict__ Mq, int Mq_max, const cplx<R>* __restrict__ craw,
    int cstride, const R* __restrict__ shift, const cplx<R>* __restrict__ GT,
    const cplx<R>* __restrict__ ST, int nbn, R dnl, cplx<R>* __restrict__ gam) {
  extern __shared__ __align__(16) unsigned char cgc_smem[];
  if (!row_live(s, blockIdx.x)) return;
  const int slot = slot_of(s, blockIdx.x);
  const int k = s.k[slot];
  const int M = min(Mq[k], Mq_max);
  const int Mr = Na + 2 * M;
  cplx<R>* c = reinterpret_cast<cplx<R>*>(cgc_smem);
  cplx<R>* wp = c + Na + 2 * Mq_max;
  const cplx<R>* cr = craw + (size_t)slot * cstride;
  for (int r = threadIdx.x; r < Mr; r += NT) c[r] = cr[r];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const R e = shift[slot];
  const cplx<R>* G = GT + (size_t)k * nbn * nbn;
  const cplx<R>* S = ST + (size_t)k * nbn * nbn;
  for (int m = lane; m < M; m += 64) {
    R cx = 0, cy = 0;
#pragma unroll 4
    for (int j = wave; j < M; j += NW) {
      const cplx<R> aj = c[Na + 2 * j];
      const cplx<R> g = G[(size_t)j * nbn + m], sv = S[(size_t)j * nbn + m];
      const R dx = g.x - e * sv.x, dy = g.y - e * sv.y;
      cx += dx * aj.x - dy * aj.y;
      cy += dx * aj.y + dy * aj.x;
    }
    wp[wave * Mq_max + m] = mk<R>(cx, cy);
  }
  __syncthreads();
  cplx<R>* o = gam + (size_t)slot * cstride;
  for (int r = threadIdx.x; r < Na; r += NT) o[r] = cscale<R>(c[r], dnl);
  for (int m = threadIdx.x; m < M; m += NT) {
    R sx = wp[m].x, sy = wp[m].y;
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      sx += wp[w * Mq_max + m].x;
      sy += wp[w * Mq_max + m].y;
    }
    const cplx<R> am = c[Na + 2 * m], hm = c[Na + 2 * m + 1];
    const R cx = hm.x - e * am.x - sx, cy = hm.y - e * am.y - sy;
    o[Na + 2 * m] = mk<R>(e * am.x - cx, e * am.y - cy);
    o[Na + 2 * m + 1] = mk<R>(-am.x, -am.y);
  }
}

// A block takes NT coefficients g of BPT bands; band groups split a tile
// when tiles are few.  LDS: gam [BPT][Mrows], -a [BPT][Mq_max].
template <typename R, int BPT>
__global__ __launch_bounds__(NT) void cg_update_kernel(
    Tiles tl, const int* __restrict__ nb, int nb_max, const cplx<R>* __restrict__ Wcg,
    size_t wk, int Na, const int* __restrict__ Mq, int Mq_max,
    const cplx<R>* __restrict__ gam, int cstride, cplx<R>* __restrict__ Wv,
    cplx<R>* __restrict__ P, R* __restrict__ dpart, int nparts) {
  constexpr int G = BT / BPT;
  extern __shared__ __align__(16) unsigned char cgu_smem[];
  const int Mr = Na + 2 * Mq_max;
  cplx<R>* cg = reinterpret_cast<cplx<R>*>(cgu_smem);   // [BPT][Mr]
  cplx<R>* ca = cg + BPT * Mr;                             // [BPT][Mq_max]
  __shared__ R red[NW * BPT];
  __shared__ int ss[BPT];
  // items (g block, tile, band group) with the band group fastest: every
  // block that reads one chunk of W_k runs back to back on one XCD
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nparts * tl.n * G) return;
  const int tid = threadIdx.x;
  const int grp = item % G, t = (item / G) % tl.n, gb = item / (G * tl.n);
  if (tl.dn && t >= *tl.dn) return;
  const int k = tl.k[t];
  const int nbg = min(BPT, tl.nb[t] - grp * BPT);
  if (nbg <= 0) return;
  const int n = nb[k];
  const int M = min(Mq[k], Mq_max);
  if (tid < BPT) ss[tid] = tid < nbg ? tslot(tl, t, grp * BPT + tid) : 0;
  __syncthreads();
  for (int i = tid; i < BPT * Mr; i += NT) {
    const int b = i / Mr, r = i % Mr;
    cg[i] = (b < nbg && r < Na + 2 * M) ? gam[(size_t)ss[b] * cstride + r] : mk<R>(0, 0);
  }
  for (int i = tid; i < BPT * Mq_max; i += NT) {   // -a_m, held by gam
    const int b = i / Mq_max, m = i % Mq_max;
    ca[i] = (b < nbg && m < M) ? gam[(size_t)ss[b] * cstride + Na + 2 * m + 1] : mk<R>(0, 0);
  }
  __syncthreads();
  const int g = gb * NT + tid;
  cplx<R> a1[BPT], a2[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) a1[b] = a2[b] = mk<R>(0, 0);
  // rows are loaded U at a time before use, so that their latencies overlap
  constexpr int U = 4;
  if (g < n) {
    const cplx<R>* W = Wcg + (size_t)k * wk + g;
    int r = 0;
    for (; r + U <= Na; r += U) {
      cplx<R> w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) w[u] = W[(size_t)(r + u) * nb_max];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int b = 0; b < BPT; ++b) a1[b] = cadd<R>(a1[b], cmul<R>(w[u], cg[b * Mr + r + u]));
    }
    for (; r < Na; ++r) {
      const cplx<R> w = W[(size_t)r * nb_max];
#pragma unroll
      for (int b = 0; b < BPT; ++b) a1[b] = cadd<R>(a1[b], cmul<R>(w, cg[b * Mr + r]));
    }
    int m = 0;
    for (; m + U <= M; m += U) {
      cplx<R> f[U], h[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        f[u] = W[(size_t)(Na + 2 * (m + u)) * nb_max];
        h[u] = W[(size_t)(Na + 2 * (m + u) + 1) * nb_max];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
          const int c0 = b * Mr + Na + 2 * (m + u);
          a1[b] = cadd<R>(a1[b], cadd<R>(cmul<R>(f[u], cg[c0]), cmul<R>(h[u], cg[c0 + 1])));
          a2[b] = cadd<R>(a2[b], cmul<R>(f[u], ca[b * Mq_max + m + u]));
        }
    }
    for (; m < M; ++m) {
      const cplx<R> f = W[(size_t)(Na + 2 * m) * nb_max];
      const cplx<R> h = W[(size_t)(Na + 2 * m + 1) * nb_max];
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        a1[b] = cadd<R>(a1[b], cadd<R>(cmul<R>(f, cg[b * Mr + Na + 2 * m]),
                                       cmul<R>(h, cg[b * Mr + Na + 2 * m + 1])));
        a2[b] = cadd<R>(a2[b], cmul<R>(f, ca[b * Mq_max + m]));
      }
    }
  }
  // outputs U bands at a time: loads first, then the stores
#pragma unroll
  for (int b0 = 0; b0 < BPT; b0 += U) {
    cplx<R> wv[U], pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      wv[u] = pv[u] = mk<R>(0, 0);
      if (b0 + u < nbg && g < n) {
        const size_t o = (size_t)ss[b0 + u] * nb_max + g;
        wv[u] = Wv[o];
        pv[u] = P[o];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u;
      R d = 0;
      if (b < nbg && g < n) {
        const size_t o = (size_t)ss[b] * nb_max + g;
        const cplx<R> ap = cadd<R>(wv[u], a1[b]);
        const cplx<R> pn = cadd<R>(pv[u], a2[b]);
        Wv[o] = ap;
        P[o] = pn;
        d = pn.x * ap.x + pn.y * ap.y;
      }
      d = wsum(d);
      if ((tid & 63) == 0) red[(tid >> 6) * BPT + b] = d;
    }
  }
  __syncthreads();
  if (tid < nbg) {
    R v = red[tid];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[w * BPT + tid];
    dpart[(size_t)ss[tid] * nparts + gb] = v;
  }
}

// The tiled update on the matrix cores: a block takes NT coefficients g of
// one 16-band tile, its wavefronts take 16 of them at a time, and each step
// of 4 rows of W_k is a 16x16x4 product (A = the tile's coefficients
// [band][row] from LDS, B = W [row][g] straight from its loads, 16 running g
// per row: 256-byte runs; D = [band][g], so a lane's results lie along g).
// Rows go in three groups: projectors (Ap only), phi rows (Ap and p) and
// H phi rows (Ap only), U steps of loads in flight.  Complex products are
// four real ones (Re += Gr Wr - Gi Wi, Im += Gr Wi + Gi Wr).  W_k is read
// once per tile whatever the number of bands, where the vector kernel reads
// it once per band group.  The <p, Ap> partials of the block's NT
// coefficients: per band over the 16 lanes of a g run, then over the
// wavefronts in order.  LDS: coefficients [Mr][16], -a [Mq_max][16].
template <typename R, int U>
__global__ __launch_bounds__(NT) void cg_update_mfma_kernel(
    Tiles tl, const int* __restrict__ nb, int nb_max, const cplx<R>* __restrict__ Wcg,
    size_t wk, int Na, const int* __restrict__ Mq, int Mq_max,
    const cplx<R>* __restrict__ gam, int cstride, cplx<R>* __restrict__ Wv,
    cplx<R>* __restrict__ P, R* __restrict__ dpart, int nparts) {
  using MF = Mfma<R>;
  extern __shared__ __align__(16) unsigned char cgm_smem[];
  const int Mr = Na + 2 * Mq_max;
  cplx<R>* cgl = reinterpret_cast<cplx<R>*>(cgm_smem);   // [Mr][16]
  cplx<R>* cal = cgl + 16 * Mr;                            // [Mq_max][16]
  __shared__ R red[NW * 16];
  __shared__ int ss[16];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nparts * tl.n) return;
  const int tid = threadIdx.x;
  const int t = item % tl.n, gb = item / tl.n;
  if (tl.dn && t >= *tl.dn) return;
  const int k = tl.k[t], nbt = tl.nb[t], n = nb[k];
  const int M = min(Mq[k], Mq_max);
  if (tid < 16) ss[tid] = tid < nbt ? tslot(tl, t, tid) : 0;
  __syncthreads();
  for (int i = tid; i < 16 * Mr; i += NT) {
    const int r = i / 16, b = i % 16;
    cgl[i] = (b < nbt && r < Na + 2 * M) ? gam[(size_t)ss[b] * cstride + r] : mk<R>(0, 0);
  }
  for (int i = tid; i < 16 * Mq_max; i += NT) {   // -a_m, held by gam
    const int m = i / 16, b = i % 16;
    cal[i] = (b < nbt && m < M) ? gam[(size_t)ss[b] * cstride + Na + 2 * m + 1] : mk<R>(0, 0);
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const cplx<R>* Wk = Wcg + (size_t)k * wk;
  R dsum[4] = {0, 0, 0, 0};
  for (int c = wave; c < NT / 16; c += NW) {
    const int g0 = gb * NT + 16 * c;
    if (g0 >= n) break;
    const int g = g0 + li;
    const bool gin = g < n;
    typename MF::acc are, aim, pre, pim;
#pragma unroll
    for (int v = 0; v < 4; ++v) are[v] = aim[v] = pre[v] = pim[v] = R(0);
    // Ap += G W over rows [r0, r0 + 4 nst) of stride rs (coefficient row of
    // step s: r0 + rs (4 s + lk)); with PHI, p += (-a) W as well
    auto group = [&](int r0, int rs, int nrows, int nst, bool phi) {
      for (int s0 = 0; s0 < nst; s0 += U) {
        cplx<R> w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = 4 * (s0 + u) + lk;
          w[u] = (s0 + u < nst && q < nrows && gin) ? Wk[(size_t)(r0 + rs * q) * nb_max + g]
                                                    : mk<R>(0, 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (s0 + u >= nst) break;
          const int q = min(4 * (s0 + u) + lk, nrows - 1);
          const cplx<R> a = cgl[(r0 + rs * q) * 16 + li];
          are = MF::mac(a.x, w[u].x, are);
          are = MF::mac(-a.y, w[u].y, are);
          aim = MF::mac(a.x, w[u].y, aim);
          aim = MF::mac(a.y, w[u].x, aim);
          if (phi) {
            const cplx<R> b = cal[q * 16 + li];
            pre = MF::mac(b.x, w[u].x, pre);
            pre = MF::mac(-b.y, w[u].y, pre);
            pim = MF::mac(b.x, w[u].y, pim);
            pim = MF::mac(b.y, w[u].x, pim);
          }
        }
      }
    };
    if (Na > 0) group(0, 1, Na, (Na + 3) / 4, false);
    if (M > 0) {
      group(Na, 2, M, (M + 3) / 4, true);
      group(Na + 1, 2, M, (M + 3) / 4, false);
    }
    // Ap = w~ + D, p = p~ + Dp for the lane's four (band, g); loads first
    cplx<R> wv[4], pv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = MF::row(lane, v);
      wv[v] = pv[v] = mk<R>(0, 0);
      if (b < nbt && gin) {
        const size_t o = (size_t)ss[b] * nb_max + g;
        wv[v] = Wv[o];
        pv[v] = P[o];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = MF::row(lane, v);
      if (b < nbt && gin) {
        const size_t o = (size_t)ss[b] * nb_max + g;
        const cplx<R> ap = mk<R>(wv[v].x + are[v], wv[v].y + aim[v]);
        const cplx<R> pn = mk<R>(pv[v].x + pre[v], pv[v].y + pim[v]);
        Wv[o] = ap;
        P[o] = pn;
        dsum[v] += pn.x * ap.x + pn.y * ap.y;
      }
    }
  }
  // per band: over the 16 lanes of a g run (fixed tree), then the wavefronts in order
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    R d = dsum[v];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) d += __shfl_xor(d, o, 16);
    if (li == 0) red[wave * 16 + MF::row(lane, v)] = d;
  }
  __syncthreads();
  if (tid < nbt) {
    R v = red[tid];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[w * 16 + tid];
    dpart[(size_t)ss[tid] * nparts + gb] = v;
  }
}

// The same update for all bands of a k-point at once, on the matrix cores:
//   Ap[b][g] = w~[b][g] + sum_r gam[b][r] W[r][g]          (all Mr rows)
//   p[b][g]  = p~[b][g] + sum_m gam[b][Na + 2m + 1] W[Na + 2m][g]   (phi rows)
// A block takes one (k, chunk of GB coefficients) item and every band of k
// (up to KT tiles: t0[k] .. t0[k+1] of the compact tiles), so W_k is read once
// per iteration.  The rows go through LDS 16 at a time with the coefficients
// of those rows (and the -a_m of the phi rows among them); the (g tile, band
// tile) pairs of the output are dealt to the 8 wavefronts round-robin.  Each
// pair holds two accumulators (Ap and p), each four real 16x16x4 products per
// 4 rows (Re = Gr Wr - Gi Wi, Im = Gr Wi + Gi Wr): A = coefficients
// [band][row], B = W [row][g], so a lane's results lie along g.  The
// <p, Ap> partial of each band goes to dpart[slot * nparts + chunk].
constexpr int UKW_NT = 512;
constexpr int UKW_RC = 16;     // rows per LDS stage

template <typename R, int KT, int GB>
__global__ __launch_bounds__(UKW_NT) void cg_update_kw_kernel(
    Tiles tl, KTileRange kr, const int* __restrict__ nb, int nb_max,
    const cplx<R>* __restrict__ Wcg, size_t wk, int Na, const int* __restrict__ Mq, int Mq_max,
    const cplx<R>* __restrict__ gam, int cstride, cplx<R>* __restrict__ Wv,
    cplx<R>* __restrict__ P, R* __restrict__ dpart, int nparts) {
  using M = Mfma<R>;
  constexpr int NBT = KT * 16, GT = GB / 16, NPAIR = KT * GT;
  constexpr int PW = (NPAIR + 7) / 8;
  constexpr int LW = GB + 1, LG = UKW_RC + 1, LA = UKW_RC / 2 + 1;
  __shared__ cplx<R> Ws[UKW_RC * LW];     // W rows [r][g]
  __shared__ cplx<R> Gs[NBT * LG];        // gam [band][r]
  __shared__ cplx<R> As[NBT * LA];        // -a of the chunk's phi rows [band][m]
  __shared__ int ss[NBT];
  __shared__ R red[GT * NBT];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nparts * kr.nk) return;
  const int k = item / nparts, gc = item % nparts, tid = threadIdx.x;
  int t0 = kr.t0[k], nt = kr.t0[k + 1] - t0;
  if (tl.dn) nt = min(nt, *tl.dn - t0);
  if (nt <= 0) return;
  nt = min(nt, KT);
  const int n = nb[k], g0 = gc * GB;
  if (g0 >= n) {   // past this k's sphere: zero partials (the vector step sums all nparts)
    if (tid < NBT) {
      const int t = tid / 16, b = tid % 16;
      if (t < nt && b < tl.nb[t0 + t]) dpart[(size_t)tslot(tl, t0 + t, b) * nparts + gc] = R(0);
    }
    return;
  }
  const int Mm = min(Mq[k], Mq_max), Mr = Na + 2 * Mm;
  const int wave = tid >> 6, lane = tid & 63;
  if (tid < NBT) {
    const int t = tid / 16, b = tid % 16;
    ss[tid] = (t < nt && b < tl.nb[t0 + t]) ? tslot(tl, t0 + t, b) : -1;
  }
  for (int i = tid; i < GT * NBT; i += UKW_NT) red[i] = R(0);
  __syncthreads();
  const int npair = GT * nt;
  typename M::acc c1r[PW], c1i[PW], c2r[PW], c2i[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) c1r[q][v] = c1i[q][v] = c2r[q][v] = c2i[q][v] = R(0);
  const cplx<R>* Wk = Wcg + (size_t)k * wk;
  for (int r0 = 0; r0 < Mr; r0 += UKW_RC) {
    // phi rows Na + 2m of this stage: m in [mlo, mhi)
    const int mlo = r0 <= Na ? 0 : (r0 - Na + 1) / 2;
    const int mhi = min(Mm, r0 + UKW_RC <= Na ? 0 : (r0 + UKW_RC - Na + 1) / 2);
    for (int i = tid; i < UKW_RC * GB; i += UKW_NT) {
      const int rr = i / GB, gg = i % GB, r = r0 + rr, g = g0 + gg;
      Ws[rr * LW + gg] = (r < Mr && g < n) ? Wk[(size_t)r * nb_max + g] : mk<R>(0, 0);
    }
    for (int i = tid; i < NBT * UKW_RC; i += UKW_NT) {
      const int b = i / UKW_RC, rr = i % UKW_RC, r = r0 + rr, slot = ss[b];
      Gs[b * LG + rr] = (slot >= 0 && r < Mr) ? gam[(size_t)slot * cstride + r] : mk<R>(0, 0);
    }
    for (int i = tid; i < NBT * (UKW_RC / 2); i += UKW_NT) {
      const int b = i / (UKW_RC / 2), mm = i % (UKW_RC / 2), m = mlo + mm, slot = ss[b];
      As[b * LA + mm] = (slot >= 0 && m < mhi) ? gam[(size_t)slot * cstride + Na + 2 * m + 1]
                                               : mk<R>(0, 0);
    }
    __syncthreads();
    // Ap: the 16 rows of the stage, 4 per product
#pragma unroll 1
    for (int j = 0; j < UKW_RC / 4; ++j) {
      const int rr = 4 * j + (lane >> 4);
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int pr = wave + 8 * q;
        if (pr < npair) {
          const int bt = pr / GT, gt = pr - bt * GT;
          const cplx<R> ga = Gs[(16 * bt + (lane & 15)) * LG + rr];
          const cplx<R> wb = Ws[rr * LW + 16 * gt + (lane & 15)];
          c1r[q] = M::mac(ga.x, wb.x, c1r[q]);
          c1r[q] = M::mac(-ga.y, wb.y, c1r[q]);
          c1i[q] = M::mac(ga.x, wb.y, c1i[q]);
          c1i[q] = M::mac(ga.y, wb.x, c1i[q]);
        }
      }
    }
    // p: the phi rows of the stage (at most 8), 4 per product
    for (int mb = mlo; mb < mhi; mb += 4) {
      const int m = mb + (lane >> 4);
      const bool ok = m < mhi;
      const int rr = Na + 2 * m - r0;
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int pr = wave + 8 * q;
        if (pr < npair) {
          const int bt = pr / GT, gt = pr - bt * GT;
          const cplx<R> aa = ok ? As[(16 * bt + (lane & 15)) * LA + (m - mlo)] : mk<R>(0, 0);
          const cplx<R> wb = ok ? Ws[rr * LW + 16 * gt + (lane & 15)] : mk<R>(0, 0);
          c2r[q] = M::mac(aa.x, wb.x, c2r[q]);
          c2r[q] = M::mac(-aa.y, wb.y, c2r[q]);
          c2i[q] = M::mac(aa.x, wb.y, c2i[q]);
          c2i[q] = M::mac(aa.y, wb.x, c2i[q]);
        }
      }
    }
    __syncthreads();
  }
  // Ap = w~ + ..., p = p~ + ..., and <p, Ap> summed over the 16 lanes of each
  // band row, then over the g tiles
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    const int pr = wave + 8 * q;
    if (pr >= npair) continue;
    const int bt = pr / GT, gt = pr - bt * GT;
    const int g = g0 + 16 * gt + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = 16 * bt + M::row(lane, v);
      const int slot = ss[b];
      R d = 0;
      if (slot >= 0 && g < n) {
        const size_t o = (size_t)slot * nb_max + g;
        const cplx<R> ap = cadd<R>(Wv[o], mk<R>(c1r[q][v], c1i[q][v]));
        const cplx<R> pn = cadd<R>(P[o], mk<R>(c2r[q][v], c2i[q][v]));
        Wv[o] = ap;
        P[o] = pn;
        d = pn.x * ap.x + pn.y * ap.y;
      }
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) d += __shfl_xor(d, o, 64);
      if ((lane & 15) == 0) red[gt * NBT + b] = d;
    }
  }
  __syncthreads();
  if (tid < NBT && ss[tid] >= 0) {
    R v = red[tid];
#pragma unroll
    for (int gt = 1; gt < GT; ++gt) v += red[gt * NBT + tid];
    dpart[(size_t)ss[tid] * nparts + gc] = v;
  }
}

// alpha = rz / <p, Ap> from the update's partials (every block of a slot
// forms the same sum in the same order; block 0 records alpha and, on a
// breakdown, takes the slot out of the active set), then
// x += alpha p ; r -= alpha Ap ; z = M^-1 r (into w) ; partials |r|^2, <r, z>.
// A breakdown (<p, Ap> not positive or not finite: the operator is positive
// definite on range Q, so this only comes from round-off once the residual
// is at the precision floor) leaves x and r as they are (alpha = 0).
template <typename R>
__global__ __launch_bounds__(NT) void cg_step2_kernel(
    Slots s, const int* __restrict__ nb, const double* __restrict__ kin, int nb_max, int nup,
    const R* __restrict__ dpart, const R* __restrict__ rzs, R* __restrict__ alpha,
    int* __restrict__ active, const R* __restrict__ pshift, cplx<R>* __restrict__ x,
    cplx<R>* __restrict__ r, const cplx<R>* __restrict__ p, cplx<R>* __restrict__ w,
    R* __restrict__ rpart, R* __restrict__ zpart) {
  __shared__ R red[2 * NW];
  __shared__ R a_sh;
  if (!row_live(s, blockIdx.y)) return;
  const int slot = slot_of(s, blockIdx.y);
  const int k = s.k[slot];
  const int g = blockIdx.x * NT + threadIdx.x;
  // the vector operands do not depend on alpha: they are requested before
  // its sum (rows are nb_max long; only g < nb[k] is used)
  const size_t o = (size_t)slot * nb_max + g;
  cplx<R> xv = mk<R>(0, 0), rv = xv, pv = xv, wv = xv;
  R kv = 0;
  if (g < nb_max) {
    xv = x[o];
    rv = r[o];
    pv = p[o];
    wv = w[o];
    kv = R(kin[(size_t)k * nb_max + g]);
  }
  const R ps = pshift[slot];
  if (threadIdx.x < 64) {
    R v = 0;
    for (int i = threadIdx.x; i < nup; i += 64) v += dpart[(size_t)slot * nup + i];
    v = wsum(v);
    if (threadIdx.x == 0) {
      const R a = rzs[slot] / v;
      // alpha of a positive definite, kinetic-preconditioned operator stays
      // far below 1e12; a larger value only comes from round-off in <p, Ap>
      const bool ok = v > R(0) && a == a && a < R(1e12);
      a_sh = ok ? a : R(0);
      if (blockIdx.x == 0) {
        alpha[slot] = a_sh;
        if (!ok) active[slot] = 0;
      }
    }
  }
  __syncthreads();
  R rr = 0, rz = 0;
  if (g < nb[k]) {
    const R a = a_sh;
    if (a != R(0)) {
      xv = mk<R>(xv.x + a * pv.x, xv.y + a * pv.y);
      rv = mk<R>(rv.x - a * wv.x, rv.y - a * wv.y);
      x[o] = xv;
      r[o] = rv;
    }
    const R m = R(1) / (kv + ps);
    w[o] = cscale<R>(rv, m);
    rr = rv.x * rv.x + rv.y * rv.y;
    rz = m * rr;
  }
  block_sum2(rr, rz, red);
  if (threadIdx.x == 0) {
    rpart[(size_t)slot * gridDim.x + blockIdx.x] = rr;
    zpart[(size_t)slot * gridDim.x + blockIdx.x] = rz;
  }
}

// x = p = 0 over the whole row of every listed slot (x may be null).
template <typename R>
__global__ __launch_bounds__(NT) void cg_zero_kernel(Slots s, int nb_max, cplx<R>* x,
                                                     cplx<R>* __restrict__ p) {
  if (!row_live(s, blockIdx.y)) return;
  const int slot = slot_of(s, blockIdx.y);
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= nb_max) return;
  const size_t o = (size_t)slot * nb_max + g;
  if (x) x[o] = mk<R>(0, 0);
  p[o] = mk<R>(0, 0);
}

// y += a x over the sphere of every listed slot.
template <typename R>
__global__ __launch_bounds__(NT) void cg_axpy_kernel(Slots s, const int* __restrict__ nb,
                                                     int nb_max, R a,
                                                     const cplx<R>* __restrict__ x,
                                                     cplx<R>* __restrict__ y) {
  if (!row_live(s, blockIdx.y)) return;
  const int slot = slot_of(s, blockIdx.y);
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= nb[s.k[slot]]) return;
  const size_t o = (size_t)slot * nb_max + g;
  const cplx<R> xv = x[o], yv = y[o];
  y[o] = mk<R>(yv.x + a * xv.x, yv.y + a * xv.y);
}

// Lists the active slots (k order) and their tiles of up to BT per k, with
// the whole block: the slots are taken CT at a time in order, a wave ballot
// and the wave totals place each active slot in the list, LDS atomics count
// the slots per k, and thread 0 lays out the tiles per k from those counts.
// sh holds 5 nk + CT / 64 + 2 ints.
__device__ void compact_block(const CgCompact& cp, const int* active, int* sh) {
  constexpr int NWC = CT / 64;
  const int nk = cp.nk, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int* na = sh;               // [nk] active slots per k
  int* lb = sh + nk;          // [nk] first list position of k
  int* tb = sh + 2 * nk;      // [nk + 1] first tile of k
  int* s0 = sh + 3 * nk + 1;  // [nk] slot0_k
  int* ns = sh + 4 * nk + 1;  // [nk] nslot_k
  int* wt = sh + 5 * nk + 1;  // [NWC] wave totals, [NWC] list entries so far
  for (int k = tid; k < nk; k += CT) {
    na[k] = 0;
    s0[k] = cp.slot0_k[k];
    ns[k] = cp.nslot_k[k];
  }
  if (tid == 0) wt[NWC] = 0;
  for (int j0 = 0; j0 < cp.J; j0 += CT) {
    const int j = j0 + tid;
    const bool in = j < cp.J;
    const int k = in ? cp.slot_k[j] : 0;
    const int a = in ? active[j] : 0;
    __syncthreads();   // s0, ns, the counts and wt[NWC] are set
    const bool f = a != 0 && j - s0[k] < ns[k];
    const unsigned long long m = __ballot(f);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wt[wave] = __popcll(m);
    if (f) atomicAdd(&na[k], 1);
    __syncthreads();
    int base = wt[NWC];
    for (int w = 0; w < wave; ++w) base += wt[w];
    if (f) cp.list[base + below] = j;
    __syncthreads();   // every wave has read wt
    if (tid == 0) {
      int t = wt[NWC];
      for (int w = 0; w < NWC; ++w) t += wt[w];
      wt[NWC] = t;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int a = 0, t = 0, tmax = 0;
    for (int k = 0; k < nk; ++k) {
      lb[k] = a;
      tb[k] = t;
      a += na[k];
      const int tk = (na[k] + BT - 1) / BT;
      t += tk;
      tmax = max(tmax, tk);
    }
    tb[nk] = t;
    if (cp.ktb) cp.ktb[nk] = t;
    cp.cnt[0] = a;
    cp.cnt[1] = t;
    cp.cnt[2] = tmax;
    if (cp.hist) {
      const int it = cp.step[0];
      cp.step[0] = it + 1;
      if (it < cp.hist_len) {
        cp.hist[2 * it] = a;
        cp.hist[2 * it + 1] = t;
      }
      if (cp.hcnt) {
        cp.hcnt[CNT_STRIDE * (it & 1)] = a;
        cp.hcnt[CNT_STRIDE * (it & 1) + 1] = t;
        cp.hcnt[CNT_STRIDE * (it & 1) + 2] = tmax;
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < nk; k += CT) {
    if (cp.ktb) cp.ktb[k] = tb[k];
    for (int t = tb[k]; t < tb[k + 1]; ++t) {
      const int o = (t - tb[k]) * BT;
      cp.ctk[t] = k;
      cp.cto[t] = lb[k] + o;
      cp.ctn[t] = min(BT, na[k] - o);
    }
  }
}

// Per-slot end of an iteration (lane 0 of the slot's wavefront).
template <typename R>
__device__ __forceinline__ void finish_slot(int slot, R rr, R rz, const CgScalars<R>& cs,
                                            int* active, int start) {
  if (start) {
    cs.rz[slot] = rz;
    cs.beta[slot] = 0;
    if (cs.stag) {
      cs.rbest[slot] = rr;
      cs.rlast[slot] = 0;
    }
    return;
  }
  const int it = ++cs.iters[slot];
  cs.rnorm2[slot] = rr;
  const bool conv = it >= cs.min_iter && (double)rr <= cs.tol2[slot];
  if (!active[slot] || !(rr == rr && rr - rr == R(0))) {   // breakdown this iteration
    active[slot] = 0;
    if (!conv) atomicAdd(cs.noconv, 1);
    return;
  }
  if (conv || it >= cs.max_iter) {
    active[slot] = 0;
    if (!conv) atomicAdd(cs.noconv, 1);
    return;
  }
  if (cs.stag) {   // stagnation at the precision's floor: stop, unconverged
    if (rr < R(STAG_DROP) * cs.rbest[slot]) {
      cs.rbest[slot] = rr;
      cs.rlast[slot] = it;
    } else if (it - cs.rlast[slot] >= cs.stag) {
      active[slot] = 0;
      atomicAdd(cs.noconv, 1);
      return;
    }
  }
  const R beta = cs.rz[slot] != R(0) ? rz / cs.rz[slot] : R(0);
  if (!(beta == beta && beta - beta == R(0))) {   // overflow: a breakdown
    active[slot] = 0;
    atomicAdd(cs.noconv, 1);
    return;
  }
  cs.beta[slot] = beta;
  cs.rz[slot] = rz;
}

// One wavefront per listed slot.
template <typename R>
__global__ __launch_bounds__(NT) void cg_finish_kernel(Slots s, int nparts,
                                                       const R* __restrict__ rpart,
                                                       const R* __restrict__ zpart,
                                                       CgScalars<R> cs, int* __restrict__ active,
                                                       int start) {
  const int row = blockIdx.x * NW + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= s.n || !row_live(s, row)) return;
  const int slot = slot_of(s, row);
  R rr = 0, rz = 0;
  for (int i = lane; i < nparts; i += 64) {
    rr += rpart[(size_t)slot * nparts + i];
    rz += zpart[(size_t)slot * nparts + i];
  }
  rr = wsum(rr);
  rz = wsum(rz);
  if (lane == 0) finish_slot<R>(slot, rr, rz, cs, active, start);
}

// The compaction alone (one block).
__global__ __launch_bounds__(CT) void cg_compact_kernel(CgCompact cp, const int* active) {
  extern __shared__ int cgk_smem[];
  compact_block(cp, active, cgk_smem);
}

// The end of an iteration in one block, for batches with few partials: the
// per-slot sums (FG lanes per listed slot, partials i = sub, sub + FG, ...
// in order, then the FG lanes pairwise) and finish_slot, then the compaction over the
// updated flags.  The flags are written and read by this block alone.
template <typename R>
__global__ __launch_bounds__(CT) void cg_end_kernel(Slots s, int nparts, const R* __restrict__ rpart,
                                                    const R* __restrict__ zpart, CgScalars<R> cs,
                                                    int* active, CgCompact cp) {
  extern __shared__ int cge_smem[];
  constexpr int FG = 8, RPP = CT / FG;
  const int tid = threadIdx.x, sub = tid % FG;
  const int nrow = s.dn ? min(s.n, *s.dn) : s.n;
  for (int r0 = 0; r0 < nrow; r0 += RPP) {
    const int row = r0 + tid / FG;
    const int slot = row < nrow ? slot_of(s, row) : 0;
    R rr = 0, rz = 0;
    if (row < nrow) {
      const R* rp = rpart + (size_t)slot * nparts;
      const R* zp = zpart + (size_t)slot * nparts;
      // UL partials of each kind per lane are loaded before they are added
      constexpr int UL = 16;
      for (int i0 = sub; i0 < nparts; i0 += FG * UL) {
        R a[UL], c[UL];
#pragma unroll
        for (int u = 0; u < UL; ++u) {
          const int i = i0 + u * FG;
          a[u] = i < nparts ? rp[i] : R(0);
          c[u] = i < nparts ? zp[i] : R(0);
        }
#pragma unroll
        for (int u = 0; u < UL; ++u) {
          rr += a[u];
          rz += c[u];
        }
      }
    }
#pragma unroll
    for (int o = FG / 2; o > 0; o >>= 1) {
      rr += __shfl_xor(rr, o, 64);
      rz += __shfl_xor(rz, o, 64);
    }
    if (row < nrow && sub == 0) finish_slot<R>(slot, rr, rz, cs, active, 0);
  }
  __syncthreads();
  compact_block(cp, active, cge_smem);
}

}  // namespace

static int cg_vec_blocks(int nb_max) { return (nb_max + NT - 1) / NT; }

template <typename R>
void cg_start(const Slots& sl, const int* nb, const double* kin, int nb_max, const R* pshift,
              const cplx<R>* r, cplx<R>* z, R* rpart, R* zpart, hipStream_t st) {
  if (sl.n <= 0) return;
  hipLaunchKernelGGL((cg_start_kernel<R>), dim3(cg_vec_blocks(nb_max), sl.n), dim3(NT), 0, st,
                     sl, nb, kin, nb_max, pshift, r, z, rpart, zpart);
  IKR_HIP(hipGetLastError());
}

template <typename R>
void cg_combine(const Slots& sl, int Na, const int* Mq, int Mq_max, const cplx<R>* craw,
                int cstride, const R* shift, const cplx<R>* GT, const cplx<R>* ST, int nbn,
                R dnl, cplx<R>* gam, hipStream_t st) {
  if (sl.n <= 0) return;
  IKR_CHECK(Na + 2 * Mq_max <= cstride && Mq_max <= nbn, 1, "cg_combine: row count");
  const size_t lds = ((size_t)Na + (size_t)(2 + NW) * Mq_max) * sizeof(cplx<R>);
  IKR_CHECK(lds <= 65536, 1, "cg_combine: too many projection rows");
  hipLaunchKernelGGL((cg_combine_kernel<R>), dim3(sl.n), dim3(NT), lds, st, sl, Na, Mq, Mq_max,
                     craw, cstride, shift, GT, ST, nbn, dnl, gam);
  IKR_HIP(hipGetLastError());
}

constexpr int UKW_GB = 64;     // coefficients per block of the k-wide update

// The k-wide update only when forced: on the 60 x 108^2 cell, where the CG
// batch keeps about 13 live bands per k-point on average, it took 12.2 ms per
// FP64 launch against 7.3 ms for the tiled update (its 16-row stages wait on
// their loads; the tiled kernel streams W with four rows in flight).
bool cg_update_kwide(int Mrows, const KTileRange& kr) {
  (void)Mrows;
  return kr.t0 && kr.nk > 0 && kr.ktmax <= 5 && (kernel_paths() & PATH_KWIDE) &&
         !(kernel_paths() & PATH_VECTOR_GRAM);
}

int cg_update_parts(int nb_max, int Mrows, const KTileRange& kr) {
  return cg_update_kwide(Mrows, kr) ? (nb_max + UKW_GB - 1) / UKW_GB : update_nblocks(nb_max);
}

template <typename R>
void cg_update(const Tiles& tl, const int* nb, int nb_max, const cplx<R>* Wcg, size_t wk,
               int Na, const int* Mq, int Mq_max, const cplx<R>* gam, int cstride,
               cplx<R>* Wv, cplx<R>* P, R* dpart, hipStream_t st, const KTileRange& kr,
               const KernelTune* kt) {
  if (tl.n <= 0) return;
  IKR_CHECK(Na + 2 * Mq_max <= cstride, 1, "cg_update: row count");
  if (cg_update_kwide(Na + 2 * Mq_max, kr)) {
    const int nparts = (nb_max + UKW_GB - 1) / UKW_GB;
    hipLaunchKernelGGL((cg_update_kw_kernel<R, 5, UKW_GB>), dim3(round8(nparts * kr.nk)),
                       dim3(UKW_NT), 0, st, tl, kr, nb, nb_max, Wcg, wk, Na, Mq, Mq_max, gam,
                       cstride, Wv, P, dpart, nparts);
    IKR_HIP(hipGetLastError());
    return;
  }
  const int ngb = update_nblocks(nb_max);
  const int blocks = ngb * tl.n;
  // the matrix cores unless the vector paths are forced or a band group is asked for
  const size_t lds_mf = (size_t)16 * (Na + 3 * Mq_max) * sizeof(cplx<R>);
  if (!(kernel_paths() & PATH_VECTOR_GRAM) && !(kt && kt->upd_bpt) && lds_mf <= 65536) {
    hipLaunchKernelGGL((cg_update_mfma_kernel<R, 8>), dim3(round8(ngb * tl.n)), dim3(NT), lds_mf,
                       st, tl, nb, nb_max, Wcg, wk, Na, Mq, Mq_max, gam, cstride, Wv, P, dpart,
                       ngb);
    IKR_HIP(hipGetLastError());
    return;
  }
  // FP64 caps the band group at 8 (16 would leave one wavefront per SIMD)
  int bpt = blocks >= 1024 ? 16 : (2 * blocks >= 1024 ? 8 : 4);
  if (sizeof(R) == 8 && bpt > 8) bpt = 8;
  if (kt && (kt->upd_bpt == 4 || kt->upd_bpt == 8 || kt->upd_bpt == 16) &&
      (size_t)kt->upd_bpt * (Na + 3 * Mq_max) * sizeof(cplx<R>) <= 65536)
    bpt = kt->upd_bpt;
  const size_t lds = (size_t)bpt * (Na + 3 * Mq_max) * sizeof(cplx<R>);
  IKR_CHECK(lds <= 65536, 1, "cg_update: too many projection rows");
  const dim3 grid(round8(ngb * (BT / bpt) * tl.n));
#define IKR_CGU(B)                                                                         \
  hipLaunchKernelGGL((cg_update_kernel<R, B>), grid, dim3(NT), lds, st, tl, nb, nb_max, Wcg, \
                     wk, Na, Mq, Mq_max, gam, cstride, Wv, P, dpart, ngb)
  if (bpt == 16) IKR_CGU(16);
  else if (bpt == 8) IKR_CGU(8);
  else IKR_CGU(4);
#undef IKR_CGU
  IKR_HIP(hipGetLastError());
}

template <typename R>
void cg_step2(const Slots& sl, const int* nb, const double* kin, int nb_max, const R* dpart,
              int nup, const R* rz, R* alpha, int* active, const R* pshift, cplx<R>* x,
              cplx<R>* r, const cplx<R>* p, cplx<R>* w, R* rpart, R* zpart, hipStream_t st) {
  if (sl.n <= 0) return;
  IKR_CHECK(rpart != dpart, 1, "cg_step2: the residual partials must not overwrite <p, Ap>");
  hipLaunchKernelGGL((cg_step2_kernel<R>), dim3(cg_vec_blocks(nb_max), sl.n), dim3(NT), 0, st,
                     sl, nb, kin, nb_max, nup, dpart, rz, alpha, active,
                     pshift, x, r, p, w, rpart, zpart);
  IKR_HIP(hipGetLastError());
}

template <typename R>
void cg_axpy(const Slots& sl, const int* nb, int nb_max, R a, const cplx<R>* x, cplx<R>* y,
             hipStream_t st) {
  if (sl.n <= 0) return;
  hipLaunchKernelGGL((cg_axpy_kernel<R>), dim3(cg_vec_blocks(nb_max), sl.n), dim3(NT), 0, st, sl,
                     nb, nb_max, a, x, y);
  IKR_HIP(hipGetLastError());
}

template <typename R>
void cg_zero(const Slots& sl, int nb_max, cplx<R>* x, cplx<R>* p, hipStream_t st) {
  if (sl.n <= 0) return;
  hipLaunchKernelGGL((cg_zero_kernel<R>), dim3(cg_vec_blocks(nb_max), sl.n), dim3(NT), 0, st, sl,
                     nb_max, x, p);
  IKR_HIP(hipGetLastError());
}

static size_t compact_lds(const CgCompact& cp) {
  return (5 * (size_t)cp.nk + CT / 64 + 2) * sizeof(int);
}

template <typename R>
void cg_finish(const Slots& sl, int nparts, const R* rpart, const R* zpart,
               const CgScalars<R>& cs, int* active, int start, hipStream_t st) {
  if (sl.n <= 0) return;
  hipLaunchKernelGGL((cg_finish_kernel<R>), dim3((sl.n + NW - 1) / NW), dim3(NT), 0, st, sl,
                     nparts, rpart, zpart, cs, active, start);
  IKR_HIP(hipGetLastError());
}

void cg_compact(const CgCompact& cp, const int* active, hipStream_t st) {
  IKR_CHECK(cp.list && cp.cnt && cp.slot_k && cp.nk > 0 && cp.J >= 0, 8,
            "cg_compact: incomplete arguments");
  const size_t lds = compact_lds(cp);
  IKR_CHECK(lds <= 65536, 1, "cg_compact: too many k-points");
  hipLaunchKernelGGL(cg_compact_kernel, dim3(1), dim3(CT), lds, st, cp, active);
  IKR_HIP(hipGetLastError());
}

// Partials per thread up to which the end of an iteration runs as one block.
constexpr size_t CG_END_FUSED_MAX = 16 * (size_t)CT;

template <typename R>
void cg_end(const Slots& sl, int nparts, const R* rpart, const R* zpart, const CgScalars<R>& cs,
            int* active, const CgCompact& cp, hipStream_t st) {
  if ((size_t)std::max(sl.n, 0) * nparts > CG_END_FUSED_MAX ||
      (kernel_paths() & PATH_SPLIT_END)) {
    cg_finish<R>(sl, nparts, rpart, zpart, cs, active, 0, st);
    cg_compact(cp, active, st);
    return;
  }
  IKR_CHECK(cp.list && cp.cnt && cp.slot_k && cp.nk > 0 && cp.J >= 0, 8,
            "cg_end: incomplete arguments");
  const size_t lds = compact_lds(cp);
  IKR_CHECK(lds <= 65536, 1, "cg_end: too many k-points");
  hipLaunchKernelGGL((cg_end_kernel<R>), dim3(1), dim3(CT), lds, st, sl, nparts, rpart, zpart,
                     cs, active, cp);
  IKR_HIP(hipGetLastError());
}

#define IKR_INST(R)                                                                            \
  template void cg_start<R>(const Slots&, const int*, const double*, int, const R*,            \
                            const cplx<R>*, cplx<R>*, R*, R*, hipStream_t);                    \
  template void cg_combine<R>(const Slots&, int, const int*, int, const cplx<R>*, int,         \
                              const R*, const cplx<R>*, const cplx<R>*, int, R, cplx<R>*,      \
                              hipStream_t);                                                    \
  template void cg_update<R>(const Tiles&, const int*, int, const cplx<R>*, size_t, int,       \
                             const int*, int, const cplx<R>*, int, cplx<R>*, cplx<R>*, R*,     \
                             hipStream_t, const KTileRange&, const KernelTune*);               \
  template void cg_step2<R>(const Slots&, const int*, const double*, int, const R*, int,       \
                            const R*, R*, int*, const R*, cplx<R>*, cplx<R>*, const cplx<R>*,  \
                            cplx<R>*, R*, R*, hipStream_t);                                    \
  template void cg_zero<R>(const Slots&, int, cplx<R>*, cplx<R>*, hipStream_t);               \
  template void cg_axpy<R>(const Slots&, const int*, int, R, const cplx<R>*, cplx<R>*,         \
                           hipStream_t);                                                       \
  template void cg_finish<R>(const Slots&, int, const R*, const R*, const CgScalars<R>&, int*,  \
                             int, hipStream_t);                                                \
  template void cg_end<R>(const Slots&, int, const R*, const R*, const CgScalars<R>&, int*,     \
                          const CgCompact&, hipStream_t);
IKR_INST(double)
IKR_INST(float)
#undef IKR_INST

}  // namespace ikr
