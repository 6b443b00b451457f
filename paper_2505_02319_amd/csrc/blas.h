// Declarations of the batched vector kernels (blas.hip).
#pragma once

#include "common.h"

namespace ikr {

constexpr int BT = 16;     // slots per tile (bands of one k-point)
constexpr int MAXM = 96;   // max projector rows in one update pass

// Tiles of up to BT slots sharing a k-point.  Slot b of tile t is
// slot0[t] + b, or idx[slot0[t] + b] when a compact index list is given.
struct Tiles {
  int n;
  const int* k;
  const int* slot0;
  const int* nb;           // slots in the tile (<= BT)
  const int* idx = nullptr;
  const int* dn = nullptr; // device count of live tiles (n is then an upper bound)
};

__device__ __forceinline__ int tslot(const Tiles& tl, int t, int b) {
  return tl.idx ? tl.idx[tl.slot0[t] + b] : tl.slot0[t] + b;
}

// One term  alpha * sum_m W[k][m][g] * C[slot][m]  of an update.
template <typename R> struct UpdTerm {
  const cplx<R>* W = nullptr;
  size_t wk = 0;           // k stride of W (elements)
  int ws = 0;              // row stride of W
  const int* Mk = nullptr; // rows per k
  const cplx<R>* C = nullptr;
  int cs = 0;              // slot stride of C
  R alpha = 0;
  int Mmax = MAXM;         // bound on Mk over all k (sizes the coefficient LDS)
};

template <typename R> struct CgScalars {
  R* rz;
  R* alpha;
  R* beta;
  R* rnorm2;
  const double* tol2;      // squared absolute tolerance per slot
  int* iters;
  int* nactive;            // device counter of still-active slots
  int* noconv;             // device counter of slots that hit the cap
  int min_iter, max_iter;
  // stagnation stop (0: off): a slot whose |r|^2 has not fallen below
  // STAG_DROP times its best value for `stag` iterations stops unconverged
  int stag = 0;
  R* rbest = nullptr;      // best |r|^2 per slot
  int* rlast = nullptr;    // iteration of the last such fall per slot
};
constexpr double STAG_DROP = 0.5;

// Internal <-> external grid layout.
struct Layout {
  int C, P, Q;
  int st_c, st_p, st_q;    // external strides of the internal axes
};

// Process-wide choice of kernel paths, for tests and tuning.  0: by size
// (the default); each bit forces one path at any size.
enum KernelPath : int {
  PATH_VECTOR_GRAM = 1,   // projections (gram and CG update) by the vector-FMA kernels
  PATH_SPLIT_END = 2,     // CG iteration end as two launches (finish, compaction)
  PATH_KWIDE = 4,         // k-wide matrix-core gram at any row count
  PATH_FIXED = 8,         // no setup-time tuning: launch shapes by the size rules alone
};

// Launch shapes chosen by the setup-time tuner (0 / 1: the size rules).
struct KernelTune {
  int gram = 0;            // 0 by size; 1 per-tile matrix-core; 2 k-wide matrix-core; 3 vector
  float gram_scale = 1;    // multiplier of the gram's block-count target (0.5 .. 2)
  int upd_bpt = 0;         // 0 by size (the matrix-core update); else the vector update with
                           // this many bands per block (4, 8, 16)
  int plane_pt = 0;        // 0 by size; else threads per block of the plane kernel (256, 512)
};

// Tiles grouped by k-point: the tiles of k are t0[k] .. t0[k + 1] - 1 of the
// tile list (device array of nk + 1 entries, consecutive per k); ktmax bounds
// the tiles of any one k.  Lets the gram take all bands of a k-point at once.
struct KTileRange {
  int nk = 0;
  const int* t0 = nullptr;
  int ktmax = 0;
};

void set_kernel_paths(int mask);
int kernel_paths();

// Elements of the gram's partial-sum buffer for up to ntiles tiles of Mmax
// rows (nk: k-points of the tile list, when the k-wide gram may be used;
// max_scale: the largest KernelTune::gram_scale the calls may take).
size_t gram_part_elems(int ntiles, int nb_max, int Mmax, int nk = 0, double max_scale = 1.0);
int update_nblocks(int nb_max);
int vec_nblocks(int nb_max);
int multidot_nblocks(int n);

// coef[slot * cstride + m] = <W[k][m], X[slot]> for the slots of the tiles;
// with kr given (and few enough tiles per k), above 64 rows the k-wide gram.
template <typename R>
void gram(const Tiles& tl, const int* nb, int nb_max, const int* Mk, int Mmax,
          const cplx<R>* W, size_t wk_stride, int w_stride, const cplx<R>* X,
          int x_stride, cplx<R>* part, cplx<R>* coef, int cstride, hipStream_t st,
          const int* active = nullptr, const KTileRange& kr = KTileRange{});

// The first stage of gram alone: partial sums over the super-chunks,
// part[((t * nsc + sc) * Mmax + m) * BT + b] for rows m < Mk[k]; returns nsc.
template <typename R>
int gram_partials(const Tiles& tl, const int* nb, int nb_max, const int* Mk, int Mmax,
                  const cplx<R>* W, size_t wk_stride, int w_stride, const cplx<R>* X,
                  int x_stride, cplx<R>* part, hipStream_t st, const int* active = nullptr,
                  const KTileRange& kr = KTileRange{}, const KernelTune* kt = nullptr);
// Which gram a call with these arguments takes (1 per-tile matrix-core, 2 k-wide, 3 vector).
int gram_variant(int Mmax, const KTileRange& kr, const KernelTune* kt);

// The second stage: coef[slot * cstride + m] = sum over the nsc super-chunks.
template <typename R>
void gram_reduce(const Tiles& tl, const int* Mk, int Mmax, int nsc, const cplx<R>* part,
                 cplx<R>* coef, int cstride, hipStream_t st, const int* active = nullptr);

template <typename R>
void update(const Tiles& tl, const int* nb, int nb_max, const int* active,
            cplx<R>* Y, int y_stride, R a, const UpdTerm<R>& t1,
            const UpdTerm<R>& t2, const cplx<R>* D, R* dpart, hipStream_t st);

void sum_groups(int n, int ngroups, const double* part, double scale, double* out,
                hipStream_t st);
// precision changes: listed slots over their spheres, or whole arrays
void convert_slots(int n, const int* list, const int* slot_k, const int* nb, int nb_max,
                   const double2* in, float2* out, hipStream_t st);
void convert_slots(int n, const int* list, const int* slot_k, const int* nb, int nb_max,
                   const float2* in, double2* out, hipStream_t st);
void convert_array(size_t n, const double* in, float* out, hipStream_t st);
void convert_array(size_t n, const double2* in, float2* out, hipStream_t st);
void resid_norms(int nslots, int nb_max, const int* slot_k, const int* nb, const double2* HX,
                 const double2* X, const double* lam, double* part, hipStream_t st);
// out[slot * nv + l] = <V[l][slot], x[slot]> (complex, over each slot's sphere) for all
// nslots slots, through partials part (slot_dots_part_elems entries).
void slot_dots(int nslots, int nb_max, const int* slot_k, const int* nb, int nv,
               const double2* V, size_t vstride, const double2* x, double2* part,
               double2* out, hipStream_t st);
size_t slot_dots_part_elems(int nslots, int nb_max, int nv);
// y[slot] = sum_l c[slot * nv + l] V[l][slot] for the nlist listed slots.
void slot_combine(int nlist, const int* list, int nb_max, const int* slot_k, const int* nb,
                  int nv, const double2* V, size_t vstride, const double2* c, double2* y,
                  hipStream_t st);
void to_internal(const Layout& L, const double* ext, double* in, hipStream_t st);
void to_external(const Layout& L, const double* in, double* ext, double a,
                 const double* base, double bscale, hipStream_t st);
void multidot(int n, int nv, const double* V, size_t vstride, const double* w,
              double* partial, hipStream_t st);
void multiaxpy(int n, int nv, const double* V, size_t vstride, const double* c, double a,
               double* y, hipStream_t st);
void scale_copy(size_t n, const double* x, double a, double* y, hipStream_t st);
// full[i] = sum_n |G[n][i]|^2, re[i] = sum_n (Re(phase[n] G[n][i]))^2 for n < nv
// (grid rows; phase[n] = (cos, sin), null for none)
void grid_row_norms(size_t ng, int nv, const double2* G, const double2* phase, double* full,
                    double* re, hipStream_t st);
// part[n * grid_square_nblocks(ng) + b]: block partial sums of G[n][i]^2 (complex)
int grid_square_nblocks(size_t ng);
void grid_square_sums(size_t ng, int nv, const double2* G, double2* part, hipStream_t st);
template <typename R>
void cscale_vec(size_t n, cplx<R>* x, R a, hipStream_t st);

}  // namespace ikr
