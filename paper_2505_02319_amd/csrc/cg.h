// Declarations of the fused Sternheimer CG kernels (cg.hip).
//
// One CG iteration on the projected operator Q (H - e_n) Q (paper: the
// discretised Sternheimer equation, with the iterates kept in range Q as in
// the remark on re-projection) needs one pass over p~ = z + beta p for all
// projections: with W_k = [projectors | phi_1, H phi_1, phi_2, H phi_2, ...]
// the gram coefficients q = P^H p~, a = Phi^H p~, h = (H Phi)^H p~ give
//   p   = p~ - Phi a                                   (p in range Q)
//   c   = Phi^H (H - e) p = h - e a - (G - e S) a,     G = Phi^H H Phi, S = Phi^H Phi
//   A p = (H_loc - e) p~ + P D q - (H Phi) a + Phi (e a - c),
// all from that one gram and one update.  With the preconditioned residual
// z = M^-1 r and r in range Q, <r, Q z> = <r, z>, so no projection of z is
// needed: the next p~ is projected by the next iteration's update.
#pragma once

#include "blas.h"
#include "common.h"

namespace ikr {

// z = M^-1 r over the listed slots; partials |r|^2 -> rpart, <r, z> -> zpart
// ([slot * nparts + block], nparts = vec_nblocks(nb_max)).
template <typename R>
void cg_start(const Slots& sl, const int* nb, const double* kin, int nb_max,
              const R* pshift, const cplx<R>* r, cplx<R>* z, R* rpart, R* zpart,
              hipStream_t st);

// Per-slot update coefficients from the gram of p~ against W_k (rows: Na
// projectors, then phi_m / H phi_m interleaved for m < Mq[k]):
//   gam[r < Na]       = dnl q_r
//   gam[Na + 2m]      = e a_m - c_m
//   gam[Na + 2m + 1]  = -a_m
// GT[k][j][m] = <phi_m, H phi_j>, ST[k][j][m] = <phi_m, phi_j> (row stride nbn).
template <typename R>
void cg_combine(const Slots& sl, int Na, const int* Mq, int Mq_max, const cplx<R>* craw,
                int cstride, const R* shift, const cplx<R>* GT, const cplx<R>* ST, int nbn,
                R dnl, cplx<R>* gam, hipStream_t st);

// Ap = w~ + sum_r W[r] gam[r] (in place in Wv), p = p~ - sum_m phi_m a_m (in
// place in P), partial <p, Ap> -> dpart[slot * nparts + gb] with nparts =
// cg_update_parts(...).  By default one 16-band tile per block on the matrix
// cores; the vector-FMA kernel when the vector paths are forced or kt asks
// for a band group; with kr given and the k-wide path forced, all bands of a
// k-point per block on the matrix cores.
template <typename R>
void cg_update(const Tiles& tl, const int* nb, int nb_max, const cplx<R>* Wcg, size_t wk,
               int Na, const int* Mq, int Mq_max, const cplx<R>* gam, int cstride,
               cplx<R>* Wv, cplx<R>* P, R* dpart, hipStream_t st,
               const KTileRange& kr = KTileRange{}, const KernelTune* kt = nullptr);
bool cg_update_kwide(int Mrows, const KTileRange& kr);
int cg_update_parts(int nb_max, int Mrows, const KTileRange& kr);

// alpha = rz / <p, Ap> per listed slot (from the nup partials per slot in
// dpart); on a breakdown (<p, Ap>
// <= 0 or a non-finite alpha) alpha = 0 and the slot leaves the active set.
// Then x += alpha p ; r -= alpha Ap ; z = M^-1 r (into w) ; partials |r|^2
// and <r, z> (rpart must not alias dpart).
template <typename R>
void cg_step2(const Slots& sl, const int* nb, const double* kin, int nb_max, const R* dpart,
              int nup, const R* rz, R* alpha, int* active, const R* pshift, cplx<R>* x,
              cplx<R>* r, const cplx<R>* p, cplx<R>* w, R* rpart, R* zpart, hipStream_t st);

// x = p = 0 on the whole rows of the listed slots (the CG's start; x may be
// null: p only).
template <typename R>
void cg_zero(const Slots& sl, int nb_max, cplx<R>* x, cplx<R>* p, hipStream_t st);

// y += a x over the spheres of the listed slots.
template <typename R>
void cg_axpy(const Slots& sl, const int* nb, int nb_max, R a, const cplx<R>* x, cplx<R>* y,
             hipStream_t st);

// Active-set compaction: list[] of active slots (k order), tiles of up to BT
// of them per k (ctk, cto = offset into list, ctn), cnt[0] = active slots,
// cnt[1] = tiles; with hist set, hist[2 * it ..] the same, it = step[0]
// (a device counter, then incremented; entries past hist_len pairs are
// dropped).
constexpr int CNT = 3;          // counts the compaction writes
constexpr int CNT_STRIDE = 4;   // their stride in the host-mapped double buffer

struct CgCompact {
  int nk;
  const int* slot0_k;
  const int* nslot_k;
  const int* slot_k;   // k of each slot; the slots of k are slot0_k[k] + i, i < nslot_k[k]
  int J;               // slots
  int* list;
  int* ctk;
  int* cto;
  int* ctn;
  int* cnt;            // [CNT]: live slots, live tiles, most live tiles of one k-point
  int* hist;
  int hist_len;
  int* step;
  int* hcnt = nullptr;   // host-mapped [2][CNT_STRIDE]: with hist, step s also writes the
                         // counts to hcnt[CNT_STRIDE (s & 1)], for the host loop to read
                         // without a copy
  int* ktb = nullptr;    // [nk + 1]: first compact tile of each k (nullable)
};

// start: rz = <r, z>, beta = 0.  Otherwise: iteration count, |r|^2,
// convergence (|r|^2 <= tol2 after at least min_iter iterations, or the
// cap), and for slots still active beta = <r, z> / rz, rz = <r, z>.
template <typename R>
void cg_finish(const Slots& sl, int nparts, const R* rpart, const R* zpart,
               const CgScalars<R>& cs, int* active, int start, hipStream_t st);

// The compaction (one block).
void cg_compact(const CgCompact& cp, const int* active, hipStream_t st);

// cg_finish (start = 0) followed by cg_compact; one block does both when
// the batch has few partials.
template <typename R>
void cg_end(const Slots& sl, int nparts, const R* rpart, const R* zpart, const CgScalars<R>& cs,
            int* active, const CgCompact& cp, hipStream_t st);

}  // namespace ikr
