// Response solver: chi0 through batched Sternheimer CG (paper eq. kchi0,
// eq. delta_phi_P, eq. sternheimer_equation, eq. delta_f), the dielectric
// adjoint E v = v - ||Kv|| chi0(Kv/||Kv||) (eq. op_discretised), the CG
// tolerance strategies of Table 1 / Table strategies_k, and inexact
// GMRES(m) with the adaptive estimate s (Algorithm 1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "cg.h"
#include "hostmath.h"
#include "ktimer.h"
#include "system.h"

namespace ikr {

namespace {

constexpr double DEGEN_TOL = 1e-8;
constexpr double TOL_FLOOR = 1e-13;   // CG tolerances never below this times ||b_j||
constexpr double CHECK_REL = 1e-3;    // FP32 results with tau_j below this times ||b_j||
                                      // get an FP64 true-residual check
constexpr double WARM_REL = 0.1;      // warm start when it leaves under this of ||b_j||
constexpr int FP32_STAG_ITERS = 30;   // an FP32 band whose |r|^2 has not halved in this many
                                      // iterations stops (and is solved again in FP64)

using host::sigma_min;
using host::small_ls;

template <typename T> std::vector<T> download(const T* d, size_t n, hipStream_t st) {
  std::vector<T> h(n);
  if (n) IKR_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st));
  IKR_HIP(hipStreamSynchronize(st));
  return h;
}

}  // namespace

// ---------------------------------------------------------------- H psi
size_t HamWork::bytes(const System& s, int nvec) {
  const int ntiles = (nvec + BT - 1) / BT;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t tcol = (size_t)nvec * s.L.C * s.ncol_max * sizeof(double2);
  return al(nvec * sizeof(int)) + 3 * al(ntiles * sizeof(int)) + 2 * al(tcol) +
         al((size_t)nvec * MAXM * sizeof(double2)) +
         al(gram_part_elems(ntiles, s.nb_max, std::max(s.natoms, 1)) * sizeof(double2));
}

void HamWork::carve(const System& s, int nvec, unsigned char* base) {
  const int ntiles = (nvec + BT - 1) / BT;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t tcol = (size_t)nvec * s.L.C * s.ncol_max * sizeof(double2);
  unsigned char* p = base;
  sk = reinterpret_cast<int*>(p); p += al(nvec * sizeof(int));
  tk = reinterpret_cast<int*>(p); p += al(ntiles * sizeof(int));
  ts = reinterpret_cast<int*>(p); p += al(ntiles * sizeof(int));
  tn = reinterpret_cast<int*>(p); p += al(ntiles * sizeof(int));
  T1 = reinterpret_cast<double2*>(p); p += al(tcol);
  T2 = reinterpret_cast<double2*>(p); p += al(tcol);
  coef = reinterpret_cast<double2*>(p); p += al((size_t)nvec * MAXM * sizeof(double2));
  part = reinterpret_cast<double2*>(p);
}

// y = H_k x with the work space in w (tables filled by the caller or here).
void apply_hamiltonian_ws(System& s, int k, int nvec, const double2* x, double2* y,
                          const HamWork& w) {
  const hipStream_t st = s.stream;
  const int ntiles = (nvec + BT - 1) / BT;
  Tiles tl{ntiles, w.tk, w.ts, w.tn};
  Slots sl{nvec, w.sk, nullptr};
  launch_col_inv<double>(s.geom, s.fft, sl, x, s.nb_max, w.T1, nullptr, nullptr, nullptr, st);
  launch_plane_hv<double>(s.geom, s.fft, sl, w.T1, w.T2, s.d_vloc.get(), 0, st);
  launch_col_fwd<double>(s.geom, s.fft, sl, w.T2, y, s.nb_max, x, nullptr, 1.0 / s.ng, st);
  if (s.natoms > 0) {
    gram<double>(tl, s.d_nb.get(), s.nb_max, s.d_natoms_k.get(), s.natoms, s.d_proj.get(),
                 (size_t)s.natoms * s.nb_max, s.nb_max, x, s.nb_max, w.part, w.coef, MAXM, st);
    UpdTerm<double> t1{s.d_proj.get(), (size_t)s.natoms * s.nb_max, s.nb_max,
                       s.d_natoms_k.get(), w.coef, MAXM, s.dnl, s.natoms};
    update<double>(tl, s.d_nb.get(), s.nb_max, nullptr, y, s.nb_max, 1.0, t1, UpdTerm<double>{},
                   nullptr, nullptr, st);
  }
}

void apply_hamiltonian(System& s, int k, int nvec, const double2* x, double2* y) {
  const hipStream_t st = s.stream;
  DBuf<unsigned char> ws;
  ws.alloc(HamWork::bytes(s, nvec));
  HamWork w;
  w.carve(s, nvec, ws.get());
  std::vector<int> sk(nvec, k), tk, ts, tn;
  for (int v0 = 0; v0 < nvec; v0 += BT) {
    tk.push_back(k);
    ts.push_back(v0);
    tn.push_back(std::min(BT, nvec - v0));
  }
  IKR_HIP(hipMemcpyAsync(w.sk, sk.data(), sk.size() * sizeof(int), hipMemcpyHostToDevice, st));
  IKR_HIP(hipMemcpyAsync(w.tk, tk.data(), tk.size() * sizeof(int), hipMemcpyHostToDevice, st));
  IKR_HIP(hipMemcpyAsync(w.ts, ts.data(), ts.size() * sizeof(int), hipMemcpyHostToDevice, st));
  IKR_HIP(hipMemcpyAsync(w.tn, tn.data(), tn.size() * sizeof(int), hipMemcpyHostToDevice, st));
  apply_hamiltonian_ws(s, k, nvec, x, y, w);
  IKR_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- K
double apply_kernel(System& s, const double* v_int, double* kv_int) {
  launch_kernel_apply(s.geom, s.fft, v_int, s.d_khat.get(), s.xc ? s.d_fx.get() : nullptr,
                      kv_int, s.d_kw1.get(), s.d_kw2.get(), s.d_kpart.get(), s.stream);
  const std::vector<double> part = download(s.d_kpart.get(), s.L.C, s.stream);
  double ss = 0;
  for (double v : part) ss += v;
  return std::sqrt(ss);
}

// ---------------------------------------------------------------- CG
namespace {

struct CgOut {
  long long n_ham = 0;
  int noconv = 0;
};

template <typename R> const cplx<R>* phi_of(const System& s);
template <> const double2* phi_of<double>(const System& s) { return s.d_phi.get(); }
template <> const float2* phi_of<float>(const System& s) { return s.w32.phi.get(); }
template <typename R> const cplx<R>* proj_of(const System& s);
template <> const double2* proj_of<double>(const System& s) { return s.d_proj.get(); }
template <> const float2* proj_of<float>(const System& s) { return s.w32.proj.get(); }
template <typename R> const R* vloc_of(const System& s);
template <> const double* vloc_of<double>(const System& s) { return s.d_vloc.get(); }
template <> const float* vloc_of<float>(const System& s) { return s.w32.vloc.get(); }

// ||r_j|| of every slot (host vector)
std::vector<double> slot_norms(System& s, const double2* r) {
  const int J = s.J, nrb = vec_nblocks(s.nb_max);
  DBuf<double> zero, part;
  zero.upload(std::vector<double>(J, 0.0), s.stream);
  part.alloc((size_t)J * nrb);
  resid_norms(J, s.nb_max, s.d_slot_k.get(), s.d_nb.get(), r, r, zero.get(), part.get(),
              s.stream);
  const std::vector<double> p = download(part.get(), (size_t)J * nrb, s.stream);
  std::vector<double> out(J, 0.0);
  for (int j = 0; j < J; ++j) {
    double a = 0;
    for (int b = 0; b < nrb; ++b) a += p[(size_t)j * nrb + b];
    out[j] = std::sqrt(a);
  }
  return out;
}

template <typename R> const cplx<R>* wcg_of(const System& s);
template <> const double2* wcg_of<double>(const System& s) { return s.w64.wcg.get(); }
template <> const float2* wcg_of<float>(const System& s) { return s.w32.wcg.get(); }

// ------------------------------------------------------------ launch tuning
// Three launch shapes of the CG iteration are measured rather than only set
// by size: the projection gram's kernel (per-tile or k-wide matrix-core, or
// vector) and its block count, the tiled update's band group, and the
// threads of the plane kernel.  At the first CG run of a precision, each
// candidate runs once untimed and three times between HIP events on the CG
// stream, each time after the kernels that precede it in a CG iteration (so
// that it meets the caches as in the solve), on the batch the run starts with (when
// it has more tiles than k-points: the "thick" class) and on thin batches of
// at most 8 and 2 bands per k-point, with the run's own batch when that is
// thin too (the "thin" class; its times are added).  The size rule is a
// candidate too and stays unless another is more than 15% faster: the size
// rules also adapt to the shrinking batch, a fixed pick does not, and picks
// with smaller margins did not hold in whole solves.
// All candidates compute the same quantities.  The runs write only scratch:
// gram partials and coefficients, the plane buffer, and the direction rows
// p, Ap of the batch's slots, which the CG run overwrites before reading.
constexpr double TUNE_MARGIN = 0.85;
constexpr int TUNE_REPS = 3;

template <typename R>
static void tune_class(System& s, CgWork<R>& w, const std::vector<std::vector<int>>& sets,
                       int cls, const int* dMq, int Mq_max, const int* dMcg, hipStream_t st) {
  const int pi = sizeof(R) == 8 ? 0 : 1;
  const int J = s.J, nbm = s.nb_max, Na = s.natoms;
  const int Mrows = Na + 2 * Mq_max;
  const size_t wk = (size_t)s.mcg * nbm;
  const R* vloc = vloc_of<R>(s);
  const cplx<R>* wcg = wcg_of<R>(s);
  const KTileRange kr = s.krange_compact();
  int* cnt = s.d_cnt.get();
  struct Batch { Slots sl; Tiles tl; int ktmax; };
  // compacts one set into the device lists (each timing starts with this)
  auto select = [&](const std::vector<int>& set) {
    int na = 0, nt = 0, kt = 0;
    for (int v : set) na += v != 0;
    for (int k = 0; k < s.nk; ++k) {
      int c = 0;
      for (int j = s.slot0_k[k]; j < s.slot0_k[k] + s.nocc_k[k]; ++j) c += set[j] != 0;
      nt += (c + BT - 1) / BT;
      kt = std::max(kt, (c + BT - 1) / BT);
    }
    IKR_HIP(hipMemcpyAsync(s.d_active.get(), set.data(), J * sizeof(int),
                           hipMemcpyHostToDevice, st));
    cg_compact(CgCompact{s.nk, s.d_slot0_k.get(), s.d_nocc_k.get(), s.d_slot_k.get(), J,
                         s.d_list.get(), s.d_ctk.get(), s.d_cto.get(), s.d_ctn.get(), cnt,
                         nullptr, 0, s.d_counters.get() + 2, nullptr, s.d_ktb.get()},
               s.d_active.get(), st);
    IKR_HIP(hipStreamSynchronize(st));   // the host vector may go
    return Batch{Slots{na, s.d_slot_k.get(), s.d_active.get(), s.d_list.get(), cnt},
                 Tiles{nt, s.d_ctk.get(), s.d_cto.get(), s.d_ctn.get(), s.d_list.get(),
                       cnt + 1},
                 kt};
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  IKR_HIP(hipEventCreate(&e0));
  IKR_HIP(hipEventCreate(&e1));
  auto elapsed_us = [&] {
    IKR_HIP(hipEventSynchronize(e1));
    float ms = 0;
    IKR_HIP(hipEventElapsedTime(&ms, e0, e1));
    return 1000.0 * ms;
  };
  // Each timed launch runs where it runs in a CG iteration: after the
  // kernels before it in the iteration (prefix), so that it meets the caches
  // as they are there; back to back, or after a flush, a launch finds its
  // operands cached, or not at all, and the picks do not hold in the solve.
  const R inv_ng = R(1.0 / s.ng);
  auto col_inv = [&](const Batch& bt) {
    launch_col_inv<R>(s.geom, s.fft, bt.sl, w.p.get(), nbm, w.T1.get(), w.w.get(),
                      w.beta.get(), w.p.get(), st);
  };
  auto to_gram = [&](const Batch& bt, const KernelTune& kt) {   // p~ and w~ of an iteration
    col_inv(bt);
    launch_plane_hv<R>(s.geom, s.fft, bt.sl, w.T1.get(), w.T2.get(), vloc, 0, st, kt.plane_pt);
    launch_col_fwd<R>(s.geom, s.fft, bt.sl, w.T2.get(), w.w.get(), nbm, w.p.get(),
                      w.shift.get(), inv_ng, st);
  };
  auto gram_and_reduce = [&](const Batch& bt, const KernelTune& kt) {
    const KTileRange krg{s.nk, s.d_ktb.get(), bt.ktmax};
    const int nsc = gram_partials<R>(bt.tl, s.d_nb.get(), nbm, dMcg, Mrows, wcg, wk, nbm,
                                     w.p.get(), nbm, w.part.get(), st, nullptr, krg, &kt);
    gram_reduce<R>(bt.tl, dMcg, Mrows, nsc, w.part.get(), w.craw.get(), s.mcg, st);
  };
  auto one = [&](auto&& prefix, auto&& launch, const Batch& bt) {
    prefix(bt);
    IKR_HIP(hipEventRecord(e0, st));
    launch(bt);
    IKR_HIP(hipEventRecord(e1, st));
    return elapsed_us();
  };
  // summed time (us per launch) over the sets: one untimed run, then
  // TUNE_REPS timed ones; a candidate already 30% behind the best after a
  // set is not run further
  auto time_us = [&](auto&& prefix, auto&& launch, double best) {
    double tot = 0;
    for (const auto& set : sets) {
      const Batch bt = select(set);
      (void)one(prefix, launch, bt);   // untimed: first use
      double t = 0;
      for (int r = 0; r < TUNE_REPS; ++r) t += one(prefix, launch, bt);
      tot += t / TUNE_REPS;
      if (best > 0 && tot > 1.3 * best) return 1e300;
    }
    return tot;
  };
  // keeps the first candidate (the size rule) unless one is clearly faster
  auto better = [](double t, double best, bool first) {
    return first || t < TUNE_MARGIN * best;
  };
  KernelTune best{};
  std::string log;
  char buf[96];
  try {
    // the gram with the reduction of its partials (the block count sets both)
    double tg = 0;
    bool first = true;
    const int vdef = gram_variant(Mrows, kr, nullptr);
    for (int v = 0; v <= 3; ++v)
      for (float sc : {1.0f, 0.5f, 2.0f}) {
        KernelTune c{};
        c.gram = v;
        c.gram_scale = sc;
        if (v == 0 && sc != 1.0f) continue;
        if (v > 0 && (gram_variant(Mrows, kr, &c) != v || (v == vdef && sc == 1.0f))) continue;
        const double t = time_us([&](const Batch& bt) { to_gram(bt, KernelTune{}); },
                                 [&](const Batch& bt) { gram_and_reduce(bt, c); }, tg);
        std::snprintf(buf, sizeof buf, t < 1e300 ? " %c%.1f:%.1f" : " %c%.1f:-", "SPKV"[v], sc, t);
        log += buf;
        if (better(t, tg, first)) { tg = t; best.gram = v; best.gram_scale = sc; }
        first = false;
      }
    s.tune_us[pi][cls][0] = tg;
    // the update's band group (the coefficients are whatever the gram left)
    double tu = 0;
    first = true;
    log += " |";
    for (int bpt : {0, 4, 8, 16}) {
      if (bpt && (size_t)bpt * (Na + 3 * Mq_max) * sizeof(cplx<R>) > 65536) continue;
      KernelTune c = best;
      c.upd_bpt = bpt;
      const double t = time_us(
          [&](const Batch& bt) {
            to_gram(bt, KernelTune{});
            gram_and_reduce(bt, best);
            cg_combine<R>(bt.sl, Na, dMq, Mq_max, w.craw.get(), s.mcg, w.shift.get(),
                          w.gT.get(), w.sT.get(), s.nbands, R(s.dnl), w.gam.get(), st);
          },
          [&](const Batch& bt) {
            cg_update<R>(bt.tl, s.d_nb.get(), nbm, wcg, wk, Na, dMq, Mq_max, w.gam.get(),
                         s.mcg, w.w.get(), w.p.get(), w.dpart.get(), st, kr, &c);
          },
          tu);
      std::snprintf(buf, sizeof buf, t < 1e300 ? " b%d:%.1f" : " b%d:-", bpt, t);
      log += buf;
      if (better(t, tu, first)) { tu = t; best.upd_bpt = bpt; }
      first = false;
    }
    s.tune_us[pi][cls][1] = tu;
    // the plane kernel's block size, where two are built
    double tp = 0;
    first = true;
    log += " |";
    const int pdef = plane_hv_threads(s.geom, 0, sizeof(R) == 8);
    for (int pt : {0, 256, 512}) {
      if (pt && (pt == pdef || plane_hv_threads(s.geom, pt, sizeof(R) == 8) != pt)) continue;
      const double t = time_us(col_inv, [&](const Batch& bt) {
        launch_plane_hv<R>(s.geom, s.fft, bt.sl, w.T1.get(), w.T2.get(), vloc, 0, st, pt);
      }, tp);
      std::snprintf(buf, sizeof buf, t < 1e300 ? " t%d:%.1f" : " t%d:-", pt ? pt : pdef, t);
      log += buf;
      if (better(t, tp, first)) { tp = t; best.plane_pt = pt; }
      first = false;
    }
    s.tune_us[pi][cls][2] = tp;
  } catch (...) {
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  IKR_HIP(hipEventDestroy(e0));
  IKR_HIP(hipEventDestroy(e1));
  s.tune[pi][cls] = best;
  s.tuned[pi][cls] = true;
  if (std::getenv("IKR_VERBOSE"))
    std::fprintf(stderr, "[ikr] tuned %s %s batches (S: size rule, P/K/V: per-tile, k-wide, "
                 "vector gram x block scale; b: bands per update block; t: plane threads; "
                 "us):%s\n", pi ? "FP32" : "FP64", cls ? "thin" : "thick", log.c_str());
}

// Batch class of nt tiles over nkl k-points: 0 with more tiles than k-points, else 1.
static int batch_class_of(int nt, int nkl) { return nt > nkl ? 0 : 1; }

template <typename R>
static void tune_launches(System& s, CgWork<R>& w, const std::vector<int>& member,
                          const int* dMq, int Mq_max, const int* dMcg, hipStream_t st) {
  const int pi = sizeof(R) == 8 ? 0 : 1;
  if (kernel_paths() & PATH_FIXED) return;
  if (s.tuned[pi][0] && s.tuned[pi][1]) return;
  int nt = 0;
  std::vector<int> thin8(s.J, 0), thin2(s.J, 0);
  for (int k = 0; k < s.nk; ++k) {
    int c = 0;
    for (int j = s.slot0_k[k]; j < s.slot0_k[k] + s.nocc_k[k]; ++j) {
      if (!member[j]) continue;
      thin8[j] = c < 8;
      thin2[j] = c < 2;
      ++c;
    }
    nt += (c + BT - 1) / BT;
  }
  bool changed = false;
  if (batch_class_of(nt, s.nk) == 0 && !s.tuned[pi][0]) {
    tune_class<R>(s, w, {member}, 0, dMq, Mq_max, dMcg, st);
    changed = true;
  }
  if (!s.tuned[pi][1]) {
    // with the run's own batch when that is thin too (its first iterations)
    if (batch_class_of(nt, s.nk) == 1)
      tune_class<R>(s, w, {member, thin8, thin2}, 1, dMq, Mq_max, dMcg, st);
    else
      tune_class<R>(s, w, {thin8, thin2}, 1, dMq, Mq_max, dMcg, st);
    changed = true;
  }
  if (changed) s.graphs.clear();   // graphs captured before hold the size-rule shapes
}

// Device state one CG run works with (the system's compaction lists,
// counters and partial sums, and the stream the run is enqueued on).
template <typename R> struct CgCtx {
  hipStream_t st;
  int *active, *iters, *counters, *list, *ctk, *cto, *ctn, *cnt, *ktb;
  double* tol2;
  DBuf<int>* hist;
  HBuf<int>* h_cnt;
  int* d_hcnt;
  cplx<R>* part;
};

template <typename R> CgCtx<R> main_ctx(System& s, CgWork<R>& w, hipStream_t st) {
  return CgCtx<R>{st, s.d_active.get(), s.d_iters.get(), s.d_counters.get(), s.d_list.get(),
                  s.d_ctk.get(), s.d_cto.get(), s.d_ctn.get(), s.d_cnt.get(), s.d_ktb.get(),
                  s.d_tol2.get(), &s.d_hist, &s.h_cnt, s.d_hcnt, w.part.get()};
}


// Preconditioned CG on Q (H - e_n) Q x = r for the member slots, all at once (discretised Sternheimer equation; zero initial guess; at least
// min_iter iterations; absolute stopping test on |r|).  The iterates stay in
// range Q (remark after Lemma cgtol_E) through the exact projection of p and
// Ap that one gram of p~ = z + beta p against [projectors | phi, H phi]
// provides.  The active set is compacted on the device after every
// iteration; the host reads its size one iteration late (an upper bound,
// since bands only leave the set), so the stream never drains between
// iterations.  With s.cg_graph set (and no kernel timing), each
// iteration is one replay of a captured graph whose grids cover the live
// count rounded up to a power of two; the kernels skip rows past the device
// count, so a graph stays valid while the set shrinks, and a smaller one is
// taken once the count halves.  start() enqueues the set-up, step() one
// iteration and the lagged read, finish() waits and collects the counts.
//
// keep_x: the member rows of w.x hold an initial guess and rhs the initial
// residual b - A x (defect correction); otherwise the guess is zero and rhs = b.
template <typename R> struct CgRunner {
  System& s;
  CgWork<R>& w;
  CgCtx<R> c;
  const std::vector<int>& member;
  const int* dMq;
  int Mq_max;
  const int* dMcg;
  int min_iter, max_iter, nkl;
  bool use_graph, timing;
  int J, nbm, nbn, Na, Mrows, nvb, nup, nmem = 0, nact = 0, nct = 0, nt0 = 0;
  int nkt = 0;   // bound on the live tiles of any one k-point (one iteration old)
  int it = 0, iters = 0, lag_seen = 0, lag_copied = 0;
  bool done = false;
  size_t wk;
  CgScalars<R> cs{};
  CgCompact cp{};
  hipEvent_t ev[2] = {nullptr, nullptr};

  CgRunner(System& s_, CgWork<R>& w_, const CgCtx<R>& c_, const std::vector<int>& member_,
           int nkl_, int min_iter_, int max_iter_, const int* dMq_, int Mq_max_,
           const int* dMcg_, bool graph)
      : s(s_), w(w_), c(c_), member(member_), dMq(dMq_), Mq_max(Mq_max_), dMcg(dMcg_),
        min_iter(min_iter_), max_iter(max_iter_), nkl(nkl_) {
    use_graph = graph;
    timing = KTimer::enabled();
    J = s.J;
    nbm = s.nb_max;
    nbn = s.nbands;
    Na = s.natoms;
    Mrows = Na + 2 * Mq_max;
    wk = (size_t)s.mcg * nbm;
    for (int v : member) nmem += v != 0;
    done = nmem == 0 || max_iter <= 0;
  }
  ~CgRunner() {
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  KTileRange kr() const { return KTileRange{s.nk, c.ktb, s.ktmax}; }

  void start(const cplx<R>* rhs, const std::vector<double>& tol_slot, bool keep_x) {
    if (done) return;
    const hipStream_t st = c.st;
    if (st != s.stream) {   // the lane starts after the work queued so far
      hipEvent_t j0;
      IKR_HIP(hipEventCreateWithFlags(&j0, hipEventDisableTiming));
      (void)hipEventRecord(j0, s.stream);
      const hipError_t e = hipStreamWaitEvent(st, j0, 0);
      (void)hipEventDestroy(j0);
      IKR_HIP(e);
    }
    if (w.r.get() != rhs)
      IKR_HIP(hipMemcpyAsync(w.r.get(), rhs, (size_t)J * nbm * sizeof(cplx<R>),
                             hipMemcpyDeviceToDevice, st));
    std::vector<double> tol2(J);
    for (int j = 0; j < J; ++j) tol2[j] = tol_slot[j] * tol_slot[j];
    IKR_HIP(hipMemcpyAsync(c.tol2, tol2.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
    IKR_HIP(hipMemcpyAsync(c.active, member.data(), J * sizeof(int), hipMemcpyHostToDevice, st));
    IKR_HIP(hipMemsetAsync(c.iters, 0, J * sizeof(int), st));
    // counters: [1] slots that missed their tolerance, [2] compaction step
    IKR_HIP(hipMemsetAsync(c.counters, 0, 8 * sizeof(int), st));
    // (the pageable sources above are copied before the calls return)
    if (c.hist->n < (size_t)2 * (max_iter + 1)) {
      if (c.hist == &s.d_hist) s.graphs.clear();   // captured graphs hold the old pointer
      c.hist->alloc((size_t)2 * (max_iter + 1));
    }
    cs = CgScalars<R>{w.rz.get(), w.alpha.get(), w.beta.get(), w.rnorm2.get(), c.tol2,
                      c.iters, c.counters, c.counters + 1, min_iter, max_iter};
    if (sizeof(R) == 4) {   // FP32 bands stop when they stall at the FP32 floor
      cs.stag = FP32_STAG_ITERS;
      cs.rbest = w.rbest.get();
      cs.rlast = s.d_rlast.get();
    }
    nvb = vec_nblocks(nbm);
    nup = cg_update_parts(nbm, Mrows, kr());
    cp = CgCompact{s.nk, s.d_slot0_k.get(), s.d_nocc_k.get(), s.d_slot_k.get(), J,
                   c.list, c.ctk, c.cto, c.ctn, c.cnt, c.hist->get(), max_iter + 1,
                   c.counters + 2, c.d_hcnt, c.ktb};
    // host bound on the tiles of the member set
    for (int k = 0; k < s.nk; ++k) {
      int n = 0;
      for (int j = s.slot0_k[k]; j < s.slot0_k[k] + s.nocc_k[k]; ++j) n += member[j] != 0;
      nct += (n + BT - 1) / BT;
      nkt = std::max(nkt, (n + BT - 1) / BT);
    }
    nt0 = nct;
    nact = nmem;
    {
      CgCompact c0 = cp;
      c0.hist = nullptr;
      c0.hcnt = nullptr;
      cg_compact(c0, c.active, st);
    }
    // p = 0 (and x = 0 unless it is the initial guess) for the members only:
    // other slots keep what they hold
    cg_zero<R>(Slots{nact, s.d_slot_k.get(), c.active, c.list, c.cnt}, nbm,
               keep_x ? nullptr : w.x.get(), w.p.get(), st);
    {
      // z = M^-1 r, rz = <r, z>, beta = 0
      Slots sl{nact, s.d_slot_k.get(), c.active, c.list, c.cnt};
      cg_start<R>(sl, s.d_nb.get(), s.d_kin.get(), nbm, w.pshift.get(), w.r.get(), w.w.get(),
                  w.rpart.get(), w.zpart.get(), st);
      cg_finish<R>(sl, nvb, w.rpart.get(), w.zpart.get(), cs, c.active, 1, st);
    }
    IKR_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    IKR_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
      // no compaction is in flight here (every run ends with a stream sync)
    for (int i = 0; i < 2 * CNT_STRIDE; ++i) c.h_cnt->p[i] = -1;
  }

  // one CG iteration over grids of na rows and nt tiles
  void iteration(int na, int nt) {
    const hipStream_t st = c.st;
    const int pi = sizeof(R) == 8 ? 0 : 1;
    const R inv_ng = R(1.0 / s.ng);
    const R* vloc = vloc_of<R>(s);
    const cplx<R>* wcg = wcg_of<R>(s);
    Slots sl{na, s.d_slot_k.get(), c.active, c.list, c.cnt};
    Tiles ctl{nt, c.ctk, c.cto, c.ctn, c.list, c.cnt + 1};
    const int cls = batch_class_of(nt, nkl);
    const KernelTune* kt = !(kernel_paths() & PATH_FIXED) && s.tuned[pi][cls]
                               ? &s.tune[pi][cls] : nullptr;
    // p~ = z + beta p ; w~ = (H_loc - e) p~ through the pruned FFT
    KTimer::begin(kid<R>(K_COL_INV), st);
    launch_col_inv<R>(s.geom, s.fft, sl, w.p.get(), nbm, w.T1.get(), w.w.get(), w.beta.get(),
                      w.p.get(), st);
    KTimer::end(kid<R>(K_COL_INV), st, 0.0);
    KTimer::begin(kid<R>(K_PLANE_HV), st);
    launch_plane_hv<R>(s.geom, s.fft, sl, w.T1.get(), w.T2.get(), vloc, 0, st,
                       kt ? kt->plane_pt : 0);
    KTimer::end(kid<R>(K_PLANE_HV), st, 0.0);
    KTimer::begin(kid<R>(K_COL_FWD), st);
    launch_col_fwd<R>(s.geom, s.fft, sl, w.T2.get(), w.w.get(), nbm, w.p.get(), w.shift.get(),
                      inv_ng, st);
    KTimer::end(kid<R>(K_COL_FWD), st, 0.0);
    // q, a, h = W_k^H p~ ; update coefficients ; Ap and p = Q p~ ; <p, Ap>
    KTimer::begin(kid<R>(K_GRAM), st);
    // the gram's kernel may follow the live tiles per k-point (graphs keep the bound of the set-up)
    const KTileRange krg{s.nk, c.ktb, use_graph ? s.ktmax : std::min(nkt, s.ktmax)};
    const int nsc = gram_partials<R>(ctl, s.d_nb.get(), nbm, dMcg, Mrows, wcg, wk, nbm,
                                     w.p.get(), nbm, c.part, st, nullptr, krg, kt);
    KTimer::end(kid<R>(K_GRAM), st, 0.0);
    gram_reduce<R>(ctl, dMcg, Mrows, nsc, c.part, w.craw.get(), s.mcg, st);
    cg_combine<R>(sl, Na, dMq, Mq_max, w.craw.get(), s.mcg, w.shift.get(), w.gT.get(),
                  w.sT.get(), nbn, R(s.dnl), w.gam.get(), st);
    KTimer::begin(kid<R>(K_UPDATE), st);
    cg_update<R>(ctl, s.d_nb.get(), nbm, wcg, wk, Na, dMq, Mq_max, w.gam.get(), s.mcg,
                 w.w.get(), w.p.get(), w.dpart.get(), st, kr(), kt);
    KTimer::end(kid<R>(K_UPDATE), st, 0.0);
    // alpha ; x += alpha p, r -= alpha Ap, z = M^-1 r, |r|^2, <r, z>
    KTimer::begin(kid<R>(K_CG_STEP), st);
    cg_step2<R>(sl, s.d_nb.get(), s.d_kin.get(), nbm, w.dpart.get(), nup, w.rz.get(),
                w.alpha.get(), c.active, w.pshift.get(), w.x.get(), w.r.get(), w.p.get(),
                w.w.get(), w.rpart.get(), w.zpart.get(), st);
    KTimer::end(kid<R>(K_CG_STEP), st, 0.0);
    // beta, convergence, and the active set of the next iteration
    cg_end<R>(sl, nvb, w.rpart.get(), w.zpart.get(), cs, c.active, cp, st);
  }

  static int pow2_cap(int n, int cap) {
    int p = 1;
    while (p < n) p <<= 1;
    return std::min(p, cap);
  }

  // Enqueues one iteration and reads the live counts of the one before;
  // false once the run is over (converged, or max_iter iterations).
  bool step() {
    if (done) return false;
    const hipStream_t st = c.st;
    if (use_graph) {
      const int na = pow2_cap(nact, J), nt = pow2_cap(nct, s.tiles.n);
      const CgGraphs::Key key{(long long)sizeof(R), na, nt, (long long)(intptr_t)dMq,
                              min_iter, max_iter, kernel_paths()};
      const hipGraphExec_t ge = s.graphs.get(key, st, [&] { iteration(na, nt); });
      IKR_HIP(hipGraphLaunch(ge, st));
    } else {
      iteration(nact, nct);
    }
    iters = it + 1;
    if (s.cg_plain) {   // reference loop: the host waits for every iteration's count
      IKR_HIP(hipMemcpyAsync(c.h_cnt->p, c.cnt, CNT * sizeof(int), hipMemcpyDeviceToHost, st));
      IKR_HIP(hipStreamSynchronize(st));
      nact = c.h_cnt->p[0];
      nct = c.h_cnt->p[1];
      nkt = c.h_cnt->p[2];
      for (int i = 0; i < CNT; ++i) c.h_cnt->p[i] = -1;
    } else {
      // the compaction of iteration it writes its counts to h_cnt[CNT_STRIDE (it & 1)]
      IKR_HIP(hipEventRecord(ev[it & 1], st));
      if (it >= 1) {
        IKR_HIP(hipEventSynchronize(ev[(it - 1) & 1]));
        volatile int* hc = c.h_cnt->p + CNT_STRIDE * ((it - 1) & 1);
        if (hc[0] < 0 || hc[1] < 0 || hc[2] < 0) {
          // not seen yet: the device counts are as fresh or fresher, so also a bound
          IKR_HIP(hipMemcpyAsync((void*)hc, c.cnt, CNT * sizeof(int), hipMemcpyDeviceToHost, st));
          IKR_HIP(hipStreamSynchronize(st));
          ++lag_copied;
        } else {
          ++lag_seen;
        }
        nact = hc[0];
        nct = hc[1];
        nkt = hc[2];
        for (int i = 0; i < CNT; ++i) hc[i] = -1;   // consumed: iteration it + 1 writes here next
      }
    }
    ++it;
    if (nact == 0 || it >= max_iter) done = true;
    return !done;
  }

  CgOut finish() {
    CgOut out;
    if (nmem == 0 || max_iter <= 0) return out;
    const hipStream_t st = c.st;
    IKR_HIP(hipStreamSynchronize(st));
    const char* vb = std::getenv("IKR_VERBOSE");
    if (vb && std::atoi(vb) >= 2)
      std::fprintf(stderr, "[ikr] CG run %s: %d iterations, %d bands; live counts read from "
                   "pinned memory %d times, copied %d times\n",
                   sizeof(R) == 8 ? "FP64" : "FP32", iters, nmem, lag_seen, lag_copied);
    const std::vector<int> hits = download(c.iters, J, st);
    for (int j = 0; j < J; ++j) out.n_ham += hits[j];
    const std::vector<int> ctr = download(c.counters, 4, st);
    const std::vector<int> last = download(c.cnt, 2, st);
    out.noconv = ctr[1] + last[0];
    if (timing) {
      // algorithmic bytes of the launches, from the live counts of each iteration
      double nb_avg = 0, ncol_avg = 0;
      for (int j = 0; j < J; ++j) {
        nb_avg += s.kp[s.slot_k[j]].nb;
        ncol_avg += s.kp[s.slot_k[j]].ncol;
      }
      nb_avg /= J;
      ncol_avg /= J;
      const double SZ = sizeof(cplx<R>), colC = ncol_avg * s.L.C;
      const std::vector<int> hist = download(c.hist->get(), (size_t)2 * iters, st);
      double b[K_COUNT] = {};
      int na = nmem, nt = nt0;
      for (int i = 0; i < iters; ++i) {
        b[K_COL_INV] += na * (3.0 * nb_avg + colC) * SZ;
        b[K_PLANE_HV] += na * 2.0 * colC * SZ + (na > 0 ? sizeof(R) * (double)s.ng : 0.0);
        b[K_COL_FWD] += na * (colC * SZ + nb_avg * (2.0 * SZ + 8.0));
        b[K_GRAM] += nt * Mrows * nb_avg * SZ + na * nb_avg * SZ;
        b[K_UPDATE] += nt * Mrows * nb_avg * SZ + na * 4.0 * nb_avg * SZ;
        b[K_CG_STEP] += na * nb_avg * (7.0 * SZ + 8.0);
        na = hist[2 * i];
        nt = hist[2 * i + 1];
      }
      for (int id = 0; id < K_PLANE_RHO; ++id)
        if (b[id] > 0) KTimer::add_bytes(kid<R>(id), b[id]);
    }
    return out;
  }
};

template <typename R>
CgOut run_cg(System& s, CgWork<R>& w, const cplx<R>* rhs, const std::vector<int>& member,
             const std::vector<double>& tol_slot, int min_iter, int max_iter,
             const int* dMq, int Mq_max, const int* dMcg, bool keep_x = false) {
  const bool use_graph = s.cg_graph != 0 && !KTimer::enabled();
  int nmem = 0;
  for (int v : member) nmem += v != 0;
  if (nmem == 0 || max_iter <= 0) return CgOut{};
  tune_launches<R>(s, w, member, dMq, Mq_max, dMcg, s.stream);
  // (a graph's private stream starts after the work queued so far: start())
  const hipStream_t st = use_graph ? s.graphs.get_stream() : s.stream;
  CgRunner<R> r(s, w, main_ctx<R>(s, w, st), member, s.nk, min_iter, max_iter, dMq, Mq_max,
                dMcg, use_graph);
  try {
    r.start(rhs, tol_slot, keep_x);
    while (r.step()) {}
    return r.finish();
  } catch (...) {
    (void)hipStreamSynchronize(st);
    throw;
  }
}

// w.w := Q (H - e_j) Q v (FP64) for the member slots, with v in the member
// rows of w.w on entry; w.p := Q v.  It is the front half of a fused CG
// iteration with p~ = v (p = 0, beta = 0).  On return s.d_list / s.d_cnt
// hold the compacted member set.
void apply_sternheimer_op(System& s, const std::vector<int>& member, const int* dMq,
                          int Mq_max, const int* dMcg) {
  const hipStream_t st = s.stream;
  CgWork<double>& w = s.w64;
  const int J = s.J, nbm = s.nb_max, nbn = s.nbands, Na = s.natoms;
  const int Mrows = Na + 2 * Mq_max;
  const size_t wk = (size_t)s.mcg * nbm;
  int nact = 0, nct = 0;
  for (int v : member) nact += v != 0;
  if (nact == 0) return;
  for (int k = 0; k < s.nk; ++k) {
    int c = 0;
    for (int j = s.slot0_k[k]; j < s.slot0_k[k] + s.nocc_k[k]; ++j) c += member[j] != 0;
    nct += (c + BT - 1) / BT;
  }
  IKR_HIP(hipMemcpyAsync(s.d_active.get(), member.data(), J * sizeof(int), hipMemcpyHostToDevice,
                         st));
  int* cnt = s.d_cnt.get();
  cg_compact(CgCompact{s.nk, s.d_slot0_k.get(), s.d_nocc_k.get(), s.d_slot_k.get(), J,
                       s.d_list.get(), s.d_ctk.get(), s.d_cto.get(), s.d_ctn.get(), cnt,
                       nullptr, 0, s.d_counters.get() + 2, nullptr, s.d_ktb.get()},
             s.d_active.get(), st);
  Slots sl{nact, s.d_slot_k.get(), s.d_active.get(), s.d_list.get(), cnt};
  Tiles ctl{nct, s.d_ctk.get(), s.d_cto.get(), s.d_ctn.get(), s.d_list.get(), cnt + 1};
  IKR_HIP(hipMemsetAsync(w.beta.get(), 0, J * sizeof(double), st));
  cg_zero<double>(sl, nbm, nullptr, w.p.get(), st);
  launch_col_inv<double>(s.geom, s.fft, sl, w.p.get(), nbm, w.T1.get(), w.w.get(), w.beta.get(),
                         w.p.get(), st);
  launch_plane_hv<double>(s.geom, s.fft, sl, w.T1.get(), w.T2.get(), s.d_vloc.get(), 0, st);
  launch_col_fwd<double>(s.geom, s.fft, sl, w.T2.get(), w.w.get(), nbm, w.p.get(), w.shift.get(),
                         1.0 / s.ng, st);
  const int nsc = gram_partials<double>(ctl, s.d_nb.get(), nbm, dMcg, Mrows, w.wcg.get(), wk,
                                        nbm, w.p.get(), nbm, w.part.get(), st, nullptr,
                                        s.krange_compact());
  gram_reduce<double>(ctl, dMcg, Mrows, nsc, w.part.get(), w.craw.get(), s.mcg, st);
  cg_combine<double>(sl, Na, dMq, Mq_max, w.craw.get(), s.mcg, w.shift.get(), w.gT.get(),
                     w.sT.get(), nbn, s.dnl, w.gam.get(), st);
  cg_update<double>(ctl, s.d_nb.get(), nbm, w.wcg.get(), wk, Na, dMq, Mq_max, w.gam.get(),
                    s.mcg, w.w.get(), w.p.get(), w.dpart.get(), st, s.krange_compact());
}

}  // namespace

void tune_launches_now(System& s, int precision, int schur) {
  IKR_CHECK(s.have_gs, 2, "ground state not set up");
  const bool use_schur = schur && s.nbands > s.nocc_max;
  const int* dMq = use_schur ? s.d_nbands_k.get() : s.d_nocc_k.get();
  const int* dMcg = use_schur ? s.d_mcg_all.get() : s.d_mcg_occ.get();
  const int Mq_max = use_schur ? s.nbands : s.nocc_max;
  const std::vector<int> all(s.J, 1);
  tune_launches<double>(s, s.w64, all, dMq, Mq_max, dMcg, s.stream);
  if (precision) {
    ensure_fp32(s);
    tune_launches<float>(s, s.w32, all, dMq, Mq_max, dMcg, s.stream);
  }
  IKR_HIP(hipStreamSynchronize(s.stream));
}


// ---------------------------------------------------------------- chi0
Chi0Result apply_chi0_internal(System& s, const double* u_int, double* drho_int,
                               const std::vector<double>& tol_in, int min_iter,
                               int max_iter, int precision, double theta, int schur,
                               const Chi0Extra* ex) {
  IKR_CHECK(s.have_gs, 2, "ground state not set up");
  const hipStream_t st = s.stream;
  CgWork<double>& w = s.w64;
  const int J = s.J, nbm = s.nb_max, nbn = s.nbands;
  const double inv_ng = 1.0 / s.ng;
  Slots all{J, s.d_slot_k.get(), nullptr};
  const size_t phik = (size_t)nbn * nbm;
  UpdTerm<double> none{};
  Chi0Result res;
  // Q-projection rows: the occupied bands, or every computed band when the
  // extra bands are treated by sum over states.
  const bool use_schur = schur && s.nbands > s.nocc_max;
  const int* dMq = use_schur ? s.d_nbands_k.get() : s.d_nocc_k.get();
  const int* dMcg = use_schur ? s.d_mcg_all.get() : s.d_mcg_occ.get();
  const int Mq_max = use_schur ? s.nbands : s.nocc_max;

  // right-hand sides t_j = F(u F^-1 phi_j) into r (or given ones)
  if (ex && ex->rhs_pw) {
    if (ex->rhs_pw != w.r.get())
      IKR_HIP(hipMemcpyAsync(w.r.get(), ex->rhs_pw, (size_t)J * nbm * sizeof(double2),
                             hipMemcpyDeviceToDevice, st));
  } else {
    launch_plane_hv<double>(s.geom, s.fft, all, s.d_Tphi.get(), w.T2.get(), u_int, 0, st);
    launch_col_fwd<double>(s.geom, s.fft, all, w.T2.get(), w.r.get(), nbm, nullptr, nullptr,
                           inv_ng, st);
  }
  // M[j][m] = <phi_m, t_j>
  gram<double>(s.tiles, s.d_nb.get(), nbm, dMq, Mq_max, s.d_phi.get(), phik,
               nbm, w.r.get(), nbm, w.part.get(), w.coefA.get(), MAXM, st, nullptr, s.krange());
  const std::vector<double2> M = download(w.coefA.get(), (size_t)J * MAXM, st);
  if (ex && ex->m_out) *ex->m_out = M;

  // occupation response and occupied-space part (minimal gauge)
  std::vector<double> de(J), df(J, 0.0);
  std::vector<double2> dp((size_t)J * MAXM, mk<double>(0, 0));
  double num = 0, den = 0;
  for (int j = 0; j < J; ++j) {
    const int k = s.slot_k[j], n = s.slot_n[j];
    de[j] = M[(size_t)j * MAXM + n].x;
    const double fpn = s.docc[(size_t)k * nbn + n];
    num += s.kp[k].weight * fpn * de[j];
    den += s.kp[k].weight * fpn;
    const double fn = s.occ[(size_t)k * nbn + n], en = s.eps[(size_t)k * nbn + n];
    for (int m = 0; m < s.nocc_k[k]; ++m) {
      if (m == n) continue;
      const double fm = s.occ[(size_t)k * nbn + m], em = s.eps[(size_t)k * nbn + m];
      const double d = host::occupation_divided_difference(fn, fm, en, em, s.fermi,
                                                           s.temperature, DEGEN_TOL);
      if (d == 0.0) continue;
      const double al = fn * d / (fn * fn + fm * fm);
      dp[(size_t)j * MAXM + m] = cscale<double>(M[(size_t)j * MAXM + m], al);
    }
    // extra computed bands: their part of the unoccupied response,
    // <phi_m, t_n> / (e_n - e_m), by sum over states.  A pair within
    // DEGEN_TOL across the occupation cut-off (smearing) takes the limit of
    // the divided difference, f'(midpoint) / f_n, as the occupied pairs do.
    if (use_schur)
      for (int m = s.nocc_k[k]; m < nbn; ++m) {
        const double em = s.eps[(size_t)k * nbn + m];
        const double c = host::extra_band_coefficient(fn, en, em, s.fermi, s.temperature,
                                                      DEGEN_TOL);
        dp[(size_t)j * MAXM + m] = cscale<double>(M[(size_t)j * MAXM + m], c);
      }
  }
  const double defermi = den != 0.0 ? num / den : 0.0;
  for (int j = 0; j < J; ++j)
    df[j] = s.docc[(size_t)s.slot_k[j] * nbn + s.slot_n[j]] * (de[j] - defermi);

  // b = -Q t   (r = -t + Phi M)
  UpdTerm<double> phiM{s.d_phi.get(), phik, nbm, dMq, w.coefA.get(), MAXM, 1.0, Mq_max};
  update<double>(s.tiles, s.d_nb.get(), nbm, nullptr, w.r.get(), nbm, -1.0, phiM, none,
                 nullptr, nullptr, st);

  // Per-band precision: bands whose tolerance is loose relative to their
  // right-hand side run the CG in FP32 (FP32 FFTs and projections); the
  // others, and everything after the CG, stay in FP64.
  // Tolerances are floored at TOL_FLOOR ||b_j||: below that the FP64
  // recursion stagnates at round-off on the ill-conditioned bands.
  std::vector<double> tol_slot(tol_in);
  std::vector<int> m64(J, 1), m32(J, 0);
  int n32 = 0;
  const std::vector<double> bn = slot_norms(s, w.r.get());   // ||b_j||
  {
    for (int j = 0; j < J; ++j) {
      if (ex && ex->tol_relative) tol_slot[j] *= bn[j];
      tol_slot[j] = std::max(tol_slot[j], TOL_FLOOR * bn[j]);
    }
    if (precision == 1 && !s.cg_plain)
      for (int j = 0; j < J; ++j)
        if (tol_slot[j] >= theta * bn[j]) { m32[j] = 1; m64[j] = 0; ++n32; }
  }
  // Warm starts (solver option recycle): x0 = the least-squares combination of
  // the band's stored solutions for its stored right-hand sides, where that
  // leaves under WARM_REL of b; the CG then runs on A d = b - A x0.
  const int L = s.cg_recycle;
  std::vector<double2> hdot;   // <b_l, b_j> of the stored right-hand sides
  bool any_warm = false;
  if (L > 0) {
    if (s.rec_cap != L) {
      s.rec_cap = L;
      s.rec_count = s.rec_head = 0;
      s.d_rec_b.alloc((size_t)L * J * nbm);
      s.d_rec_x.alloc((size_t)L * J * nbm);
      s.d_rec_tb.alloc((size_t)J * nbm);
      s.d_rec_part.alloc(slot_dots_part_elems(J, nbm, L));
      s.d_rec_h.alloc((size_t)J * L);
      s.d_rec_c.alloc((size_t)J * L);
      s.d_rec_list.alloc(J);
      s.rec_G.assign((size_t)J * L * L, mk<double>(0, 0));
    }
    IKR_HIP(hipMemcpyAsync(s.d_rec_tb.get(), w.r.get(), (size_t)J * nbm * sizeof(double2),
                           hipMemcpyDeviceToDevice, st));
    const int nv = s.rec_count;
    if (nv > 0) {
      const size_t vs = (size_t)J * nbm;
      slot_dots(J, nbm, s.d_slot_k.get(), s.d_nb.get(), nv, s.d_rec_b.get(), vs, w.r.get(),
                s.d_rec_part.get(), s.d_rec_h.get(), st);
      hdot = download(s.d_rec_h.get(), (size_t)J * nv, st);
      std::vector<double2> c((size_t)J * nv, mk<double>(0, 0));
      std::vector<int> wl;
      std::vector<double> ratio(J);
      for (int j = 0; j < J; ++j) {
        const double2* h = hdot.data() + (size_t)j * nv;
        std::vector<host::zd> c_j;
        const double pred = host::warm_coefficients(
            reinterpret_cast<const host::zd*>(s.rec_G.data() + (size_t)j * L * L), L, nv,
            reinterpret_cast<const host::zd*>(h), bn[j] * bn[j], c_j);
        ratio[j] = std::sqrt(std::max(pred, 0.0)) / std::max(bn[j], 1e-300);
        if (pred < WARM_REL * WARM_REL * bn[j] * bn[j]) {
          for (int l = 0; l < nv; ++l)
            c[(size_t)j * nv + l] = mk<double>(c_j[l].real(), c_j[l].imag());
          wl.push_back(j);
        }
      }
      if (std::getenv("IKR_VERBOSE")) {
        std::vector<double> r = ratio;
        std::sort(r.begin(), r.end());
        std::fprintf(stderr, "[ikr warm] stored %d: residual left by the stored solutions, "
                     "min %.3f median %.3f max %.3f of ||b||; %zu warm\n", nv, r.front(),
                     r[r.size() / 2], r.back(), wl.size());
      }
      if (!wl.empty()) {
        any_warm = true;
        res.warm = (int)wl.size();
        IKR_HIP(hipMemcpyAsync(s.d_rec_c.get(), c.data(), c.size() * sizeof(double2),
                               hipMemcpyHostToDevice, st));
        IKR_HIP(hipMemcpyAsync(s.d_rec_list.get(), wl.data(), wl.size() * sizeof(int),
                               hipMemcpyHostToDevice, st));
        // x = 0 for every slot, then x0 on the warm ones; r = b - A x0 there
        cg_zero<double>(Slots{J, s.d_slot_k.get(), nullptr}, nbm, w.x.get(), w.p.get(), st);
        slot_combine((int)wl.size(), s.d_rec_list.get(), nbm, s.d_slot_k.get(), s.d_nb.get(), nv,
                     s.d_rec_x.get(), vs, s.d_rec_c.get(), w.x.get(), st);
        slot_combine((int)wl.size(), s.d_rec_list.get(), nbm, s.d_slot_k.get(), s.d_nb.get(), nv,
                     s.d_rec_x.get(), vs, s.d_rec_c.get(), w.w.get(), st);
        std::vector<int> mw(J, 0);
        for (int j : wl) mw[j] = 1;
        IKR_HIP(hipStreamSynchronize(st));
        apply_sternheimer_op(s, mw, dMq, Mq_max, dMcg);
        cg_axpy<double>(Slots{(int)wl.size(), s.d_slot_k.get(), nullptr, s.d_rec_list.get()},
                        s.d_nb.get(), nbm, -1.0, w.w.get(), w.r.get(), st);
        res.n_ham64 += (long long)wl.size();
      }
    }
  }
  CgOut o64;
  if (s.cg_plain) {
    // plain FP64 reference: the k-points one after the other
    for (int k = 0; k < s.nk; ++k) {
      std::vector<int> mk_(J, 0);
      for (int j = s.slot0_k[k]; j < s.slot0_k[k] + s.nocc_k[k]; ++j) mk_[j] = 1;
      const CgOut ok = run_cg<double>(s, s.w64, w.r.get(), mk_, tol_slot, min_iter, max_iter,
                                      dMq, Mq_max, dMcg, any_warm);
      o64.n_ham += ok.n_ham;
      o64.noconv += ok.noconv;
    }
  } else {
    o64 = run_cg<double>(s, s.w64, w.r.get(), m64, tol_slot, min_iter, max_iter, dMq, Mq_max,
                         dMcg, any_warm);
  }
  res.n_ham64 += o64.n_ham;
  res.noconv = o64.noconv;
  if (n32 > 0) {
    ensure_fp32(s);
    std::vector<int> l32;
    for (int j = 0; j < J; ++j)
      if (m32[j]) l32.push_back(j);
    DBuf<int> dl32;
    dl32.upload(l32, st);
    convert_slots(n32, dl32.get(), s.d_slot_k.get(), s.d_nb.get(), nbm, w.r.get(), s.w32.r.get(), st);
    if (any_warm)
      convert_slots(n32, dl32.get(), s.d_slot_k.get(), s.d_nb.get(), nbm, w.x.get(),
                    s.w32.x.get(), st);
    const CgOut o32 = run_cg<float>(s, s.w32, s.w32.r.get(), m32, tol_slot, min_iter,
                                      max_iter, dMq, Mq_max, dMcg, any_warm);
    convert_slots(n32, dl32.get(), s.d_slot_k.get(), s.d_nb.get(), nbm, s.w32.x.get(), w.x.get(), st);
    res.n_ham32 = o32.n_ham;
    // FP64 check of the FP32 results: the true residual b - A x of every
    // FP32 band whose tolerance is below CHECK_REL ||b_j||, and of every band
    // the FP32 CG did not bring below its tolerance (stalled at the FP32
    // floor, or at the cap; one FP64 H application each).  A band that fails
    // continues in FP64 from its FP32 iterate (defect correction); one that
    // did not converge restarts from zero, as its iterate may be far off.
    if (any_warm)   // the check below forms b - A x from r = b
      IKR_HIP(hipMemcpyAsync(w.r.get(), s.d_rec_tb.get(), (size_t)J * nbm * sizeof(double2),
                             hipMemcpyDeviceToDevice, st));
    const std::vector<float> rn = download(s.w32.rnorm2.get(), J, st);
    std::vector<int> mc(J, 0), mz(J, 0);
    int nc = 0, nz = 0;
    for (int j = 0; j < J; ++j) {
      if (!m32[j]) continue;
      const bool conv = (double)rn[j] <= tol_slot[j] * tol_slot[j];
      if (!conv || tol_slot[j] < CHECK_REL * bn[j]) {
        mc[j] = 1;
        ++nc;
        if (!conv) { mz[j] = 1; ++nz; }
      }
    }
    if (nc > 0) {
      if (nz > 0) {
        std::vector<int> lz;
        for (int j = 0; j < J; ++j)
          if (mz[j]) lz.push_back(j);
        DBuf<int> dlz;
        dlz.upload(lz, st);
        cg_zero<double>(Slots{nz, s.d_slot_k.get(), nullptr, dlz.get()}, nbm, w.x.get(),
                        w.p.get(), st);
        IKR_HIP(hipStreamSynchronize(st));
      }
      IKR_HIP(hipMemcpyAsync(w.w.get(), w.x.get(), (size_t)J * nbm * sizeof(double2),
                             hipMemcpyDeviceToDevice, st));
      apply_sternheimer_op(s, mc, dMq, Mq_max, dMcg);
      // r = b - A x on the checked rows (r still holds b there)
      cg_axpy<double>(Slots{nc, s.d_slot_k.get(), s.d_active.get(), s.d_list.get(),
                            s.d_cnt.get()},
                      s.d_nb.get(), nbm, -1.0, w.w.get(), w.r.get(), st);
      res.n_ham64 += nc;
      res.checked += nc;
      const std::vector<double> rt = slot_norms(s, w.r.get());
      std::vector<int> mf(J, 0);
      int nf = 0;
      for (int j = 0; j < J; ++j)
        if (mc[j] && !(rt[j] <= tol_slot[j])) { mf[j] = 1; ++nf; }
      if (nf > 0) {
        const CgOut of = run_cg<double>(s, s.w64, w.r.get(), mf, tol_slot, min_iter, max_iter,
                                        dMq, Mq_max, dMcg, /*keep_x=*/true);
        res.n_ham64 += of.n_ham;
        res.noconv += of.noconv;
        res.fallback += nf;
      }
    }
  }
  res.n_ham = res.n_ham64 + res.n_ham32;
  if (L > 0) {   // keep this right-hand side and solution (the oldest pair goes)
    const int pos = s.rec_head, nv = s.rec_count;
    const size_t vs = (size_t)J * nbm;
    IKR_HIP(hipMemcpyAsync(s.d_rec_b.get() + pos * vs, s.d_rec_tb.get(), vs * sizeof(double2),
                           hipMemcpyDeviceToDevice, st));
    IKR_HIP(hipMemcpyAsync(s.d_rec_x.get() + pos * vs, w.x.get(), vs * sizeof(double2),
                           hipMemcpyDeviceToDevice, st));
    for (int j = 0; j < J; ++j) {
      double2* G = s.rec_G.data() + (size_t)j * L * L;
      for (int l = 0; l < nv; ++l) {
        if (l == pos) continue;
        const double2 h = hdot[(size_t)j * nv + l];        // <b_l, b_new>
        G[l * L + pos] = h;
        G[pos * L + l] = mk<double>(h.x, -h.y);
      }
      G[pos * L + pos] = mk<double>(bn[j] * bn[j], 0);
    }
    s.rec_head = (pos + 1) % L;
    s.rec_count = std::min(nv + 1, L);
  }
  UpdTerm<double> phiA{s.d_phi.get(), phik, nbm, dMq, w.coefA.get(), MAXM, -1.0, Mq_max};
  const double S16 = 16.0;
  double ncol_avg = 0;
  for (int j = 0; j < J; ++j) ncol_avg += s.kp[s.slot_k[j]].ncol;
  ncol_avg /= J;
  const double colC = ncol_avg * s.L.C;

  // final projection and occupied part: dphi = x - Phi Phi^H x + Phi dP
  gram<double>(s.tiles, s.d_nb.get(), nbm, dMq, Mq_max, s.d_phi.get(), phik,
               nbm, w.x.get(), nbm, w.part.get(), w.coefA.get(), MAXM, st, nullptr, s.krange());
  IKR_HIP(hipMemcpyAsync(w.coefB.get(), dp.data(), dp.size() * sizeof(double2),
                         hipMemcpyHostToDevice, st));
  UpdTerm<double> phiB{s.d_phi.get(), phik, nbm, dMq, w.coefB.get(), MAXM, 1.0, Mq_max};
  update<double>(s.tiles, s.d_nb.get(), nbm, nullptr, w.x.get(), nbm, 1.0, phiA, phiB, nullptr,
                 nullptr, st);
  if (ex && ex->dphi_out)
    IKR_HIP(hipMemcpyAsync(ex->dphi_out, w.x.get(), (size_t)J * nbm * sizeof(double2),
                           hipMemcpyDeviceToDevice, st));
  if (!drho_int) {
    IKR_HIP(hipStreamSynchronize(st));
    return res;
  }

  // drho = sum_k w_k sum_n 2 f Re(conj psi dpsi) + df |psi|^2
  launch_col_inv<double>(s.geom, s.fft, all, w.x.get(), nbm, w.T1.get(), nullptr, nullptr,
                         nullptr, st);
  std::vector<double> wa(J), wb(J);
  for (int j = 0; j < J; ++j) {
    const int k = s.slot_k[j];
    wa[j] = 2.0 * s.kp[k].weight * s.occ[(size_t)k * nbn + s.slot_n[j]] / s.volume;
    wb[j] = s.kp[k].weight * df[j] / s.volume;
  }
  IKR_HIP(hipMemcpyAsync(s.d_wa.get(), wa.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
  IKR_HIP(hipMemcpyAsync(s.d_wb.get(), wb.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
  const int gsz = 8;
  KTimer::begin(K_PLANE_RHO, st);
  launch_plane_rho(s.geom, s.fft, J, s.d_slot_k.get(), s.d_Tphi.get(), w.T1.get(), s.d_wa.get(),
                   s.d_wb.get(), gsz, s.d_rhopart.get(), st);
  KTimer::end(K_PLANE_RHO, st, J * 2.0 * colC * S16 + (J + gsz - 1) / gsz * 8.0 * s.ng);
  sum_groups(s.ng, (J + gsz - 1) / gsz, s.d_rhopart.get(), 1.0, drho_int, st);
  IKR_HIP(hipStreamSynchronize(st));
  return res;
}

// ---------------------------------------------------------------- tolerances
// Prefactor of Table 1 in its k-point form (Table strategies_k, with the
// per-k occupied counts replaced by the total N_occ as in the paper's runs).
static std::vector<double> prefactors(const System& s, int strategy, double knorm,
                                      double bnorm, bool schur) {
  std::vector<double> p(s.J, 1.0);
  for (int j = 0; j < s.J; ++j) {
    const int k = s.slot_k[j], n = s.slot_n[j], no = s.nocc_k[k];
    host::BandTolInputs a;
    a.volume = s.volume;
    a.ng = (double)s.ng;
    a.nocc_tot = s.J;
    a.f = s.occ[(size_t)k * s.nbands + n];
    a.wk = s.kp[k].weight;
    a.knorm = knorm;
    a.orbnorm = s.orbnorm_k[k];
    a.orbnorm_full = s.orbnorm_full_k[k];
    a.nk = s.nk;
    a.nocc_k = no;
    a.bnorm = bnorm;
    if (strategy == IKR_THM2) {
      // where every computed band is occupied the gap is taken to the highest
      // computed band (>= 1e-4 Ha); with the extra bands taken by sum over
      // states the CG operator's smallest eigenvalue is e_{nbands+1} - e_n >=
      // e_{nbands} - e_n
      const double en = s.eps[(size_t)k * s.nbands + n];
      const bool above = no < s.nbands && !schur;
      const double eup = s.eps[(size_t)k * s.nbands + (above ? no : s.nbands - 1)];
      a.gap = std::max(eup - en, above ? 0.0 : 1e-4);
    }
    p[j] = host::band_prefactor(strategy, a);
  }
  return p;
}

// ---------------------------------------------------------------- E v
// Euclidean norm of a grid vector (fixed-order reduction).
static double grid_norm(System& s, const double* v) {
  const int nbl = multidot_nblocks(s.ng);
  multidot(s.ng, 1, v, s.ng, v, s.d_multi.get(), s.stream);
  const std::vector<double> h = download(s.d_multi.get(), nbl, s.stream);
  double a = 0;
  for (double x : h) a += x;
  return std::sqrt(a);
}

// Rejects a non-finite chi0 result with what went into it.
static void check_finite_response(System& s, const Chi0Result& r, const std::vector<double>& tol) {
  const double nr = grid_norm(s, s.d_drho.get());
  if (std::isfinite(nr)) return;
  double tmin = 1e300, tmax = 0;
  for (double t : tol) { tmin = std::min(tmin, t); tmax = std::max(tmax, t); }
  char msg[256];
  std::snprintf(msg, sizeof msg,
                "non-finite chi0 response (H applications FP64 %lld, FP32 %lld, unconverged %d, "
                "CG tolerances %.2e..%.2e)",
                r.n_ham64, r.n_ham32, r.noconv, tmin, tmax);
  throw Error(5, msg);
}

void apply_dielectric_ext(System& s, const double* v_ext, double* ev_ext, double common,
                          const ikr_solver_opts& o, double bnorm, ikr_stats* stt) {
  const hipStream_t st = s.stream;
  to_internal(s.L, v_ext, s.d_tmpg.get(), st);
  const double nu = apply_kernel(s, s.d_tmpg.get(), s.d_u.get());
  IKR_CHECK(std::isfinite(nu), 5, "non-finite input: ||K v|| is not finite");
  s.knorm_hist.push_back(nu);
  if (stt) stt->knorm_last = nu;
  if (nu == 0.0) {
    IKR_HIP(hipMemcpyAsync(ev_ext, v_ext, s.ng * sizeof(double), hipMemcpyDeviceToDevice, st));
    IKR_HIP(hipStreamSynchronize(st));
    return;
  }
  scale_copy(s.ng, s.d_u.get(), 1.0 / nu, s.d_u.get(), st);
  std::vector<double> tol = prefactors(s, o.strategy, nu, bnorm,
                                       o.schur && s.nbands > s.nocc_max);
  for (double& t : tol) t *= common;
  Chi0Result r = apply_chi0_internal(s, s.d_u.get(), s.d_drho.get(), tol, o.cg_min_iter,
                                     o.cg_max_iter, o.precision, o.fp32_theta, o.schur);
  if (stt) {
    stt->n_ham += r.n_ham;
    stt->n_ham_fp64 += r.n_ham64;
    stt->n_ham_fp32 += r.n_ham32;
    stt->cg_unconverged += r.noconv;
    stt->fp64_fallback += r.fallback;
    stt->fp32_checked += r.checked;
    stt->warm_started += r.warm;
  }
  check_finite_response(s, r, tol);
  to_external(s.L, s.d_drho.get(), ev_ext, -nu, v_ext, 1.0, st);
  IKR_HIP(hipStreamSynchronize(st));
}

// ev = E~^T v = v - ||v|| K chi0~(v / ||v||).  K and chi0 are symmetric in
// the grid inner product, so the transpose of E = 1 - chi0 K is 1 - K chi0.
// The CG error enters through K, bounded by ||K||_2 ||v|| ||(chi0 - chi0~) v^||,
// so the strategies that use ||K v_i|| take ||K||_2 ||v_i|| instead.
void apply_dielectric_adjoint_ext(System& s, const double* v_ext, double* ev_ext,
                                  double common, const ikr_solver_opts& o, double bnorm,
                                  ikr_stats* stt) {
  const hipStream_t st = s.stream;
  const double nu = grid_norm(s, v_ext);
  IKR_CHECK(std::isfinite(nu), 5, "non-finite input: ||v|| is not finite");
  if (stt) stt->knorm_last = nu;
  if (nu == 0.0) {
    IKR_HIP(hipMemcpyAsync(ev_ext, v_ext, s.ng * sizeof(double), hipMemcpyDeviceToDevice, st));
    IKR_HIP(hipStreamSynchronize(st));
    return;
  }
  to_internal(s.L, v_ext, s.d_tmpg.get(), st);
  scale_copy(s.ng, s.d_tmpg.get(), 1.0 / nu, s.d_u.get(), st);
  std::vector<double> tol = prefactors(s, o.strategy, s.knorm_bound * nu, bnorm,
                                       o.schur && s.nbands > s.nocc_max);
  for (double& t : tol) t *= common;
  Chi0Result r = apply_chi0_internal(s, s.d_u.get(), s.d_drho.get(), tol, o.cg_min_iter,
                                     o.cg_max_iter, o.precision, o.fp32_theta, o.schur);
  if (stt) {
    stt->n_ham += r.n_ham;
    stt->n_ham_fp64 += r.n_ham64;
    stt->n_ham_fp32 += r.n_ham32;
    stt->cg_unconverged += r.noconv;
    stt->fp64_fallback += r.fallback;
    stt->fp32_checked += r.checked;
    stt->warm_started += r.warm;
  }
  check_finite_response(s, r, tol);
  apply_kernel(s, s.d_drho.get(), s.d_u.get());
  to_external(s.L, s.d_u.get(), ev_ext, -nu, v_ext, 1.0, st);
  IKR_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- Kerker
// T v = W^-1 (D + (1 - D_11) e_1 e_1^T) W v (eq. kerker and the proof of
// Lemma kerker_properties): the symbol |G|^2 / (|G|^2 + alpha^2) with the
// G = 0 entry set to 1, applied by the density-grid FFT pair of the Hxc
// kernel.
void apply_kerker_ext(System& s, double alpha, const double* v_ext, double* out_ext) {
  const hipStream_t st = s.stream;
  if (s.kerker_alpha != alpha || !s.d_kerker.get()) {
    const int C = s.L.C, P = s.L.P, Q = s.L.Q;
    std::vector<double> d((size_t)s.ng);
    for (int c = 0; c < C; ++c)
      for (int p = 0; p < P; ++p)
        for (int q = 0; q < Q; ++q) {
          const int cs = c < C / 2 ? c : c - C, ps = p < P / 2 ? p : p - P,
                    qs = q < Q / 2 ? q : q - Q;
          const double gc = cs * s.b[s.cax], gp = ps * s.b[s.pax], gq = qs * s.b[s.qax];
          const double gg = gc * gc + gp * gp + gq * gq;
          d[((size_t)c * P + p) * Q + q] = gg > 0 ? gg / (gg + alpha * alpha) : 1.0;
        }
    s.d_kerker.upload(d, st);
    s.kerker_alpha = alpha;
  }
  to_internal(s.L, v_ext, s.d_tmpg.get(), st);
  launch_kernel_apply(s.geom, s.fft, s.d_tmpg.get(), s.d_kerker.get(), nullptr, s.d_u.get(),
                      s.d_kw1.get(), s.d_kw2.get(), s.d_kpart.get(), st);
  to_external(s.L, s.d_u.get(), out_ext, 1.0, nullptr, 0.0, st);
}

// ---------------------------------------------------------------- Alg. 1
// Inexact GMRES(m) on E (adjoint = false) or on E^T (adjoint = true).
//
// With o.kerker the system is T E x = T b (eq. precond_dyson): every operator
// application is followed by T, and the right-hand side is T b; tau (taken
// relative to ||b|| when tol_is_relative) then bounds ||T (b - E x)||, which
// Theorem 2 still controls as ||T|| = 1.  With o.x0 the iteration starts from
// x0 (Alg. 1, first line, at tolerance tau/3).
void solve_response(System& s, const double* b_ext, double* x_ext, const ikr_solver_opts& o,
                    ikr_stats* stt, bool adjoint) {
  const bool kerker = o.kerker != 0;
  IKR_CHECK(!(kerker && adjoint), 1, "Kerker preconditioning is for forward solves only");
  s.rec_count = s.rec_head = 0;   // warm starts only from this solve's own applications
  auto apply_op = [&](const double* v, double* ev, double common, double bn, ikr_stats* sp) {
    if (adjoint) apply_dielectric_adjoint_ext(s, v, ev, common, o, bn, sp);
    else apply_dielectric_ext(s, v, ev, common, o, bn, sp);
    if (kerker) apply_kerker_ext(s, o.kerker_alpha, ev, ev);
  };
  const auto t0 = std::chrono::steady_clock::now();
  const hipStream_t st = s.stream;
  const int n = s.ng, m = o.restart_m;
  IKR_CHECK(m >= 1 && m <= 60, 1, "restart size out of range");
  const bool adaptive = o.strategy == IKR_AGR || o.strategy == IKR_BAL ||
                        o.strategy == IKR_GRT || o.strategy == IKR_THM2;
  DBuf<double> V, coef, part, tmp;
  V.alloc((size_t)(m + 1) * n);
  coef.alloc(64);
  const int nbl = multidot_nblocks(n);
  part.alloc((size_t)(m + 1) * nbl);
  tmp.alloc(n);

  auto dots = [&](int nv, const double* Vp, const double* w) {
    multidot(n, nv, Vp, n, w, part.get(), st);
    const std::vector<double> h = download(part.get(), (size_t)nv * nbl, st);
    std::vector<double> out(nv, 0.0);
    for (int j = 0; j < nv; ++j)
      for (int b = 0; b < nbl; ++b) out[j] += h[(size_t)j * nbl + b];
    return out;
  };
  auto axpy = [&](int nv, const double* Vp, const std::vector<double>& c, double a, double* y) {
    IKR_HIP(hipMemcpyAsync(coef.get(), c.data(), nv * sizeof(double), hipMemcpyHostToDevice, st));
    IKR_HIP(hipStreamSynchronize(st));
    multiaxpy(n, nv, Vp, n, coef.get(), a, y, st);
  };

  const double bnorm = std::sqrt(dots(1, b_ext, b_ext)[0]);
  const double tau = o.tol_is_relative ? o.tol * bnorm : o.tol;
  IKR_CHECK(std::isfinite(bnorm), 5, "non-finite right-hand side");
  bool x0_zero = true;
  if (o.x0) {
    const double x0n = std::sqrt(dots(1, o.x0, o.x0)[0]);
    IKR_CHECK(std::isfinite(x0n), 5, "non-finite initial guess");
    if (o.x0 != x_ext)
      IKR_HIP(hipMemcpyAsync(x_ext, o.x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice,
                             st));
    x0_zero = x0n == 0.0;
  } else {
    IKR_HIP(hipMemsetAsync(x_ext, 0, (size_t)n * sizeof(double), st));
  }
  // right-hand side of the (preconditioned) system
  DBuf<double> tb;
  const double* rhs = b_ext;
  if (kerker) {
    tb.alloc(n);
    apply_kerker_ext(s, o.kerker_alpha, b_ext, tb.get());
    rhs = tb.get();
  }
  double s_est = o.s0;
  int restarts = 0, iters = 0;
  double resid = bnorm;
  std::vector<double> H((size_t)(m + 1) * m);
  bool done = bnorm == 0.0;
  if (done) IKR_HIP(hipMemsetAsync(x_ext, 0, (size_t)n * sizeof(double), st));   // E^-1 0 = 0
  while (!done) {
    // the initial residual r0 = b - E~(0) x0, applied to tolerance tau/3
    double* v0 = V.get();
    if (x0_zero) {
      IKR_HIP(hipMemcpyAsync(v0, rhs, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
      apply_op(x_ext, v0, adaptive ? tau / 3.0 : tau, bnorm, stt);
      axpy(1, rhs, {1.0}, -1.0, v0);
    }
    const double beta = std::sqrt(dots(1, v0, v0)[0]);
    if (beta == 0.0) break;
    scale_copy(n, v0, 1.0 / beta, v0, st);
    std::fill(H.begin(), H.end(), 0.0);
    resid = beta;
    bool conv = false;
    int i_used = 0;
    std::vector<double> y;
    for (int i = 1; i <= m; ++i) {
      const double common = adaptive ? (s_est / (3.0 * m)) * tau / resid : tau;
      double* vi = V.get() + (size_t)i * n;
      apply_op(V.get() + (size_t)(i - 1) * n, vi, common, bnorm, stt);
      ++iters;
      // classical Gram-Schmidt, twice
      std::vector<double> h = dots(i, V.get(), vi);
      std::vector<double> neg(i);
      for (int j = 0; j < i; ++j) neg[j] = -h[j];
      axpy(i, V.get(), neg, 1.0, vi);
      std::vector<double> h2 = dots(i, V.get(), vi);
      for (int j = 0; j < i; ++j) { neg[j] = -h2[j]; h[j] += h2[j]; }
      axpy(i, V.get(), neg, 1.0, vi);
      const double hn = std::sqrt(dots(1, vi, vi)[0]);
      if (!std::isfinite(hn)) {
        char msg[128];
        std::snprintf(msg, sizeof msg, "non-finite Krylov vector at GMRES step %d (restart %d)",
                      iters, restarts);
        throw Error(5, msg);
      }
      for (int j = 0; j < i; ++j) H[(size_t)j * m + (i - 1)] = h[j];
      H[(size_t)i * m + (i - 1)] = hn;
      if (hn > 0) scale_copy(n, vi, 1.0 / hn, vi, st);
      resid = small_ls(H, m, i, beta, y);
      i_used = i;
      if (resid <= tau / 3.0) {
        std::vector<double> Hi((size_t)(i + 1) * i);
        for (int a = 0; a <= i; ++a)
          for (int c = 0; c < i; ++c) Hi[(size_t)a * i + c] = H[(size_t)a * m + c];
        const double sig = sigma_min(Hi, i + 1, i);
        axpy(i, V.get(), y, 1.0, x_ext);
        x0_zero = false;
        if (stt) stt->sigma_min = sig;
        if (s_est <= sig) { done = true; conv = true; break; }
        s_est = sig;            // restart with s = sigma_i(H_i)
        conv = true;
        break;
      }
      if (hn == 0.0) break;     // exact invariant subspace
    }
    if (!conv) {
      std::vector<double> Hm((size_t)(i_used + 1) * i_used);
      for (int a = 0; a <= i_used; ++a)
        for (int c = 0; c < i_used; ++c) Hm[(size_t)a * i_used + c] = H[(size_t)a * m + c];
      const double sig = sigma_min(Hm, i_used + 1, i_used);
      axpy(i_used, V.get(), y, 1.0, x_ext);
      x0_zero = false;
      s_est = sig;
      if (stt) stt->sigma_min = sig;
    }
    if (done) break;
    if (++restarts > o.max_restarts) {
      if (stt) { stt->restarts = restarts; stt->gmres_iters = iters; }
      throw Error(4, "GMRES restart cap reached");
    }
  }
  if (stt) {
    stt->gmres_iters = iters;
    stt->restarts = restarts;
    stt->est_res = resid;
    stt->s_final = s_est;
    stt->true_res = -1;
  }
  if (o.want_true_residual && stt) {
    ikr_solver_opts ot = o;
    ot.strategy = IKR_FIXED;
    ikr_stats dummy{};
    const int rec = s.cg_recycle;   // the check starts every CG from zero
    s.cg_recycle = 0;
    if (adjoint) apply_dielectric_adjoint_ext(s, x_ext, tmp.get(), o.true_res_cg_tol, ot, bnorm, &dummy);
    else apply_dielectric_ext(s, x_ext, tmp.get(), o.true_res_cg_tol, ot, bnorm, &dummy);
    s.cg_recycle = rec;
    axpy(1, b_ext, {1.0}, -1.0, tmp.get());
    stt->true_res = std::sqrt(dots(1, tmp.get(), tmp.get())[0]);
  }
  IKR_HIP(hipStreamSynchronize(st));
  if (stt)
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace ikr
