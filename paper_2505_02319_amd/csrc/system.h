// Host-side state of one response system (opaque ikr_handle).
#pragma once

#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/ikr.h"
#include "blas.h"
#include "common.h"

namespace ikr {

// Owning device buffer.
template <typename T> struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { if (p) (void)hipFree(p); }
  void alloc(size_t count) {
    if (p) { (void)hipFree(p); p = nullptr; }
    n = count;
    if (count) IKR_HIP(hipMalloc(&p, count * sizeof(T)));
  }
  // Copies from pageable host memory complete before returning, so the
  // source vector may be released right after the call.
  void upload(const std::vector<T>& h, hipStream_t st) {
    alloc(h.size());
    if (n) {
      IKR_HIP(hipMemcpyAsync(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
      IKR_HIP(hipStreamSynchronize(st));
    }
  }
  T* get() const { return p; }
};

struct KPoint {
  double kfrac[3];
  double kcart[3];
  double weight;
  int nb = 0;
  int ncol = 0;
  std::vector<int> miller;   // [nb][3] external axes
  std::vector<double> kin;   // [nb]
  std::vector<int> col_start, col_pq, col_clo;
};

// Per-precision Sternheimer CG work space.
template <typename R> struct CgWork {
  DBuf<cplx<R>> x, r, p, w, T1, T2, coefA, coefB, part;
  DBuf<R> rz, alpha, beta, rnorm2, dpart, pshift, shift, rbest;
  DBuf<cplx<R>> phi, proj;     // copies of Phi / projectors in this precision
  DBuf<R> vloc;
  // fused CG projections: W_k = [projectors | phi_1, H phi_1, phi_2, ...]
  // ([nk][mcg][nb_max]), G^T and S^T ([nk][nbands][nbands]), raw gram
  // coefficients and update coefficients ([J][mcg]), |r|^2 and <r, z> partials
  DBuf<cplx<R>> wcg, gT, sT, craw, gam;
  DBuf<R> rpart, zpart;
};

// Page-locked host memory (for asynchronous device-to-host copies).
template <typename T> struct HBuf {
  T* p = nullptr;
  HBuf() = default;
  HBuf(const HBuf&) = delete;
  HBuf& operator=(const HBuf&) = delete;
  ~HBuf() { if (p) (void)hipHostFree(p); }
  void alloc(size_t count, unsigned flags = hipHostMallocDefault) {
    if (p) { (void)hipHostFree(p); p = nullptr; }
    if (count) IKR_HIP(hipHostMalloc((void**)&p, count * sizeof(T), flags));
  }
};

// Executable HIP graphs of one Sternheimer CG iteration, keyed by precision
// and grid bounds, and the private stream they are captured and replayed on
// (a caller's stream may be the legacy default stream, which cannot capture).
struct CgGraphs {
  using Key = std::array<long long, 7>;
  hipStream_t stream = nullptr;
  std::map<Key, hipGraphExec_t> exec;
  long long captures = 0;
  CgGraphs() = default;
  CgGraphs(const CgGraphs&) = delete;
  CgGraphs& operator=(const CgGraphs&) = delete;
  ~CgGraphs() {
    clear();
    if (stream) (void)hipStreamDestroy(stream);
  }
  void clear() {
    for (auto& e : exec) (void)hipGraphExecDestroy(e.second);
    exec.clear();
  }
  hipStream_t get_stream() {
    if (!stream) IKR_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    return stream;
  }
  // The cached graph for key, else one captured from record() on st.
  template <typename F> hipGraphExec_t get(const Key& key, hipStream_t st, F&& record) {
    const auto it = exec.find(key);
    if (it != exec.end()) return it->second;
    hipGraph_t g = nullptr;
    IKR_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      record();
    } catch (...) {
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    IKR_HIP(hipStreamEndCapture(st, &g));
    hipGraphExec_t ge = nullptr;
    const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    IKR_HIP(e);
    exec.emplace(key, ge);
    ++captures;
    return ge;
  }
};

struct System {
  // model
  double a[3], b[3], volume = 0;
  int N[3], ng = 0;
  int natoms = 0;
  std::vector<double> pos, amp;   // cartesian [natoms][3]
  double sigma_loc = 0, sigma_proj = 0, dnl = 0, ecut = 0, temperature = 0;
  int kgrid[3];
  int nocc = 0, nextra = 0, nbands = 0, xc = 0;
  hipStream_t stream = nullptr;
  int device = 0;                  // device current at setup

  // layout
  int cax = 0, pax = 1, qax = 2;
  Layout L{};
  Geom geom{};
  FftTables fft{};
  DBuf<double2> tw64;
  DBuf<float2> tw32;

  // k-points and spheres
  int nk = 0, nb_max = 0, ncol_max = 0;
  std::vector<KPoint> kp;
  DBuf<int> d_nb, d_ncol, d_col_start, d_col_pq, d_col_clo, d_prow, d_nprow;
  DBuf<double> d_kin;
  DBuf<double> d_vloc;             // internal layout
  DBuf<double2> d_proj;            // [nk][natoms][nb_max]

  // ground state
  bool have_gs = false;
  int gs_outer_iters = 0;          // eigensolver outer steps (0 if imported)
  double gs_residual = 0;          // largest eigen-residual norm at exit
  std::vector<double> eps, occ, docc;   // [nk][nbands]
  double fermi = 0;
  std::vector<int> nocc_k;
  std::vector<double> gap_k;
  DBuf<double2> d_phi;             // [nk][nbands][nb_max]

  // occupied slots and tiles
  int J = 0;
  std::vector<int> slot_k, slot_n, slot0_k;   // slot0_k: first slot of each k
  DBuf<int> d_slot_k, d_nocc_k, d_natoms_k, d_nbands_k;
  std::vector<int> tile_k, tile_slot0, tile_nb;
  DBuf<int> d_tile_k, d_tile_slot0, d_tile_nb;
  Tiles tiles{};
  int nocc_max = 0;
  DBuf<int> d_kt0;                 // [nk + 1] first tile of each k in `tiles`
  DBuf<int> d_ktb;                 // [nk + 1] the same for the compacted active tiles
  int ktmax = 0;                   // most tiles of one k
  KTileRange krange() const { return KTileRange{nk, d_kt0.get(), ktmax}; }
  KTileRange krange_compact() const { return KTileRange{nk, d_ktb.get(), ktmax}; }

  // caches
  DBuf<double2> d_Tphi;            // [J][C][ncol_max] column transforms of occupied phi
  DBuf<double> d_rho, d_fx, d_khat;   // internal layout
  DBuf<double> d_kerker;           // Kerker symbol with G = 0 -> 1 (internal layout)
  double kerker_alpha = -1;        // alpha d_kerker was built for
  std::vector<double> orbnorm_k;   // ||Re F_k^-1 Phi_k||_{2,inf}
  std::vector<double> orbnorm_full_k;  // ||F_k^-1 Phi_k||_{2,inf}
  double knorm_bound = 0;          // ||K||_2 <= max 4 pi / |G|^2 + max |f_x|

  // work
  CgWork<double> w64;
  CgWork<float> w32;
  DBuf<double> d_u, d_drho, d_tmpg, d_kpart, d_rhopart, d_wa, d_wb, d_multi;
  DBuf<double2> d_kw1, d_kw2;
  DBuf<int> d_active, d_iters, d_counters, d_rlast;
  DBuf<int> d_list, d_ctk, d_cto, d_ctn;   // compact active slots and their tiles
  DBuf<int> d_slot0_k;             // first slot of each k
  int mcg = 0;                     // rows of W_k: natoms + 2 nbands
  DBuf<int> d_mcg_occ, d_mcg_all;  // rows used per k: natoms + 2 nocc_k / + 2 nbands
  DBuf<int> d_cnt, d_hist;         // live counts of the compaction, per-iteration history
  HBuf<int> h_cnt;                 // [2][CNT_STRIDE] lagged copies of d_cnt (coherent pinned memory)
  int* d_hcnt = nullptr;           // h_cnt as a device address: the compaction writes it
  std::vector<double> dvloc;       // [natoms][ng] dV_loc/dA_a, internal layout (lazy)
  DBuf<double> d_tol2;
  std::vector<double> knorm_hist;
  int cg_graph = 0;                // 1: CG iterations replayed from captured graphs
  int cg_plain = 0;                // 1: plain FP64 reference: one k-point per CG run,
                                   //    the host reads the live count every iteration
  // Sternheimer warm starts: ring of the last rec_cap right-hand sides and CG
  // solutions per slot ([rec_cap][J][nb_max]), the Gram matrices of the stored
  // right-hand sides per slot ([J][rec_cap][rec_cap], host)
  int cg_recycle = 0;              // capacity asked for by the current call (0: off)
  int rec_cap = 0, rec_count = 0, rec_head = 0;
  DBuf<double2> d_rec_b, d_rec_x, d_rec_tb, d_rec_part, d_rec_h, d_rec_c;
  DBuf<int> d_rec_list;
  std::vector<double2> rec_G;
  CgGraphs graphs;
  // Launch shapes of the CG iteration, measured at the first CG run that
  // needs them: [precision: 0 FP64, 1 FP32][batch: 0 more tiles than
  // k-points, 1 at most one tile per k-point on average]
  KernelTune tune[2][2];
  bool tuned[2][2] = {{false, false}, {false, false}};
  double tune_us[2][2][3] = {};    // measured times of the picks (gram, update, plane)

  std::string name;
};

// noalloc.hip: the no-allocation work space (one fixed device array per GPU)
void init_scratch(int device);
void apply_hamiltonian_noalloc(System& s, int k, int nvec, const double2* x, double2* y);

// setup.cpp
System* create_system(const ikr_system_desc* d, hipStream_t st);
void import_ground_state(System& s, const double* eps, const double* coeffs);
void finish_setup(System& s);

// groundstate.cpp
void compute_ground_state(System& s);

// solver.cpp
// Work space of one Hamiltonian application to nvec vectors of one k-point:
// slot and tile tables, the two column buffers of the pruned FFT, projector
// coefficients and gram partials, carved from one block of device memory.
struct HamWork {
  int *sk = nullptr, *tk = nullptr, *ts = nullptr, *tn = nullptr;
  double2 *T1 = nullptr, *T2 = nullptr, *coef = nullptr, *part = nullptr;
  static size_t bytes(const System& s, int nvec);
  void carve(const System& s, int nvec, unsigned char* base);
};
void apply_hamiltonian(System& s, int k, int nvec, const double2* x, double2* y);
// The same with a caller-provided work space whose tables are already filled;
// enqueues only (no synchronisation).
void apply_hamiltonian_ws(System& s, int k, int nvec, const double2* x, double2* y,
                          const HamWork& w);
double apply_kernel(System& s, const double* v_int, double* kv_int);
struct Chi0Result {
  long long n_ham = 0, n_ham32 = 0, n_ham64 = 0;
  int noconv = 0;
  int warm = 0;         // Sternheimer solves warm-started from earlier solutions
  int fallback = 0;     // FP32 bands continued in FP64 (true residual above tolerance)
  int checked = 0;      // FP32 bands whose true residual was checked in FP64
};
// Optional inputs/outputs of the chi0 path beyond the density.
struct Chi0Extra {
  const double2* rhs_pw = nullptr;     // t_j [J][nb_max] instead of F(u psi_j)
  double2* dphi_out = nullptr;         // delta phi_j [J][nb_max] (device copy)
  std::vector<double2>* m_out = nullptr;   // M[j][m] = <phi_m, t_j> (host, stride MAXM)
  bool tol_relative = false;           // tolerances scale with ||b_j||
};
Chi0Result apply_chi0_internal(System& s, const double* u_int, double* drho_int,
                               const std::vector<double>& tol_slot, int min_iter,
                               int max_iter, int precision = 0, double theta = 1e-5,
                               int schur = 0, const Chi0Extra* ex = nullptr);
// dL/dA for every atom from drho = E^-1 b and lambda = E^-T dL/d(drho)
// (fixed occupations only), CG tolerances relative to each right-hand side.
std::vector<double> grad_amplitudes(System& s, const double* drho_ext, const double* lam_ext,
                                    double cg_tol, ikr_stats* st);
void ensure_fp32(System& s);   // FP32 work space and operator copies (lazy)
// Measures the CG launch shapes now (FP64, and FP32 too when precision != 0)
// for the projection rows of the schur option, where not measured yet.
void tune_launches_now(System& s, int precision, int schur);
// out = T v (Kerker, eq. kerker), grid vectors in the external layout (may alias)
void apply_kerker_ext(System& s, double alpha, const double* v_ext, double* out_ext);
// b = chi0 dV0 for the displacement of one atom (local and nonlocal parts)
Chi0Result displacement_rhs(System& s, int atom, int dir, double cg_tol, double* dv0_ext,
                            double* b_ext);
void apply_dielectric_ext(System& s, const double* v_ext, double* ev_ext,
                          double common, const ikr_solver_opts& o, double bnorm,
                          ikr_stats* st);
void apply_dielectric_adjoint_ext(System& s, const double* v_ext, double* ev_ext,
                                  double common, const ikr_solver_opts& o, double bnorm,
                                  ikr_stats* st);
void solve_response(System& s, const double* b_ext, double* x_ext,
                    const ikr_solver_opts& o, ikr_stats* st, bool adjoint = false);

}  // namespace ikr
