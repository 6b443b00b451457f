// System setup: plane-wave spheres (paper eq. fourier_bases, k-point form of
// Sec. 4.1.1), grid layout for the pruned transforms, local potential and
// projectors of the model, occupations, density and per-band caches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>

#include "cg.h"
#include "hostmath.h"
#include "system.h"

namespace ikr {

bool plane_supported(int P, int Q);

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double EPS_OCC = 1e-10;    // occupied when f > EPS_OCC

int fold(int i, int n) { return i < 0 ? i + n : i; }

using host::focc;
using host::focc_dx;

}  // namespace

System* create_system(const ikr_system_desc* d, hipStream_t st) {
  IKR_CHECK(d, 1, "null system description");
  for (int i = 0; i < 3; ++i) {
    IKR_CHECK(d->lattice[i] > 0 && std::isfinite(d->lattice[i]), 1, "lattice must be positive");
    IKR_CHECK(fft_length_supported(d->fft[i]), 1,
              "unsupported FFT length " + std::to_string(d->fft[i]));
    IKR_CHECK(d->kgrid[i] >= 1 && d->kgrid[i] <= 64, 1, "kgrid entries must be in [1, 64]");
  }
  IKR_CHECK(d->natoms >= 0 && d->natoms <= MAXM / 2, 1, "natoms out of range");
  IKR_CHECK(d->natoms == 0 || (d->frac_pos && d->amp), 1, "null atom arrays");
  IKR_CHECK(d->sigma_loc > 0 && d->sigma_proj > 0, 1, "widths must be positive");
  IKR_CHECK(d->ecut > 0, 1, "ecut must be positive");
  IKR_CHECK(d->nocc >= 1 && d->nextra >= 0, 1, "bad band counts");
  IKR_CHECK(d->nocc + d->nextra <= MAXM - 1, 1, "too many bands");
  IKR_CHECK(d->temperature >= 0, 1, "negative temperature");

  std::unique_ptr<System> sp(new System());
  System& s = *sp;
  s.stream = st;
  IKR_HIP(hipGetDevice(&s.device));
  init_scratch(s.device);
  for (int i = 0; i < 3; ++i) {
    s.a[i] = d->lattice[i];
    s.b[i] = 2.0 * PI / d->lattice[i];
    s.N[i] = d->fft[i];
    s.kgrid[i] = d->kgrid[i];
  }
  s.volume = s.a[0] * s.a[1] * s.a[2];
  s.ng = s.N[0] * s.N[1] * s.N[2];
  s.natoms = d->natoms;
  s.pos.resize(3 * s.natoms);
  s.amp.assign(d->amp, d->amp + s.natoms);
  for (int a = 0; a < s.natoms; ++a)
    for (int i = 0; i < 3; ++i) s.pos[3 * a + i] = d->frac_pos[3 * a + i] * s.a[i];
  s.sigma_loc = d->sigma_loc;
  s.sigma_proj = d->sigma_proj;
  s.dnl = d->d_proj;
  s.ecut = d->ecut;
  s.temperature = d->temperature;
  s.nocc = d->nocc;
  s.nextra = d->nextra;
  s.nbands = d->nocc + d->nextra;
  s.xc = d->xc;

  // -- layout: the longest axis is the column axis, the other two the plane
  s.cax = 0;
  for (int i = 1; i < 3; ++i)
    if (s.N[i] > s.N[s.cax]) s.cax = i;
  int rest[2], nr = 0;
  for (int i = 0; i < 3; ++i)
    if (i != s.cax) rest[nr++] = i;
  s.pax = rest[0];
  s.qax = rest[1];
  const int stride[3] = {s.N[1] * s.N[2], s.N[2], 1};
  s.L = Layout{s.N[s.cax], s.N[s.pax], s.N[s.qax], stride[s.cax], stride[s.pax], stride[s.qax]};
  const int C = s.L.C, P = s.L.P, Q = s.L.Q;
  IKR_CHECK(plane_supported(P, Q), 1,
            "unsupported FFT plane " + std::to_string(P) + "x" + std::to_string(Q));

  // -- k-points: Gamma-centred grid folded into [-1/2, 1/2)
  s.nk = s.kgrid[0] * s.kgrid[1] * s.kgrid[2];
  s.kp.resize(s.nk);
  int ik = 0;
  for (int i = 0; i < s.kgrid[0]; ++i)
    for (int j = 0; j < s.kgrid[1]; ++j)
      for (int l = 0; l < s.kgrid[2]; ++l, ++ik) {
        KPoint& K = s.kp[ik];
        const int idx[3] = {i, j, l};
        for (int x = 0; x < 3; ++x) {
          double f = double(idx[x]) / s.kgrid[x];
          if (f >= 0.5) f -= 1.0;
          K.kfrac[x] = f;
          K.kcart[x] = f * s.b[x];
        }
        K.weight = 1.0 / s.nk;
      }

  // -- spheres, ordered column by column (columns along the c axis)
  const double two_ecut = 2.0 * s.ecut;
  for (KPoint& K : s.kp) {
    K.col_start.push_back(0);
    for (int ps = -P / 2; ps < P / 2; ++ps)
      for (int qs = -Q / 2; qs < Q / 2; ++qs) {
        int first = 0, count = 0;
        for (int cs = -C / 2; cs < C / 2; ++cs) {
          int m[3];
          m[s.cax] = cs;
          m[s.pax] = ps;
          m[s.qax] = qs;
          const double q0 = m[0] * s.b[0] + K.kcart[0];
          const double q1 = m[1] * s.b[1] + K.kcart[1];
          const double q2 = m[2] * s.b[2] + K.kcart[2];
          const double qq = q0 * q0 + q1 * q1 + q2 * q2;
          if (qq <= two_ecut) {
            IKR_CHECK(count == 0 || first + count == cs, 8, "sphere column not contiguous");
            if (count == 0) first = cs;
            ++count;
            K.miller.insert(K.miller.end(), {m[0], m[1], m[2]});
            K.kin.push_back(0.5 * qq);
          }
        }
        if (count) {
          K.col_pq.push_back(fold(ps, P) * Q + fold(qs, Q));
          K.col_clo.push_back(first);
          K.col_start.push_back(K.col_start.back() + count);
        }
      }
    K.nb = (int)K.kin.size();
    K.ncol = (int)K.col_pq.size();
    IKR_CHECK(K.nb > s.nbands, 1, "plane-wave sphere smaller than the band count");
    s.nb_max = std::max(s.nb_max, K.nb);
    s.ncol_max = std::max(s.ncol_max, K.ncol);
  }
  {
    std::vector<int> nb(s.nk), ncol(s.nk), cst((size_t)s.nk * (s.ncol_max + 1)),
        cpq((size_t)s.nk * s.ncol_max, 0), clo((size_t)s.nk * s.ncol_max, 0);
    std::vector<double> kin((size_t)s.nk * s.nb_max, 0.0);
    for (int k = 0; k < s.nk; ++k) {
      const KPoint& K = s.kp[k];
      nb[k] = K.nb;
      ncol[k] = K.ncol;
      for (int c = 0; c <= s.ncol_max; ++c)
        cst[(size_t)k * (s.ncol_max + 1) + c] = K.col_start[std::min(c, K.ncol)];
      for (int c = 0; c < K.ncol; ++c) {
        cpq[(size_t)k * s.ncol_max + c] = K.col_pq[c];
        clo[(size_t)k * s.ncol_max + c] = K.col_clo[c];
      }
      std::copy(K.kin.begin(), K.kin.end(), kin.begin() + (size_t)k * s.nb_max);
    }
    s.d_nb.upload(nb, st);
    s.d_ncol.upload(ncol, st);
    s.d_col_start.upload(cst, st);
    s.d_col_pq.upload(cpq, st);
    s.d_col_clo.upload(clo, st);
    s.d_kin.upload(kin, st);
    // rows of the (P, Q) plane that hold sphere columns, per k
    std::vector<int> prow((size_t)s.nk * P, 0), nprow(s.nk, 0);
    for (int k = 0; k < s.nk; ++k) {
      std::vector<char> has(P, 0);
      for (int pq : s.kp[k].col_pq) has[pq / Q] = 1;
      for (int p = 0; p < P; ++p)
        if (has[p]) prow[(size_t)k * P + nprow[k]++] = p;
    }
    s.d_prow.upload(prow, st);
    s.d_nprow.upload(nprow, st);
  }
  s.geom = Geom{C, P, Q, s.nk, s.nb_max, s.ncol_max, s.d_nb.get(), s.d_ncol.get(),
                s.d_col_start.get(), s.d_col_pq.get(), s.d_col_clo.get(), s.d_kin.get(),
                s.d_prow.get(), s.d_nprow.get()};

  // -- twiddle tables e^{-2 pi i m / N} for the C, P and Q lengths
  {
    std::vector<double2> t64;
    std::vector<float2> t32;
    auto add = [&](int n) {
      const int off = (int)t64.size();
      for (int m = 0; m < n; ++m) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * m / n;
        const double cr = (double)std::cos(ang), ci = (double)-std::sin(ang);
        t64.push_back(mk<double>(cr, ci));
        t32.push_back(mk<float>((float)cr, (float)ci));
      }
      return off;
    };
    s.fft.offC = add(C);
    s.fft.offP = add(P);
    s.fft.offQ = add(Q);
    s.tw64.upload(t64, st);
    s.tw32.upload(t32, st);
    s.fft.tw64 = s.tw64.get();
    s.fft.tw32 = s.tw32.get();
  }

  // -- local potential on the grid, internal layout [C][P][Q].  The cube sum
  // sum_G (-A/|Omega|) e^{-s^2 |G|^2/2} e^{iG.(r - R)} factorises into three
  // one-dimensional sums per atom; V(r) is its real part.
  {
    std::vector<double> v((size_t)s.ng, 0.0);
    const double s2 = s.sigma_loc * s.sigma_loc;
    std::vector<std::vector<double2>> f1(3);
    for (int a = 0; a < s.natoms; ++a) {
      for (int x = 0; x < 3; ++x) {
        const int n = s.N[x];
        f1[x].assign(n, mk<double>(0, 0));
        for (int i = 0; i < n; ++i) {
          const double rx = i * s.a[x] / n - s.pos[3 * a + x];
          double re = 0, im = 0;
          for (int m = -n / 2; m < n / 2; ++m) {
            const double g = m * s.b[x];
            const double amp = std::exp(-s2 * g * g / 2.0);
            re += amp * std::cos(g * rx);
            im += amp * std::sin(g * rx);
          }
          f1[x][i] = mk<double>(re, im);
        }
      }
      const double pref = -s.amp[a] / s.volume;
      for (int c = 0; c < C; ++c)
        for (int p = 0; p < P; ++p)
          for (int q = 0; q < Q; ++q) {
            int e[3];
            e[s.cax] = c;
            e[s.pax] = p;
            e[s.qax] = q;
            const double2 t = cmul<double>(cmul<double>(f1[0][e[0]], f1[1][e[1]]), f1[2][e[2]]);
            v[((size_t)c * P + p) * Q + q] += pref * t.x;
          }
    }
    s.d_vloc.upload(v, st);
  }

  // -- projectors p_a(G+k) = (4 pi s^2)^{3/4} e^{-s^2 |q|^2/2} e^{-iq.R}/sqrt|Omega|
  {
    std::vector<double2> pr((size_t)s.nk * s.natoms * s.nb_max, mk<double>(0, 0));
    const double sp2 = s.sigma_proj * s.sigma_proj;
    const double norm = std::pow(4.0 * PI * sp2, 0.75) / std::sqrt(s.volume);
    for (int k = 0; k < s.nk; ++k) {
      const KPoint& K = s.kp[k];
      for (int a = 0; a < s.natoms; ++a)
        for (int g = 0; g < K.nb; ++g) {
          double q[3], qr = 0;
          for (int x = 0; x < 3; ++x) {
            q[x] = K.miller[3 * g + x] * s.b[x] + K.kcart[x];
            qr += q[x] * s.pos[3 * a + x];
          }
          const double rad = norm * std::exp(-sp2 * (2.0 * K.kin[g]) / 2.0);
          pr[((size_t)k * s.natoms + a) * s.nb_max + g] =
              mk<double>(rad * std::cos(qr), -rad * std::sin(qr));
        }
    }
    s.d_proj.upload(pr, st);
    // projector rows per k-point (the gram/update kernels read it per tile)
    s.d_natoms_k.upload(std::vector<int>(s.nk, s.natoms), st);
  }

  // -- Hartree kernel 4 pi/|G|^2 (G = 0 -> 0) in the internal layout
  {
    std::vector<double> kh((size_t)s.ng);
    for (int c = 0; c < C; ++c)
      for (int p = 0; p < P; ++p)
        for (int q = 0; q < Q; ++q) {
          const int cs = c < C / 2 ? c : c - C, ps = p < P / 2 ? p : p - P,
                    qs = q < Q / 2 ? q : q - Q;
          const double gc = cs * s.b[s.cax], gp = ps * s.b[s.pax], gq = qs * s.b[s.qax];
          const double gg = gc * gc + gp * gp + gq * gq;
          kh[((size_t)c * P + p) * Q + q] = gg > 0 ? 4.0 * PI / gg : 0.0;
        }
    s.d_khat.upload(kh, st);
  }
  s.d_kw1.alloc((size_t)s.ng);
  s.d_kw2.alloc((size_t)s.ng);
  s.d_kpart.alloc(C);
  s.d_u.alloc(s.ng);
  s.d_drho.alloc(s.ng);
  s.d_tmpg.alloc(s.ng);
  IKR_HIP(hipStreamSynchronize(st));
  return sp.release();
}

// FP32 copies of the operator data and an FP32 CG work space, made on first
// use of the mixed-precision path.
void ensure_fp32(System& s) {
  if (s.w32.x.get()) return;
  const hipStream_t st = s.stream;
  const CgWork<double>& d = s.w64;
  CgWork<float>& w = s.w32;
  const size_t vec = (size_t)s.J * s.nb_max, tbuf = (size_t)s.J * s.L.C * s.ncol_max;
  w.x.alloc(vec); w.r.alloc(vec); w.p.alloc(vec); w.w.alloc(vec);
  w.T1.alloc(tbuf); w.T2.alloc(tbuf);
  w.coefA.alloc(d.coefA.n); w.coefB.alloc(d.coefB.n); w.part.alloc(d.part.n);
  w.rz.alloc(s.J); w.alpha.alloc(s.J); w.beta.alloc(s.J); w.rnorm2.alloc(s.J);
  w.rbest.alloc(s.J);
  w.dpart.alloc(d.dpart.n);
  w.pshift.alloc(s.J); w.shift.alloc(s.J);
  convert_array(s.J, d.pshift.get(), w.pshift.get(), st);
  convert_array(s.J, d.shift.get(), w.shift.get(), st);
  w.phi.alloc(s.d_phi.n);
  convert_array(s.d_phi.n, s.d_phi.get(), w.phi.get(), st);
  w.proj.alloc(s.d_proj.n);
  convert_array(s.d_proj.n, s.d_proj.get(), w.proj.get(), st);
  w.vloc.alloc(s.ng);
  convert_array(s.ng, s.d_vloc.get(), w.vloc.get(), st);
  w.wcg.alloc(d.wcg.n);
  convert_array(d.wcg.n, d.wcg.get(), w.wcg.get(), st);
  w.gT.alloc(d.gT.n);
  convert_array(d.gT.n, d.gT.get(), w.gT.get(), st);
  w.sT.alloc(d.sT.n);
  convert_array(d.sT.n, d.sT.get(), w.sT.get(), st);
  w.craw.alloc(d.craw.n); w.gam.alloc(d.gam.n); w.rpart.alloc(d.rpart.n);
  w.zpart.alloc(d.zpart.n);
  IKR_HIP(hipStreamSynchronize(st));
}

void import_ground_state(System& s, const double* eps, const double* coeffs) {
  IKR_CHECK(eps && coeffs, 1, "null ground-state arrays");
  s.eps.assign(eps, eps + (size_t)s.nk * s.nbands);
  for (double e : s.eps) IKR_CHECK(std::isfinite(e), 5, "non-finite eigenvalue");
  const size_t n = (size_t)s.nk * s.nbands * s.nb_max;
  s.d_phi.alloc(n);
  IKR_HIP(hipMemcpyAsync(s.d_phi.get(), coeffs, n * sizeof(double2), hipMemcpyHostToDevice,
                         s.stream));
  // zero the padding beyond nb_k so projections never see stale values
  for (int k = 0; k < s.nk; ++k)
    for (int b = 0; b < s.nbands; ++b) {
      const int nbk = s.kp[k].nb;
      if (nbk < s.nb_max)
        IKR_HIP(hipMemsetAsync(s.d_phi.get() + ((size_t)k * s.nbands + b) * s.nb_max + nbk, 0,
                               (s.nb_max - nbk) * sizeof(double2), s.stream));
    }
  finish_setup(s);
}

// Occupations (eq. density with f = 2/(1+e^x)), Fermi level, occupied
// slots, column transforms of the occupied orbitals, density, the Slater
// kernel and the grt orbital norms.
// Setup progress on stderr when IKR_VERBOSE is set (large cells take minutes).
static void progress(const char* stage) {
  static const bool on = std::getenv("IKR_VERBOSE") != nullptr;
  if (on) std::fprintf(stderr, "[ikr setup] %s\n", stage);
}

void finish_setup(System& s) {
  s.graphs.clear();   // captured CG graphs refer to the buffers set up here
  const int nk = s.nk, nbn = s.nbands;
  s.w32.x.alloc(0);   // FP32 copies are rebuilt from this ground state on demand
  s.mcg = s.natoms + 2 * nbn;
  s.occ.assign((size_t)nk * nbn, 0.0);
  s.docc.assign((size_t)nk * nbn, 0.0);
  if (s.temperature <= 0) {
    for (int k = 0; k < nk; ++k)
      for (int n = 0; n < s.nocc; ++n) s.occ[(size_t)k * nbn + n] = 2.0;
    double homo = -1e300, lumo = 1e300;
    for (int k = 0; k < nk; ++k) {
      homo = std::max(homo, s.eps[(size_t)k * nbn + s.nocc - 1]);
      if (s.nocc < nbn) lumo = std::min(lumo, s.eps[(size_t)k * nbn + s.nocc]);
    }
    s.fermi = s.nocc < nbn ? 0.5 * (homo + lumo) : homo;
  } else {
    const double T = s.temperature, nel = 2.0 * s.nocc;
    double lo = 1e300, hi = -1e300;
    for (double e : s.eps) { lo = std::min(lo, e); hi = std::max(hi, e); }
    lo -= 50 * T;
    hi += 50 * T;
    auto count = [&](double ef) {
      double c = 0;
      for (int k = 0; k < nk; ++k) {
        double ck = 0;
        for (int n = 0; n < nbn; ++n) ck += focc((s.eps[(size_t)k * nbn + n] - ef) / T);
        c += s.kp[k].weight * ck;
      }
      return c;
    };
    for (int it = 0; it < 200 && hi - lo >= 1e-15; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (count(mid) < nel) lo = mid; else hi = mid;
    }
    s.fermi = 0.5 * (lo + hi);
    for (size_t i = 0; i < s.eps.size(); ++i) {
      const double x = (s.eps[i] - s.fermi) / T;
      s.occ[i] = focc(x);
      s.docc[i] = focc_dx(x) / T;
    }
  }
  s.nocc_k.assign(nk, 0);
  s.gap_k.assign(nk, NAN);
  for (int k = 0; k < nk; ++k) {
    int no = 0;
    for (int n = 0; n < nbn; ++n)
      if (s.occ[(size_t)k * nbn + n] > EPS_OCC) no = n + 1;
    IKR_CHECK(no >= 1, 1, "k-point without occupied bands");
    s.nocc_k[k] = no;
    if (no < nbn) s.gap_k[k] = s.eps[(size_t)k * nbn + no] - s.eps[(size_t)k * nbn + no - 1];
  }
  s.nocc_max = *std::max_element(s.nocc_k.begin(), s.nocc_k.end());

  // -- slots (occupied (k, n)) and tiles of <= BT slots per k
  s.slot_k.clear(); s.slot_n.clear(); s.slot0_k.clear();
  s.tile_k.clear(); s.tile_slot0.clear(); s.tile_nb.clear();
  for (int k = 0; k < nk; ++k) {
    s.slot0_k.push_back((int)s.slot_k.size());
    for (int n0 = 0; n0 < s.nocc_k[k]; n0 += BT) {
      s.tile_k.push_back(k);
      s.tile_slot0.push_back((int)s.slot_k.size() + n0);
      s.tile_nb.push_back(std::min(BT, s.nocc_k[k] - n0));
    }
    for (int n = 0; n < s.nocc_k[k]; ++n) {
      s.slot_k.push_back(k);
      s.slot_n.push_back(n);
    }
  }
  s.J = (int)s.slot_k.size();
  const hipStream_t st = s.stream;
  s.d_slot_k.upload(s.slot_k, st);
  s.d_nocc_k.upload(s.nocc_k, st);
  s.d_nbands_k.upload(std::vector<int>(nk, s.nbands), st);
  s.d_tile_k.upload(s.tile_k, st);
  s.d_tile_slot0.upload(s.tile_slot0, st);
  s.d_tile_nb.upload(s.tile_nb, st);
  s.tiles = Tiles{(int)s.tile_k.size(), s.d_tile_k.get(), s.d_tile_slot0.get(),
                  s.d_tile_nb.get()};
  {
    std::vector<int> kt0(nk + 1, 0);
    s.ktmax = 0;
    for (int k = 0; k < nk; ++k) {
      const int nt = (s.nocc_k[k] + BT - 1) / BT;
      kt0[k + 1] = kt0[k] + nt;
      s.ktmax = std::max(s.ktmax, nt);
    }
    s.d_kt0.upload(kt0, st);
    s.d_ktb.alloc(nk + 1);
  }

  // -- work space (FP64 CG)
  const size_t vec = (size_t)s.J * s.nb_max;
  const size_t tbuf = (size_t)s.J * s.L.C * s.ncol_max;
  CgWork<double>& w = s.w64;
  w.x.alloc(vec); w.r.alloc(vec); w.p.alloc(vec); w.w.alloc(vec);
  w.T1.alloc(tbuf); w.T2.alloc(tbuf);
  const int mrows = std::max(s.nocc_max, s.natoms) + 1;
  w.coefA.alloc((size_t)s.J * MAXM);
  w.coefB.alloc((size_t)s.J * MAXM);
  w.part.alloc(gram_part_elems(s.tiles.n, s.nb_max, std::max({mrows, s.nbands, s.mcg}), nk, 2.0));
  w.craw.alloc((size_t)s.J * s.mcg);
  w.gam.alloc((size_t)s.J * s.mcg);
  w.rpart.alloc((size_t)s.J * vec_nblocks(s.nb_max));
  w.zpart.alloc((size_t)s.J * vec_nblocks(s.nb_max));
  w.rz.alloc(s.J); w.alpha.alloc(s.J); w.beta.alloc(s.J); w.rnorm2.alloc(s.J);
  w.rbest.alloc(s.J);
  w.dpart.alloc((size_t)s.J * std::max({update_nblocks(s.nb_max), vec_nblocks(s.nb_max),
                                         (s.nb_max + 63) / 64}));
  w.pshift.alloc(s.J); w.shift.alloc(s.J);
  s.d_active.alloc(s.J);
  s.d_list.alloc(s.J);
  s.d_ctk.alloc(s.tiles.n);
  s.d_cto.alloc(s.tiles.n);
  s.d_ctn.alloc(s.tiles.n);
  s.d_iters.alloc(s.J);
  s.d_rlast.alloc(s.J);
  s.d_counters.alloc(8);
  s.d_slot0_k.upload(s.slot0_k, st);
  {
    std::vector<int> mo(nk), ma(nk, s.mcg);
    for (int k = 0; k < nk; ++k) mo[k] = s.natoms + 2 * s.nocc_k[k];
    s.d_mcg_occ.upload(mo, st);
    s.d_mcg_all.upload(ma, st);
  }
  s.d_cnt.alloc(CNT);
  s.h_cnt.alloc(2 * CNT_STRIDE, hipHostMallocCoherent);
  for (int i = 0; i < 2 * CNT_STRIDE; ++i) s.h_cnt.p[i] = -1;
  IKR_HIP(hipHostGetDevicePointer((void**)&s.d_hcnt, s.h_cnt.p, 0));
  s.d_tol2.alloc(s.J);
  s.d_wa.alloc(s.J);
  s.d_wb.alloc(s.J);
  s.d_multi.alloc((size_t)64 * 256);

  progress("occupations, slots and work space ready");
  // -- column transforms of the occupied orbitals (slot order)
  s.d_Tphi.alloc(tbuf);
  for (int j = 0; j < s.J; ++j)
    IKR_HIP(hipMemcpyAsync(w.x.get() + (size_t)j * s.nb_max,
                           s.d_phi.get() + ((size_t)s.slot_k[j] * nbn + s.slot_n[j]) * s.nb_max,
                           s.nb_max * sizeof(double2), hipMemcpyDeviceToDevice, st));
  Slots all{s.J, s.d_slot_k.get(), nullptr};
  launch_col_inv<double>(s.geom, s.fft, all, w.x.get(), s.nb_max, s.d_Tphi.get(), nullptr,
                         nullptr, nullptr, st);

  // -- per-slot eigenvalues and preconditioner shifts c_nk = max(<phi, kin phi>, 0.1)
  {
    std::vector<double> sh(s.J), ps(s.J);
    std::vector<double2> hphi((size_t)s.J * s.nb_max);
    IKR_HIP(hipMemcpyAsync(hphi.data(), w.x.get(), hphi.size() * sizeof(double2),
                           hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < s.J; ++j) {
      const KPoint& K = s.kp[s.slot_k[j]];
      double c = 0;
      for (int g = 0; g < K.nb; ++g) {
        const double2 v = hphi[(size_t)j * s.nb_max + g];
        c += K.kin[g] * (v.x * v.x + v.y * v.y);
      }
      ps[j] = std::max(c, 0.1);
      sh[j] = s.eps[(size_t)s.slot_k[j] * nbn + s.slot_n[j]];
    }
    s.w64.pshift.upload(ps, st);
    s.w64.shift.upload(sh, st);
  }

  progress("column transforms and preconditioner shifts ready");
  // -- fused CG projections: W_k = [projectors | phi_1, H phi_1, phi_2, H phi_2, ...],
  //    G^T[k][j][m] = <phi_m, H phi_j> and S^T[k][j][m] = <phi_m, phi_j>
  {
    const int Na = s.natoms;
    const size_t kb = (size_t)nbn * s.nb_max, rowb = s.nb_max * sizeof(double2);
    DBuf<double2> hphi;
    hphi.alloc((size_t)nk * kb);
    IKR_HIP(hipMemsetAsync(hphi.get(), 0, hphi.n * sizeof(double2), st));
    for (int k = 0; k < nk; ++k)
      apply_hamiltonian(s, k, nbn, s.d_phi.get() + k * kb, hphi.get() + k * kb);
    w.wcg.alloc((size_t)nk * s.mcg * s.nb_max);
    for (int k = 0; k < nk; ++k) {
      double2* dst = w.wcg.get() + (size_t)k * s.mcg * s.nb_max;
      if (Na > 0)
        IKR_HIP(hipMemcpyAsync(dst, s.d_proj.get() + (size_t)k * Na * s.nb_max, Na * rowb,
                               hipMemcpyDeviceToDevice, st));
      IKR_HIP(hipMemcpy2DAsync(dst + (size_t)Na * s.nb_max, 2 * rowb, s.d_phi.get() + k * kb,
                               rowb, rowb, nbn, hipMemcpyDeviceToDevice, st));
      IKR_HIP(hipMemcpy2DAsync(dst + (size_t)(Na + 1) * s.nb_max, 2 * rowb, hphi.get() + k * kb,
                               rowb, rowb, nbn, hipMemcpyDeviceToDevice, st));
    }
    std::vector<int> tk, ts, tn;
    for (int k = 0; k < nk; ++k)
      for (int n0 = 0; n0 < nbn; n0 += BT) {
        tk.push_back(k);
        ts.push_back(k * nbn + n0);
        tn.push_back(std::min(BT, nbn - n0));
      }
    DBuf<int> dtk, dts, dtn;
    dtk.upload(tk, st); dts.upload(ts, st); dtn.upload(tn, st);
    Tiles tl{(int)tk.size(), dtk.get(), dts.get(), dtn.get()};
    DBuf<double2> part;
    part.alloc(gram_part_elems(tl.n, s.nb_max, nbn));
    w.gT.alloc((size_t)nk * nbn * nbn);
    w.sT.alloc((size_t)nk * nbn * nbn);
    gram<double>(tl, s.d_nb.get(), s.nb_max, s.d_nbands_k.get(), nbn, s.d_phi.get(), kb,
                 s.nb_max, hphi.get(), s.nb_max, part.get(), w.gT.get(), nbn, st);
    gram<double>(tl, s.d_nb.get(), s.nb_max, s.d_nbands_k.get(), nbn, s.d_phi.get(), kb,
                 s.nb_max, s.d_phi.get(), s.nb_max, part.get(), w.sT.get(), nbn, st);
    IKR_HIP(hipStreamSynchronize(st));
  }

  progress("fused CG tables ready");
  // -- density rho = sum_k w_k sum_n f |psi|^2 (grid values)
  {
    const int gs = 8;
    const int ngrp = (s.J + gs - 1) / gs;
    s.d_rhopart.alloc((size_t)std::max(ngrp, 1) * s.ng);
    std::vector<double> wa(s.J, 0.0), wb(s.J);
    for (int j = 0; j < s.J; ++j)
      wb[j] = s.kp[s.slot_k[j]].weight * s.occ[(size_t)s.slot_k[j] * nbn + s.slot_n[j]] / s.volume;
    s.d_wa.upload(wa, st);
    s.d_wb.upload(wb, st);
    launch_plane_rho(s.geom, s.fft, s.J, s.d_slot_k.get(), s.d_Tphi.get(), s.d_Tphi.get(),
                     s.d_wa.get(), s.d_wb.get(), gs, s.d_rhopart.get(), st);
    s.d_rho.alloc(s.ng);
    sum_groups(s.ng, ngrp, s.d_rhopart.get(), 1.0, s.d_rho.get(), st);
  }
  // -- Slater exchange kernel f_x = -(1/3)(3/pi)^{1/3} max(rho, 1e-10)^{-2/3}
  {
    std::vector<double> rho(s.ng), fx(s.ng, 0.0);
    IKR_HIP(hipMemcpyAsync(rho.data(), s.d_rho.get(), s.ng * sizeof(double),
                           hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
    if (s.xc)
      for (int i = 0; i < s.ng; ++i)
        fx[i] = -(1.0 / 3.0) * std::cbrt(3.0 / PI) * std::pow(std::max(rho[i], 1e-10), -2.0 / 3.0);
    s.d_fx.upload(fx, st);
    // ||K||_2 bound: largest Hartree eigenvalue (smallest nonzero |G| = min b_i on
    // an orthorhombic grid) plus the largest |f_x|
    double fxmax = 0;
    for (double v : fx) fxmax = std::max(fxmax, std::fabs(v));
    const double bmin = std::min({s.b[0], s.b[1], s.b[2]});
    s.knorm_bound = 4.0 * PI / (bmin * bmin) + fxmax;
  }
  progress("density and exchange kernel ready");
  // -- ||Re F_k^-1 Phi_k||_{2,inf} per k (grt strategy, Sec. 3.4.1).  The real
  // part depends on the phase of each orbital, which the eigensolver leaves
  // arbitrary: each orbital is taken with the phase that makes sum_r psi^2
  // real and positive (the real representation when one exists), and the
  // result is floored at ||F_k^-1 Phi_k||_{2,inf} / sqrt(2).
  {
    s.orbnorm_k.assign(nk, 0.0);
    s.orbnorm_full_k.assign(nk, 0.0);
    DBuf<double2> grid, sq, ph;
    DBuf<double> dfull, dre;
    int maxo = s.nocc_max;
    const int nsq = grid_square_nblocks(s.ng);
    grid.alloc((size_t)maxo * s.ng);
    sq.alloc((size_t)maxo * nsq);
    ph.alloc(maxo);
    dfull.alloc(s.ng);
    dre.alloc(s.ng);
    std::vector<double> hf(s.ng), hr(s.ng);
    std::vector<double2> hsq((size_t)maxo * nsq), hph(maxo);
    for (int k = 0; k < nk; ++k) {
      const int j0 = s.slot0_k[k], no = s.nocc_k[k];
      launch_plane_grid(s.geom, s.fft, no, s.d_slot_k.get() + j0,
                        s.d_Tphi.get() + (size_t)j0 * s.L.C * s.ncol_max, grid.get(), st);
      grid_square_sums(s.ng, no, grid.get(), sq.get(), st);
      IKR_HIP(hipMemcpyAsync(hsq.data(), sq.get(), (size_t)no * nsq * sizeof(double2),
                             hipMemcpyDeviceToHost, st));
      IKR_HIP(hipStreamSynchronize(st));
      for (int n = 0; n < no; ++n) {
        double x = 0, y = 0;
        for (int b = 0; b < nsq; ++b) {
          x += hsq[(size_t)n * nsq + b].x;
          y += hsq[(size_t)n * nsq + b].y;
        }
        const double th = -0.5 * std::atan2(y, x);
        hph[n] = make_double2(std::cos(th), std::sin(th));
      }
      IKR_HIP(hipMemcpyAsync(ph.get(), hph.data(), no * sizeof(double2), hipMemcpyHostToDevice,
                             st));
      grid_row_norms(s.ng, no, grid.get(), ph.get(), dfull.get(), dre.get(), st);
      IKR_HIP(hipMemcpyAsync(hf.data(), dfull.get(), s.ng * sizeof(double), hipMemcpyDeviceToHost, st));
      IKR_HIP(hipMemcpyAsync(hr.data(), dre.get(), s.ng * sizeof(double), hipMemcpyDeviceToHost, st));
      IKR_HIP(hipStreamSynchronize(st));
      double mx = 0, mxf = 0;
      for (int i = 0; i < s.ng; ++i) {
        mx = std::max(mx, hr[i]);
        mxf = std::max(mxf, hf[i]);
      }
      s.orbnorm_full_k[k] = std::sqrt(mxf / s.volume);
      s.orbnorm_k[k] = std::max(std::sqrt(mx / s.volume), s.orbnorm_full_k[k] / std::sqrt(2.0));
    }
  }
  IKR_HIP(hipStreamSynchronize(st));
  progress("orbital norms ready");
  s.have_gs = true;
}

}  // namespace ikr
