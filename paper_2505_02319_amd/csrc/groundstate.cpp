// Ground state of the fixed model Hamiltonian on the GPU: the lowest bands
// of every H_k (eq. KS / eq. discretised_KS, Bloch form) by Chebyshev-
// filtered subspace iteration over all k-points at once.  Each outer step
// filters the block with a scaled Chebyshev polynomial of H_k that damps
// the spectrum above the block's largest Ritz value, re-orthonormalises it
// (Cholesky QR, twice) and performs a Rayleigh-Ritz step.  The H psi
// products use the same pruned-FFT kernels as the Sternheimer CG; the small
// dense problems (Gram Cholesky, Hermitian eigenproblem) run on the host.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "system.h"

namespace ikr {

void cheb_combine(int nslots, int nb_max, const int* slot_k, const int* nb, const double2* Z,
                  double2* X, const double* alpha, const double* beta, hipStream_t st);
void resid_norms(int nslots, int nb_max, const int* slot_k, const int* nb, const double2* HX,
                 const double2* X, const double* lam, double* part, hipStream_t st);

namespace {

using cd = double2;

// Batched Hermitian eigenproblems A_k U_k = U_k diag(lam_k) on the device
// (rocSOLVER zheevd, eigenvalues ascending); A_k row-major on the host, U_k
// returned row-major (U[i * n + c] = component i of eigenvector c).
struct BatchEig {
  rocblas_handle h = nullptr;
  DBuf<cd> A;
  DBuf<double> D, E;
  DBuf<int> info;
  BatchEig() = default;
  BatchEig(const BatchEig&) = delete;
  BatchEig& operator=(const BatchEig&) = delete;
  ~BatchEig() { if (h) (void)rocblas_destroy_handle(h); }
  void run(hipStream_t st, int n, const std::vector<std::vector<cd>>& mats,
           std::vector<double>& lam, std::vector<std::vector<cd>>& U) {
    const int nb = (int)mats.size();
    const size_t nn = (size_t)n * n;
    if (!h) {
      IKR_CHECK(rocblas_create_handle(&h) == rocblas_status_success, 7, "rocblas handle");
      A.alloc(nn * nb);
      D.alloc((size_t)n * nb);
      E.alloc((size_t)n * nb);
      info.alloc(nb);
    }
    IKR_CHECK(rocblas_set_stream(h, st) == rocblas_status_success, 7, "rocblas stream");
    std::vector<cd> cm(nn * nb);
    for (int k = 0; k < nb; ++k)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) cm[k * nn + (size_t)j * n + i] = mats[k][(size_t)i * n + j];
    IKR_HIP(hipMemcpyAsync(A.get(), cm.data(), cm.size() * sizeof(cd), hipMemcpyHostToDevice, st));
    const rocblas_status r = rocsolver_zheevd_strided_batched(
        h, rocblas_evect_original, rocblas_fill_upper, n,
        reinterpret_cast<rocblas_double_complex*>(A.get()), n, (rocblas_stride)nn, D.get(), n,
        E.get(), n, info.get(), nb);
    IKR_CHECK(r == rocblas_status_success, 7, "rocsolver zheevd failed");
    std::vector<int> inf(nb);
    std::vector<double> d((size_t)n * nb);
    IKR_HIP(hipMemcpyAsync(cm.data(), A.get(), cm.size() * sizeof(cd), hipMemcpyDeviceToHost, st));
    IKR_HIP(hipMemcpyAsync(d.data(), D.get(), d.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    IKR_HIP(hipMemcpyAsync(inf.data(), info.get(), nb * sizeof(int), hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < nb; ++k) IKR_CHECK(inf[k] == 0, 4, "Hermitian eigensolver did not converge");
    lam.assign((size_t)nb * n, 0.0);
    U.assign(nb, std::vector<cd>(nn));
    for (int k = 0; k < nb; ++k)
      for (int c = 0; c < n; ++c) {
        lam[(size_t)k * n + c] = d[(size_t)k * n + c];
        for (int i = 0; i < n; ++i) U[k][(size_t)i * n + c] = cm[k * nn + (size_t)c * n + i];
      }
  }
};

// M = L^{-H} for G = L L^H (in place Cholesky with a diagonal shift on
// failure); returns the upper-triangular M (row-major n x n).
std::vector<cd> chol_inv_upper(int n, std::vector<cd> G) {
  double tr = 0;
  for (int i = 0; i < n; ++i) tr += G[(size_t)i * n + i].x;
  for (int attempt = 0; attempt < 6; ++attempt) {
    std::vector<cd> L((size_t)n * n, mk<double>(0, 0));
    bool ok = true;
    const double shift = attempt == 0 ? 0.0 : tr / n * std::pow(10.0, -15 + 2 * attempt);
    for (int j = 0; j < n && ok; ++j) {
      double d = G[(size_t)j * n + j].x + shift;
      for (int k = 0; k < j; ++k) {
        const cd l = L[(size_t)j * n + k];
        d -= l.x * l.x + l.y * l.y;
      }
      if (!(d > 0)) { ok = false; break; }
      const double ljj = std::sqrt(d);
      L[(size_t)j * n + j] = mk<double>(ljj, 0);
      for (int i = j + 1; i < n; ++i) {
        cd v = G[(size_t)i * n + j];
        for (int k = 0; k < j; ++k)
          v = csub<double>(v, cmulc<double>(L[(size_t)j * n + k], L[(size_t)i * n + k]));
        // L[i][j] = (G[i][j] - sum_k L[i][k] conj(L[j][k])) / L[j][j]
        L[(size_t)i * n + j] = cscale<double>(v, 1.0 / ljj);
      }
    }
    if (!ok) continue;
    // invert lower-triangular L, then M = (L^-1)^H
    std::vector<cd> Li((size_t)n * n, mk<double>(0, 0));
    for (int j = 0; j < n; ++j) {
      Li[(size_t)j * n + j] = mk<double>(1.0 / L[(size_t)j * n + j].x, 0);
      for (int i = j + 1; i < n; ++i) {
        cd v = mk<double>(0, 0);
        for (int k = j; k < i; ++k) v = cadd<double>(v, cmul<double>(L[(size_t)i * n + k], Li[(size_t)k * n + j]));
        Li[(size_t)i * n + j] = cscale<double>(v, -1.0 / L[(size_t)i * n + i].x);
      }
    }
    std::vector<cd> M((size_t)n * n, mk<double>(0, 0));
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const cd v = Li[(size_t)j * n + i];
        M[(size_t)i * n + j] = mk<double>(v.x, -v.y);
      }
    return M;
  }
  throw Error(8, "Gram matrix not positive definite in the eigensolver");
}

}  // namespace

void compute_ground_state(System& s) {
  const hipStream_t st = s.stream;
  const int nk = s.nk, nbm = s.nb_max, nbn = s.nbands;
  // Guard vectors above the wanted bands keep the filter's damping cut away
  // from clusters that straddle band nbands.
  const int nblk = std::min(MAXM - 1, nbn + std::max(8, nbn / 2));
  const int ns = nk * nblk;
  const double tol = 1e-11;
  const int degree = 24, max_outer = 400;
  const bool verbose = std::getenv("IKR_VERBOSE") != nullptr;

  // slots (k, i) and tiles of <= BT per k
  std::vector<int> sk(ns), tk, ts, tn;
  for (int k = 0; k < nk; ++k)
    for (int i = 0; i < nblk; ++i) sk[(size_t)k * nblk + i] = k;
  for (int k = 0; k < nk; ++k)
    for (int i0 = 0; i0 < nblk; i0 += BT) {
      tk.push_back(k);
      ts.push_back(k * nblk + i0);
      tn.push_back(std::min(BT, nblk - i0));
    }
  DBuf<int> dsk, dtk, dts, dtn, dM, dkt0;
  dsk.upload(sk, st); dtk.upload(tk, st); dts.upload(ts, st); dtn.upload(tn, st);
  dM.upload(std::vector<int>(nk, nblk), st);
  Tiles tl{(int)tk.size(), dtk.get(), dts.get(), dtn.get()};
  const int tpk = (nblk + BT - 1) / BT;   // tiles per k
  {
    std::vector<int> kt0(nk + 1);
    for (int k = 0; k <= nk; ++k) kt0[k] = k * tpk;
    dkt0.upload(kt0, st);
  }
  const KTileRange kr{nk, dkt0.get(), tpk};
  Slots sl{ns, dsk.get(), nullptr};

  const size_t vec = (size_t)ns * nbm;
  DBuf<cd> A, B, Cb, HX, T1, T2, coef, part, pcoef;
  A.alloc(vec); B.alloc(vec); Cb.alloc(vec); HX.alloc(vec);
  for (cd* b : {A.get(), B.get(), Cb.get(), HX.get()})
    IKR_HIP(hipMemsetAsync(b, 0, vec * sizeof(cd), st));
  T1.alloc((size_t)ns * s.L.C * s.ncol_max);
  T2.alloc((size_t)ns * s.L.C * s.ncol_max);
  coef.alloc((size_t)ns * MAXM);
  pcoef.alloc((size_t)ns * MAXM);
  part.alloc(gram_part_elems(tl.n, nbm, std::max(nblk, s.natoms), nk));
  DBuf<double> dshift, dal, dbe, dlam, rpart;
  dshift.alloc(ns); dal.alloc(ns); dbe.alloc(ns); dlam.alloc(ns);
  const int nrb = vec_nblocks(nbm);
  rpart.alloc((size_t)ns * nrb);
  const size_t wk = (size_t)nblk * nbm;

  // Z = (H - shift) Y  for all slots
  auto hpsi = [&](const cd* Y, cd* Z, const double* shift) {
    launch_col_inv<double>(s.geom, s.fft, sl, Y, nbm, T1.get(), nullptr, nullptr, nullptr, st);
    launch_plane_hv<double>(s.geom, s.fft, sl, T1.get(), T2.get(), s.d_vloc.get(), 0, st);
    launch_col_fwd<double>(s.geom, s.fft, sl, T2.get(), Z, nbm, Y, shift, 1.0 / s.ng, st);
    if (s.natoms > 0) {
      gram<double>(tl, s.d_nb.get(), nbm, s.d_natoms_k.get(), s.natoms, s.d_proj.get(),
                   (size_t)s.natoms * nbm, nbm, Y, nbm, part.get(), pcoef.get(), MAXM, st);
      UpdTerm<double> t{s.d_proj.get(), (size_t)s.natoms * nbm, nbm, s.d_natoms_k.get(),
                        pcoef.get(), MAXM, s.dnl, s.natoms};
      update<double>(tl, s.d_nb.get(), nbm, nullptr, Z, nbm, 1.0, t, UpdTerm<double>{}, nullptr,
                     nullptr, st);
    }
  };
  // G[k][m][j] = <Y_m, X_j> per k (host, nblk x nblk per k)
  auto gram_host = [&](const cd* Yw, const cd* Xs) {
    gram<double>(tl, s.d_nb.get(), nbm, dM.get(), nblk, Yw, wk, nbm, Xs, nbm, part.get(),
                 coef.get(), MAXM, st, nullptr, kr);
    std::vector<cd> c((size_t)ns * MAXM);
    IKR_HIP(hipMemcpyAsync(c.data(), coef.get(), c.size() * sizeof(cd), hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
    std::vector<std::vector<cd>> G(nk, std::vector<cd>((size_t)nblk * nblk));
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < nblk; ++j)
        for (int m = 0; m < nblk; ++m)
          G[k][(size_t)m * nblk + j] = c[((size_t)k * nblk + j) * MAXM + m];
    return G;
  };
  // Out[k][j] = sum_m Yw[k][m] Mk[m][j]
  auto combine = [&](const cd* Yw, const std::vector<std::vector<cd>>& Mk, cd* Out) {
    std::vector<cd> c((size_t)ns * MAXM, mk<double>(0, 0));
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < nblk; ++j)
        for (int m = 0; m < nblk; ++m)
          c[((size_t)k * nblk + j) * MAXM + m] = Mk[k][(size_t)m * nblk + j];
    IKR_HIP(hipMemcpyAsync(coef.get(), c.data(), c.size() * sizeof(cd), hipMemcpyHostToDevice, st));
    IKR_HIP(hipStreamSynchronize(st));
    UpdTerm<double> t{Yw, wk, nbm, dM.get(), coef.get(), MAXM, 1.0};
    update<double>(tl, s.d_nb.get(), nbm, nullptr, Out, nbm, 0.0, t, UpdTerm<double>{}, nullptr,
                   nullptr, st);
  };
  // Y <- Y L^{-H} (Cholesky QR), Y in buffer `Y`, scratch `W`
  auto cholqr = [&](cd*& Y, cd*& W) {
    for (int pass = 0; pass < 2; ++pass) {
      auto G = gram_host(Y, Y);
      std::vector<std::vector<cd>> M(nk);
      for (int k = 0; k < nk; ++k) M[k] = chol_inv_upper(nblk, G[k]);
      combine(Y, M, W);
      std::swap(Y, W);
    }
  };

  // -- initial block: random coefficients damped by e^{-|G+k|^2/2}
  {
    std::vector<cd> h(vec, mk<double>(0, 0));
    std::mt19937_64 rng(20250502);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int k = 0; k < nk; ++k)
      for (int i = 0; i < nblk; ++i)
        for (int g = 0; g < s.kp[k].nb; ++g) {
          const double d = std::exp(-s.kp[k].kin[g]);
          const double re = nd(rng), im = nd(rng);
          h[((size_t)k * nblk + i) * nbm + g] = mk<double>(re * d, im * d);
        }
    IKR_HIP(hipMemcpyAsync(A.get(), h.data(), vec * sizeof(cd), hipMemcpyHostToDevice, st));
    IKR_HIP(hipStreamSynchronize(st));
  }
  // Upper bound of the spectrum of every H_k (Weyl): max kinetic + max V +
  // D ||P_k^H P_k|| (D > 0), the last bounded by the largest Gershgorin row
  // sum of the projectors' Gram matrix (natoms x natoms, nearly the identity
  // for well-separated atoms) or its trace.  A tight bound makes the filter
  // sharper.
  double bup = 0;
  {
    std::vector<double> v((size_t)s.ng);
    IKR_HIP(hipMemcpyAsync(v.data(), s.d_vloc.get(), v.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    std::vector<cd> pr((size_t)nk * s.natoms * nbm);
    if (s.natoms)
      IKR_HIP(hipMemcpyAsync(pr.data(), s.d_proj.get(), pr.size() * sizeof(cd), hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
    double vmax = -1e300;
    for (double x : v) vmax = std::max(vmax, x);
    const int na = s.natoms;
    for (int k = 0; k < nk; ++k) {
      double kmax = 0;
      for (double x : s.kp[k].kin) kmax = std::max(kmax, x);
      double nl = 0;
      if (na > 0 && s.dnl > 0) {
        std::vector<cd> G((size_t)na * na, mk<double>(0, 0));
        const cd* P = pr.data() + (size_t)k * na * nbm;
        double tr = 0;
        for (int a = 0; a < na; ++a)
          for (int b = 0; b < na; ++b) {
            double re = 0, im = 0;
            for (int g = 0; g < s.kp[k].nb; ++g) {
              const cd x = P[(size_t)a * nbm + g], y = P[(size_t)b * nbm + g];
              re += x.x * y.x + x.y * y.y;
              im += x.x * y.y - x.y * y.x;
            }
            G[(size_t)a * na + b] = mk<double>(re, im);
            if (a == b) tr += re;
          }
        double gersh = 0;   // largest eigenvalue <= max row sum of |G| (Gershgorin)
        for (int a = 0; a < na; ++a) {
          double row = 0;
          for (int b = 0; b < na; ++b)
            row += std::hypot(G[(size_t)a * na + b].x, G[(size_t)a * na + b].y);
          gersh = std::max(gersh, row);
        }
        nl = s.dnl * std::min(gersh, tr);
      }
      bup = std::max(bup, kmax + std::max(vmax, 0.0) + nl);
    }
    bup *= 1.01;
  }

  cd* Y = A.get();
  cd* W = B.get();
  cd* Z = Cb.get();
  std::vector<double> lam((size_t)nk * nblk, 0.0);
  std::vector<double> rnorm(ns, 1.0);

  // Rayleigh-Ritz on the orthonormal block Y: X = Y U, HX = (HY) U
  BatchEig eig;
  auto rayleigh_ritz = [&]() {
    std::vector<double> zero(ns, 0.0);
    IKR_HIP(hipMemcpyAsync(dshift.get(), zero.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
    hpsi(Y, Z, dshift.get());
    auto Hs = gram_host(Y, Z);
    std::vector<std::vector<cd>> U;
    for (int k = 0; k < nk; ++k) {
      std::vector<cd>& Ak = Hs[k];
      for (int i = 0; i < nblk; ++i)
        for (int j = 0; j < i; ++j) {   // Hermitian average
          const cd a = Ak[(size_t)i * nblk + j], b = Ak[(size_t)j * nblk + i];
          const cd m = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
          Ak[(size_t)i * nblk + j] = m;
          Ak[(size_t)j * nblk + i] = mk<double>(m.x, -m.y);
        }
      for (int i = 0; i < nblk; ++i) Ak[(size_t)i * nblk + i].y = 0;
    }
    eig.run(st, nblk, Hs, lam, U);
    combine(Y, U, W);      // X
    combine(Z, U, HX.get());
    std::swap(Y, W);       // Y now holds X
    IKR_HIP(hipMemcpyAsync(dlam.get(), lam.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
    resid_norms(ns, nbm, dsk.get(), s.d_nb.get(), HX.get(), Y, dlam.get(), rpart.get(), st);
    std::vector<double> p((size_t)ns * nrb);
    IKR_HIP(hipMemcpyAsync(p.data(), rpart.get(), p.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < ns; ++i) {
      double a = 0;
      for (int b = 0; b < nrb; ++b) a += p[(size_t)i * nrb + b];
      rnorm[i] = std::sqrt(a);
    }
  };

  cholqr(Y, W);
  rayleigh_ritz();
  int outer = 0;
  for (; outer < max_outer; ++outer) {
    double worst = 0;
    for (int k = 0; k < nk; ++k)
      for (int n = 0; n < nbn; ++n) worst = std::max(worst, rnorm[(size_t)k * nblk + n]);
    if (verbose)
      std::fprintf(stderr, "[ikr eig] step %d worst residual %.3e  cut %.5f  top %.5f\n", outer,
                   worst, lam[nblk - 1], bup);
    if (worst <= tol) break;
    // scaled Chebyshev filter of the given degree on [a, bup], anchored at a0
    std::vector<double> cc(ns), ee(ns), sg(ns), al(ns), be(ns);
    for (int k = 0; k < nk; ++k) {
      const double a0 = lam[(size_t)k * nblk], a = lam[(size_t)k * nblk + nblk - 1];
      const double e = (bup - a) / 2, c = (bup + a) / 2;
      for (int i = 0; i < nblk; ++i) {
        const int j = k * nblk + i;
        cc[j] = c; ee[j] = e; sg[j] = e / (a0 - c);
      }
    }
    IKR_HIP(hipMemcpyAsync(dshift.get(), cc.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
    // Y1 = (H - c) X * (sigma1 / e)
    cd* Xp = Y;          // X_{i-1}
    hpsi(Xp, Z, dshift.get());
    for (int j = 0; j < ns; ++j) { al[j] = sg[j] / ee[j]; be[j] = 0.0; }
    IKR_HIP(hipMemcpyAsync(dal.get(), al.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
    IKR_HIP(hipMemcpyAsync(dbe.get(), be.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
    IKR_HIP(hipMemsetAsync(W, 0, vec * sizeof(cd), st));
    cheb_combine(ns, nbm, dsk.get(), s.d_nb.get(), Z, W, dal.get(), dbe.get(), st);     // W = al * Z
    IKR_HIP(hipStreamSynchronize(st));
    cd* Yc = W;          // Y_i
    std::vector<double> sigma(sg), s1(sg);
    for (int deg = 2; deg <= degree; ++deg) {
      for (int j = 0; j < ns; ++j) {
        const double sn = 1.0 / (2.0 / s1[j] - sigma[j]);
        al[j] = 2.0 * sn / ee[j];
        be[j] = -sigma[j] * sn;
        sigma[j] = sn;
      }
      hpsi(Yc, Z, dshift.get());
      IKR_HIP(hipMemcpyAsync(dal.get(), al.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
      IKR_HIP(hipMemcpyAsync(dbe.get(), be.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
      cheb_combine(ns, nbm, dsk.get(), s.d_nb.get(), Z, Xp, dal.get(), dbe.get(), st);  // Xp <- al Z + be Xp
      IKR_HIP(hipStreamSynchronize(st));
      std::swap(Xp, Yc);
    }
    // the filtered block is in Yc; the other buffer of the pair is scratch
    Y = Yc;
    W = Xp;
    cholqr(Y, W);
    rayleigh_ritz();
  }
  double worst = 0;
  for (int k = 0; k < nk; ++k)
    for (int n = 0; n < nbn; ++n) worst = std::max(worst, rnorm[(size_t)k * nblk + n]);
  IKR_CHECK(worst <= 1e3 * tol, 4, "ground-state eigensolver did not converge");

  // keep the lowest nbands of every k
  s.eps.assign((size_t)nk * nbn, 0.0);
  for (int k = 0; k < nk; ++k)
    for (int n = 0; n < nbn; ++n) s.eps[(size_t)k * nbn + n] = lam[(size_t)k * nblk + n];
  s.d_phi.alloc((size_t)nk * nbn * nbm);
  for (int k = 0; k < nk; ++k)
    IKR_HIP(hipMemcpyAsync(s.d_phi.get() + (size_t)k * nbn * nbm, Y + (size_t)k * nblk * nbm,
                           (size_t)nbn * nbm * sizeof(cd), hipMemcpyDeviceToDevice, st));
  IKR_HIP(hipStreamSynchronize(st));
  s.gs_outer_iters = outer;
  s.gs_residual = worst;
  finish_setup(s);
}

}  // namespace ikr
