// Gradient of a loss of the density response with respect to the
// local-potential amplitudes A_a (V_loc = sum_a A_a a_a(r), linear in A).
//
// With drho = E^-1 b, lambda = E^-T dL/d(drho) and u = K drho:
//   dL/dA_a = lambda^T (d chi0/dA_a) u + lambda^T chi0 (dK/dA_a) drho
//           = sum_r a_a(r) [ G(r) + (chi0 s)(r) ],  s = (chi0 lambda) f_x'(rho) drho,
// the ground state not being self-consistent (dK/dA_a = f_x'(rho) chi0 a_a).
// The first term is the third derivative of the band energy in the
// directions (a, u, lambda) (rho is N_g/|Omega| times its potential
// derivative on the grid), evaluated with first-order orbitals only (2n+1
// rule, equal occupations):
//   psi^x_n = -Q (H - e_n)^-1 Q x phi_n,   L^x_mn = <phi_m, x phi_n>,
//   C_n     = u psi^l_n + l psi^u_n - sum_m (L^u_mn psi^l_m + L^l_mn psi^u_m),
//   eta_n   = Q (H - e_n)^-1 Q C_n      (one adjoint Sternheimer solve per band),
//   zeta_n  = sum_m <psi^l_m, psi^u_n> phi_m,
//   G       = sum_k w_k 2 f sum_n [Re(conj psi^u_n psi^l_n) - Re(conj psi_n (eta_n + zeta_n))].
// Every Sternheimer solve, FFT, projection and density accumulation runs in
// the same kernels as chi0; the host only assembles scalars and the final
// grid contractions.
#include <algorithm>
#include <cmath>

#include "system.h"

namespace ikr {
namespace {

constexpr double PI = 3.14159265358979323846;

template <typename T> std::vector<T> fetch(const T* d, size_t n, hipStream_t st) {
  std::vector<T> h(n);
  if (n) {
    IKR_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
  }
  return h;
}

// dV_loc/dA_a on the grid (internal layout): the local-potential sum of the
// setup with amplitude 1 for atom a and 0 for the others.
void build_dvloc(System& s) {
  if (!s.dvloc.empty()) return;
  const int C = s.L.C, P = s.L.P, Q = s.L.Q;
  s.dvloc.assign((size_t)s.natoms * s.ng, 0.0);
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
    const double pref = -1.0 / s.volume;
    double* out = s.dvloc.data() + (size_t)a * s.ng;
    for (int c = 0; c < C; ++c)
      for (int p = 0; p < P; ++p)
        for (int q = 0; q < Q; ++q) {
          int e[3];
          e[s.cax] = c;
          e[s.pax] = p;
          e[s.qax] = q;
          const double2 t = cmul<double>(cmul<double>(f1[0][e[0]], f1[1][e[1]]), f1[2][e[2]]);
          out[((size_t)c * P + p) * Q + q] = pref * t.x;
        }
  }
}

}  // namespace

std::vector<double> grad_amplitudes(System& s, const double* drho_ext, const double* lam_ext,
                                    double cg_tol, ikr_stats* stt) {
  IKR_CHECK(s.have_gs, 2, "ground state not set up");
  IKR_CHECK(s.temperature <= 0, 1, "amplitude gradient: fixed occupations only");
  for (int k = 0; k < s.nk; ++k)
    IKR_CHECK(s.nocc_k[k] == s.nocc, 1, "amplitude gradient: fixed occupations only");
  IKR_CHECK(cg_tol > 0 && cg_tol < 1, 1, "cg_tol must lie in (0, 1)");
  const hipStream_t st = s.stream;
  const int J = s.J, nbm = s.nb_max, ng = s.ng, no = s.nocc, nbn = s.nbands;
  const size_t vec = (size_t)J * nbm;
  const double inv_ng = 1.0 / ng;
  CgWork<double>& w = s.w64;
  Slots all{J, s.d_slot_k.get(), nullptr};
  const int schur = s.nbands > s.nocc_max ? 1 : 0;
  const int max_iter = 2000;
  const std::vector<double> tol(J, cg_tol);
  auto count = [&](const Chi0Result& r) {
    if (!stt) return;
    stt->n_ham += r.n_ham;
    stt->n_ham_fp64 += r.n_ham64;
    stt->cg_unconverged += r.noconv;
    stt->fp64_fallback += r.fallback;
    stt->fp32_checked += r.checked;
  };

  DBuf<double> drho, lam, u, g1, g2, chil, sv, chis, one;
  drho.alloc(ng); lam.alloc(ng); u.alloc(ng); g1.alloc(ng); g2.alloc(ng);
  chil.alloc(ng); sv.alloc(ng); chis.alloc(ng);
  one.upload(std::vector<double>{1.0}, st);
  DBuf<double2> psu, psl, cbuf, tmp, mu, ml, cz;
  psu.alloc(vec); psl.alloc(vec); cbuf.alloc(vec); tmp.alloc(vec);
  to_internal(s.L, drho_ext, drho.get(), st);
  to_internal(s.L, lam_ext, lam.get(), st);
  apply_kernel(s, drho.get(), u.get());                      // u = K drho

  // first-order orbitals psi^u, psi^l and L^u, L^l
  std::vector<double2> Mu, Ml;
  Chi0Extra eu;
  eu.dphi_out = psu.get();
  eu.m_out = &Mu;
  eu.tol_relative = true;
  count(apply_chi0_internal(s, u.get(), nullptr, tol, 1, max_iter, 0, 1e-5, schur, &eu));
  Chi0Extra el;
  el.dphi_out = psl.get();
  el.m_out = &Ml;
  el.tol_relative = true;
  count(apply_chi0_internal(s, lam.get(), nullptr, tol, 1, max_iter, 0, 1e-5, schur, &el));
  mu.upload(Mu, st);
  ml.upload(Ml, st);

  // C = F(u psi^l) + F(l psi^u) - sum_m (L^u_mn psi^l_m + L^l_mn psi^u_m)
  IKR_HIP(hipMemsetAsync(cbuf.get(), 0, vec * sizeof(double2), st));
  IKR_HIP(hipMemsetAsync(tmp.get(), 0, vec * sizeof(double2), st));
  launch_col_inv<double>(s.geom, s.fft, all, psl.get(), nbm, w.T1.get(), nullptr, nullptr,
                         nullptr, st);
  launch_plane_hv<double>(s.geom, s.fft, all, w.T1.get(), w.T2.get(), u.get(), 0, st);
  launch_col_fwd<double>(s.geom, s.fft, all, w.T2.get(), cbuf.get(), nbm, nullptr, nullptr,
                         inv_ng, st);
  launch_col_inv<double>(s.geom, s.fft, all, psu.get(), nbm, w.T1.get(), nullptr, nullptr,
                         nullptr, st);
  launch_plane_hv<double>(s.geom, s.fft, all, w.T1.get(), w.T2.get(), lam.get(), 0, st);
  launch_col_fwd<double>(s.geom, s.fft, all, w.T2.get(), tmp.get(), nbm, nullptr, nullptr,
                         inv_ng, st);
  multiaxpy((int)(2 * vec), 1, reinterpret_cast<const double*>(tmp.get()), 2 * vec, one.get(),
            1.0, reinterpret_cast<double*>(cbuf.get()), st);
  // the occupied slots of k are slot0 = k * nocc .. (fixed occupations)
  const size_t ok = (size_t)no * nbm;
  UpdTerm<double> tl{psl.get(), ok, nbm, s.d_nocc_k.get(), mu.get(), MAXM, -1.0, no};
  UpdTerm<double> tu{psu.get(), ok, nbm, s.d_nocc_k.get(), ml.get(), MAXM, -1.0, no};
  update<double>(s.tiles, s.d_nb.get(), nbm, nullptr, cbuf.get(), nbm, 1.0, tl, tu, nullptr,
                 nullptr, st);

  // E = -Q (H - e)^-1 Q C (the chi0 solve with C as right-hand side), so eta = -E
  Chi0Extra ec;
  ec.rhs_pw = cbuf.get();
  ec.dphi_out = tmp.get();
  ec.tol_relative = true;
  count(apply_chi0_internal(s, nullptr, nullptr, tol, 1, max_iter, 0, 1e-5, schur, &ec));
  // zeta coefficients <psi^l_m, psi^u_n>, then tmp = eta + zeta = -E + Phi coef
  cz.alloc((size_t)J * MAXM);
  gram<double>(s.tiles, s.d_nb.get(), nbm, s.d_nocc_k.get(), no, psl.get(), ok, nbm, psu.get(),
               nbm, w.part.get(), cz.get(), MAXM, st);
  UpdTerm<double> tz{s.d_phi.get(), (size_t)nbn * nbm, nbm, s.d_nocc_k.get(), cz.get(), MAXM,
                     1.0, no};
  update<double>(s.tiles, s.d_nb.get(), nbm, nullptr, tmp.get(), nbm, -1.0, tz,
                 UpdTerm<double>{}, nullptr, nullptr, st);

  // G = sum_k w_k 2 f sum_n [Re(conj psi^u psi^l) - Re(conj psi (eta + zeta))]
  const int gsz = 8, ngrp = (J + gsz - 1) / gsz;
  std::vector<double> wa(J), wb(J, 0.0);
  for (int j = 0; j < J; ++j) {
    const int k = s.slot_k[j];
    wa[j] = 2.0 * s.kp[k].weight * s.occ[(size_t)k * nbn + s.slot_n[j]] / s.volume;
  }
  IKR_HIP(hipMemcpyAsync(s.d_wb.get(), wb.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
  IKR_HIP(hipMemcpyAsync(s.d_wa.get(), wa.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
  launch_col_inv<double>(s.geom, s.fft, all, psu.get(), nbm, w.T1.get(), nullptr, nullptr,
                         nullptr, st);
  launch_col_inv<double>(s.geom, s.fft, all, psl.get(), nbm, w.T2.get(), nullptr, nullptr,
                         nullptr, st);
  launch_plane_rho(s.geom, s.fft, J, s.d_slot_k.get(), w.T1.get(), w.T2.get(), s.d_wa.get(),
                   s.d_wb.get(), gsz, s.d_rhopart.get(), st);
  sum_groups(ng, ngrp, s.d_rhopart.get(), 1.0, g1.get(), st);
  IKR_HIP(hipStreamSynchronize(st));
  for (double& v : wa) v = -v;
  IKR_HIP(hipMemcpyAsync(s.d_wa.get(), wa.data(), J * sizeof(double), hipMemcpyHostToDevice, st));
  launch_col_inv<double>(s.geom, s.fft, all, tmp.get(), nbm, w.T1.get(), nullptr, nullptr,
                         nullptr, st);
  launch_plane_rho(s.geom, s.fft, J, s.d_slot_k.get(), s.d_Tphi.get(), w.T1.get(), s.d_wa.get(),
                   s.d_wb.get(), gsz, s.d_rhopart.get(), st);
  sum_groups(ng, ngrp, s.d_rhopart.get(), 1.0, g2.get(), st);

  // lambda^T chi0 (dK/dA) drho = sum_r a (chi0 s),  s = (chi0 lambda) f_x'(rho) drho
  std::vector<double> total = fetch(g1.get(), ng, st);
  {
    const std::vector<double> h2 = fetch(g2.get(), ng, st);
    for (int i = 0; i < ng; ++i) total[i] += h2[i];
  }
  if (s.xc) {
    Chi0Extra er;
    er.tol_relative = true;
    count(apply_chi0_internal(s, lam.get(), chil.get(), tol, 1, max_iter, 0, 1e-5, schur, &er));
    const std::vector<double> hc = fetch(chil.get(), ng, st);
    const std::vector<double> hd = fetch(drho.get(), ng, st);
    const std::vector<double> hr = fetch(s.d_rho.get(), ng, st);
    std::vector<double> hs(ng);
    double sn = 0;
    for (int i = 0; i < ng; ++i) {
      const double fxp = hr[i] > 1e-10
                             ? (2.0 / 9.0) * std::cbrt(3.0 / PI) * std::pow(hr[i], -5.0 / 3.0)
                             : 0.0;
      hs[i] = hc[i] * fxp * hd[i];
      sn += hs[i] * hs[i];
    }
    if (sn > 0) {
      sv.upload(hs, st);
      count(apply_chi0_internal(s, sv.get(), chis.get(), tol, 1, max_iter, 0, 1e-5, schur, &er));
      const std::vector<double> h3 = fetch(chis.get(), ng, st);
      for (int i = 0; i < ng; ++i) total[i] += h3[i];
    }
  }

  build_dvloc(s);
  std::vector<double> grad(s.natoms, 0.0);
  for (int a = 0; a < s.natoms; ++a) {
    const double* da = s.dvloc.data() + (size_t)a * ng;
    double acc = 0;
    for (int i = 0; i < ng; ++i) acc += da[i] * total[i];
    grad[a] = acc;
  }
  IKR_HIP(hipStreamSynchronize(st));
  return grad;
}

}  // namespace ikr
