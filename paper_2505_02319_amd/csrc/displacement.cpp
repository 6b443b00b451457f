// Right-hand side of the Dyson equation for a displaced atom (paper
// Sec. 4.1.2, "Implementation and computational setup": the perturbing
// potential dV0 from displacing atomic positions, and b = chi0 dV0).
//
// For the model potential both parts move with the atom a:
//   - local: the Gaussian's Fourier coefficients -A e^{-s^2|G|^2/2} e^{-iG.R}
//     / |Omega| gain a factor -i G_dir, so dV_loc/dR_{a,dir} is the real part
//     of the same separable cube sum with the axis `dir` differentiated;
//   - nonlocal: p_a(q) carries e^{-iq.R}, so dp_a = -i q_dir p_a (q = G + k)
//     and dV_nl = D (|dp_a><p_a| + |p_a><dp_a|).
// The nonlocal part is not a multiplicative potential, so chi0 is applied
// through the Sternheimer route with its right-hand sides
// t_n = F(dV_loc psi_n) + dV_nl phi_n formed here (eq. kchi0 and
// eq. sternheimer_equation only ever use dV0 phi_n).
#include <cmath>

#include "system.h"

namespace ikr {

Chi0Result displacement_rhs(System& s, int atom, int dir, double cg_tol, double* dv0_ext,
                            double* b_ext) {
  const hipStream_t st = s.stream;
  const int C = s.L.C, P = s.L.P, Q = s.L.Q, nk = s.nk, nbm = s.nb_max, J = s.J;

  // -- dV_loc / dR_{atom, dir} on the grid, internal layout
  DBuf<double> dv;
  {
    const double s2 = s.sigma_loc * s.sigma_loc;
    std::vector<std::vector<double2>> f1(3);
    for (int x = 0; x < 3; ++x) {
      const int n = s.N[x];
      f1[x].assign(n, mk<double>(0, 0));
      for (int i = 0; i < n; ++i) {
        const double rx = i * s.a[x] / n - s.pos[3 * atom + x];
        double re = 0, im = 0;
        for (int m = -n / 2; m < n / 2; ++m) {
          const double g = m * s.b[x];
          const double amp = std::exp(-s2 * g * g / 2.0);
          if (x == dir) {   // (-i g) e^{i g rx}
            re += amp * g * std::sin(g * rx);
            im -= amp * g * std::cos(g * rx);
          } else {
            re += amp * std::cos(g * rx);
            im += amp * std::sin(g * rx);
          }
        }
        f1[x][i] = mk<double>(re, im);
      }
    }
    const double pref = -s.amp[atom] / s.volume;
    std::vector<double> v((size_t)s.ng);
    for (int c = 0; c < C; ++c)
      for (int p = 0; p < P; ++p)
        for (int q = 0; q < Q; ++q) {
          int e[3];
          e[s.cax] = c;
          e[s.pax] = p;
          e[s.qax] = q;
          const double2 t = cmul<double>(cmul<double>(f1[0][e[0]], f1[1][e[1]]), f1[2][e[2]]);
          v[((size_t)c * P + p) * Q + q] = pref * t.x;
        }
    dv.upload(v, st);
  }
  if (dv0_ext) to_external(s.L, dv.get(), dv0_ext, 1.0, nullptr, 0.0, st);

  CgWork<double>& w = s.w64;
  // -- local part of the right-hand sides, t_j = F(dV_loc psi_j), into w.r
  Slots all{J, s.d_slot_k.get(), nullptr};
  launch_plane_hv<double>(s.geom, s.fft, all, s.d_Tphi.get(), w.T2.get(), dv.get(), 0, st);
  launch_col_fwd<double>(s.geom, s.fft, all, w.T2.get(), w.r.get(), nbm, nullptr, nullptr,
                         1.0 / s.ng, st);

  // -- nonlocal part, t_j += D (dp <p, phi_j> + p <dp, phi_j>)
  {
    std::vector<double2> pr((size_t)nk * s.natoms * nbm);
    IKR_HIP(hipMemcpyAsync(pr.data(), s.d_proj.get(), pr.size() * sizeof(double2),
                           hipMemcpyDeviceToHost, st));
    IKR_HIP(hipStreamSynchronize(st));
    // rows [p, dp] (for the gram) and [dp, p] (for the update) per k
    std::vector<double2> w2((size_t)nk * 2 * nbm, mk<double>(0, 0)), w2s(w2.size());
    for (int k = 0; k < nk; ++k) {
      const KPoint& K = s.kp[k];
      for (int g = 0; g < K.nb; ++g) {
        const double2 pv = pr[((size_t)k * s.natoms + atom) * nbm + g];
        const double qd = K.miller[3 * g + dir] * s.b[dir] + K.kcart[dir];
        const double2 dp = mk<double>(qd * pv.y, -qd * pv.x);   // -i q p
        w2[((size_t)k * 2 + 0) * nbm + g] = pv;
        w2[((size_t)k * 2 + 1) * nbm + g] = dp;
        w2s[((size_t)k * 2 + 0) * nbm + g] = dp;
        w2s[((size_t)k * 2 + 1) * nbm + g] = pv;
      }
    }
    DBuf<double2> dw2, dw2s;
    DBuf<int> dm2;
    dw2.upload(w2, st);
    dw2s.upload(w2s, st);
    dm2.upload(std::vector<int>(nk, 2), st);
    // occupied orbitals in slot order (w.p is free here)
    for (int k = 0; k < nk; ++k)
      if (s.nocc_k[k] > 0)
        IKR_HIP(hipMemcpyAsync(w.p.get() + (size_t)s.slot0_k[k] * nbm,
                               s.d_phi.get() + (size_t)k * s.nbands * nbm,
                               (size_t)s.nocc_k[k] * nbm * sizeof(double2),
                               hipMemcpyDeviceToDevice, st));
    gram<double>(s.tiles, s.d_nb.get(), nbm, dm2.get(), 2, dw2.get(), (size_t)2 * nbm, nbm,
                 w.p.get(), nbm, w.part.get(), w.coefA.get(), MAXM, st);
    UpdTerm<double> t{dw2s.get(), (size_t)2 * nbm, nbm, dm2.get(), w.coefA.get(), MAXM, s.dnl, 2};
    update<double>(s.tiles, s.d_nb.get(), nbm, nullptr, w.r.get(), nbm, 1.0, t, UpdTerm<double>{},
                   nullptr, nullptr, st);
    IKR_HIP(hipStreamSynchronize(st));
  }

  // -- chi0 through the Sternheimer route with these right-hand sides
  Chi0Extra ex;
  ex.rhs_pw = w.r.get();
  ex.tol_relative = true;
  std::vector<double> tol(J, cg_tol);
  Chi0Result r = apply_chi0_internal(s, nullptr, s.d_drho.get(), tol, 1, 1000, 0, 1e-5, 0, &ex);
  to_external(s.L, s.d_drho.get(), b_ext, 1.0, nullptr, 0.0, st);
  IKR_HIP(hipStreamSynchronize(st));
  return r;
}

}  // namespace ikr
