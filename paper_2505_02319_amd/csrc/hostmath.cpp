// Host-side numerics of the response solver (declarations and their sources
// in the paper: hostmath.h).
#include "hostmath.h"

#include <algorithm>
#include <cmath>

#include "../../include/ikr.h"

namespace ikr {
namespace host {

double focc(double x) {
  const double e = std::exp(-std::fabs(x));
  return x > 0 ? 2.0 * e / (1.0 + e) : 2.0 / (1.0 + e);
}

double focc_dx(double x) {
  const double e = std::exp(-std::fabs(x));
  return -2.0 * e / ((1.0 + e) * (1.0 + e));
}

double sigma_min(const std::vector<double>& H, int r, int c) {
  std::vector<double> A(H);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int p = 0; p < c; ++p)
      for (int q = p + 1; q < c; ++q) {
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < r; ++i) {
          al += A[i * c + p] * A[i * c + p];
          be += A[i * c + q] * A[i * c + q];
          ga += A[i * c + p] * A[i * c + q];
        }
        if (ga == 0) continue;
        off = std::max(off, std::fabs(ga) / (std::sqrt(al) * std::sqrt(be)));
        const double zeta = (be - al) / (2 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        const double cs = 1 / std::sqrt(1 + t * t), sn = cs * t;
        for (int i = 0; i < r; ++i) {
          const double x = A[i * c + p], y = A[i * c + q];
          A[i * c + p] = cs * x - sn * y;
          A[i * c + q] = sn * x + cs * y;
        }
      }
    if (off < 1e-15) break;
  }
  double mn = 1e300;
  for (int p = 0; p < c; ++p) {
    double n2 = 0;
    for (int i = 0; i < r; ++i) n2 += A[i * c + p] * A[i * c + p];
    mn = std::min(mn, std::sqrt(n2));
  }
  return mn;
}

double small_ls(const std::vector<double>& H, int ld, int i, double beta, std::vector<double>& y) {
  std::vector<double> R((size_t)(i + 1) * i), g(i + 1, 0.0);
  for (int a = 0; a <= i; ++a)
    for (int b = 0; b < i; ++b) R[a * i + b] = H[a * ld + b];
  g[0] = beta;
  for (int j = 0; j < i; ++j) {
    const double a = R[j * i + j], b = R[(j + 1) * i + j];
    const double rr = std::hypot(a, b);
    const double c = rr > 0 ? a / rr : 1.0, sn = rr > 0 ? b / rr : 0.0;
    for (int col = j; col < i; ++col) {
      const double x = R[j * i + col], z = R[(j + 1) * i + col];
      R[j * i + col] = c * x + sn * z;
      R[(j + 1) * i + col] = -sn * x + c * z;
    }
    const double x = g[j], z = g[j + 1];
    g[j] = c * x + sn * z;
    g[j + 1] = -sn * x + c * z;
  }
  y.assign(i, 0.0);
  double miss = 0;   // rows a zero diagonal leaves unsolved (rank-deficient H only)
  for (int j = i - 1; j >= 0; --j) {
    double v = g[j];
    for (int col = j + 1; col < i; ++col) v -= R[j * i + col] * y[col];
    if (R[j * i + j] != 0)
      y[j] = v / R[j * i + j];
    else
      miss = std::hypot(miss, v);
  }
  return miss > 0 ? std::hypot(g[i], miss) : std::fabs(g[i]);
}

double warm_coefficients(const zd* G, int ld, int nv, const zd* h, double bb, std::vector<zd>& c) {
  double tr = 0;
  for (int i = 0; i < nv; ++i) tr += G[i * ld + i].real();
  const double ridge = 1e-12 * tr + 1e-300;
  std::vector<zd> L((size_t)nv * nv, zd(0, 0));
  for (int j = 0; j < nv; ++j) {
    double d = G[j * ld + j].real() + ridge;
    for (int k = 0; k < j; ++k) d -= std::norm(L[(size_t)j * nv + k]);
    if (!(d > 0)) { c.assign(nv, zd(0, 0)); return bb; }
    const double ljj = std::sqrt(d);
    L[(size_t)j * nv + j] = zd(ljj, 0);
    for (int i = j + 1; i < nv; ++i) {
      zd v = G[i * ld + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * nv + k] * std::conj(L[(size_t)j * nv + k]);
      L[(size_t)i * nv + j] = v / ljj;
    }
  }
  // G c = h: L u = h, then L^H c = u
  std::vector<zd> u(nv);
  for (int i = 0; i < nv; ++i) {
    zd v = h[i];
    for (int k = 0; k < i; ++k) v -= L[(size_t)i * nv + k] * u[k];
    u[i] = v / L[(size_t)i * nv + i].real();
  }
  c.assign(nv, zd(0, 0));
  for (int i = nv - 1; i >= 0; --i) {
    zd v = u[i];
    for (int k = i + 1; k < nv; ++k) v -= std::conj(L[(size_t)k * nv + i]) * c[k];
    c[i] = v / L[(size_t)i * nv + i].real();
  }
  double hc = 0;
  for (int i = 0; i < nv; ++i) hc += (std::conj(h[i]) * c[i]).real();
  return bb - hc;
}

double occupation_divided_difference(double fn, double fm, double en, double em, double fermi,
                                     double T, double degen_tol) {
  if (std::fabs(en - em) < degen_tol)
    return T > 0 ? focc_dx((0.5 * (en + em) - fermi) / T) / T : 0.0;
  return (fn - fm) / (en - em);
}

double extra_band_coefficient(double fn, double en, double em, double fermi, double T,
                              double degen_tol) {
  if (std::fabs(en - em) < degen_tol)
    return (T > 0 && fn > 0) ? focc_dx((0.5 * (en + em) - fermi) / T) / (T * fn) : 0.0;
  return 1.0 / (en - em);
}

double band_prefactor(int strategy, const BandTolInputs& a) {
  switch (strategy) {
    case IKR_AGR: return 1.0;
    case IKR_BAL: return a.volume / (2.0 * a.f * a.wk * a.nocc_tot * std::sqrt(a.ng));
    case IKR_GRT:
      return std::sqrt(a.volume) /
             (2.0 * a.f * a.wk * std::sqrt(a.ng) * std::sqrt(a.nocc_tot) * a.knorm * a.orbnorm);
    case IKR_THM2:
      return std::sqrt(a.volume) * a.gap /
             (2.0 * a.f * a.wk * a.knorm * a.orbnorm_full * a.nk * std::sqrt(a.ng * a.nocc_k));
    case IKR_D10: return 0.1;
    case IKR_D100: return 0.01;
    case IKR_D10N: return 0.1 / a.bnorm;
    default: return 1.0;
  }
}

}  // namespace host
}  // namespace ikr
