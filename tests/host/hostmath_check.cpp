// Check program for the library's host-side numerics (hostmath.cpp), built
// by the host compiler with the address and undefined-behaviour sanitizers.
// Reads one command per line on stdin and answers each with one line of
// numbers (%.17g) on stdout; test_host_numerics.py drives it and compares
// the answers with numpy.
//
//   ls ld i beta H[(i+1)*ld]         -> resid y[0..i-1]
//   sv r c H[r*c]                    -> sigma_min
//   warm ld nv bb G[nv*ld] h[nv]     -> pred c[0..nv-1]   (complex: re im pairs)
//   focc x                           -> f(x) f'(x)
//   odd fn fm en em fermi T tol      -> divided difference
//   ebc fn en em fermi T tol         -> extra-band coefficient
//   pref strategy volume ng nocc_tot f wk knorm orbnorm orbnorm_full nk nocc_k gap bnorm
//                                    -> prefactor
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../../paper_2505_02319_amd/csrc/hostmath.h"

using namespace ikr::host;

static void put(double v) { std::printf(" %.17g", v); }

// one number (strtod: also nan and inf)
static double num(std::istream& in) {
  std::string t;
  in >> t;
  return std::strtod(t.c_str(), nullptr);
}

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string cmd;
    if (!(in >> cmd)) continue;
    if (cmd == "ls") {
      int ld, i;
      in >> ld >> i;
      const double beta = num(in);
      std::vector<double> H((size_t)(i + 1) * ld);
      for (double& v : H) v = num(in);
      std::vector<double> y;
      std::printf("%.17g", small_ls(H, ld, i, beta, y));
      for (double v : y) put(v);
    } else if (cmd == "sv") {
      int r, c;
      in >> r >> c;
      std::vector<double> H((size_t)r * c);
      for (double& v : H) v = num(in);
      std::printf("%.17g", sigma_min(H, r, c));
    } else if (cmd == "warm") {
      int ld, nv;
      in >> ld >> nv;
      const double bb = num(in);
      std::vector<zd> G((size_t)nv * ld), h(nv);
      for (zd& v : G) { const double a = num(in); v = zd(a, num(in)); }
      for (zd& v : h) { const double a = num(in); v = zd(a, num(in)); }
      std::vector<zd> c;
      std::printf("%.17g", warm_coefficients(G.data(), ld, nv, h.data(), bb, c));
      for (const zd& v : c) { put(v.real()); put(v.imag()); }
    } else if (cmd == "focc") {
      const double x = num(in);
      std::printf("%.17g %.17g", focc(x), focc_dx(x));
    } else if (cmd == "odd") {
      double v[7];
      for (double& x : v) x = num(in);
      std::printf("%.17g", occupation_divided_difference(v[0], v[1], v[2], v[3], v[4], v[5], v[6]));
    } else if (cmd == "ebc") {
      double v[6];
      for (double& x : v) x = num(in);
      std::printf("%.17g", extra_band_coefficient(v[0], v[1], v[2], v[3], v[4], v[5]));
    } else if (cmd == "pref") {
      int strategy;
      in >> strategy;
      BandTolInputs a;
      for (double* x : {&a.volume, &a.ng, &a.nocc_tot, &a.f, &a.wk, &a.knorm, &a.orbnorm,
                        &a.orbnorm_full, &a.nk, &a.nocc_k, &a.gap, &a.bnorm})
        *x = num(in);
      std::printf("%.17g", band_prefactor(strategy, a));
    } else {
      std::fprintf(stderr, "unknown command %s\n", cmd.c_str());
      return 2;
    }
    if (in.fail()) {
      std::fprintf(stderr, "short input for %s\n", cmd.c_str());
      return 2;
    }
    std::printf("\n");
  }
  return 0;
}
