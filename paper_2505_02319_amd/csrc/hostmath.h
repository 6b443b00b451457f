// Host-side numerics of the response solver, free of HIP so that they also
// build with the host sanitizers into a check program of their own:
//  - the small dense problems of Algorithm 1 (the GMRES least-squares problem
//    on the Hessenberg matrix, the smallest singular value that serves as the
//    estimate s of the smallest singular value of the operator),
//  - the smeared occupations and the divided differences of the minimal-gauge
//    occupied-space term (eq. delta_phi_P, eq. delta_f),
//  - the per-band CG tolerance prefactors (Table 1 in its k-point form,
//    Table strategies_k, Theorem 2),
//  - the least-squares warm start over stored right-hand sides.
#pragma once

#include <complex>
#include <vector>

namespace ikr {
namespace host {

using zd = std::complex<double>;

// 2 / (1 + e^x) (spin-degenerate Fermi-Dirac occupation at x = (e - e_F) / T),
// without overflow at any finite x, and its derivative in x.
double focc(double x);
double focc_dx(double x);

// Smallest singular value of the r x c row-major matrix H (one-sided Jacobi,
// at most 60 sweeps).  c = 0 gives +inf's stand-in 1e300.
double sigma_min(const std::vector<double>& H, int r, int c);

// min_y || beta e_1 - H y || over the (i + 1) x i upper Hessenberg matrix
// stored row-major with leading size ld (rows 0..i, columns 0..i-1 used), by
// Givens rotations; y gets i entries (0 where a rotated diagonal entry is 0,
// which only a rank-deficient H has).  Returns || beta e_1 - H y || for that
// y (the least-squares residual when H has full column rank); i = 0 returns
// |beta|.
double small_ls(const std::vector<double>& H, int ld, int i, double beta, std::vector<double>& y);

// Least squares over nv stored right-hand sides b_l of one band: c minimising
// || b - sum_l c_l b_l || from their Gram matrix G (G[i * ld + j] = <b_i, b_j>,
// row-major) and h_l = <b_l, b>, by Cholesky of G with a ridge of 1e-12 of its
// trace.  Returns the predicted squared residual ||b||^2 - Re(h^H c) (bb =
// ||b||^2); a G that is not positive definite even with the ridge gives c = 0
// and bb.
double warm_coefficients(const zd* G, int ld, int nv, const zd* h, double bb, std::vector<zd>& c);

// (f_n - f_m) / (e_n - e_m), the divided difference of the occupations of an
// occupied pair, with its limit f'((e_n + e_m) / 2) (f' in energy) when the
// energies lie within degen_tol; 0 in that limit at T = 0.
double occupation_divided_difference(double fn, double fm, double en, double em, double fermi,
                                     double T, double degen_tol);

// Coefficient of <phi_m, t_n> for an extra (unoccupied) computed band m taken
// by sum over states: 1 / (e_n - e_m), or within degen_tol the limit of the
// divided difference over f_n, f'((e_n + e_m) / 2) / f_n (0 at T = 0 or f_n = 0).
double extra_band_coefficient(double fn, double en, double em, double fermi, double T,
                              double degen_tol);

// What the prefactor of one band (k, n) depends on.
struct BandTolInputs {
  double volume = 1;        // cell volume |Omega|
  double ng = 1;            // real-space grid points
  double nocc_tot = 1;      // occupied (k, n) pairs in all (the paper's N_occ)
  double f = 1;             // occupation f_nk
  double wk = 1;            // k-point weight
  double knorm = 1;         // ||K v|| (or its bound for the adjoint)
  double orbnorm = 1;       // (2, inf) norm of the real parts of k's orbitals (grt)
  double orbnorm_full = 1;  // (2, inf) norm of k's computed orbitals (Theorem 2)
  double nk = 1;            // k-points
  double nocc_k = 1;        // occupied bands at k
  double gap = 1;           // e_up - e_n, the CG operator's spectral gap (Theorem 2)
  double bnorm = 1;         // ||b|| of the GMRES right-hand side (D10n)
};

// The prefactor C_{nk} that multiplies the common factor of a GMRES step to
// give band (k, n) its CG tolerance, for strategy (the IKR_* values of the
// library's header: agr, bal, grt, D10, D100, D10n, fixed, thm2).
double band_prefactor(int strategy, const BandTolInputs& a);

}  // namespace host
}  // namespace ikr
