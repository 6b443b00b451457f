/*
 * ikr.h -- C ABI of the MI355X (gfx950) inexact-Krylov linear-response library.
 *
 * The library solves the discretised Dyson equation  E drho = b  with
 * E = 1 - chi0 K  (the dielectric adjoint; paper Sec. 2.2, eq. dyson_discretised)
 * by inexact GMRES(m) (paper Alg. 1) whose operator applications solve the
 * Sternheimer equations of every occupied band and k-point by preconditioned
 * CG under the adaptive per-band tolerances of paper Table 1 / Table
 * strategies_k, then accumulate the density response (eq. kchi0).
 *
 * Conventions shared by every entry point
 *   - Grid vectors (potentials, densities, b, drho) are real FP64 arrays of
 *     length N_g = fft[0]*fft[1]*fft[2] in C order [N0][N1][N2] (index 2
 *     fastest), values on the real-space grid of paper Sec. 2.3.1.  Norms of
 *     grid vectors are plain Euclidean norms of these values.
 *   - Orbital-coefficient vectors are complex128 (interleaved re, im) with a
 *     row stride of nb_max complex numbers, in the basis order returned by
 *     ikr_get_basis (per k-point).
 *   - Pointers named *_dev are device pointers (hipMalloc'd memory of the
 *     device that was current at setup); *_host are host pointers.  The
 *     caller owns every buffer it passes; the library never frees them.
 *   - Every call enqueues its work on the HIP stream given at setup and
 *     returns after that work has completed (host-side scalars are needed
 *     by the GMRES loop).  A handle is not thread-safe; separate handles are
 *     independent.
 *   - Errors are returned as ikr_status codes; no C++ exception crosses the
 *     ABI.  ikr_last_error() returns a message for the last failing call on
 *     the calling thread.
 */
#ifndef IKR_H
#define IKR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ikr_system* ikr_handle;

typedef enum {
  IKR_OK = 0,
  IKR_E_ARG = 1,       /* invalid argument (null pointer, size, unsupported grid) */
  IKR_E_STATE = 2,     /* handle not ready for this call */
  IKR_E_NOGAP = 3,     /* no gap above the occupied bands of some k-point */
  IKR_E_NOCONV = 4,    /* a CG or GMRES iteration cap was hit (best result written) */
  IKR_E_NAN = 5,       /* non-finite input or intermediate */
  IKR_E_OOM = 6,       /* device allocation failed */
  IKR_E_HIP = 7,       /* HIP runtime error */
  IKR_E_INTERNAL = 8
} ikr_status;

/* CG-tolerance strategies: paper Table 1 (agr, bal, grt and the baselines
 * D10, D100, D10n) in the k-point form of Table strategies_k.  IKR_FIXED
 * applies the common factor unchanged to every band.  IKR_THM2 is the
 * prefactor C_{i,nk} of Theorem 2 itself (k-point form of the supplement:
 * gap e_{Nocc,k + 1} - e_{nk}, ||K v_i||, the full ||F_k^-1 Phi_k||_{2,inf},
 * N_mp sqrt(N_g Nocc,k)), i.e. the guarantee without the approximations
 * behind grt. */
typedef enum {
  IKR_AGR = 0, IKR_BAL = 1, IKR_GRT = 2, IKR_D10 = 3, IKR_D100 = 4,
  IKR_D10N = 5, IKR_FIXED = 6, IKR_THM2 = 7
} ikr_strategy;

/* Model system (host memory, read during ikr_setup_system only).
 * Orthorhombic cell; per atom a Gaussian local potential with Fourier
 * coefficients -amp * exp(-sigma_loc^2 |G|^2 / 2) e^{-iG.R} / |Omega| and an
 * L2-normalised Gaussian separable projector of width sigma_proj and
 * strength d_proj (Ha).  Gamma-centred k-grid kgrid (no symmetry reduction).
 * temperature = 0: nocc doubly occupied bands per k; > 0: Fermi-Dirac
 * smearing of 2*nocc electrons over nocc + nextra bands. */
typedef struct {
  double lattice[3];        /* cell lengths a_i (bohr) */
  int natoms;
  const double* frac_pos;   /* [natoms][3] fractional positions */
  const double* amp;        /* [natoms] local-potential amplitudes */
  double sigma_loc;         /* bohr */
  double sigma_proj;        /* bohr */
  double d_proj;            /* Ha */
  double ecut;              /* Ha; sphere |G + k|^2 <= 2 ecut (eq. fourier_bases) */
  int fft[3];               /* real-space grid; each a product of 2, 3, 5 in the
                               supported set (see ikr_supported_fft_size) */
  int kgrid[3];
  int nocc;
  int nextra;
  double temperature;       /* Ha */
  int xc;                   /* 0: Hartree kernel only, 1: + Slater exchange */
} ikr_system_desc;

/* Optional imported ground state (host memory).  eps [nk][nbands] ascending
 * per k; coeffs complex128 [nk][nbands][nb_max] orthonormal per k, in the
 * ikr_get_basis order of each k (entries beyond nb_k ignored).  The basis
 * order is known only after setup, so an import is made by
 * ikr_import_ground_state on a handle set up with compute_ground_state = 0. */
typedef struct {
  const double* eps;
  const double* coeffs;
} ikr_ground_state;

typedef struct {
  int strategy;             /* ikr_strategy */
  double tol;               /* GMRES tolerance tau */
  int tol_is_relative;      /* 1: tau = tol * ||b|| */
  int restart_m;            /* GMRES restart size m (default 20) */
  double s0;                /* initial estimate s of sigma_m(H_m) (default 1) */
  int max_restarts;         /* default 50 */
  int precision;            /* 0: FP64 Sternheimer CG, 1: FP32 CG where loose */
  int cg_min_iter;          /* default 1 (paper Sec. 4.1.2) */
  int cg_max_iter;          /* default 1000 */
  double fp32_theta;        /* FP32 used when tau_nk >= theta * ||b_nk|| */
  double b_norm;            /* ||b|| for D10n inside ikr_apply_dielectric */
  int want_true_residual;   /* 1: report ||b - E x|| with tight CG at exit */
  double true_res_cg_tol;   /* CG tolerance of the true-residual apply (1e-14) */
  int schur;                /* 1: the computed unoccupied bands take their part of
                               the orbital response by sum over states and the CG
                               runs on the complement of all computed bands (the
                               extra-band / Schur-complement treatment the paper's
                               runs use, Sec. 4.1.2); 0: CG on the complement of
                               the occupied bands only (default 1) */
  int batching;             /* 0: one launch per kernel in every Sternheimer CG
                               iteration; 1: each iteration is one replay of a
                               captured HIP graph (graphs are cached on the handle
                               per grid size; the caller's stream may be the
                               default stream: capture and replay use a private
                               stream joined to it).  Results agree with mode 0
                               to rounding (grids sized to a power of two may
                               split sums differently); replays are bitwise
                               reproducible.
                               Kernel profiling (ikr_profile_enable) switches
                               graphs off.  2: the plain FP64 reference path:
                               the k-points' Sternheimer CGs one after the
                               other, the host reading the live count after
                               every CG iteration, FP64 throughout (precision
                               ignored).  Default 0 */
  const double* x0;         /* device, nullable: initial guess x0 of Alg. 1 (grid
                               values, C order, caller-owned, not written).  With
                               x0 != 0 the first residual b - E~ x0 is formed with
                               the tolerance tau/3 (Alg. 1, first line), so a solve
                               can resume from a saved iterate; s0 can carry the
                               saved estimate s.  Default NULL (x0 = 0) */
  int kerker;               /* 1: solve the Kerker-preconditioned equation
                               T E drho = T b (eq. precond_dyson) with T of
                               eq. kerker; the estimated residual and tau then refer
                               to T (b - E x), which Theorem 2 still bounds since
                               ||T|| = 1 (Lemma kerker_properties); true_res stays
                               ||b - E x||.  Forward solves only.  Default 0 */
  double kerker_alpha;      /* alpha of the Kerker symbol |G|^2/(|G|^2 + alpha^2),
                               1/bohr (default 0.8) */
  int recycle;              /* Sternheimer warm starts across dielectric
                               applications (0..8, default 0: off): the last
                               `recycle` right-hand sides and CG solutions of every
                               band are kept on the device (2 recycle J nb_max
                               complex), and a band's CG starts from the
                               least-squares combination of its earlier solutions
                               whenever that leaves under a tenth of the new
                               right-hand side (its residual b - A x0 is formed
                               with one FP64 H application).  Reset at the start
                               of every solve. */
} ikr_solver_opts;

typedef struct {
  long long n_ham;          /* Hamiltonian band-applications (one per CG iter) */
  long long n_ham_fp32;
  long long n_ham_fp64;
  int gmres_iters;
  int restarts;
  int cg_unconverged;       /* Sternheimer solves that hit the iteration cap or
                               broke down (after any FP64 fallback) */
  double est_res;           /* final estimated GMRES residual */
  double true_res;          /* ||b - E x|| if requested, else -1 */
  double s_final;
  double sigma_min;
  double knorm_last;        /* ||K v|| of the last dielectric application */
  double seconds;
  long long fp64_fallback;  /* FP32 Sternheimer solves continued in FP64 because their
                               true residual b - A x was above the tolerance (defect
                               correction from the FP32 iterate; from zero if the FP32
                               CG did not converge) */
  long long fp32_checked;   /* FP32 Sternheimer solves whose true residual was checked
                               with one FP64 H application (tolerance below 1e-3 ||b||,
                               or FP32 CG not converged) */
  long long warm_started;   /* Sternheimer solves started from earlier solutions
                               (solver option recycle) */
} ikr_stats;

/* Fill opts with the defaults above (strategy bal, tol 1e-8 relative). */
void ikr_default_opts(ikr_solver_opts* opts);

/* 1 if n is a supported FFT length (products of 2, 3, 5 in the library's
 * compiled set), else 0. */
int ikr_supported_fft_size(int n);

/* Build the discretisation (paper Sec. 2.3.1), the local potential on the
 * grid, the projectors, and -- if gs is NULL -- the ground state by the
 * library's own block eigensolver on the GPU; occupations, Fermi level,
 * density, per-k gaps.  stream: hipStream_t (may be NULL for the default
 * stream).  Returns IKR_E_NOGAP if some k has e_{Nocc+1} - e_{Nocc} < 1e-6 Ha
 * (Lemma cgtol_E needs a gap); the handle is still created in that case. */
ikr_status ikr_setup_system(const ikr_system_desc* desc, void* stream,
                            int compute_ground_state, ikr_handle* out);

/* Import eigenpairs (host) for a handle created with compute_ground_state=0;
 * completes setup (occupations, density, caches). */
ikr_status ikr_import_ground_state(ikr_handle h, const ikr_ground_state* gs);

/* Sizes: nk, nbands, nb_max, N_g, and per-k occupied counts (host [nk]). */
ikr_status ikr_get_info(ikr_handle h, int* nk, int* nbands, int* nb_max,
                        int* ng, int* nocc_k_host);

/* Basis of k-point k: nb_k and the Miller indices [nb_k][3] in the order the
 * library uses (G = sum_i m_i b_i, |G + k|^2 <= 2 ecut).  miller_host may be
 * NULL to query nb_k only. */
ikr_status ikr_get_basis(ikr_handle h, int k, int* nb_k, int* miller_host);

/* Ground state (host): eps [nk][nbands], occupations [nk][nbands],
 * coefficients complex128 [nk][nbands][nb_max] (may be NULL), Fermi level. */
ikr_status ikr_get_ground_state(ikr_handle h, double* eps_host,
                                double* occ_host, double* coeffs_host,
                                double* fermi_host);

/* Setup diagnostics (host): gaps_host [nk] = e_{Nocc,k + 1} - e_{Nocc,k}
 * (NaN where every computed band is occupied), the number of outer steps of
 * the library's eigensolver (0 for an imported ground state) and the largest
 * eigen-residual norm ||H phi - e phi|| it reached.  Any pointer may be NULL. */
ikr_status ikr_get_setup_info(ikr_handle h, double* gaps_host, int* gs_iters,
                              double* gs_residual);

/* Orbital terms of the tolerance strategies (host, [nk] each, may be NULL):
 * full_host[k] = ||F_k^-1 Phi_k||_{2,inf} over the occupied orbitals (the
 * maximum over grid points of the row norm, with psi normalised on the cell;
 * Lemma cgtol_E and Theorem 2) and re_host[k] the same of the real parts
 * (grt, Sec. 3.4.1), each orbital taken with the phase that makes
 * sum_r psi(r)^2 real and positive, floored at full_host[k] / sqrt(2). */
ikr_status ikr_get_orbital_norms(ikr_handle h, double* re_host, double* full_host);

/* Ground-state density on the grid (device, C order). */
ikr_status ikr_get_density(ikr_handle h, double* rho_dev);

/* y = H_k x for nvec vectors (device, complex128 [nvec][nb_max]); the
 * kinetic, local (FFT) and nonlocal terms of eq. Hamiltonian, Bloch form. */
ikr_status ikr_apply_hamiltonian(ikr_handle h, int k, int nvec,
                                 const double* x_dev, double* y_dev);

/* y = H_k x exactly as ikr_apply_hamiltonian, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the call allocates nothing.  Its
 * work space (2 nvec * C * ncol_max complex column buffers plus small tables)
 * is a fixed 64 MiB device array per GPU, held until the process ends;
 * nvec beyond what fits returns IKR_E_ARG with the limit in the message
 * (e.g. about 40 vectors on a 48^3 grid).  All calls on one GPU share that
 * array, so calls that overlap in time on one GPU race.  On a stream under
 * graph capture the call only enqueues its work; otherwise it returns after
 * completion.  Same arguments, layout and ownership as
 * ikr_apply_hamiltonian. */
ikr_status ikr_apply_hamiltonian_noalloc(ikr_handle h, int k, int nvec,
                                         const double* x_dev, double* y_dev);

/* kv = K v, K = K_H + K_xc at the ground-state density (device grid
 * vectors).  Hartree 4 pi/|G|^2 with G = 0 -> 0 (paper Sec. 3.4.3). */
ikr_status ikr_apply_hxc_kernel(ikr_handle h, const double* v_dev,
                                double* kv_dev);

/* out = T v with the Kerker preconditioner of eq. kerker:
 * T = W^-1 (D + (1 - D_11) e_1 e_1^T) W, D = diag(|G|^2 / (|G|^2 + alpha^2))
 * over the FFT cube (|G| from the signed index), i.e. the charge-conserving
 * form that keeps the G = 0 component (Lemma kerker_properties: T Hermitian
 * positive definite, ||T|| = 1).  v_dev, out_dev: device FP64 grid values
 * (C order), caller-owned, may alias.  alpha > 0 (1/bohr), else IKR_E_ARG. */
ikr_status ikr_apply_kerker(ikr_handle h, double alpha, const double* v_dev,
                            double* out_dev);

/* Right-hand side of the Dyson equation for the displacement of one atom
 * (Sec. 4.1.2: the perturbing potential dV0 of displaced atomic positions):
 * b = chi0 dV0 with dV0 = dV_ext / dR_{atom, direction}, the derivative of
 * both parts of the model potential -- the local Gaussian (whose Fourier
 * coefficients gain a factor -i G_dir) and the nonlocal projector of that
 * atom (dV_nl = D (|dp><p| + |p><dp|), dp = -i q_dir p, q = G + k).  The
 * nonlocal part acts on the orbitals' coefficients, so chi0 is applied with
 * the Sternheimer right-hand sides dV0 phi_n formed directly.  dv0_dev
 * (nullable, device, grid values) receives the local part of dV0; b_dev
 * (device) receives b.  cg_tol: CG tolerance relative to each band's
 * Sternheimer right-hand side, in (0, 1) (1e-10 gives b to about 1e-9).
 * Errors: IKR_E_ARG for an atom or direction out of range or a
 * non-positive tolerance; IKR_E_STATE without a ground state; IKR_E_NOCONV
 * when a CG hit its cap (b still written). */
ikr_status ikr_displacement_rhs(ikr_handle h, int atom, int direction, double cg_tol,
                                double* dv0_dev, double* b_dev, ikr_stats* stats);

/* drho = chi0 dv through the Sternheimer route (eq. kchi0, eq.
 * delta_phi_P, eq. sternheimer_equation, eq. delta_f).  CG tolerances are
 * absolute on the Sternheimer right-hand sides of dv: cg_tol for every band,
 * or per band from cg_tol_host [nk][nbands] (entries of unoccupied bands
 * ignored) when non-NULL. */
ikr_status ikr_apply_chi0(ikr_handle h, const double* dv_dev, double* drho_dev,
                          double cg_tol, const double* cg_tol_host,
                          ikr_stats* stats);

/* ev = E~ v = v - ||K v|| chi0~(K v / ||K v||)  (eq. op_discretised), the
 * per-band CG tolerances being prefactor(strategy) * common  (Table 1). */
ikr_status ikr_apply_dielectric(ikr_handle h, const double* v_dev,
                                double* ev_dev, double common,
                                const ikr_solver_opts* opts, ikr_stats* stats);

/* drho solving E drho = b by inexact GMRES(m), Alg. 1. */
ikr_status ikr_solve_response(ikr_handle h, const double* b_dev,
                              double* drho_dev, const ikr_solver_opts* opts,
                              ikr_stats* stats);

/* ev = E~^T v = v - ||v|| K chi0~(v / ||v||), the transpose of eq.
 * op_discretised's operator (E^T = 1 - K chi0, K and chi0 being symmetric in
 * the grid inner product; the transpose is not in the paper).  The per-band
 * CG tolerances are prefactor(strategy) * common as in ikr_apply_dielectric,
 * with ||K v|| replaced by ||K||_2 ||v|| (the CG error now passes through K).
 * Same arguments, layout, ownership and errors as ikr_apply_dielectric. */
ikr_status ikr_apply_dielectric_adjoint(ikr_handle h, const double* v_dev,
                                        double* ev_dev, double common,
                                        const ikr_solver_opts* opts,
                                        ikr_stats* stats);

/* lambda solving E^T lambda = g by the inexact GMRES(m) of Alg. 1 applied to
 * the transposed operator: lambda = dL/db for a loss L(drho) with
 * g = dL/d(drho) and drho = E^-1 b.  g_dev, lambda_dev: device, FP64, N_g
 * grid values in C order; caller-owned; must not alias.  Errors as
 * ikr_solve_response (IKR_E_NOCONV when the restart cap is hit, lambda then
 * holding the last iterate). */
ikr_status ikr_solve_response_adjoint(ikr_handle h, const double* g_dev,
                                      double* lambda_dev,
                                      const ikr_solver_opts* opts,
                                      ikr_stats* stats);

/* dL/dA_a for every atom a, the A_a being the local-potential amplitudes
 * (V_loc = sum_a A_a a_a(r)), given drho = E^-1 b and lambda = E^-T dL/d(drho)
 * (ikr_solve_response / ikr_solve_response_adjoint).  With u = K drho:
 *   dL/dA_a = lambda^T (d chi0/dA_a) u + lambda^T chi0 (dK/dA_a) drho,
 * the first term by the third-order (2n+1) form of the band energy with the
 * first-order orbitals psi^u, psi^lambda and one adjoint Sternheimer solve per
 * band, the second through two chi0 applications (dK/dA_a = f_x' chi0 a_a,
 * the potential being fixed, not self-consistent).  Not in the paper; built
 * on its Sternheimer route (eq. sternheimer_equation, eq. kchi0).
 * drho_dev, lambda_dev: device FP64 grid values (C order), caller-owned.
 * dlda_host: host array of natoms doubles, written on success.  cg_tol: CG
 * tolerance relative to each right-hand side, in (0, 1) (1e-12 for
 * gradients good to ~1e-8).  Errors: IKR_E_ARG for null pointers, a bad
 * tolerance or smeared occupations (only fixed occupations are supported),
 * IKR_E_STATE without a ground state, IKR_E_NAN for a non-finite result. */
ikr_status ikr_grad_amplitudes(ikr_handle h, const double* drho_dev,
                               const double* lambda_dev, double cg_tol,
                               double* dlda_host, ikr_stats* stats);

/* Kernel-path selection (process-wide; for tests and tuning).  Every path
 * computes the same quantities; by default (mask 0) each launch picks its
 * path by size.  Bit 0 forces the vector-FMA projections: the gram (otherwise
 * the per-tile matrix-core gram below 65 projection rows, the k-wide
 * matrix-core gram above) and the CG update (otherwise on the matrix cores,
 * one 16-band tile per block), bit 1 the two-launch end of a CG iteration (otherwise one
 * block while the batch has few partials), bit 2 the k-wide matrix-core gram
 * (all bands of a k-point per block) at any row count, bit 3 the size rules
 * alone for every launch shape (no setup-time tuning, below).
 * Unknown bits: IKR_E_ARG.  ikr_get_kernel_paths returns the current mask. */
ikr_status ikr_set_kernel_paths(int mask);
int ikr_get_kernel_paths(void);

/* Launch shapes picked by measurement.  At the first Sternheimer CG run of
 * each precision, a system times the candidates of three launch shapes of
 * the CG iteration with HIP events on its stream (one untimed and three
 * timed runs each, each after the kernels that precede it in a CG
 * iteration) and keeps the fastest: the projection gram's kernel and block
 * count, the CG update's band group, and the plane kernel's block size.  It
 * does so for the batch the run starts with, when that batch has more tiles
 * of 16 bands than k-points ("thick"), and for batches of at most 8 and at
 * most 2 bands per k-point, with the run's own batch when that is thin too
 * ("thin": the late iterations, times added); each iteration then takes the
 * shapes of its class.  The size rule is one of the candidates and is kept
 * unless another is more than 15% faster.
 * IKR_VERBOSE=1 in the environment logs every candidate's time to stderr.
 * ikr_get_tuning fills out[24]: for precision p (0 FP64, 1 FP32) and class c
 * (0 thick, 1 thin), the 6 entries from out[12 p + 6 c] are: measured (1) or
 * not yet (0); the gram kernel (0 size rule, 1 per-tile matrix-core, 2
 * k-wide matrix-core, 3 vector-FMA); the gram's block-count scale in percent
 * (50, 100, 200); the CG update's bands per block (0: the size rule, the
 * matrix-core update; 4, 8, 16: the vector update with that band group); the
 * plane kernel's threads per block (0 size rule, 256, 512); the picked
 * gram's time in ns (summed over the class's batches).  Errors: IKR_E_ARG for
 * a null handle or out. */
ikr_status ikr_get_tuning(ikr_handle h, int* out);
/* Measures the launch shapes now rather than at the first CG run (so that a
 * caller can count it as set-up): FP64, and FP32 too when precision != 0,
 * on all occupied bands with the projection rows of the schur option
 * (0: occupied bands, 1: every computed band); classes already measured or
 * set are kept.  Synchronises the system's stream.  Errors: IKR_E_ARG for a
 * null handle, IKR_E_STATE without a ground state. */
ikr_status ikr_tune_launches(ikr_handle h, int precision, int schur);
/* Sets the launch shapes by hand (tests, and callers that measured them
 * before): in[24] in ikr_get_tuning's layout.  An entry whose first value is
 * 0 is cleared (measured again at the next CG run that needs it); otherwise
 * its gram kernel (0..3; a kernel the shape does not admit falls back to the
 * size rule), scale (50, 100, 200), bands per block (0, 4, 8, 16; a group
 * whose coefficients do not fit 64 KiB of LDS falls back to the size rule)
 * and plane threads (0, 256, 512) are used as given, and its time is ignored.
 * Errors: IKR_E_ARG for a null handle or in, or a value outside those sets. */
ikr_status ikr_set_tuning(ikr_handle h, const int* in);

/* Opt-in kernel timing (process-wide).  Bit i of kernel_mask brackets every
 * launch of hot kernel i of the Sternheimer CG by HIP events on the launching
 * stream (0 disables, -1 times all); each launch carries its algorithmic
 * byte count (bytes the kernel must move to or from HBM by its definition,
 * not by measurement).  kernel_id indexes ikr_profile_kernel_name
 * (0 .. ikr_profile_kernel_count()-1); the FP32 launches of the mixed-
 * precision CG are timed under their own ids (names ending in "_fp32"). */
ikr_status ikr_profile_enable(int kernel_mask);
ikr_status ikr_profile_reset(void);
int ikr_profile_kernel_count(void);
const char* ikr_profile_kernel_name(int kernel_id);
ikr_status ikr_profile_query(int kernel_id, long long* launches, double* total_ms,
                             double* total_bytes);

const char* ikr_last_error(void);
void ikr_destroy(ikr_handle h);

#ifdef __cplusplus
}
#endif
#endif /* IKR_H */
