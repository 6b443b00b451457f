// extern "C" boundary of the library (declared in include/ikr.h).  Every
// entry point validates its arguments, converts C++ exceptions to status
// codes and records a thread-local message for ikr_last_error().
#include <cmath>
#include <cstring>
#include <string>

#include "ktimer.h"
#include <algorithm>
#include <cmath>

#include "system.h"

using ikr::Error;
using ikr::System;

namespace {

thread_local std::string g_last_error;

template <typename F> ikr_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return IKR_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return (ikr_status)e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return IKR_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return IKR_E_INTERNAL;
  } catch (...) {
    g_last_error = "unknown error";
    return IKR_E_INTERNAL;
  }
}

System* sys_of(ikr_handle h) {
  IKR_CHECK(h, IKR_E_ARG, "null handle");
  return reinterpret_cast<System*>(h);
}

void check_opts(const ikr_solver_opts* o) {
  IKR_CHECK(o, IKR_E_ARG, "null solver options");
  IKR_CHECK(o->strategy >= IKR_AGR && o->strategy <= IKR_THM2, IKR_E_ARG, "bad strategy");
  IKR_CHECK(o->tol > 0 && std::isfinite(o->tol), IKR_E_ARG, "tolerance must be positive");
  IKR_CHECK(o->restart_m >= 1 && o->restart_m <= 60, IKR_E_ARG, "restart size must be in [1, 60]");
  IKR_CHECK(o->cg_min_iter >= 0 && o->cg_max_iter >= 1, IKR_E_ARG, "bad CG iteration limits");
  IKR_CHECK(o->s0 > 0, IKR_E_ARG, "s0 must be positive");
  IKR_CHECK(o->precision == 0 || o->precision == 1, IKR_E_ARG, "precision must be 0 or 1");
  IKR_CHECK(o->batching >= 0 && o->batching <= 2, IKR_E_ARG, "batching must be 0, 1 or 2");
  IKR_CHECK(o->kerker == 0 || o->kerker == 1, IKR_E_ARG, "kerker must be 0 or 1");
  IKR_CHECK(o->recycle >= 0 && o->recycle <= 8, IKR_E_ARG, "recycle must be in [0, 8]");
  IKR_CHECK(!o->kerker || (o->kerker_alpha > 0 && std::isfinite(o->kerker_alpha)), IKR_E_ARG,
            "kerker_alpha must be positive");
}

// The CG launch mode of one call (restored on exit, also on errors).
struct GraphMode {
  System* s;
  GraphMode(System* sys, const ikr_solver_opts* o) : s(sys) {
    s->cg_graph = o->batching == 1;
    s->cg_plain = o->batching == 2;
    s->cg_recycle = o->recycle;
  }
  ~GraphMode() { s->cg_graph = 0; s->cg_plain = 0; s->cg_recycle = 0; }
};

}  // namespace

extern "C" {

void ikr_default_opts(ikr_solver_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->strategy = IKR_BAL;
  o->tol = 1e-8;
  o->tol_is_relative = 1;
  o->restart_m = 20;
  o->s0 = 1.0;
  o->max_restarts = 50;
  o->precision = 0;
  o->cg_min_iter = 1;
  o->cg_max_iter = 1000;
  o->fp32_theta = 1e-5;
  o->b_norm = 1.0;
  o->want_true_residual = 0;
  o->true_res_cg_tol = 1e-14;
  o->schur = 1;
  o->x0 = nullptr;
  o->kerker = 0;
  o->kerker_alpha = 0.8;
  o->recycle = 0;
}

int ikr_supported_fft_size(int n) { return ikr::fft_length_supported(n) ? 1 : 0; }

ikr_status ikr_setup_system(const ikr_system_desc* desc, void* stream,
                            int compute_ground_state, ikr_handle* out) {
  return guarded([&] {
    IKR_CHECK(out, IKR_E_ARG, "null output handle");
    *out = nullptr;
    System* s = ikr::create_system(desc, reinterpret_cast<hipStream_t>(stream));
    try {
      if (compute_ground_state) ikr::compute_ground_state(*s);
    } catch (...) {
      delete s;
      throw;
    }
    *out = reinterpret_cast<ikr_handle>(s);
    if (s->have_gs)
      for (double g : s->gap_k)
        IKR_CHECK(!(g < 1e-6), IKR_E_NOGAP, "gap above the occupied bands below 1e-6 Ha");
  });
}

ikr_status ikr_import_ground_state(ikr_handle h, const ikr_ground_state* gs) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(gs, IKR_E_ARG, "null ground state");
    ikr::import_ground_state(*s, gs->eps, gs->coeffs);
    for (double g : s->gap_k)
      IKR_CHECK(!(g < 1e-6), IKR_E_NOGAP, "gap above the occupied bands below 1e-6 Ha");
  });
}

ikr_status ikr_get_info(ikr_handle h, int* nk, int* nbands, int* nb_max, int* ng,
                        int* nocc_k_host) {
  return guarded([&] {
    System* s = sys_of(h);
    if (nk) *nk = s->nk;
    if (nbands) *nbands = s->nbands;
    if (nb_max) *nb_max = s->nb_max;
    if (ng) *ng = s->ng;
    if (nocc_k_host) {
      IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
      for (int k = 0; k < s->nk; ++k) nocc_k_host[k] = s->nocc_k[k];
    }
  });
}

ikr_status ikr_get_basis(ikr_handle h, int k, int* nb_k, int* miller_host) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(k >= 0 && k < s->nk, IKR_E_ARG, "k-point index out of range");
    if (nb_k) *nb_k = s->kp[k].nb;
    if (miller_host)
      std::memcpy(miller_host, s->kp[k].miller.data(), s->kp[k].miller.size() * sizeof(int));
  });
}

ikr_status ikr_get_ground_state(ikr_handle h, double* eps_host, double* occ_host,
                                double* coeffs_host, double* fermi_host) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    if (eps_host) std::memcpy(eps_host, s->eps.data(), s->eps.size() * sizeof(double));
    if (occ_host) std::memcpy(occ_host, s->occ.data(), s->occ.size() * sizeof(double));
    if (fermi_host) *fermi_host = s->fermi;
    if (coeffs_host) {
      IKR_HIP(hipMemcpyAsync(coeffs_host, s->d_phi.get(),
                             (size_t)s->nk * s->nbands * s->nb_max * sizeof(double2),
                             hipMemcpyDeviceToHost, s->stream));
      IKR_HIP(hipStreamSynchronize(s->stream));
    }
  });
}

ikr_status ikr_get_setup_info(ikr_handle h, double* gaps_host, int* gs_iters,
                              double* gs_residual) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    if (gaps_host) std::memcpy(gaps_host, s->gap_k.data(), s->gap_k.size() * sizeof(double));
    if (gs_iters) *gs_iters = s->gs_outer_iters;
    if (gs_residual) *gs_residual = s->gs_residual;
  });
}

ikr_status ikr_get_orbital_norms(ikr_handle h, double* re_host, double* full_host) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    if (re_host) std::memcpy(re_host, s->orbnorm_k.data(), s->orbnorm_k.size() * sizeof(double));
    if (full_host)
      std::memcpy(full_host, s->orbnorm_full_k.data(), s->orbnorm_full_k.size() * sizeof(double));
  });
}

ikr_status ikr_get_density(ikr_handle h, double* rho_dev) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(rho_dev, IKR_E_ARG, "null output");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr::to_external(s->L, s->d_rho.get(), rho_dev, 1.0, nullptr, 0.0, s->stream);
    IKR_HIP(hipStreamSynchronize(s->stream));
  });
}

ikr_status ikr_apply_hamiltonian(ikr_handle h, int k, int nvec, const double* x_dev,
                                 double* y_dev) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(k >= 0 && k < s->nk, IKR_E_ARG, "k-point index out of range");
    IKR_CHECK(nvec >= 1 && nvec <= 4096, IKR_E_ARG, "nvec out of range");
    IKR_CHECK(x_dev && y_dev && x_dev != y_dev, IKR_E_ARG, "bad vector pointers");
    ikr::apply_hamiltonian(*s, k, nvec, reinterpret_cast<const double2*>(x_dev),
                           reinterpret_cast<double2*>(y_dev));
  });
}

ikr_status ikr_apply_hamiltonian_noalloc(ikr_handle h, int k, int nvec, const double* x_dev,
                                         double* y_dev) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(k >= 0 && k < s->nk, IKR_E_ARG, "k-point index out of range");
    IKR_CHECK(nvec >= 1 && nvec <= 4096, IKR_E_ARG, "nvec out of range");
    IKR_CHECK(x_dev && y_dev && x_dev != y_dev, IKR_E_ARG, "bad vector pointers");
    ikr::apply_hamiltonian_noalloc(*s, k, nvec, reinterpret_cast<const double2*>(x_dev),
                                   reinterpret_cast<double2*>(y_dev));
  });
}

ikr_status ikr_apply_hxc_kernel(ikr_handle h, const double* v_dev, double* kv_dev) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(v_dev && kv_dev, IKR_E_ARG, "null vector");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr::to_internal(s->L, v_dev, s->d_tmpg.get(), s->stream);
    ikr::apply_kernel(*s, s->d_tmpg.get(), s->d_u.get());
    ikr::to_external(s->L, s->d_u.get(), kv_dev, 1.0, nullptr, 0.0, s->stream);
    IKR_HIP(hipStreamSynchronize(s->stream));
  });
}

ikr_status ikr_apply_kerker(ikr_handle h, double alpha, const double* v_dev, double* out_dev) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(v_dev && out_dev, IKR_E_ARG, "null vector");
    IKR_CHECK(alpha > 0 && std::isfinite(alpha), IKR_E_ARG, "alpha must be positive");
    ikr::apply_kerker_ext(*s, alpha, v_dev, out_dev);
    IKR_HIP(hipStreamSynchronize(s->stream));
  });
}

ikr_status ikr_displacement_rhs(ikr_handle h, int atom, int direction, double cg_tol,
                                double* dv0_dev, double* b_dev, ikr_stats* stats) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(b_dev, IKR_E_ARG, "null output");
    IKR_CHECK(atom >= 0 && atom < s->natoms, IKR_E_ARG, "atom index out of range");
    IKR_CHECK(direction >= 0 && direction < 3, IKR_E_ARG, "direction must be 0, 1 or 2");
    IKR_CHECK(cg_tol > 0 && cg_tol < 1, IKR_E_ARG, "CG tolerance must be in (0, 1)");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr::Chi0Result r = ikr::displacement_rhs(*s, atom, direction, cg_tol, dv0_dev, b_dev);
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->n_ham = r.n_ham;
      stats->n_ham_fp64 = r.n_ham64;
      stats->n_ham_fp32 = r.n_ham32;
      stats->cg_unconverged = r.noconv;
      stats->true_res = -1;
    }
    IKR_CHECK(r.noconv == 0, IKR_E_NOCONV, "a Sternheimer CG hit the iteration cap");
  });
}

ikr_status ikr_apply_chi0(ikr_handle h, const double* dv_dev, double* drho_dev, double cg_tol,
                          const double* cg_tol_host, ikr_stats* stats) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(dv_dev && drho_dev, IKR_E_ARG, "null vector");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    IKR_CHECK(cg_tol_host || cg_tol > 0, IKR_E_ARG, "CG tolerance must be positive");
    std::vector<double> tol(s->J, cg_tol);
    if (cg_tol_host)
      for (int j = 0; j < s->J; ++j)
        tol[j] = cg_tol_host[(size_t)s->slot_k[j] * s->nbands + s->slot_n[j]];
    ikr::to_internal(s->L, dv_dev, s->d_tmpg.get(), s->stream);
    ikr::Chi0Result r = ikr::apply_chi0_internal(*s, s->d_tmpg.get(), s->d_drho.get(), tol, 1, 1000);
    ikr::to_external(s->L, s->d_drho.get(), drho_dev, 1.0, nullptr, 0.0, s->stream);
    IKR_HIP(hipStreamSynchronize(s->stream));
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->n_ham = r.n_ham;
      stats->n_ham_fp64 = r.n_ham64;
      stats->n_ham_fp32 = r.n_ham32;
      stats->cg_unconverged = r.noconv;
      stats->fp64_fallback = r.fallback;
      stats->fp32_checked = r.checked;
      stats->true_res = -1;
    }
    IKR_CHECK(r.noconv == 0, IKR_E_NOCONV, "a Sternheimer CG hit the iteration cap");
  });
}

ikr_status ikr_apply_dielectric(ikr_handle h, const double* v_dev, double* ev_dev,
                                double common, const ikr_solver_opts* opts, ikr_stats* stats) {
  return guarded([&] {
    System* s = sys_of(h);
    check_opts(opts);
    GraphMode mode(s, opts);
    IKR_CHECK(v_dev && ev_dev && v_dev != ev_dev, IKR_E_ARG, "bad vector pointers");
    IKR_CHECK(common > 0, IKR_E_ARG, "common tolerance factor must be positive");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr_stats local{};
    ikr::apply_dielectric_ext(*s, v_dev, ev_dev, common, *opts, opts->b_norm, &local);
    local.true_res = -1;
    if (stats) *stats = local;
  });
}

ikr_status ikr_solve_response(ikr_handle h, const double* b_dev, double* drho_dev,
                              const ikr_solver_opts* opts, ikr_stats* stats) {
  return guarded([&] {
    System* s = sys_of(h);
    check_opts(opts);
    GraphMode mode(s, opts);
    IKR_CHECK(b_dev && drho_dev && b_dev != drho_dev, IKR_E_ARG, "bad vector pointers");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr_stats local{};
    local.true_res = -1;
    try {
      ikr::solve_response(*s, b_dev, drho_dev, *opts, &local);
    } catch (...) {
      if (stats) *stats = local;
      throw;
    }
    if (stats) *stats = local;
  });
}

ikr_status ikr_apply_dielectric_adjoint(ikr_handle h, const double* v_dev, double* ev_dev,
                                        double common, const ikr_solver_opts* opts,
                                        ikr_stats* stats) {
  return guarded([&] {
    System* s = sys_of(h);
    check_opts(opts);
    GraphMode mode(s, opts);
    IKR_CHECK(v_dev && ev_dev && v_dev != ev_dev, IKR_E_ARG, "bad vector pointers");
    IKR_CHECK(common > 0, IKR_E_ARG, "common tolerance factor must be positive");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr_stats local{};
    ikr::apply_dielectric_adjoint_ext(*s, v_dev, ev_dev, common, *opts, opts->b_norm, &local);
    local.true_res = -1;
    if (stats) *stats = local;
  });
}

ikr_status ikr_solve_response_adjoint(ikr_handle h, const double* g_dev, double* lambda_dev,
                                      const ikr_solver_opts* opts, ikr_stats* stats) {
  return guarded([&] {
    System* s = sys_of(h);
    check_opts(opts);
    GraphMode mode(s, opts);
    IKR_CHECK(g_dev && lambda_dev && g_dev != lambda_dev, IKR_E_ARG, "bad vector pointers");
    IKR_CHECK(!opts->kerker, IKR_E_ARG, "Kerker preconditioning is for forward solves only");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr_stats local{};
    local.true_res = -1;
    try {
      ikr::solve_response(*s, g_dev, lambda_dev, *opts, &local, true);
    } catch (...) {
      if (stats) *stats = local;
      throw;
    }
    if (stats) *stats = local;
  });
}

ikr_status ikr_grad_amplitudes(ikr_handle h, const double* drho_dev, const double* lambda_dev,
                               double cg_tol, double* dlda_host, ikr_stats* stats) {
  return guarded([&] {
    System* s = sys_of(h);
    IKR_CHECK(drho_dev && lambda_dev && dlda_host, IKR_E_ARG, "null pointer");
    IKR_CHECK(s->have_gs, IKR_E_STATE, "ground state not set up");
    ikr_stats local{};
    local.true_res = -1;
    const std::vector<double> g = ikr::grad_amplitudes(*s, drho_dev, lambda_dev, cg_tol, &local);
    for (double v : g) IKR_CHECK(std::isfinite(v), IKR_E_NAN, "non-finite gradient");
    std::copy(g.begin(), g.end(), dlda_host);
    if (stats) *stats = local;
  });
}

ikr_status ikr_set_kernel_paths(int mask) {
  return guarded([&] {
    IKR_CHECK(mask >= 0 && mask <= 15, IKR_E_ARG, "unknown kernel path bits");
    ikr::set_kernel_paths(mask);
  });
}

int ikr_get_kernel_paths(void) { return ikr::kernel_paths(); }

ikr_status ikr_get_tuning(ikr_handle h, int* out) {
  return guarded([&] {
    IKR_CHECK(out, IKR_E_ARG, "null output");
    const ikr::System* s = sys_of(h);
    for (int p = 0; p < 2; ++p)
      for (int c = 0; c < 2; ++c) {
        int* o = out + 12 * p + 6 * c;
        const ikr::KernelTune& t = s->tune[p][c];
        o[0] = s->tuned[p][c] ? 1 : 0;
        o[1] = o[0] ? t.gram : 0;
        o[2] = o[0] ? (int)std::lround(100.0 * t.gram_scale) : 0;
        o[3] = o[0] ? t.upd_bpt : 0;
        o[4] = o[0] ? t.plane_pt : 0;
        o[5] = o[0] ? (int)std::lround(1000.0 * s->tune_us[p][c][0]) : 0;
      }
  });
}

ikr_status ikr_tune_launches(ikr_handle h, int precision, int schur) {
  return guarded([&] {
    ikr::System* s = sys_of(h);
    IKR_CHECK(s->have_gs, IKR_E_STATE, "no ground state");
    ikr::tune_launches_now(*s, precision, schur);
  });
}

ikr_status ikr_set_tuning(ikr_handle h, const int* in) {
  return guarded([&] {
    IKR_CHECK(in, IKR_E_ARG, "null input");
    ikr::System* s = sys_of(h);
    for (int i = 0; i < 4; ++i) {
      const int* o = in + 6 * i;
      if (!o[0]) continue;
      IKR_CHECK(o[1] >= 0 && o[1] <= 3, IKR_E_ARG, "tuning: gram kernel not in 0..3");
      IKR_CHECK(o[2] == 50 || o[2] == 100 || o[2] == 200, IKR_E_ARG,
                "tuning: gram scale not 50, 100 or 200");
      IKR_CHECK(o[3] == 0 || o[3] == 4 || o[3] == 8 || o[3] == 16, IKR_E_ARG,
                "tuning: bands per block not 0, 4, 8 or 16");
      IKR_CHECK(o[4] == 0 || o[4] == 256 || o[4] == 512, IKR_E_ARG,
                "tuning: plane threads not 0, 256 or 512");
    }
    for (int p = 0; p < 2; ++p)
      for (int c = 0; c < 2; ++c) {
        const int* o = in + 12 * p + 6 * c;
        ikr::KernelTune t{};
        if (o[0]) {
          t.gram = o[1];
          t.gram_scale = o[2] / 100.0f;
          t.upd_bpt = o[3];
          t.plane_pt = o[4];
        }
        s->tune[p][c] = t;
        s->tuned[p][c] = o[0] != 0;
        for (double& v : s->tune_us[p][c]) v = 0;
      }
    s->graphs.clear();
  });
}

ikr_status ikr_profile_enable(int kernel_mask) {
  return guarded([&] { ikr::KTimer::enable((unsigned)kernel_mask); });
}

ikr_status ikr_profile_reset(void) {
  return guarded([&] { ikr::KTimer::reset(); });
}

int ikr_profile_kernel_count(void) { return ikr::K_COUNT; }

const char* ikr_profile_kernel_name(int kernel_id) { return ikr::kernel_name(kernel_id); }

ikr_status ikr_profile_query(int kernel_id, long long* launches, double* total_ms,
                             double* total_bytes) {
  return guarded([&] {
    IKR_CHECK(kernel_id >= 0 && kernel_id < ikr::K_COUNT, IKR_E_ARG, "kernel id out of range");
    ikr::KTimer::query(kernel_id, launches, total_ms, total_bytes);
  });
}

const char* ikr_last_error(void) { return g_last_error.c_str(); }

void ikr_destroy(ikr_handle h) {
  if (h) delete reinterpret_cast<System*>(h);
}

}  // extern "C"
