"""ctypes binding of libikr.so (the C ABI of include/ikr.h).

Argument marshalling only: every step of the response path runs in the HIP
library.  PyTorch provides device memory (tensors passed by data_ptr) and
the HIP stream.  There is no fallback: if the library is missing or fails
to load, import raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libikr.so")

IKR_AGR, IKR_BAL, IKR_GRT, IKR_D10, IKR_D100, IKR_D10N, IKR_FIXED, IKR_THM2 = range(8)
STRATEGY = {"agr": IKR_AGR, "bal": IKR_BAL, "grt": IKR_GRT, "D10": IKR_D10,
            "D100": IKR_D100, "D10n": IKR_D10N, "fixed": IKR_FIXED, "thm2": IKR_THM2}
STATUS = {0: "OK", 1: "E_ARG", 2: "E_STATE", 3: "E_NOGAP", 4: "E_NOCONV",
          5: "E_NAN", 6: "E_OOM", 7: "E_HIP", 8: "E_INTERNAL"}


class IkrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ikr {STATUS.get(code, code)}: {msg}")
        self.code = code


class SystemDesc(C.Structure):
    _fields_ = [("lattice", C.c_double * 3), ("natoms", C.c_int),
                ("frac_pos", C.POINTER(C.c_double)), ("amp", C.POINTER(C.c_double)),
                ("sigma_loc", C.c_double), ("sigma_proj", C.c_double),
                ("d_proj", C.c_double), ("ecut", C.c_double), ("fft", C.c_int * 3),
                ("kgrid", C.c_int * 3), ("nocc", C.c_int), ("nextra", C.c_int),
                ("temperature", C.c_double), ("xc", C.c_int)]


class GroundStateC(C.Structure):
    _fields_ = [("eps", C.POINTER(C.c_double)), ("coeffs", C.POINTER(C.c_double))]


class SolverOpts(C.Structure):
    _fields_ = [("strategy", C.c_int), ("tol", C.c_double), ("tol_is_relative", C.c_int),
                ("restart_m", C.c_int), ("s0", C.c_double), ("max_restarts", C.c_int),
                ("precision", C.c_int), ("cg_min_iter", C.c_int), ("cg_max_iter", C.c_int),
                ("fp32_theta", C.c_double), ("b_norm", C.c_double),
                ("want_true_residual", C.c_int), ("true_res_cg_tol", C.c_double),
                ("schur", C.c_int), ("batching", C.c_int), ("x0", C.c_void_p),
                ("kerker", C.c_int), ("kerker_alpha", C.c_double), ("recycle", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n_ham", C.c_longlong), ("n_ham_fp32", C.c_longlong),
                ("n_ham_fp64", C.c_longlong), ("gmres_iters", C.c_int),
                ("restarts", C.c_int), ("cg_unconverged", C.c_int),
                ("est_res", C.c_double), ("true_res", C.c_double),
                ("s_final", C.c_double), ("sigma_min", C.c_double),
                ("knorm_last", C.c_double), ("seconds", C.c_double),
                ("fp64_fallback", C.c_longlong), ("fp32_checked", C.c_longlong),
                ("warm_started", C.c_longlong)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# Exported symbols and their signatures (must match include/ikr.h).
_VP = C.c_void_p
SIGNATURES = {
    "ikr_default_opts": (None, [C.POINTER(SolverOpts)]),
    "ikr_supported_fft_size": (C.c_int, [C.c_int]),
    "ikr_setup_system": (C.c_int, [C.POINTER(SystemDesc), _VP, C.c_int, C.POINTER(_VP)]),
    "ikr_import_ground_state": (C.c_int, [_VP, C.POINTER(GroundStateC)]),
    "ikr_get_info": (C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ikr_get_basis": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ikr_get_ground_state": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ikr_get_setup_info": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int),
                                     C.POINTER(C.c_double)]),
    "ikr_get_density": (C.c_int, [_VP, _VP]),
    "ikr_get_orbital_norms": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ikr_apply_hamiltonian": (C.c_int, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "ikr_apply_hamiltonian_noalloc": (C.c_int, [_VP, C.c_int, C.c_int, _VP, _VP]),
    "ikr_apply_hxc_kernel": (C.c_int, [_VP, _VP, _VP]),
    "ikr_apply_kerker": (C.c_int, [_VP, C.c_double, _VP, _VP]),
    "ikr_displacement_rhs": (C.c_int, [_VP, C.c_int, C.c_int, C.c_double, _VP, _VP,
                                       C.POINTER(Stats)]),
    "ikr_apply_chi0": (C.c_int, [_VP, _VP, _VP, C.c_double, C.POINTER(C.c_double),
                                 C.POINTER(Stats)]),
    "ikr_apply_dielectric": (C.c_int, [_VP, _VP, _VP, C.c_double, C.POINTER(SolverOpts),
                                       C.POINTER(Stats)]),
    "ikr_solve_response": (C.c_int, [_VP, _VP, _VP, C.POINTER(SolverOpts), C.POINTER(Stats)]),
    "ikr_apply_dielectric_adjoint": (C.c_int, [_VP, _VP, _VP, C.c_double,
                                               C.POINTER(SolverOpts), C.POINTER(Stats)]),
    "ikr_solve_response_adjoint": (C.c_int, [_VP, _VP, _VP, C.POINTER(SolverOpts),
                                             C.POINTER(Stats)]),
    "ikr_grad_amplitudes": (C.c_int, [_VP, _VP, _VP, C.c_double, C.POINTER(C.c_double),
                                      C.POINTER(Stats)]),
    "ikr_set_kernel_paths": (C.c_int, [C.c_int]),
    "ikr_get_kernel_paths": (C.c_int, []),
    "ikr_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "ikr_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "ikr_tune_launches": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "ikr_profile_enable": (C.c_int, [C.c_int]),
    "ikr_profile_reset": (C.c_int, []),
    "ikr_profile_kernel_count": (C.c_int, []),
    "ikr_profile_kernel_name": (C.c_char_p, [C.c_int]),
    "ikr_profile_query": (C.c_int, [C.c_int, C.POINTER(C.c_longlong), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "ikr_last_error": (C.c_char_p, []),
    "ikr_destroy": (None, [_VP]),
}

_lib = None


def lib():
    """Load libikr.so (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built; run paper_2505_02319_amd.build.build()")
        # torch first: the library then binds to the HIP runtime torch has loaded,
        # so the process holds one HIP runtime (two in one process do not share
        # the GPU: whichever initialises second finds no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise IkrError(code, lib().ikr_last_error().decode())


def default_opts(**kw) -> SolverOpts:
    """Solver options with the library defaults, overridden by kw.  x0 may be
    a CUDA float64 grid tensor (it must stay alive while the options are
    used) or a device address."""
    o = SolverOpts()
    lib().ikr_default_opts(C.byref(o))
    for key, val in kw.items():
        if key == "strategy" and isinstance(val, str):
            val = STRATEGY[val]
        if key == "x0" and val is not None and hasattr(val, "data_ptr"):
            assert val.is_cuda and val.is_contiguous()
            o._x0_keep = val
            val = val.data_ptr()
        setattr(o, key, val)
    return o


PATH_VECTOR_GRAM, PATH_SPLIT_END, PATH_KWIDE, PATH_FIXED = 1, 2, 4, 8


def set_kernel_paths(mask: int):
    """Force kernel paths process-wide (0: by size; bits: PATH_*)."""
    _check(lib().ikr_set_kernel_paths(int(mask)))


def kernel_paths() -> int:
    return int(lib().ikr_get_kernel_paths())


def profile_enable(on=True):
    """True: time every hot kernel; False: none; a kernel name: only that one."""
    L = lib()
    if isinstance(on, str):
        names = [L.ikr_profile_kernel_name(i).decode() for i in range(L.ikr_profile_kernel_count())]
        mask = 1 << names.index(on)
    else:
        mask = -1 if on else 0
    _check(L.ikr_profile_enable(mask))


def profile_reset():
    _check(lib().ikr_profile_reset())


def profile_query():
    """{kernel name: (launches, total_ms, total_algorithmic_bytes)}"""
    L = lib()
    out = {}
    for i in range(L.ikr_profile_kernel_count()):
        n, ms, by = C.c_longlong(), C.c_double(), C.c_double()
        _check(L.ikr_profile_query(i, C.byref(n), C.byref(ms), C.byref(by)))
        out[L.ikr_profile_kernel_name(i).decode()] = (n.value, ms.value, by.value)
    return out


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ptr(t):
    return C.c_void_p(t.data_ptr())


@dataclass
class Info:
    nk: int
    nbands: int
    nb_max: int
    ng: int


class ResponseSystem:
    """One response system (opaque handle) on the current CUDA/HIP device.

    ``spec`` is any object with the fields of ikr_system_desc (lattice,
    frac_pos, amp, sigma_loc, sigma_proj, d_proj, ecut, fft, kgrid, nocc,
    nextra, temperature, xc).  ``ground_state``: "compute" (library's own
    GPU eigensolver) or a pair (eps [nk][nbands], coeffs [nk][nbands][nb_max]
    complex) in the library's basis order, or None to import later.
    """

    def __init__(self, spec, ground_state="compute", stream=None):
        import torch
        self._torch = torch
        L = lib()
        self.spec = spec
        self.fft = tuple(int(x) for x in spec.fft)
        pos = np.ascontiguousarray(np.asarray(spec.frac_pos, float).reshape(-1))
        amp = np.ascontiguousarray(np.asarray(spec.amp, float).reshape(-1))
        self._keep = (pos, amp)
        d = SystemDesc()
        d.lattice[:] = [float(x) for x in spec.lattice]
        d.natoms = len(amp)
        d.frac_pos = _dptr(pos)
        d.amp = _dptr(amp)
        d.sigma_loc, d.sigma_proj, d.d_proj = spec.sigma_loc, spec.sigma_proj, spec.d_proj
        d.ecut = spec.ecut
        d.fft[:] = list(self.fft)
        d.kgrid[:] = [int(x) for x in spec.kgrid]
        d.nocc, d.nextra = int(spec.nocc), int(spec.nextra)
        d.temperature = float(spec.temperature)
        d.xc = int(spec.xc)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = C.c_void_p()
        compute = 1 if isinstance(ground_state, str) and ground_state == "compute" else 0
        code = L.ikr_setup_system(C.byref(d), C.c_void_p(stream), compute, C.byref(h))
        self.h = h
        if code not in (0,):
            if h.value is None:
                _check(code)
            self.setup_status = code
        else:
            self.setup_status = 0
        if not compute and ground_state is not None:
            self.import_ground_state(*ground_state)

    # ------------------------------------------------------------ queries
    def tuning(self) -> dict:
        """The launch shapes measured at the first CG run of each precision:
        {(precision, batch): {...}} for precision "fp64"/"fp32" and batch
        "thick"/"thin"; entries not yet measured are left out."""
        out = (C.c_int * 24)()
        _check(lib().ikr_get_tuning(self.h, out))
        names = {0: "size_rule", 1: "per_tile_mfma", 2: "kwide_mfma", 3: "vector"}
        res = {}
        for p, pn in enumerate(("fp64", "fp32")):
            for c, cn in enumerate(("thick", "thin")):
                o = out[12 * p + 6 * c: 12 * p + 6 * c + 6]
                if o[0]:
                    res[(pn, cn)] = {"gram": names.get(o[1], "?"), "gram_scale": o[2] / 100.0,
                                     "update_bands_per_block": o[3], "plane_threads": o[4],
                                     "gram_us": o[5] / 1000.0}
        return res

    def tune_launches(self, precision=1, schur=1):
        """Measure the CG launch shapes now (FP64, and FP32 when precision),
        instead of at the first CG run of each precision."""
        _check(lib().ikr_tune_launches(self.h, int(precision), int(schur)))

    def pin_tuning(self, gram=None, gram_scale=1.0, update_bands_per_block=8,
                   plane_threads=0):
        """Pin every precision's and batch class's launch shapes to the given
        ones (gram: 1 per-tile matrix-core, 2 k-wide, 3 vector); gram=None
        clears them, so that the next CG runs measure them again (0 for gram,
        update_bands_per_block or plane_threads: the size rule)."""
        vals = [0] * 6 if gram is None else [1, int(gram), int(round(100 * gram_scale)),
                                            int(update_bands_per_block), int(plane_threads), 0]
        arr = (C.c_int * 24)(*(vals * 4))
        _check(lib().ikr_set_tuning(self.h, arr))

    def info(self) -> Info:
        nk, nb, nbm, ng = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        _check(lib().ikr_get_info(self.h, C.byref(nk), C.byref(nb), C.byref(nbm),
                                  C.byref(ng), None))
        return Info(nk.value, nb.value, nbm.value, ng.value)

    def nocc_k(self):
        inf = self.info()
        out = (C.c_int * inf.nk)()
        _check(lib().ikr_get_info(self.h, None, None, None, None, out))
        return list(out)

    def basis(self, k: int) -> np.ndarray:
        nb = C.c_int()
        _check(lib().ikr_get_basis(self.h, k, C.byref(nb), None))
        m = np.zeros((nb.value, 3), np.int32)
        _check(lib().ikr_get_basis(self.h, k, C.byref(nb),
                                   m.ctypes.data_as(C.POINTER(C.c_int))))
        return m

    def import_ground_state(self, eps, coeffs):
        inf = self.info()
        eps = np.ascontiguousarray(np.asarray(eps, float).reshape(inf.nk, inf.nbands))
        cf = np.ascontiguousarray(np.asarray(coeffs, np.complex128).reshape(
            inf.nk, inf.nbands, inf.nb_max))
        g = GroundStateC(_dptr(eps), cf.ctypes.data_as(C.POINTER(C.c_double)))
        code = lib().ikr_import_ground_state(self.h, C.byref(g))
        self.setup_status = code
        if code not in (0, 3):
            _check(code)

    def ground_state(self):
        inf = self.info()
        eps = np.zeros((inf.nk, inf.nbands))
        occ = np.zeros((inf.nk, inf.nbands))
        cf = np.zeros((inf.nk, inf.nbands, inf.nb_max), np.complex128)
        fermi = C.c_double()
        _check(lib().ikr_get_ground_state(self.h, _dptr(eps), _dptr(occ),
                                          cf.ctypes.data_as(C.POINTER(C.c_double)),
                                          C.byref(fermi)))
        return eps, occ, cf, fermi.value

    def orbital_norms(self):
        """(||Re F_k^-1 Phi_k||_{2,inf}, ||F_k^-1 Phi_k||_{2,inf}) per k."""
        inf = self.info()
        re, full = np.zeros(inf.nk), np.zeros(inf.nk)
        _check(lib().ikr_get_orbital_norms(self.h, _dptr(re), _dptr(full)))
        return re, full

    def setup_info(self):
        inf = self.info()
        gaps = np.zeros(inf.nk)
        it = C.c_int()
        res = C.c_double()
        _check(lib().ikr_get_setup_info(self.h, _dptr(gaps), C.byref(it), C.byref(res)))
        return {"gaps": gaps, "gs_iters": it.value, "gs_residual": res.value}

    # ------------------------------------------------------------ operators
    def _grid(self, t):
        torch = self._torch
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
        assert t.numel() == int(np.prod(self.fft))
        return t

    def density(self):
        torch = self._torch
        out = torch.empty(self.fft, dtype=torch.float64, device="cuda")
        _check(lib().ikr_get_density(self.h, _ptr(out)))
        return out

    def apply_hamiltonian(self, k: int, x):
        torch = self._torch
        inf = self.info()
        assert x.dtype == torch.complex128 and x.is_cuda and x.is_contiguous()
        assert x.shape[-1] == inf.nb_max
        y = torch.empty_like(x)
        _check(lib().ikr_apply_hamiltonian(self.h, k, x.shape[0], _ptr(x), _ptr(y)))
        return y

    def apply_hamiltonian_noalloc(self, k: int, x, y=None):
        """y = H_k x through the entry point that allocates no device memory
        (y may be given, so that the call itself allocates nothing)."""
        torch = self._torch
        inf = self.info()
        assert x.dtype == torch.complex128 and x.is_cuda and x.is_contiguous()
        assert x.shape[-1] == inf.nb_max
        if y is None:
            y = torch.empty_like(x)
        assert y.shape == x.shape and y.dtype == x.dtype and y.is_contiguous()
        _check(lib().ikr_apply_hamiltonian_noalloc(self.h, k, x.shape[0], _ptr(x), _ptr(y)))
        return y

    def apply_kernel(self, v):
        out = self._torch.empty_like(self._grid(v))
        _check(lib().ikr_apply_hxc_kernel(self.h, _ptr(v), _ptr(out)))
        return out

    def apply_kerker(self, v, alpha: float = 0.8):
        """T v with the Kerker preconditioner (eq. kerker)."""
        out = self._torch.empty_like(self._grid(v))
        _check(lib().ikr_apply_kerker(self.h, float(alpha), _ptr(v), _ptr(out)))
        return out

    def displacement_rhs(self, atom: int, direction: int, cg_tol: float = 1e-10):
        """(b, dV0_local, stats): b = chi0 dV0 for the displacement of one atom."""
        torch = self._torch
        b = torch.empty(self.fft, dtype=torch.float64, device="cuda")
        dv0 = torch.empty_like(b)
        st = Stats()
        _check(lib().ikr_displacement_rhs(self.h, int(atom), int(direction), float(cg_tol),
                                          _ptr(dv0), _ptr(b), C.byref(st)))
        return b, dv0, st.as_dict()

    def apply_chi0(self, dv, cg_tol: float = 1e-10, cg_tol_per_band=None):
        out = self._torch.empty_like(self._grid(dv))
        st = Stats()
        per = None
        if cg_tol_per_band is not None:
            arr = np.ascontiguousarray(np.asarray(cg_tol_per_band, float))
            per = _dptr(arr)
        _check(lib().ikr_apply_chi0(self.h, _ptr(dv), _ptr(out), float(cg_tol), per,
                                    C.byref(st)))
        return out, st.as_dict()

    def apply_dielectric(self, v, common: float, opts: Optional[SolverOpts] = None):
        out = self._torch.empty_like(self._grid(v))
        st = Stats()
        o = opts or default_opts()
        _check(lib().ikr_apply_dielectric(self.h, _ptr(v), _ptr(out), float(common),
                                          C.byref(o), C.byref(st)))
        return out, st.as_dict()

    def apply_dielectric_adjoint(self, v, common: float, opts: Optional[SolverOpts] = None):
        out = self._torch.empty_like(self._grid(v))
        st = Stats()
        o = opts or default_opts()
        _check(lib().ikr_apply_dielectric_adjoint(self.h, _ptr(v), _ptr(out), float(common),
                                                  C.byref(o), C.byref(st)))
        return out, st.as_dict()

    def _solve(self, fn, b, opts):
        out = self._torch.empty_like(self._grid(b))
        st = Stats()
        o = opts or default_opts()
        code = fn(self.h, _ptr(b), _ptr(out), C.byref(o), C.byref(st))
        if code != 0:
            err = IkrError(code, lib().ikr_last_error().decode())
            err.stats = st.as_dict()
            raise err
        return out, st.as_dict()

    def solve(self, b, opts: Optional[SolverOpts] = None):
        """drho = E^-1 b (Alg. 1)."""
        return self._solve(lib().ikr_solve_response, b, opts)

    def solve_adjoint(self, g, opts: Optional[SolverOpts] = None):
        """lambda = E^-T g (the same inexact GMRES on the transposed operator)."""
        return self._solve(lib().ikr_solve_response_adjoint, g, opts)

    def grad_amplitudes(self, drho, lam, cg_tol: float = 1e-12):
        """dL/dA (numpy, one per atom) from drho = E^-1 b and lam = E^-T dL/d(drho)."""
        out = np.zeros(self.spec.natoms)
        st = Stats()
        _check(lib().ikr_grad_amplitudes(self.h, _ptr(self._grid(drho)), _ptr(self._grid(lam)),
                                         float(cg_tol), _dptr(out), C.byref(st)))
        return out, st.as_dict()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ikr_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class DysonSolve(torch.autograd.Function):
        """drho = E^-1 b with its gradient dL/db = E^-T dL/d(drho): the backward
        pass is the inexact GMRES solve of the transposed dielectric operator
        (same Sternheimer kernels, nothing stored from the forward solve)."""

        @staticmethod
        def forward(ctx, b, amplitudes, rs, opts, adj_opts, grad_tol):
            x, st = rs.solve(b.contiguous(), opts)
            ctx.rs, ctx.adj_opts = rs, adj_opts if adj_opts is not None else opts
            ctx.grad_tol = grad_tol
            ctx.stats = st
            ctx.save_for_backward(x)
            return x

        @staticmethod
        def backward(ctx, g):
            (x,) = ctx.saved_tensors
            lam, st = ctx.rs.solve_adjoint(g.contiguous(), ctx.adj_opts)
            ctx.adjoint_stats = st
            gamp = None
            if ctx.needs_input_grad[1]:
                ga, _ = ctx.rs.grad_amplitudes(x, lam, ctx.grad_tol)
                gamp = torch.from_numpy(ga)
            return lam, gamp, None, None, None, None

    return DysonSolve


def dyson_solve(b, rs: "ResponseSystem", opts: Optional[SolverOpts] = None,
                adj_opts: Optional[SolverOpts] = None, amplitudes=None,
                grad_tol: float = 1e-12):
    """Differentiable solve of E drho = b (b a CUDA float64 grid tensor).

    ``amplitudes``: optional CPU float64 tensor equal to the system's
    local-potential amplitudes; when it requires grad, backward also returns
    dL/dA (the system itself is not changed: the derivative is taken at the
    amplitudes it was set up with)."""
    global _DYSON
    if _DYSON is None:
        _DYSON = _autograd_function()
    if amplitudes is not None:
        got = np.asarray(amplitudes.detach().cpu(), float)
        if got.shape != (rs.spec.natoms,) or not np.allclose(got, rs.spec.amp, rtol=0, atol=0):
            raise ValueError("amplitudes must equal the system's local-potential amplitudes")
    return _DYSON.apply(b, amplitudes, rs, opts or default_opts(), adj_opts, grad_tol)


_DYSON = None


def _chi0_function():
    import torch

    class Chi0Apply(torch.autograd.Function):
        """drho = chi0 dv through the Sternheimer route.  chi0 is symmetric in
        the grid inner product (it is a response function of a Hermitian
        Hamiltonian, eq. chi0), so the backward pass applies chi0 itself to
        the incoming gradient; nothing is stored from the forward pass."""

        @staticmethod
        def forward(ctx, dv, rs, cg_tol):
            ctx.rs, ctx.cg_tol = rs, cg_tol
            return _chi0_scaled(rs, dv, cg_tol)

        @staticmethod
        def backward(ctx, g):
            return _chi0_scaled(ctx.rs, g, ctx.cg_tol), None, None

    return Chi0Apply


def _chi0_scaled(rs, v, cg_tol):
    """chi0 v with CG tolerances relative to ||v|| (v normalised first)."""
    import torch
    v = v.contiguous()
    n = float(torch.linalg.norm(v))
    if n == 0.0:
        return torch.zeros_like(v)
    out, _ = rs.apply_chi0(v / n, cg_tol=cg_tol)
    return out * n


def chi0_apply(dv, rs: "ResponseSystem", cg_tol: float = 1e-10):
    """Differentiable drho = chi0 dv (dv a CUDA float64 grid tensor); the CG
    tolerance is relative to ||dv|| (and to ||g|| in the backward pass)."""
    global _CHI0
    if _CHI0 is None:
        _CHI0 = _chi0_function()
    return _CHI0.apply(dv, rs, cg_tol)


_CHI0 = None
