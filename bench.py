#!/usr/bin/env python3
"""Throughput of the inexact-GMRES Dyson solve on one MI355X.

One step = one full solve of E drho = b (Alg. 1 on the Kerker-preconditioned
equation T E drho = T b, grt strategy, tau = 1e-8 ||b||, m = 20, s0 = 1,
x0 = 0; computed unoccupied bands by sum over states; FP32 Sternheimer CG
where the band's tolerance allows; the true residual ||b - E drho|| of the
same solve is reported) on the 8-atom cubic cell (a = 20.52 bohr, Ecut = 15 Ha,
FFT 48^3, 2x2x2 k-points, 16 occupied + 4 extra bands, Hartree + Slater
kernel), with b the seeded smooth random field.  Inputs and the ground state
(computed by the library's own GPU eigensolver during setup) are resident in
HBM before the timed region.  Prints one JSON line.

Beside the headline (untimed by the step clock, reported in the same line):
the plain FP64 reference path (k-points one after the other, a host read per
CG iteration) and the speed-up over it, the true residuals and the paper's
efficiency eta = -log10(||r_end|| / ||b||) / N_ham of several strategies with
and without the Kerker preconditioner, eta_rel against D10, and one timed
solve on the 32-atom smeared cell (60 x 108^2, 27 k-points, 64 + 8 bands) with
its setup time, per-kernel times and true residual.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(spec, n_ham_per_solve, seconds):
    """Oracle Sternheimer CG timed on the host: per band-iteration cost on
    k-point 0 of the workload (a bounded sample), scaled to solves/s by the
    Hamiltonian applications one GPU solve needs."""
    import numpy as np

    from oracle.groundstate import eigenpairs
    from oracle.response import sternheimer_cg
    from oracle.system import WORKERS, System

    class _GS:   # the oracle's ground-state record for k-point 0 only
        pass
    t0 = time.perf_counter()
    sys_ = System(spec)
    e, v = eigenpairs(sys_, 0, spec.nbands)
    gs = _GS()
    gs.eps, gs.phi, gs.nocc_k = [e], [v], [spec.nocc]
    t_gs = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    phi = v[:spec.nocc]
    iters, t_cg, n = 0, 0.0, 0
    while t_cg < seconds and n < spec.nocc:
        rhs = rng.standard_normal(phi.shape[1]) + 1j * rng.standard_normal(phi.shape[1])
        rhs -= (phi.conj() @ rhs) @ phi
        rhs /= np.linalg.norm(rhs)
        t1 = time.perf_counter()
        res = sternheimer_cg(sys_, gs, 0, n, rhs, tol=0.0, maxiter=20)
        t_cg += time.perf_counter() - t1
        iters += res.iterations
        n += 1
    per_iter = t_cg / iters
    return {"value": 1.0 / (per_iter * n_ham_per_solve), "unit": "solves/s",
            "cores": WORKERS, "kind": "oracle",
            "sample": (f"oracle preconditioned Sternheimer CG on k-point 0 of the workload, "
                       f"{n} bands x 20 iterations ({iters} band-iterations, {t_cg:.1f} s; "
                       f"k-point-0 eigensolve {t_gs:.1f} s untimed), scaled by the "
                       f"{n_ham_per_solve:.0f} H applications of one GPU solve"),
            "seconds_per_band_iteration": per_iter}


def whole_solve_small(args):
    """The whole solve on the small cell (cfg1, the 2-atom cell at Gamma) by the
    oracle's Alg. 1 on the host and by the library on the GPU, same b, tau,
    strategy and preconditioner: an end-to-end comparison beside the sampled
    baseline of the bench workload (whose oracle solve would take hours)."""
    import numpy as np
    import torch

    from oracle.gmres import inexact_gmres
    from oracle.groundstate import ground_state
    from oracle.response import HxcKernel
    from oracle.system import WORKERS, System
    from paper_2505_02319_amd import ResponseSystem, default_opts
    from workloads import B_SEED, config, random_field
    spec = config("cfg1")
    sys_ = System(spec)
    gs = ground_state(sys_)
    kern = HxcKernel(sys_, gs.rho, xc=spec.xc)
    b = random_field(spec, B_SEED)
    tau = 1e-8 * float(np.linalg.norm(b))
    t0 = time.perf_counter()
    ref = inexact_gmres(sys_, gs, kern, b, tau, strategy=args.strategy, m=20,
                        kerker_alpha=0.8 if args.kerker else None)
    t_cpu = time.perf_counter() - t0
    rs = ResponseSystem(spec, ground_state="compute")
    bd = torch.from_numpy(b).cuda()
    opts = default_opts(strategy=args.strategy, tol=1e-8, tol_is_relative=1,
                        precision=args.precision, schur=args.schur, kerker=args.kerker)
    rs.solve(bd, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = rs.solve(bd, opts)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    diff = float(np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x))
    rs.close()
    return {"workload": "cfg1: 2-atom cell 10.26^3 bohr, Ecut 8 Ha, FFT 20^3, Gamma, 5+2 bands",
            "oracle_seconds": t_cpu, "oracle_cores": WORKERS, "oracle_n_ham": ref.n_ham,
            "oracle_gmres_iters": ref.iterations, "gpu_seconds": t_gpu, "gpu_n_ham": st["n_ham"],
            "gpu_gmres_iters": st["gmres_iters"], "rel_diff_gpu_vs_oracle": diff}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--strategy", default="grt")
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--schur", type=int, default=1)
    ap.add_argument("--kerker", type=int, default=1,
                    help="1: Kerker-preconditioned GMRES (the paper's P-strategies)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-checks", action="store_true",
                    help="skip the untimed accuracy and FP64 comparison solves")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph-steps", type=int, default=2,
                    help="solves timed again with each CG iteration replayed from a HIP graph "
                         "(reported beside the headline, which uses plain launches)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device copies of MIB MiB (counter calibration)")
    ap.add_argument("--gradient", action="store_true",
                    help="time the forward solve and the adjoint backward (dL/db, dL/dA) "
                         "and check them against central differences")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="only summarise a rocprofv3 kernel-trace CSV: durations of the last "
                         "--trace-last dispatches whose name contains --trace-kernel")
    ap.add_argument("--pmc-summary", metavar="CSV",
                    help="only summarise a rocprofv3 --pmc counter-collection CSV: the mean "
                         "per-dispatch counter value over the last --trace-last dispatches "
                         "whose name contains --trace-kernel")
    ap.add_argument("--trace-kernel", default="plane_hv_kernel<double")
    ap.add_argument("--trace-last", type=int, default=0)
    ap.add_argument("--kernel-paths", type=int, default=0,
                    help="kernel-path mask forced process-wide (0: by size)")
    ap.add_argument("--large-cell", default="cfg4",
                    help="workload of the one-solve large-cell leg ('none' to skip)")
    ap.add_argument("--large-strategy", default="grt")
    ap.add_argument("--large-kerker", type=int, default=1)
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary, args.trace_kernel, args.trace_last)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.trace_kernel, args.trace_last)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the response path here is single-GPU "
              "(k-point sharding across GPUs is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    # setup and eigensolver progress on stderr (large cells take minutes)
    os.environ.setdefault("IKR_VERBOSE", "1")
    import torch

    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return

    from paper_2505_02319_amd import (ResponseSystem, default_opts, profile_enable,
                                      profile_query, profile_reset)
    from workloads import B_SEED, config, random_field

    spec = config(args.workload)
    torch.cuda.set_device(0)
    if args.kernel_paths:
        from paper_2505_02319_amd import set_kernel_paths
        set_kernel_paths(args.kernel_paths)
    if args.gradient:
        gradient_bench(torch, spec, args)
        return
    t0 = time.perf_counter()
    rs = ResponseSystem(spec, ground_state="compute")
    info = rs.setup_info()
    t_setup = time.perf_counter() - t0
    log(f"setup {spec.name}: {t_setup:.1f} s, eigensolver steps {info['gs_iters']}, "
        f"residual {info['gs_residual']:.1e}, min gap {min(info['gaps']):.2e}")
    t0 = time.perf_counter()
    rs.tune_launches(precision=args.precision, schur=args.schur)
    t_tune = time.perf_counter() - t0
    log(f"launch tuning: {t_tune:.2f} s")
    b = torch.from_numpy(random_field(spec, B_SEED)).cuda()
    opts = default_opts(strategy=args.strategy, tol=1e-8, tol_is_relative=1,
                        precision=args.precision, schur=args.schur, kerker=args.kerker)

    # warmup; the last warmup step times every hot kernel to find the dominant
    # one, whose launches alone are then timed live inside the timed region
    dom = "plane_hv"
    for w in range(max(args.warmup, 1)):
        last = w == max(args.warmup, 1) - 1
        if last:
            profile_reset()
            profile_enable(True)
        _, st = rs.solve(b, opts)
        if last:
            profile_enable(False)
            allk = profile_query()
            dom = max(allk, key=lambda k: allk[k][1])
        log(f"warmup {w}: {st['seconds']:.3f} s, N_ham {st['n_ham']}, "
            f"GMRES iters {st['gmres_iters']}")

    profile_reset()
    profile_enable(dom)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    n_ham = 0
    gm = 0
    for s in range(args.steps):
        x, st = rs.solve(b, opts)
        n_ham += st["n_ham"]
        gm += st["gmres_iters"]
        log(f"step {s}: {st['seconds']:.3f} s, N_ham {st['n_ham']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    profile_enable(False)
    prof = profile_query()

    # the same solves with every CG iteration replayed from a captured graph
    graph = None
    if args.graph_steps > 0:
        gopts = default_opts(strategy=args.strategy, tol=1e-8, tol_is_relative=1,
                             precision=args.precision, schur=args.schur, batching=1,
                             kerker=args.kerker)
        rs.solve(b, gopts)                       # captures the graphs
        torch.cuda.synchronize()
        t_g = time.perf_counter()
        for _ in range(args.graph_steps):
            xg, stg = rs.solve(b, gopts)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t_g) / args.graph_steps
        graph = {"seconds_per_solve": sec, "solves_per_s": 1.0 / sec, "n_ham": stg["n_ham"],
                 "rel_diff_vs_launches": float(torch.linalg.norm(xg - x) / torch.linalg.norm(x))}
        log(f"graph replay: {sec:.3f} s per solve, N_ham {stg['n_ham']}")

    bnorm = float(torch.linalg.norm(b))
    true_rel, fp64, n32, other, plain, strategies = None, None, None, None, None, None
    if not args.no_checks:
        true_rel, fp64, n32, other = accuracy_checks(rs, b, bnorm, args, default_opts)
        plain = plain_fp64_leg(rs, b, bnorm, args, default_opts)
        strategies = strategy_legs(rs, b, bnorm, args, default_opts)

    launches, ms, by = prof[dom]
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3),
                   "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for k, v in allk.items()}
    bytes_per_launch = by / max(launches, 1)
    value = args.steps / elapsed
    out = {
        "metric": "drho solves/s at rel. res 1e-8",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32/f64",
        "fp64_cg_solve": fp64,
        "graph_replay_solve": graph,
        "n_ham_fp32_per_solve": n32,
        "data": "synthetic",
        "config": {"workload": describe(spec, args), "global_batch": 1,
                   "parallelism": "single-gpu"},
        "hpsi_band_applies_per_s": n_ham / elapsed,
        "n_ham_per_solve": n_ham / args.steps,
        "gmres_iters_per_solve": gm / args.steps,
        "true_rel_residual": true_rel,
        "plain_fp64_solve": plain,
        "speedup_vs_plain_fp64": (plain["seconds"] / (elapsed / args.steps)) if plain else None,
        "strategies": strategies,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(spec.name, dom),
                     "avg_launch_us": 1e3 * ms / max(launches, 1), "launches": launches,
                     "bytes_per_launch": bytes_per_launch},
        "kernels_warmup_step": kernels,
        "launch_tuning": tuning_of(rs),
        "setup_seconds": t_setup,
        "launch_tuning_seconds": t_tune,
    }
    rs.close()
    if args.large_cell != "none":
        out["large_cell_solve"] = large_cell_leg(torch, args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(spec, n_ham / args.steps, args.cpu_seconds)
        log("whole solve on the small cell, oracle and GPU ...")
        out["cpu_baseline"]["whole_solve_small_cell"] = whole_solve_small(args)
    print(json.dumps(out), flush=True)


def gradient_bench(torch, spec, args):
    """Loss L = ||drho - drho_t||^2 with drho = E^-1 b and drho_t = E^-1 b' (tight):
    forward and backward (adjoint GMRES, dL/db, and dL/dA through the adjoint
    Sternheimer solves) timed, then checked against central differences in b
    (exact for a quadratic) and in the amplitude of atom 0 (ground state
    recomputed at A +- h)."""
    import numpy as np

    from paper_2505_02319_amd import ResponseSystem, default_opts, dyson_solve
    from workloads import B_SEED, BPRIME_SEED, random_field
    opts = default_opts(strategy="grt", tol=1e-10, tol_is_relative=1, precision=0)
    t0 = time.perf_counter()
    rs = ResponseSystem(spec, ground_state="compute")
    log(f"setup {spec.name}: {time.perf_counter() - t0:.1f} s")
    b = torch.from_numpy(random_field(spec, B_SEED)).cuda()
    target, _ = rs.solve(torch.from_numpy(random_field(spec, BPRIME_SEED)).cuda(),
                         default_opts(strategy="grt", tol=1e-10, tol_is_relative=1))
    amp = torch.tensor(np.asarray(spec.amp, float), requires_grad=True)
    bl = b.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x = dyson_solve(bl, rs, opts, amplitudes=amp)
    loss = torch.sum((x - target) ** 2)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t1
    t2 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t2
    gb = bl.grad.detach()
    ga = amp.grad.numpy().copy()
    log(f"forward {t_fwd:.2f} s, backward {t_bwd:.2f} s")

    def lossval(r, bv):
        xv, _ = r.solve(bv, opts)
        return float(torch.sum((xv - target) ** 2))
    d = torch.from_numpy(random_field(spec, 7)).cuda()
    h = 1e-3
    fd_b = (lossval(rs, b + h * d) - lossval(rs, b - h * d)) / (2 * h)
    an_b = float(torch.sum(gb * d))
    ha = 1e-4
    vals = []
    for sgn in (1, -1):
        a2 = np.array(spec.amp, float)
        a2[0] += sgn * ha
        r2 = ResponseSystem(spec.with_(amp=a2), ground_state="compute")
        vals.append(lossval(r2, b))
        r2.close()
        log(f"amplitude {'+' if sgn > 0 else '-'}h done")
    fd_a = (vals[0] - vals[1]) / (2 * ha)
    out = {"metric": "gradient of ||drho - drho_t||^2 (dL/db, dL/dA)", "workload": spec.name,
           "forward_s": t_fwd, "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd,
           "dLdb_directional_rel_err_vs_fd": abs(an_b - fd_b) / abs(fd_b),
           "dLdA0": float(ga[0]), "dLdA0_fd": fd_a,
           "dLdA0_rel_err_vs_fd": abs(ga[0] - fd_a) / abs(fd_a),
           "fd_steps": {"b": h, "A": ha}, "gmres_tol": 1e-10, "loss": float(loss.detach())}
    print(json.dumps(out), flush=True)
    rs.close()


def accuracy_checks(rs, b, bnorm, args, default_opts):
    """Untimed: the true residual of the benchmarked solve (tight CG), and the
    same solve with the Sternheimer CG in FP64 throughout."""
    import torch
    vopts = default_opts(strategy=args.strategy, tol=1e-8, tol_is_relative=1,
                         precision=args.precision, schur=args.schur, kerker=args.kerker,
                         want_true_residual=1)
    xv, vst = rs.solve(b, vopts)
    bnorm = float(torch.linalg.norm(b))
    true_rel = vst["true_res"] / bnorm
    log(f"true relative residual {true_rel:.2e}")
    # the same solve with the Sternheimer CG in FP64 throughout (untimed
    # reference for the mixed-precision error and speed-up)
    popts = default_opts(strategy=args.strategy, tol=1e-8, tol_is_relative=1, precision=0,
                         schur=args.schur, kerker=args.kerker, want_true_residual=1)
    xp, pst = rs.solve(b, popts)
    fp64 = {"seconds": pst["seconds"], "n_ham": pst["n_ham"],
            "true_rel_residual": pst["true_res"] / bnorm,
            "rel_diff_vs_mixed": float(torch.linalg.norm(xv - xp) / torch.linalg.norm(xp))}
    log(f"fp64 CG: {pst['seconds']:.3f} s, true rel. residual {fp64['true_rel_residual']:.2e}")
    other = None
    return true_rel, fp64, vst["n_ham_fp32"], other


def trace_summary(path, kernel, last):
    """Durations of the last `last` dispatches (all if 0) of the kernels whose
    name contains `kernel`, from a rocprofv3 --kernel-trace CSV; with the
    bench run under the profiler and nothing launched after its timed steps,
    these are the launches its HIP events timed."""
    import csv
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    cols = {c.lower(): c for c in rows[0]} if rows else {}
    kn, ks, ke = cols["kernel_name"], cols["start_timestamp"], cols["end_timestamp"]
    sel = sorted((r for r in rows if kernel in r[kn]), key=lambda r: int(r[ks]))
    if last > 0:
        sel = sel[-last:]
    us = [(int(r[ke]) - int(r[ks])) * 1e-3 for r in sel]
    # occupancy of the GPU over the window of the selected dispatches: the
    # union of all kernels' intervals in it, and the idle time between them
    gaps = None
    if sel:
        w0, w1 = int(sel[0][ks]), int(sel[-1][ke])
        iv = sorted((int(r[ks]), int(r[ke])) for r in rows
                    if int(r[ks]) >= w0 and int(r[ke]) <= w1)
        busy, cur0, cur1, idle_n = 0, iv[0][0], iv[0][1], 0
        for a, b in iv[1:]:
            if a > cur1:
                busy += cur1 - cur0
                cur0, cur1 = a, b
                idle_n += 1
            else:
                cur1 = max(cur1, b)
        busy += cur1 - cur0
        win = w1 - w0
        gaps = {"window_ms": win * 1e-6, "busy_ms": busy * 1e-6, "idle_frac": 1 - busy / win,
                "dispatches": len(iv), "idle_us_per_dispatch": (win - busy) * 1e-3 / len(iv)}
    print(json.dumps({"trace": os.path.basename(path), "kernel": kernel, "dispatches": len(us),
                      "avg_us": sum(us) / max(len(us), 1), "min_us": min(us) if us else None,
                      "max_us": max(us) if us else None,
                      "names": sorted({r[kn] for r in sel}), "occupancy": gaps}), flush=True)


def pmc_summary(path, kernel, last):
    """Mean per-dispatch value of each counter in a rocprofv3 --pmc CSV over
    the last `last` dispatches (all if 0) of the kernels whose name contains
    `kernel` (values of one dispatch summed over their rows)."""
    import csv
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    cols = {c.lower(): c for c in rows[0]} if rows else {}
    kn, dk = cols["kernel_name"], cols["dispatch_id"]
    cn, cv = cols["counter_name"], cols["counter_value"]
    per = {}
    for r in rows:
        if kernel in r[kn]:
            per.setdefault(int(r[dk]), {}).setdefault(r[cn], 0.0)
            per[int(r[dk])][r[cn]] += float(r[cv])
    ids = sorted(per)
    if last > 0:
        ids = ids[-last:]
    names = sorted({c for i in ids for c in per[i]})
    mean = {c: sum(per[i].get(c, 0.0) for i in ids) / max(len(ids), 1) for c in names}
    print(json.dumps({"pmc": os.path.basename(path), "kernel": kernel, "dispatches": len(ids),
                      "mean_per_dispatch": mean}), flush=True)


def plain_fp64_leg(rs, b, bnorm, args, default_opts):
    """The plain FP64 reference path on the same solve: the Sternheimer CGs of
    the k-points one after the other, the host reading the live count after
    every CG iteration, FP64 throughout (solver option batching = 2)."""
    import torch
    popts = default_opts(strategy=args.strategy, tol=1e-8, tol_is_relative=1, precision=0,
                         schur=args.schur, kerker=args.kerker, batching=2)
    rs.solve(b, popts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = rs.solve(b, popts)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    log(f"plain fp64 path: {sec:.3f} s, N_ham {st['n_ham']}")
    return {"seconds": sec, "n_ham": st["n_ham"], "gmres_iters": st["gmres_iters"]}


def strategy_legs(rs, b, bnorm, args, default_opts):
    """N_ham, seconds, true residual and the paper's efficiency
    eta = -log10(||r_end|| / ||r_0||) / N_ham (r_0 = b, x0 = 0; Sec. 4.1.3) of
    the strategies with and without the Kerker preconditioner (Sec. 3.3), and
    eta_rel against D10, all in the headline's precision."""
    import math
    out = {}
    for name, strat, kerk, rec in [("grt", "grt", 0, 0), ("bal", "bal", 0, 0),
                                   ("D10", "D10", 0, 0), ("Pgrt", "grt", 1, 0),
                                   ("Pbal", "bal", 1, 0), ("PD10", "D10", 1, 0),
                                   ("Pgrt_warm", "grt", 1, 4)]:
        o = default_opts(strategy=strat, tol=1e-8, tol_is_relative=1, precision=args.precision,
                         schur=args.schur, kerker=kerk, want_true_residual=1, recycle=rec)
        _, st = rs.solve(b, o)
        tr = st["true_res"] / bnorm
        eta = -math.log10(tr) / st["n_ham"] if tr > 0 else None
        out[name] = {"n_ham": st["n_ham"], "seconds": st["seconds"],
                     "gmres_iters": st["gmres_iters"], "true_rel_residual": tr, "eta": eta,
                     "warm_started": st["warm_started"]}
    ref = out["D10"]["eta"]
    for v in out.values():
        v["eta_rel_vs_D10"] = v["eta"] / ref if (v["eta"] and ref) else None
    log("strategies: " + ", ".join(f"{k} N_ham {v['n_ham']} res {v['true_rel_residual']:.1e}"
                                   for k, v in out.items()))
    return out


def large_cell_leg(torch, args):
    """One timed solve on the large smeared cell (setup by the library's GPU
    eigensolver, timed apart), with per-kernel times and its true residual."""
    from paper_2505_02319_amd import (ResponseSystem, default_opts, profile_enable,
                                      profile_query, profile_reset)
    from workloads import B_SEED, config, random_field
    spec = config(args.large_cell)
    t0 = time.perf_counter()
    rs = ResponseSystem(spec, ground_state="compute")
    info = rs.setup_info()
    t_setup = time.perf_counter() - t0
    log(f"large cell {spec.name}: setup {t_setup:.1f} s, eigensolver steps {info['gs_iters']}")
    t0 = time.perf_counter()
    rs.tune_launches(precision=1, schur=1)
    t_tune = time.perf_counter() - t0
    log(f"large cell launch tuning: {t_tune:.2f} s")
    b = torch.from_numpy(random_field(spec, B_SEED)).cuda()
    bnorm = float(torch.linalg.norm(b))
    o = default_opts(strategy=args.large_strategy, tol=1e-8, tol_is_relative=1, precision=1,
                     schur=1, kerker=args.large_kerker)
    profile_reset()
    profile_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, st = rs.solve(b, o)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t1
    profile_enable(False)
    prof = profile_query()
    log(f"large cell solve: {sec:.2f} s, N_ham {st['n_ham']}, GMRES {st['gmres_iters']}")
    # true residual ||b - E x|| with every Sternheimer CG at 1e-14 (Sec. 4.1.3)
    ex, _ = rs.apply_dielectric(x, 1e-14, default_opts(strategy="fixed", precision=0))
    true_rel = float(torch.linalg.norm(b - ex)) / bnorm
    log(f"large cell true relative residual {true_rel:.2e}")
    tuning = tuning_of(rs)
    rs.close()
    kernels = {k: {"launches": v[0], "ms": round(v[1], 1),
                   "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for k, v in prof.items() if v[0]}
    return {"workload": describe_large(spec, args), "setup_seconds": t_setup,
            "launch_tuning_seconds": t_tune,
            "eigensolver_steps": info["gs_iters"], "seconds": sec, "solves_per_s": 1.0 / sec,
            "n_ham": st["n_ham"], "n_ham_fp32": st["n_ham_fp32"], "gmres_iters": st["gmres_iters"],
            "true_rel_residual": true_rel,
            "note": "kernel times from HIP events on every hot launch of the timed solve",
            "kernels": kernels, "launch_tuning": tuning}


def tuning_of(rs):
    """The launch shapes the system measured, keyed "fp64/thick" and so on."""
    return {f"{p}/{c}": v for (p, c), v in rs.tuning().items()}


def describe_large(spec, args):
    L = spec.lattice
    return (f"{spec.name}: {len(spec.frac_pos)}-atom cell {L[0]:g}x{L[1]:g}x{L[2]:g} bohr, "
            f"Ecut {spec.ecut:g} Ha, FFT {spec.fft[0]}x{spec.fft[1]}x{spec.fft[2]}, "
            f"{spec.kgrid[0]}x{spec.kgrid[1]}x{spec.kgrid[2]} k, {spec.nocc}+{spec.nextra} bands, "
            f"T {spec.temperature:g}, strategy {'P' if args.large_kerker else ''}"
            f"{args.large_strategy}, mixed precision, tau 1e-8||b||")


def describe(spec, args):
    L = spec.lattice
    return (f"{spec.name}: {len(spec.frac_pos)}-atom cell {L[0]:g}x{L[1]:g}x{L[2]:g} bohr, "
            f"Ecut {spec.ecut:g} Ha, FFT {spec.fft[0]}x{spec.fft[1]}x{spec.fft[2]}, "
            f"{spec.kgrid[0]}x{spec.kgrid[1]}x{spec.kgrid[2]} k, {spec.nocc}+{spec.nextra} bands, "
            f"T {spec.temperature:g}, K_H{' + Slater' if spec.xc else ''}, "
            f"strategy {'P' if args.kerker else ''}{args.strategy} "
            f"({'Kerker-preconditioned' if args.kerker else 'unpreconditioned'} GMRES), "
            f"extra bands by sum over states "
            f"{'on' if args.schur else 'off'}, CG precision "
            f"{'mixed' if args.precision else 'fp64'}, m 20, tau 1e-8||b||")


def copy_probe(torch, mib):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    for _ in range(5):
        c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "copies": 5}), flush=True)


KERNEL_SOURCES = {   # sources whose change invalidates a kernel's counter readings
    "plane_hv": ["fft.hip", "fft_core.h", "common.h"],
    "col_inv": ["fft.hip", "fft_core.h", "common.h"],
    "col_fwd": ["fft.hip", "fft_core.h", "common.h"],
    "gram": ["blas.hip", "blas.h", "common.h"],
    "update": ["cg.hip", "cg.h", "blas.h", "common.h"],
    "cg_step": ["cg.hip", "cg.h", "common.h"],
}


def source_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel.replace("_fp32", ""), []):
        with open(os.path.join(ROOT, "paper_2505_02319_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, each scaled by the same counter's reading
    for a plain copy of known size); None when there is none for this kernel
    and workload, or when the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if not line.startswith("traffic:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("kernel") != kernel or kv.get("source") != source_digest(kernel):
                continue
            return (float(kv["fetch_kib"]) * 1024 / float(kv["fetch_factor"]) +
                    float(kv["write_kib"]) * 1024 / float(kv["write_factor"]))
    return None


if __name__ == "__main__":
    main()
