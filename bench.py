#!/usr/bin/env python3
"""Benchmark of the blended-shell Stokes hot path on one MI355X.

Workload: spherical shell r in [0.55, 1], icosahedral macro mesh with 10
tangential subdivisions x 2 radial layers (12,000 macro-tets), refined to level
4: N_u = 199,680,390 velocity and N_p = 8,448,066 pressure DoFs.  Viscosity
eta = exp(ln(1e4) (0.5 - T)) from a seeded degree-8 spherical-harmonic
temperature T, density rho = exp(0.5 (1 - r)), buoyancy f = int T r_hat . phi,
no-slip inner and free-slip outer boundary.  All inputs are synthetic.

One step is one forward + backward pass of the differentiable solve:
  set_log_viscosity  (eta on every level, diag(A), FP64 Chebyshev bounds)
  rhs_buoyancy       (f from T)
  solve              (FP64 FGMRES to 1e-8 relative residual, symmetric Uzawa
                      with V-cycle BFBT, FP32 multigrid / Schur inner solves)
  solve_adjoint      (the same solver on the transposed system, J = |u|^2 / 2)
  gradient           (dJ/d ln eta and dJ/dT)
value = (N_u + N_p) / seconds per step, in MDoF/s.

Outside the timed steps the bench also reports: the A-apply throughput at the
finest level in FP32 and FP64 (N_u / time per apply), the all-FP64 forward
solve with its time and the mixed solve's difference from it, the roofline
position of the dominant kernel (the FP32 A-apply sweep) and the CPU oracle
timed on a small shell sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# counted FP32 VALU arithmetic per micro-tet of the A-apply sweep kernel
# (fma/fmac/fmamk = 2 flops, mul/add/sub = 1, rsq/rcp = 1): the VALU
# instructions of the element-loop body in the kernel's gfx950 assembly (917
# instructions, one micro-tet per lane and iteration)
A_FLOPS_PER_TET_FP32 = 1194
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flops x 2.4 GHz
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_sweep_A_fp32_shell10x2_L4.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2506_04157_amd", "csrc", "kernels.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None when absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(nt=3, nr=1, level=1):
    """The FP64 oracle (assembly + constrained direct solve, adjoint solve and
    assembled gradient) on a small shell of the same family, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import inputs
    from oracle.adjoint import grad_log_eta, grad_temperature
    from oracle.fem import assemble_A, assemble_B, rhs_buoyancy
    from oracle.mesh import RefinedMesh, shell_macros
    from oracle.system import solve_stokes, velocity_basis

    with threadpool_limits(1):
        t0 = time.perf_counter()
        m = RefinedMesh(shell_macros(nt, nr, 0.55, 1.0), level)
        field = inputs.SHField(2)
        T2, T1 = field.temperature(m.X2), field.temperature(m.X1)
        eta = inputs.viscosity_contrast(T1, 1e4)
        lnrho = inputs.ln_density(m.X1)
        A = assemble_A(m, eta)
        B = assemble_B(m)
        Bbar = B + assemble_B(m, lnrho, only_C=True)
        f = rhs_buoyancy(m, T2)
        Q, _, _ = velocity_basis(m, {1}, {2})
        u, p, _ = solve_stokes(A, Bbar, f, np.zeros(m.n1), Q, Bt=B.T)
        lam, _, _ = solve_stokes(A, B, u, np.zeros(m.n1), Q, Bt=Bbar.T)
        grad_log_eta(m, eta, u, lam)
        grad_temperature(m, lam)
        dt = time.perf_counter() - t0
    ndof = 3 * m.n2 + m.n1
    return {"value": ndof / dt / 1e6, "unit": "MDoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"shell {nt}x{nr} ({60 * nt * nt * nr} macro-tets) level {level}, N_u={3 * m.n2}, "
                       f"N_p={m.n1}, same fields and BCs; mesh + assembly + direct forward and adjoint "
                       f"solves + gradient in FP64, {dt:.1f} s on 1 thread"),
            "seconds": dt}


def _rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


ROOF_KERNEL = "k_sweep<float, true, 1>"


def summarize_profile(d, out, cmd):
    """Text summary of a rocprofv3 --kernel-trace --stats run: the kernels by
    total time and, from the trace, the roofline kernel's launches grouped by
    grid size (the finest level has the largest grid)."""
    lines = [f"# rocprofv3 kernel summary", f"# command: {cmd}", ""]
    stats = _rows(os.path.join(d, "run_kernel_stats.csv"))
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    lines.append(f"total kernel time {tot / 1e9:.3f} s over {len(stats)} kernels")
    lines.append(f"{'total_s':>9} {'calls':>8} {'avg_us':>10} {'pct':>6}  kernel")
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:30]:
        lines.append(f"{float(r['TotalDurationNs']) / 1e9:9.3f} {int(r['Calls']):8d} "
                     f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}  {r['Name'][:110]}")
    tr = os.path.join(d, "run_kernel_trace.csv")
    if os.path.exists(tr):
        import csv
        groups = {}
        with open(tr) as fh:
            for r in csv.DictReader(fh):
                if ROOF_KERNEL not in r["Kernel_Name"]:
                    continue
                g = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)
                dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                s_, c_ = groups.get(g, (0, 0))
                groups[g] = (s_ + dt, c_ + 1)
        lines += ["", f"{ROOF_KERNEL} launches by grid size (work-items):"]
        for g in sorted(groups, reverse=True):
            s_, c_ = groups[g]
            lines.append(f"  grid {g:>10d}: {c_:6d} launches, average {s_ / c_ / 1e3:10.1f} us")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_traffic(dfetch, dwrite, n_u, out, cmd):
    """HBM bytes per launch of the roofline kernel at the finest level from
    FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled by the ratio of
    known bytes to the counter's reading on the plain copy of n_u floats that
    bench.py --apply-only performs before the timings."""
    def per_kernel(d, counter):
        acc = {}
        for r in _rows(os.path.join(d, "run_counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            key = (r["Kernel_Name"], int(r["Grid_Size"]))
            acc.setdefault(key, []).append(float(r["Counter_Value"]))
        return acc
    f, w = per_kernel(dfetch, "FETCH_SIZE"), per_kernel(dwrite, "WRITE_SIZE")
    known = 4.0 * n_u
    def copy_kib(acc):
        # the copy kernel reading/writing the most bytes is the calibration copy
        cands = [(sum(v) / len(v), k) for k, v in acc.items() if "copyBuffer" in k[0] or "copy" in k[0].lower()]
        return max(cands)[0]
    kf, kw = known / (copy_kib(f) * 1024.0), known / (copy_kib(w) * 1024.0)
    def roof(acc):
        cands = [(k[1], sum(v) / len(v)) for k, v in acc.items() if ROOF_KERNEL in k[0]]
        return max(cands)[1]
    fb, wb = roof(f) * 1024.0 * kf, roof(w) * 1024.0 * kw
    lines = ["# HBM traffic of the roofline kernel (finest level, largest grid)",
             f"# fetch command: {cmd[0]}", f"# write command: {cmd[1]}",
             f"kernel: {ROOF_KERNEL}",
             f"kernel_source_sha256_16: {kernel_sha()}",
             f"copy_bytes_known: {known:.0f}",
             f"fetch_scale: {kf:.4f}", f"write_scale: {kw:.4f}",
             f"fetch_bytes_per_launch: {fb:.0f}", f"write_bytes_per_launch: {wb:.0f}",
             f"hbm_bytes_per_launch: {fb + wb:.0f}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_counters(d, out, cmd, match):
    """Per-kernel averages of every counter of a rocprofv3 --pmc run over the
    dispatches whose kernel name contains `match`, grouped by grid size."""
    acc = {}
    for r in _rows(os.path.join(d, "run_counter_collection.csv")):
        if match not in r["Kernel_Name"]:
            continue
        key = (r["Kernel_Name"][:90], int(r["Grid_Size"]), r["Counter_Name"])
        acc.setdefault(key, []).append(float(r["Counter_Value"]))
    lines = ["# rocprofv3 counter summary (average per dispatch)", f"# command: {cmd}", ""]
    for (k, g, c) in sorted(acc, key=lambda t: (t[0], -t[1], t[2])):
        v = acc[(k, g, c)]
        lines.append(f"{k}  grid {g:>10d}  {c:<16s} {sum(v) / len(v):14.4f}  ({len(v)} dispatches)")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        # bench.py --summarize-counters DIR OUT "COMMAND" KERNEL_SUBSTRING
        summarize_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-profile":
        # bench.py --summarize-profile DIR OUT "COMMAND"
        summarize_profile(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-traffic":
        # bench.py --summarize-traffic FETCH_DIR WRITE_DIR N_U OUT "FETCH_CMD" "WRITE_CMD"
        summarize_traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], (sys.argv[6], sys.argv[7]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=4)
    ap.add_argument("--n-tan", type=int, default=10)
    ap.add_argument("--n-rad", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--apply-only", action="store_true",
                    help="only the A-apply timings (for counter collection)")
    ap.add_argument("--transfer-only", action="store_true",
                    help="only the finest-level FP32 restriction and prolongation (for counter collection)")
    ap.add_argument("--l-eta-study", action="store_true",
                    help="only the coarse-viscosity study: A-block CG iterations and time of 10 FGMRES "
                         "iterations with the viscosity model of eq. ViscosityDef for l_eta = -1, 0, 1")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not "
              "part of this build", file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("STK_VERBOSE", "1")   # solver progress on stderr
    import numpy as np
    import torch

    import inputs
    from paper_2506_04157_amd import StokesContext, default_params

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    sc = StokesContext("shell", level=args.level, min_level=0, n_tan=args.n_tan, n_rad=args.n_rad, device=dev)
    n2, n1 = sc.sizes()
    Nu, Np = 3 * n2, n1
    log(f"context {time.perf_counter() - t0:.1f}s  N_u={Nu} N_p={Np}")
    X2 = torch.tensor(sc.coords(which=2)[0], device=dev)
    X1 = torch.tensor(sc.coords(which=1)[0], device=dev)
    field = inputs.SHField(2)
    T2 = field.temperature_torch(X2).contiguous()
    T1 = field.temperature_torch(X1)
    mlog = (float(np.log(1e4)) * (0.5 - T1)).contiguous()
    lnrho = (0.5 * (1.0 - torch.linalg.norm(X1, dim=1))).contiguous()
    del X2, X1, T1
    mixed = default_params(precision=32, tol_rel=1e-8)
    full = default_params(precision=64, tol_rel=1e-8)
    n_tets = 60 * args.n_tan ** 2 * args.n_rad * 8 ** args.level
    result = {}

    def a_apply():
        out = {}
        for dt_, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            x = torch.tensor(inputs.uniform(0, Nu), dtype=dt_, device=dev)
            y = torch.empty_like(x)
            sc.time_apply_A(x, y, reps=2)
            ms, mk = sc.time_apply_A(x, y, reps=20)
            out[name] = {"gdof_s": Nu / ms / 1e6, "ms_per_apply": ms, "ms_sweep_kernel": mk}
            log(f"A-apply {name}: {ms:.3f} ms/apply ({Nu / ms / 1e6:.1f} GDoF/s), sweep kernel {mk:.3f} ms")
            del x, y
        return out

    if args.apply_only:
        # A-apply timings, preceded by plain device copies of known size that
        # calibrate the HBM byte counters (FETCH_SIZE / WRITE_SIZE)
        sc.set_log_viscosity(mlog, lnrho, mixed)
        a = torch.ones(Nu, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {3} copies of {4 * Nu} bytes")
        del a, b
        result["a_apply"] = a_apply()
        print(json.dumps(result["a_apply"]), flush=True)
        return

    if args.transfer_only:
        # five FP32 restrictions to and prolongations from the next coarser
        # level; each call zero-fills its output and returns synchronised
        sc.set_log_viscosity(mlog, lnrho, mixed)
        lf = args.level
        nc = 3 * sc.sizes(lf - 1)[0]
        rf = torch.tensor(inputs.uniform(1, Nu), dtype=torch.float32, device=dev)
        ec = torch.tensor(inputs.uniform(2, nc), dtype=torch.float32, device=dev)
        out = {}
        for name, fn in (("restrict", lambda: sc.restrict(rf, lf)), ("prolong", lambda: sc.prolong(ec, lf))):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            out[name] = {"ms_per_call": (time.perf_counter() - t1) / 5 * 1e3}
            log(f"{name} level {lf}: {out[name]['ms_per_call']:.3f} ms per call")
        print(json.dumps(out), flush=True)
        return

    if args.l_eta_study:
        # Fig. AIterations setting: the first 10 FGMRES iterations of a solve,
        # A-block CG iterations and their time, per choice of l_eta (-1: P1
        # viscosity on every level)
        base = inputs.base_viscosity_profile()
        f = None
        study = {}
        for l_eta in (-1, 0, 1):
            prm = default_params(precision=32, tol_rel=1e-12, max_outer=10)
            sc.set_temperature_viscosity(T2, base, l_eta=l_eta, lnrho=lnrho, params=prm)
            if f is None:
                f = sc.rhs_buoyancy(T2)
            u, p, rep = sc.solve(f, params=prm, allow_noconv=True)
            torch.cuda.synchronize()
            study[str(l_eta)] = {k: rep[k] for k in ("iterations", "rel_residual", "a_solves", "a_cg_its",
                                                    "vcycles", "coarse_its", "seconds")}
            log(f"l_eta {l_eta}: {rep['iterations']} FGMRES its, rel res {rep['rel_residual']:.2e}, "
                f"A-block CG its {rep['a_cg_its']}, {rep['seconds']:.1f}s")
        print(json.dumps({"l_eta_study": study, "E_A": 4.610, "V_A": 2.996,
                          "eta_base": "inputs.base_viscosity_profile()", "level": args.level}), flush=True)
        return

    def step():
        tt = {}
        s = time.perf_counter()
        sc.set_log_viscosity(mlog, lnrho, mixed)
        f = sc.rhs_buoyancy(T2)
        torch.cuda.synchronize()
        tt["setup_s"] = time.perf_counter() - s
        u, p, rep = sc.solve(f, params=mixed)
        torch.cuda.synchronize()
        tt["forward"] = rep
        lu, lp, rep2 = sc.solve_adjoint(u, None, mixed)
        torch.cuda.synchronize()
        tt["adjoint"] = rep2
        s = time.perf_counter()
        gm, gT = sc.gradient(u, lu)
        torch.cuda.synchronize()
        tt["gradient_s"] = time.perf_counter() - s
        return u, p, gm, gT, tt

    for i in range(args.warmup):
        log(f"warmup step {i + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()
    log(f"timed steps: {args.steps}")
    t_start = time.perf_counter()
    for i in range(args.steps):
        u, p, gm, gT, tt = step()
        log(f"step {i + 1}: forward {tt['forward']['seconds']:.2f}s ({tt['forward']['iterations']} its), "
            f"adjoint {tt['adjoint']['seconds']:.2f}s ({tt['adjoint']['iterations']} its)")
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t_start) / args.steps
    fw, ad = tt["forward"], tt["adjoint"]
    result["step_breakdown"] = {
        "setup_s": tt["setup_s"], "forward_solve_s": fw["seconds"], "adjoint_solve_s": ad["seconds"],
        "gradient_s": tt["gradient_s"], "forward_iterations": fw["iterations"],
        "forward_rel_residual": fw["rel_residual"], "adjoint_iterations": ad["iterations"],
        "adjoint_rel_residual": ad["rel_residual"],
        "forward_counts": {k: fw[k] for k in ("a_solves", "a_cg_its", "s_solves", "s_cg_its", "vcycles",
                                              "coarse_its", "mass_its")},
        "grad_finite": bool(torch.isfinite(gm).all().item() and torch.isfinite(gT).all().item()),
    }

    result["a_apply"] = a_apply()

    if not args.no_fp64:
        log("all-FP64 forward solve")
        sc.set_log_viscosity(mlog, lnrho, full)
        f = sc.rhs_buoyancy(T2)
        u64, p64, r64 = sc.solve(f, params=full)
        torch.cuda.synchronize()
        du = (torch.linalg.norm(u - u64) / torch.linalg.norm(u64)).item()
        dp = (torch.linalg.norm(p - p64) / torch.linalg.norm(p64)).item()
        result["solve_fp32mg_vs_fp64"] = {
            "mixed_s": fw["seconds"], "fp64_s": r64["seconds"], "speedup": r64["seconds"] / fw["seconds"],
            "mixed_iterations": fw["iterations"], "fp64_iterations": r64["iterations"],
            "mixed_rel_residual": fw["rel_residual"], "fp64_rel_residual": r64["rel_residual"],
            "u_rel_diff_vs_fp64": du, "p_rel_diff_vs_fp64": dp}
        log(f"FP64 solve {r64['seconds']:.2f}s ({r64['iterations']} its); mixed {fw['seconds']:.2f}s; "
            f"|u-u64|/|u64| = {du:.2e}, |p-p64|/|p64| = {dp:.2e}")
        del u64, p64

    fp32 = result["a_apply"]["fp32"]
    achieved = A_FLOPS_PER_TET_FP32 * n_tets / (fp32["ms_sweep_kernel"] * 1e-3) / 1e12
    traffic = read_traffic() if (args.level, args.n_tan, args.n_rad) == (4, 10, 2) else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                "kernel": "k_sweep<float, blend, A> (A-apply plane sweep, finest level)",
                "flops_per_launch": A_FLOPS_PER_TET_FP32 * n_tets,
                "frac_of_nonpacked_fp32_peak": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                "hbm_gbs_algorithmic": (2 * Nu + Np) * 4 / (fp32["ms_sweep_kernel"] * 1e-3) / 1e9,
                "hbm_frac_algorithmic": (2 * Nu + Np) * 4 / (fp32["ms_sweep_kernel"] * 1e-3) / 1e9 / PEAK_HBM_GBS}

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline()
        log(f"oracle: {cpu['sample']}")

    value = (Nu + Np) / t_step / 1e6
    line = {
        "metric": "A-apply GDoF/s + time-to-1e-8 Stokes solve, FP32-MG vs FP64, 1 MI355X",
        "value": value, "unit": "MDoF/s",
        "value_definition": "(N_u + N_p) / seconds per step; step = set_log_viscosity + rhs + mixed forward "
                            "solve to 1e-8 + adjoint solve to 1e-8 + gradient",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"blended spherical shell [0.55,1], icosahedral {args.n_tan}x{args.n_rad} macro mesh "
                                f"({60 * args.n_tan ** 2 * args.n_rad} macro-tets), level {args.level}, P2-P1, "
                                "viscosity contrast 1e4, compressible (rho=exp(0.5(1-r))), tol 1e-8"),
                   "N_u": Nu, "N_p": Np, "micro_tets": n_tets, "parallelism": "single GPU"},
        "a_apply_gdof_s": {"fp32": fp32["gdof_s"], "fp64": result["a_apply"]["fp64"]["gdof_s"]},
        "a_apply": result["a_apply"],
        "solve_fp32mg_vs_fp64": result.get("solve_fp32mg_vs_fp64"),
        "step_breakdown": result["step_breakdown"],
        "roofline": roofline,
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
