#!/usr/bin/env python3
"""Benchmark of the blended-shell Stokes hot path on one MI355X.

Workload: spherical shell r in [0.55, 1], icosahedral macro mesh with 10
tangential subdivisions x 2 radial layers (12,000 macro-tets), refined to level
4: N_u = 199,680,390 velocity and N_p = 8,448,066 pressure DoFs.  Viscosity
eta = exp(ln(1e4) (0.5 - T)) from a seeded degree-8 spherical-harmonic
temperature T, density rho = exp(0.5 (1 - r)), buoyancy f = int T r_hat . phi,
no-slip inner and free-slip outer boundary.  All inputs are synthetic.

One timed step is one finest-level FP64 A-apply y = P A P x (the plane-sweep
kernel, the gather of shared nodes and the boundary projection) on a resident
seeded vector: value = N_u / seconds per step in GDoF/s.  The sweep kernel of
every timed step is bracketed by HIP events on the library's stream
(stk_kernel_timer); its average duration gives the roofline position.

After the timed steps, each once, within a wall-clock budget (STK_BENCH_BUDGET_S,
default 420 s from the start; legs that would not fit are listed as skipped):
  the FP32 A-apply (events, 20 applies);
  the CPU oracle: scipy FP64 SpMV of the assembled A on the 10x2 shell at
    level 1 (1 core, median of 20; the same product on all host cores beside
    it), and the oracle's direct solve pipeline on a 3x1 level-1 shell;
  the mixed-precision forward solve to 1e-8 (FP32 multigrid / Schur inner
    solves inside FP64 FGMRES) and the all-FP64 forward solve, with times,
    iterations, residuals and their difference;
  the mixed adjoint solve (J = |u|^2 / 2) and the gradient kernel;
  two temperature steps of the splitting scheme driven by the solved velocity.
The JSON line is printed once at the end, also when a leg fails or the
process receives SIGTERM.
"""
import argparse
import hashlib
import json
import os
import signal
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic arithmetic of the blended A-apply per micro-tet (4 quadrature
# points): the FP32 sweep's element loop counted from its gfx950 assembly
# (fma/fmac/fmamk = 2 flops, mul/add/sub = 1, rsq/rcp = 1).  The FP64 kernel
# executes about 100 more per micro-tet, the Newton steps of its rsq/rcp; they
# are not counted as algorithmic work.  The committed counter summary
# (FLOPS_FILE) holds this figure with the sweep-source hash it was checked on
# and the executed flops the VALU counters report per micro-tet; a figure whose
# hash no longer matches is reported as unverified.
A_FLOPS_PER_TET = 1194
PEAK_FP64_TFLOPS = 78.6           # MI355X published FP64 vector peak
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak (packed)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flops x 2.4 GHz
PEAK_HBM_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILES = {64: os.path.join(PROFILES, "traffic_k_sweep_A_fp64_shell10x2_L4.txt"),
                 32: os.path.join(PROFILES, "traffic_k_sweep_A_fp32_shell10x2_L4.txt")}
FLOPS_FILE = os.path.join(PROFILES, "flops_k_sweep_A_shell10x2_L4.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2506_04157_amd", "csrc", "kernels.hip")
DEVICE_HDR = os.path.join(ROOT, "paper_2506_04157_amd", "csrc", "device.hpp")
ROOF_KERNELS = {64: "k_sweep<double, true, 1>", 32: "k_sweep<float, true, 1>"}
METRIC = "A-apply GDoF/s + time-to-1e-8 Stokes solve, FP32-MG vs FP64, 1 MI355X"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _between(text, start, end):
    i = text.index(start) if start else 0
    return text[i:text.index(end, i)]


def kernel_sha():
    """Hash of the source the roofline kernel is built from: kernels.hip up to
    the end of the plane sweep (its helpers, the element arithmetic and the
    kernel), the sweep's launch wrapper, and device.hpp up to the sweep's LDS
    layout.  Kernels elsewhere in the files do not change it."""
    with open(KERNEL_SRC) as fh:
        k = fh.read()
    with open(DEVICE_HDR) as fh:
        d = fh.read()
    parts = [_between(k, None, "// Element-parallel variant for coarse levels"),
             _between(k, "void launch_stokes(", "\n}\n"),
             _between(d, None, "size_t sweep_lds_bytes")]
    return hashlib.sha256("\0".join(parts).encode()).hexdigest()[:16]


def _kv(path):
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def read_flops():
    """(algorithmic flops per micro-tet, verified): verified when the counter
    summary was taken on the current sweep source."""
    if not os.path.exists(FLOPS_FILE):
        return A_FLOPS_PER_TET, False
    kv = _kv(FLOPS_FILE)
    return A_FLOPS_PER_TET, kv.get("kernel_source_sha256_16") == kernel_sha()


def read_traffic(prec=64):
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None when absent or taken on a different kernel source."""
    path = TRAFFIC_FILES[prec]
    if not os.path.exists(path):
        return None
    kv = _kv(path)
    if kv.get("kernel_source_sha256_16") != kernel_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return {"os_cpu_count": os.cpu_count(), "lscpu_model": model}


def cpu_baseline(nt=10, nr=2, level=1, solve_nt=3, solve_nr=1, solve_level=1):
    """The FP64 oracle timed on the host: scipy SpMV of the assembled A (1
    thread, median of 20) on the 10x2 shell at level 1, in GDoF/s; and, as a
    secondary figure, the oracle's direct-solve pipeline (assembly,
    constrained forward and adjoint direct solves, gradient) on a small shell."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import inputs
    from oracle.adjoint import grad_log_eta, grad_temperature
    from oracle.fem import assemble_A, assemble_B, rhs_buoyancy
    from oracle.mesh import RefinedMesh, shell_macros
    from oracle.system import solve_stokes, velocity_basis

    field = inputs.SHField(2)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        m = RefinedMesh(shell_macros(nt, nr, 0.55, 1.0), level)
        eta = inputs.viscosity_contrast(field.temperature(m.X1), 1e4)
        A = assemble_A(m, eta)
        t_asm = time.perf_counter() - t0
        x = inputs.uniform(0, A.shape[0])
        ts = []
        for _ in range(20):
            s = time.perf_counter()
            y = A @ x
            ts.append(time.perf_counter() - s)
        t_spmv = float(np.median(ts))
        nu = A.shape[0]
    # the same product on all host cores (the oracle's OpenMP CSR product)
    omp = None
    try:
        from oracle import cspmv
        if not os.path.exists(cspmv.LIB):
            cspmv.build()
        yo = cspmv.spmv(A, x)
        tso = []
        for _ in range(20):
            s = time.perf_counter()
            cspmv.spmv(A, x, yo)
            tso.append(time.perf_counter() - s)
        t_omp = float(np.median(tso))
        omp = {"threads": cspmv.threads(), "ms": t_omp * 1e3, "gdof_s": nu / t_omp / 1e9,
               "max_rel_diff_vs_scipy": float(np.abs(yo - y).max() / np.abs(y).max())}
    except Exception as exc:   # a missing gcc/OpenMP only loses this secondary figure
        omp = {"error": str(exc)[:200]}
    with threadpool_limits(1):
        del A, y
        # secondary: the direct-solve pipeline on a small shell
        t1 = time.perf_counter()
        ms = RefinedMesh(shell_macros(solve_nt, solve_nr, 0.55, 1.0), solve_level)
        T2, T1 = field.temperature(ms.X2), field.temperature(ms.X1)
        eta_s = inputs.viscosity_contrast(T1, 1e4)
        lnrho = inputs.ln_density(ms.X1)
        As = assemble_A(ms, eta_s)
        B = assemble_B(ms)
        Bbar = B + assemble_B(ms, lnrho, only_C=True)
        f = rhs_buoyancy(ms, T2)
        Q, _, _ = velocity_basis(ms, {1}, {2})
        u, p, _ = solve_stokes(As, Bbar, f, np.zeros(ms.n1), Q, Bt=B.T)
        lam, _, _ = solve_stokes(As, B, u, np.zeros(ms.n1), Q, Bt=Bbar.T)
        grad_log_eta(ms, eta_s, u, lam)
        grad_temperature(ms, lam)
        t_pipe = time.perf_counter() - t1
    ndof_s = 3 * ms.n2 + ms.n1
    return {"value": nu / t_spmv / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"assembled FP64 A of the oracle (scipy CSR SpMV, 1 thread, median of 20) on the "
                       f"{nt}x{nr} shell ({60 * nt * nt * nr} macro-tets) at level {level}: N_u={nu}; "
                       f"{t_spmv * 1e3:.1f} ms per SpMV; mesh + assembly {t_asm:.1f} s"),
            "spmv_ms": t_spmv * 1e3, "assembly_s": t_asm,
            "openmp_spmv_all_host_cores": omp,
            "direct_solve_pipeline": {
                "sample": (f"{solve_nt}x{solve_nr} shell level {solve_level} (N_u={3 * ms.n2}, N_p={ms.n1}): "
                           "mesh, assembly, constrained direct forward and adjoint solves, gradient, FP64, 1 thread"),
                "seconds": t_pipe, "mdof_s": ndof_s / t_pipe / 1e6},
            "host": host_cpu()}


def _rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


ROOF_KERNEL = ROOF_KERNELS[64]


def summarize_profile(d, out, cmd, kernel=ROOF_KERNEL):
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
                if kernel not in r["Kernel_Name"]:
                    continue
                g = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)
                dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                s_, c_ = groups.get(g, (0, 0))
                groups[g] = (s_ + dt, c_ + 1)
        lines += ["", f"{kernel} launches by grid size (work-items):"]
        for g in sorted(groups, reverse=True):
            s_, c_ = groups[g]
            lines.append(f"  grid {g:>10d}: {c_:6d} launches, average {s_ / c_ / 1e3:10.1f} us")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_traffic(dfetch, dwrite, n_u, out, cmd, kernel=ROOF_KERNEL):
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
        cands = [(k[1], sum(v) / len(v)) for k, v in acc.items() if kernel in k[0]]
        return max(cands)[1]
    fb, wb = roof(f) * 1024.0 * kf, roof(w) * 1024.0 * kw
    lines = ["# HBM traffic of the roofline kernel (finest level, largest grid)",
             f"# fetch command: {cmd[0]}", f"# write command: {cmd[1]}",
             f"kernel: {kernel}",
             f"kernel_source_sha256_16: {kernel_sha()}",
             f"copy_bytes_known: {known:.0f}",
             f"fetch_scale: {kf:.4f}", f"write_scale: {kw:.4f}",
             f"fetch_bytes_per_launch: {fb:.0f}", f"write_bytes_per_launch: {wb:.0f}",
             f"hbm_bytes_per_launch: {fb + wb:.0f}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_flops(d, n_tets, out, cmd):
    """Executed VALU flops per micro-tet of the two finest-level sweep kernels
    (the largest grid of each) from a rocprofv3 --pmc SQ_INSTS_VALU_FLOPS_FP64
    SQ_INSTS_VALU_FLOPS_FP32 run, next to the algorithmic count, with the hash
    of the sweep source they were taken on."""
    acc = {}
    for r in _rows(os.path.join(d, "run_counter_collection.csv")):
        key = (r["Kernel_Name"], int(r["Grid_Size"]), r["Counter_Name"])
        acc.setdefault(key, []).append(float(r["Counter_Value"]))
    lines = ["# VALU flops of the A-apply sweep kernels (finest level, largest grid)", f"# command: {cmd}",
             f"kernel_source_sha256_16: {kernel_sha()}", f"micro_tets: {n_tets}",
             f"algorithmic_flops_per_micro_tet: {A_FLOPS_PER_TET}"]
    for prec, counter in ((64, "SQ_INSTS_VALU_FLOPS_FP64"), (32, "SQ_INSTS_VALU_FLOPS_FP32")):
        name = ROOF_KERNELS[prec]
        cands = [(g, sum(v) / len(v)) for (k, g, c), v in acc.items() if name in k and c == counter]
        if not cands:
            lines.append(f"executed_flops_per_micro_tet_fp{prec}: n/a")
            continue
        g, val = max(cands)
        lines.append(f"executed_flops_per_micro_tet_fp{prec}: {val / n_tets:.1f}  ({counter}, grid {g})")
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


def _roofline(prec, n_tets, nu, np_, ms_kernel, traffic):
    """Roofline position of the A-apply sweep kernel from its average event
    time: algorithmic flops (A_FLOPS_PER_TET per micro-tet) against the VALU
    peak of its precision, and algorithmic bytes (x, y and eta once) against
    HBM."""
    peak = PEAK_FP64_TFLOPS if prec == 64 else PEAK_FP32_TFLOPS
    wb = 8 if prec == 64 else 4
    fpt, verified = read_flops()
    flops = fpt * n_tets
    achieved = flops / (ms_kernel * 1e-3) / 1e12
    algo_bytes = (2 * nu + np_) * wb
    r = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
         "traffic": traffic,
         "kernel": f"{ROOF_KERNELS[prec]} (A-apply plane sweep, finest level)",
         "ms_per_launch": ms_kernel, "flops_per_launch": flops, "flops_per_micro_tet": fpt,
         "flops_checked_on_current_source": verified,
         "hbm_gbs_algorithmic": algo_bytes / (ms_kernel * 1e-3) / 1e9,
         "hbm_frac_algorithmic": algo_bytes / (ms_kernel * 1e-3) / 1e9 / PEAK_HBM_GBS,
         "algorithmic_bytes_per_launch": algo_bytes}
    if prec == 32:
        r["frac_of_nonpacked_fp32_peak"] = achieved / PEAK_FP32_NONPACKED_TFLOPS
    if traffic:
        r["traffic_over_algorithmic"] = traffic / algo_bytes
    return r


def main():
    t_begin = time.perf_counter()
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        # bench.py --summarize-counters DIR OUT "COMMAND" KERNEL_SUBSTRING
        summarize_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-flops":
        # bench.py --summarize-flops DIR MICRO_TETS OUT "COMMAND"
        summarize_flops(sys.argv[2], int(sys.argv[3]), sys.argv[4], sys.argv[5])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-profile":
        # bench.py --summarize-profile DIR OUT "COMMAND" [KERNEL]
        summarize_profile(sys.argv[2], sys.argv[3], sys.argv[4], *sys.argv[5:6])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-traffic":
        # bench.py --summarize-traffic FETCH_DIR WRITE_DIR N_U OUT "FETCH_CMD" "WRITE_CMD" [KERNEL]
        summarize_traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], (sys.argv[6], sys.argv[7]),
                          *sys.argv[8:9])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--level", type=int, default=4)
    ap.add_argument("--n-tan", type=int, default=10)
    ap.add_argument("--n-rad", type=int, default=2)
    ap.add_argument("--budget", type=float, default=float(os.environ.get("STK_BENCH_BUDGET_S", 420)),
                    help="wall seconds from the start after which no further once-only leg is started")
    ap.add_argument("--no-solves", action="store_true", help="skip the solve legs")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--apply-only", action="store_true",
                    help="only the A-apply timings (for counter collection)")
    ap.add_argument("--transfer-only", action="store_true",
                    help="only the finest-level FP32 restriction and prolongation (for counter collection)")
    ap.add_argument("--contrast-study", action="store_true",
                    help="only the high-contrast study: viscosity contrast 1e6 (depth factor, temperature, a "
                         "seeded slab), mixed and all-FP64 solves to 1e-8 on the shell and level given")
    ap.add_argument("--large-apply", action="store_true",
                    help="only the A-apply throughput (FP64 and FP32) with the device memory in use; "
                         "use with --n-tan 20 --n-rad 4 for the largest shell")
    ap.add_argument("--schur-study", action="store_true",
                    help="only the comparison of block preconditioners and Schur approximations (Sec. 7.4 "
                         "setting): every Uzawa variant with the V-cycle BFBT, mass, and symmetric and "
                         "asymmetric weighted BFBT, stopped at an absolute residual of 1e-8; use with "
                         "--n-tan 2 --n-rad 1")
    ap.add_argument("--temp-study", action="store_true",
                    help="only the temperature step (Sec. 3 splitting, eq. WeakTemp) on the shell and level "
                         "given: MMOC, right-hand side and FGMRES solve timings, kernel times")
    ap.add_argument("--time-loop-study", action="store_true",
                    help="only the coupled time loop: STEPS steps of temperature then Stokes (from the previous "
                         "solution, absolute tolerance 1e-5) with the viscosity model, per-step times")
    ap.add_argument("--loop-steps", type=int, default=5)
    ap.add_argument("--l-eta-study", action="store_true",
                    help="only the coarse-viscosity study: A-block CG iterations and time of 10 FGMRES "
                         "iterations with the viscosity model of eq. ViscosityDef for l_eta = -1, 0, 1")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)
    if (args.apply_only or args.transfer_only or args.l_eta_study or args.contrast_study or args.large_apply
            or args.schur_study or args.temp_study or args.time_loop_study):
        return studies(args)

    n_tets = 60 * args.n_tan ** 2 * args.n_rad * 8 ** args.level
    workload = (f"blended spherical shell [0.55,1], icosahedral {args.n_tan}x{args.n_rad} macro mesh "
                f"({60 * args.n_tan ** 2 * args.n_rad} macro-tets), level {args.level}, P2-P1; viscosity "
                "contrast 1e4 from a seeded SH temperature, rho=exp(0.5(1-r)), no-slip inner / free-slip outer")
    line = {
        "metric": METRIC, "value": None, "unit": "GDoF/s",
        "value_definition": "N_u / seconds per step; step = one finest-level FP64 A-apply y = P A P x "
                            "(plane sweep + shared-node gather + projection), input resident in HBM",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "N_u": None, "N_p": None, "micro_tets": n_tets,
                   "parallelism": "single GPU"},
        "roofline": None, "cpu_baseline": None, "skipped": [], "errors": [],
    }
    printed = []

    def emit(*_):
        if printed:
            return
        printed.append(True)
        line["wall_s"] = time.perf_counter() - t_begin
        print(json.dumps(line), flush=True)

    def on_term(signum, frame):
        line["errors"].append(f"terminated by signal {signum}")
        emit()
        os._exit(128 + signum)

    signal.signal(signal.SIGTERM, on_term)

    def fits(name, seconds):
        left = args.budget - (time.perf_counter() - t_begin)
        if seconds > left:
            line["skipped"].append({"leg": name, "estimated_s": seconds, "budget_left_s": round(left, 1)})
            log(f"skip {name}: needs ~{seconds:.0f} s, {left:.0f} s left of the budget")
            return False
        return True

    try:
        run_bench(args, line, fits, n_tets)
    except Exception as e:   # a late leg must not erase what was measured
        import traceback
        traceback.print_exc()
        line["errors"].append(f"{type(e).__name__}: {e}")
    finally:
        emit()


def run_bench(args, line, fits, n_tets):
    import numpy as np
    import torch

    import inputs
    from paper_2506_04157_amd import StokesContext, default_params

    os.environ.setdefault("STK_VERBOSE", "1")   # solver progress lines on stderr
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    with StokesContext("shell", level=args.level, min_level=0, n_tan=args.n_tan, n_rad=args.n_rad,
                       device=dev) as sc:
        n2, n1 = sc.sizes()
        Nu, Np = 3 * n2, n1
        line["config"]["N_u"], line["config"]["N_p"] = Nu, Np
        line["setup_s"] = {"context": time.perf_counter() - t0}
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
        s = time.perf_counter()
        sc.set_log_viscosity(mlog, lnrho, mixed)
        torch.cuda.synchronize()
        line["setup_s"]["fields"] = time.perf_counter() - s

        # ---- timed steps: one finest-level FP64 A-apply each ---------------------
        x = torch.tensor(inputs.uniform(0, Nu), device=dev)
        y = torch.empty_like(x)
        for i in range(args.warmup):
            sc.apply_A(x, out=y, bc=3)
        torch.cuda.synchronize()
        log(f"warmup {args.warmup} applies done; timing {args.steps}")
        sc.kernel_timer(True)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for i in range(args.steps):
            sc.apply_A(x, out=y, bc=3)
        torch.cuda.synchronize()
        te = time.perf_counter()
        ms_k, nk = sc.kernel_timer(False)
        ms_step = (te - ts) / args.steps * 1e3
        line["ms_per_step"] = ms_step
        line["value"] = Nu / (ms_step * 1e-3) / 1e9
        line["step_timing"] = {"host_clock_ms_per_step": ms_step, "sweep_kernel_ms_per_launch": ms_k / max(nk, 1),
                               "sweep_kernel_launches_timed": nk,
                               "sweep_share_of_step": (ms_k / max(nk, 1)) / ms_step}
        line["roofline"] = _roofline(64, n_tets, Nu, Np, ms_k / max(nk, 1),
                                     read_traffic(64) if (args.level, args.n_tan, args.n_rad) == (4, 10, 2) else None)
        log(f"FP64 A-apply: {ms_step:.3f} ms/step ({line['value']:.1f} GDoF/s), sweep kernel "
            f"{ms_k / max(nk, 1):.3f} ms ({line['roofline']['frac'] * 100:.1f} % of FP64 peak)")
        ynorm = torch.linalg.norm(y).item()
        line["step_output_finite"] = bool(np.isfinite(ynorm))
        del x, y

        # ---- FP32 A-apply --------------------------------------------------------------
        x32 = torch.tensor(inputs.uniform(0, Nu), dtype=torch.float32, device=dev)
        y32 = torch.empty_like(x32)
        sc.time_apply_A(x32, y32, reps=2)
        ms32, mk32 = sc.time_apply_A(x32, y32, reps=20)
        line["a_apply_fp32"] = {"gdof_s": Nu / (ms32 * 1e-3) / 1e9, "ms_per_apply": ms32, "ms_sweep_kernel": mk32,
                                "roofline": _roofline(32, n_tets, Nu, Np, mk32,
                                                      read_traffic(32) if (args.level, args.n_tan, args.n_rad)
                                                      == (4, 10, 2) else None)}
        log(f"FP32 A-apply: {ms32:.3f} ms ({Nu / ms32 / 1e6:.1f} GDoF/s), sweep kernel {mk32:.3f} ms")
        del x32, y32

        # ---- CPU oracle -------------------------------------------------------------------
        if not args.no_cpu and fits("cpu_baseline", 60):
            log("CPU oracle baseline")
            cpu = cpu_baseline()
            line["cpu_baseline"] = {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")}
            line["cpu_baseline_detail"] = {k: cpu[k] for k in ("spmv_ms", "assembly_s", "direct_solve_pipeline",
                                                               "openmp_spmv_all_host_cores", "host")}
            log(f"oracle: {cpu['sample']}")

        if args.no_solves:
            return
        # ---- solves -----------------------------------------------------------------------------
        f = sc.rhs_buoyancy(T2)
        solves = {}
        line["solves"] = solves
        u = p = None
        if fits("mixed_forward_solve", 90):
            log("mixed-precision forward solve")
            u, p, rep = sc.solve(f, params=mixed)
            torch.cuda.synchronize()
            solves["mixed"] = _rep(rep)
            log(f"mixed solve {rep['seconds']:.2f}s ({rep['iterations']} its, rel {rep['rel_residual']:.2e})")
        if not args.no_fp64 and fits("fp64_forward_solve", 130):
            log("all-FP64 forward solve")
            u64, p64, r64 = sc.solve(f, params=full)
            torch.cuda.synchronize()
            solves["fp64"] = _rep(r64)
            log(f"FP64 solve {r64['seconds']:.2f}s ({r64['iterations']} its)")
            if u is not None:
                du = (torch.linalg.norm(u - u64) / torch.linalg.norm(u64)).item()
                dp = (torch.linalg.norm(p - p64) / torch.linalg.norm(p64)).item()
                solves["mixed_vs_fp64"] = {
                    "speedup": r64["seconds"] / solves["mixed"]["seconds"],
                    "u_rel_diff": du, "p_rel_diff": dp}
                log(f"mixed vs FP64: speed-up {solves['mixed_vs_fp64']['speedup']:.2f}, |du| {du:.2e}, |dp| {dp:.2e}")
            del u64, p64
        if u is not None and fits("adjoint_solve_and_gradient", 90):
            log("mixed adjoint solve + gradient")
            lu, lp, ra = sc.solve_adjoint(u, None, mixed)
            torch.cuda.synchronize()
            s = time.perf_counter()
            gm, gT = sc.gradient(u, lu)
            torch.cuda.synchronize()
            solves["adjoint"] = _rep(ra)
            solves["adjoint"]["gradient_s"] = time.perf_counter() - s
            solves["adjoint"]["gradient_finite"] = bool(torch.isfinite(gm).all().item()
                                                        and torch.isfinite(gT).all().item())
            log(f"adjoint {ra['seconds']:.2f}s ({ra['iterations']} its)")
        if u is not None and fits("temperature_step", 30):
            # the splitting's temperature step driven by the solved velocity
            # (Sec. 3): two steps from T^n = T^{n-1} = T, u^n = u^{n-1} = u, with
            # the paper's Ra, Pe, Di and a step of a third of a micro-tet's
            # radial height over max |u|; the second is reported
            from paper_2506_04157_amd import temp_params
            umax = float(u.abs().max().item())
            tau = (1.0 / 3.0) * (0.45 / args.n_rad / 2 ** args.level) / max(umax, 1e-30)
            prm = temp_params(tau1=tau, tau0=tau, k=1.0, Pe=2.822e4, Cp=1.0, Di=0.4538, alpha=1.0, H=1.0,
                              Ra=1.692e7, T_in=4200.0 / 3900.0, T_out=300.0 / 3900.0, tol_abs=1e-10)
            eta1 = torch.exp(mlog).contiguous()
            T_prev, T_cur = T2, T2
            reps = []
            for _ in range(2):
                T_new, rt = sc.temperature_step(T_cur, T_prev, u, u, eta1, prm, lnrho=lnrho)
                torch.cuda.synchronize()
                reps.append(rt)
                T_prev, T_cur = T_cur, T_new
            rt = reps[-1]
            line["temperature_step"] = {
                "workload": f"P2 temperature nodes {Nu // 3}, the velocity of the mixed forward solve, tau {tau:.3e}",
                "ms_mmoc": rt["ms_mmoc"], "ms_rhs": rt["ms_rhs"], "ms_solve": rt["ms_solve"],
                "fgmres_iterations": rt["iterations"], "cg_iterations": rt["cg_its"],
                "abs_residual": rt["abs_residual"], "stored_S": rt["stored_S"],
                "T_finite": bool(torch.isfinite(T_cur).all().item())}
            log(f"temperature step: mmoc {rt['ms_mmoc']:.1f} ms, rhs {rt['ms_rhs']:.1f} ms, solve "
                f"{rt['ms_solve']:.1f} ms ({rt['iterations']} FGMRES its, {rt['cg_its']} CG its)")


def _rep(rep):
    keys = ("seconds", "iterations", "rel_residual", "a_solves", "a_cg_its", "s_solves", "s_cg_its", "vcycles",
            "coarse_its", "mass_its")
    return {k: rep[k] for k in keys}


def studies(args):
    """Single-purpose runs for counter collection and the coarse-viscosity study."""
    import numpy as np
    import torch

    import inputs
    from paper_2506_04157_amd import StokesContext, default_params

    os.environ.setdefault("STK_VERBOSE", "1")
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    free_before = torch.cuda.mem_get_info(dev)
    with StokesContext("shell", level=args.level, min_level=0, n_tan=args.n_tan, n_rad=args.n_rad,
                       device=dev) as sc:
        n2, n1 = sc.sizes()
        Nu, Np = 3 * n2, n1
        log(f"context {time.perf_counter() - t0:.1f}s  N_u={Nu} N_p={Np}")
        if args.large_apply:
            return large_apply(args, sc, dev, Nu, Np, free_before, time.perf_counter() - t0)
        if args.contrast_study:
            return contrast_study(args, sc, dev, Nu, Np)
        if args.schur_study:
            return schur_study(args, sc, dev, Nu, Np)
        if args.temp_study:
            return temp_study(args, sc, dev, Nu, Np)
        if args.time_loop_study:
            return time_loop_study(args, sc, dev, Nu, Np)
        X2 = torch.tensor(sc.coords(which=2)[0], device=dev)
        X1 = torch.tensor(sc.coords(which=1)[0], device=dev)
        field = inputs.SHField(2)
        T2 = field.temperature_torch(X2).contiguous()
        T1 = field.temperature_torch(X1)
        mlog = (float(np.log(1e4)) * (0.5 - T1)).contiguous()
        lnrho = (0.5 * (1.0 - torch.linalg.norm(X1, dim=1))).contiguous()
        del X2, X1, T1
        mixed = default_params(precision=32, tol_rel=1e-8)

        if args.apply_only:
            # A-apply timings, preceded by plain device copies of known size that
            # calibrate the HBM byte counters (FETCH_SIZE / WRITE_SIZE)
            sc.set_log_viscosity(mlog, lnrho, mixed)
            a = torch.ones(Nu, dtype=torch.float32, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            log(f"copy calibration: 3 copies of {4 * Nu} bytes")
            del a, b
            out = {}
            for dt_, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
                x = torch.tensor(inputs.uniform(0, Nu), dtype=dt_, device=dev)
                y = torch.empty_like(x)
                sc.time_apply_A(x, y, reps=2)
                ms, mk = sc.time_apply_A(x, y, reps=20)
                out[name] = {"gdof_s": Nu / ms / 1e6, "ms_per_apply": ms, "ms_sweep_kernel": mk}
                log(f"A-apply {name}: {ms:.3f} ms/apply ({Nu / ms / 1e6:.1f} GDoF/s), sweep kernel {mk:.3f} ms")
                del x, y
            print(json.dumps(out), flush=True)
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


def large_apply(args, sc, dev, Nu, Np, free_before, t_ctx):
    """A-apply throughput on a large shell in both precisions, with the device
    memory the context and the vectors occupy (hipMemGetInfo through torch)."""
    import torch

    import inputs
    n_tets = 60 * args.n_tan ** 2 * args.n_rad * 8 ** args.level
    X1 = sc.coords(which=1)[0]
    T1 = inputs.SHField(2).temperature_torch(torch.tensor(X1, device=dev)).cpu().numpy()
    eta = torch.tensor(inputs.viscosity_1e6(X1, T1), device=dev)
    del X1, T1
    log("viscosity set up")
    sc.set_fields(eta)
    del eta
    out = {"workload": f"shell {args.n_tan}x{args.n_rad} ({60 * args.n_tan ** 2 * args.n_rad} macro-tets), "
                       f"level {args.level}, viscosity contrast 1e6", "N_u": Nu, "N_p": Np, "micro_tets": n_tets,
           "context_s": t_ctx}
    for dt_, name in ((torch.float64, "fp64"), (torch.float32, "fp32")):
        # a seeded vector drawn on the device (the host draw of 1.6e9 values is slow)
        g = torch.Generator(device=dev)
        g.manual_seed(0)
        x = (2.0 * torch.rand(Nu, dtype=torch.float64, device=dev, generator=g) - 1.0).to(dt_)
        y = torch.empty_like(x)
        sc.time_apply_A(x, y, reps=2)
        free, total = torch.cuda.mem_get_info(dev)
        ms, mk = sc.time_apply_A(x, y, reps=10)
        prec = 64 if name == "fp64" else 32
        out[name] = {"gdof_s": Nu / ms / 1e6, "ms_per_apply": ms, "ms_sweep_kernel": mk,
                     "roofline": _roofline(prec, n_tets, Nu, Np, mk, None),
                     "device_bytes_in_use": total - free, "device_bytes_total": total,
                     "in_use_before_context": free_before[1] - free_before[0]}
        log(f"{name}: {ms:.2f} ms per apply ({Nu / ms / 1e6:.1f} GDoF/s), sweep {mk:.2f} ms; "
            f"{(total - free) / 2**30:.1f} GiB of {total / 2**30:.1f} in use")
        del x, y
    print(json.dumps({"large_apply": out}), flush=True)


def contrast_study(args, sc, dev, Nu, Np):
    """Mixed-precision against all-FP64 solves to 1e-8 at viscosity contrast
    1e6 (Sec. 5.2.2: FP64 Chebyshev bounds, FP32 smoothing)."""
    import torch

    import inputs
    from paper_2506_04157_amd import default_params
    field = inputs.SHField(2)
    X1 = sc.coords(which=1)[0]
    T1 = field.temperature_torch(torch.tensor(X1, device=dev)).cpu().numpy()
    log("P1 temperature evaluated")
    eta1 = inputs.viscosity_1e6(X1, T1)
    log(f"viscosity: contrast {eta1.max() / eta1.min():.3e}")
    lnrho = torch.tensor(inputs.ln_density(X1), device=dev)
    del X1, T1
    T2 = field.temperature_torch(torch.tensor(sc.coords(which=2)[0], device=dev)).contiguous()
    log("P2 temperature evaluated")
    out = {"workload": f"shell {args.n_tan}x{args.n_rad} level {args.level}, N_u={Nu}, N_p={Np}",
           "eta_max_over_min": float(eta1.max() / eta1.min()), "eta_min": float(eta1.min()),
           "eta_max": float(eta1.max())}
    eta = torch.tensor(eta1, device=dev)
    del eta1
    res = {}
    for prec in (32, 64):
        prm = default_params(precision=prec, tol_rel=1e-8, max_outer=200)
        sc.set_fields(eta, lnrho, prm)
        f = sc.rhs_buoyancy(T2)
        u, p, rep = sc.solve(f, params=prm, allow_noconv=True)
        torch.cuda.synchronize()
        res[prec] = (u, p)
        out["fp64" if prec == 64 else "mixed"] = {k: rep[k] for k in (
            "seconds", "iterations", "rel_residual", "a_cg_its", "s_cg_its", "vcycles", "coarse_its", "mass_its")}
        log(f"prec {prec}: {rep['iterations']} its, rel {rep['rel_residual']:.2e}, {rep['seconds']:.1f}s")
    (u32, p32), (u64, p64) = res[32], res[64]
    out["mixed_vs_fp64"] = {"speedup": out["fp64"]["seconds"] / out["mixed"]["seconds"],
                            "u_rel_diff": (torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64)).item(),
                            "p_rel_diff": (torch.linalg.norm(p32 - p64) / torch.linalg.norm(p64)).item()}
    print(json.dumps({"contrast_study": out}), flush=True)


def temp_study(args, sc, dev, Nu, Np):
    """The temperature step at the given size with the paper's nondimensional
    numbers (Ra = 1.692e7, Pe = 2.822e4, Di = 0.4538, alpha = k = Cp = H = 1,
    T_in = 4200/3900, T_out = 300/3900, tol_T = 1e-10): a seeded SH
    temperature, a smooth seeded velocity of magnitude about 1, viscosity
    contrast 1e4 at the temperature, rho = exp(0.5 (1 - r)), tau = 2e-3
    (displacements of about a sixth of a micro-tet).  Three steps (the first
    builds the point locator), then single launches of the MMOC and of the
    operator timed with HIP events on the library's stream."""
    import numpy as np
    import torch

    import inputs
    from paper_2506_04157_amd import temp_params
    n2 = Nu // 3
    field = inputs.SHField(2)
    X2 = torch.tensor(sc.coords(which=2)[0], device=dev)
    T2 = field.temperature_torch(X2).contiguous()
    u_n = inputs.smooth_vector_field_torch(11, X2).contiguous()
    u_nm1 = (0.9 * u_n).contiguous()
    del X2
    X1 = torch.tensor(sc.coords(which=1)[0], device=dev)
    eta = torch.exp(float(np.log(1e4)) * (0.5 - field.temperature_torch(X1))).contiguous()
    lnrho = (0.5 * (1.0 - torch.linalg.norm(X1, dim=1))).contiguous()
    del X1
    log("temperature inputs ready")
    prm = temp_params(tau1=2e-3, tau0=2e-3, k=1.0, Pe=2.822e4, Cp=1.0, Di=0.4538, alpha=1.0, H=1.0, Ra=1.692e7,
                      T_in=4200.0 / 3900.0, T_out=300.0 / 3900.0, tol_abs=1e-10)
    T_nm1 = T2.clone()
    T_n = T2
    steps, steps_mf = [], []
    for it in range(4):
        # the last step with the matrix-free S in the preconditioner's CG
        prm.stored_S = 1 if it < 3 else 0
        T_np1, rep = sc.temperature_step(T_n, T_nm1, u_n, u_nm1, eta, prm, lnrho=lnrho)
        torch.cuda.synchronize()
        (steps if it < 3 else steps_mf).append(rep)
        log(f"step {it}: mmoc {rep['ms_mmoc']:.1f} ms, rhs {rep['ms_rhs']:.1f} ms, solve {rep['ms_solve']:.1f} ms, "
            f"{rep['iterations']} FGMRES its, {rep['cg_its']} CG its, residual {rep['abs_residual']:.2e}, "
            f"stored S {rep['stored_S']}")
        T_nm1, T_n = T_n, T_np1
    prm.stored_S = 1
    st = torch.cuda.current_stream(dev)

    def timed(fn, reps=5):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    out_buf = torch.empty_like(T2)
    ms_mmoc = timed(lambda: sc.mmoc(T_n, u_n, u_nm1, 2e-3, out=out_buf))
    ms_apply = timed(lambda: sc.temp_apply(T_n, prm, 0, u_star=u_n, lnrho=lnrho, out=out_buf))
    ms_sym = timed(lambda: sc.temp_apply(T_n, prm, 1, lnrho=lnrho, out=out_buf))
    n_tets = 60 * args.n_tan ** 2 * args.n_rad * 8 ** args.level
    last = steps[-1]
    out = {"workload": f"shell {args.n_tan}x{args.n_rad} level {args.level}, temperature nodes {n2}, "
                       f"micro-tets {n_tets}",
           "params": {k: getattr(prm, k) for k, _ in prm._fields_},
           "steps": steps, "step_matrix_free_S": steps_mf,
           "solve_ms_per_cg_iteration": steps[-1]["ms_solve"] / max(steps[-1]["cg_its"], 1),
           "solve_ms_per_cg_iteration_matrix_free": steps_mf[-1]["ms_solve"] / max(steps_mf[-1]["cg_its"], 1),
           "mmoc_launch_ms": ms_mmoc, "mmoc_gnodes_per_s": n2 / ms_mmoc * 1e-6,
           "apply_L_ms": ms_apply, "apply_L_gdof_per_s": n2 / ms_apply * 1e-6,
           "apply_S_ms": ms_sym, "apply_S_gdof_per_s": n2 / ms_sym * 1e-6,
           "step_ms": last["ms_mmoc"] + last["ms_rhs"] + last["ms_solve"],
           "mmoc_share": last["ms_mmoc"] / (last["ms_mmoc"] + last["ms_rhs"] + last["ms_solve"])}
    print(json.dumps({"temp_study": out}), flush=True)


def time_loop_study(args, sc, dev, Nu, Np):
    """The coupled time loop of Sec. 3 and Sec. 6 at the given size: an initial
    Stokes solve from zero, then --loop-steps coupled steps (temperature step
    with the viscosity at the extrapolated temperature, then the Stokes solve
    started from the previous solution to the absolute tolerance
    tol_(u,p) = 1e-5 of table parametertable).  The viscosity model of eq.
    ViscosityDef with the paper's E_A, V_A and the synthetic base profile; the
    paper's Ra, Pe, Di; buoyancy scale Ra/Pe = 600; the initial temperature
    linear in r between the Dirichlet values plus a seeded SH perturbation of
    amplitude 0.1 that vanishes on both spheres; rho = exp(0.5 (1 - r)); a
    step of a third of a micro-tet's radial height over max |u|.  Per-step
    times of the MMOC, the temperature solve and the Stokes solve, and their
    shares."""
    import numpy as np
    import torch

    import inputs
    from paper_2506_04157_amd import default_params, temp_params
    field = inputs.SHField(2)
    X2 = torch.tensor(sc.coords(which=2)[0], device=dev)
    T_in, T_out = 4200.0 / 3900.0, 300.0 / 3900.0
    s_ = (torch.linalg.norm(X2, dim=1) - 0.55) / 0.45
    T0 = (T_in + (T_out - T_in) * s_ + 0.1 * (field.temperature_torch(X2) - 0.5) * torch.sin(np.pi * s_))
    T0 = T0.contiguous()
    del X2, s_
    X1 = torch.tensor(sc.coords(which=1)[0], device=dev)
    lnrho = (0.5 * (1.0 - torch.linalg.norm(X1, dim=1))).contiguous()
    del X1
    base = inputs.base_viscosity_profile()
    E_A, V_A, scale = 4.610, 2.996, 1.692e7 / 2.822e4
    cold = default_params(precision=32, tol_rel=1e-30, tol_abs=1e-5, max_outer=200)
    warm = default_params(precision=32, tol_rel=1e-30, tol_abs=1e-5, max_outer=200, initial_guess=1)
    sc.set_temperature_viscosity(T0, base, E_A, V_A, lnrho=lnrho, params=cold)
    u, p, rep0 = sc.solve(sc.rhs_buoyancy(T0, scale=scale), params=cold, allow_noconv=True)
    torch.cuda.synchronize()
    log(f"initial solve: {rep0['iterations']} its, abs {rep0['abs_residual']:.2e}, {rep0['seconds']:.1f} s")
    umax = float(u.abs().max().item())
    tau = (1.0 / 3.0) * (0.45 / args.n_rad / 2 ** args.level) / max(umax, 1e-30)
    tp = temp_params(tau1=tau, tau0=tau, k=1.0, Pe=2.822e4, Cp=1.0, Di=0.4538, alpha=1.0, H=1.0, Ra=1.692e7,
                     T_in=T_in, T_out=T_out, tol_abs=1e-10)
    T_prev, T_cur, u_prev, u_cur, p_cur = T0, T0, u, u, p
    steps = []
    for it in range(args.loop_steps):
        t0 = time.perf_counter()
        T_new, u_new, p_new, trep, srep = sc.coupled_step(T_cur, T_prev, u_cur, u_prev, base, tp, params=warm,
                                                          E_A=E_A, V_A=V_A, buoyancy_scale=scale, lnrho=lnrho,
                                                          p_n=p_cur, allow_noconv=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = {"wall_s": wall, "temperature": {k: trep[k] for k in ("ms_mmoc", "ms_rhs", "ms_solve", "iterations",
                                                                   "cg_its")},
              "stokes": {k: srep[k] for k in ("iterations", "seconds", "initial_residual", "abs_residual",
                                              "a_cg_its", "s_cg_its")}}
        steps.append(st)
        log(f"step {it}: {wall:.1f} s; temperature mmoc {trep['ms_mmoc']:.0f} ms, solve {trep['ms_solve']:.0f} ms "
            f"({trep['iterations']} its); Stokes {srep['iterations']} its from {srep['initial_residual']:.2e} "
            f"to {srep['abs_residual']:.2e}, {srep['seconds']:.1f} s")
        T_prev, T_cur, u_prev, u_cur, p_cur = T_cur, T_new, u_cur, u_new, p_new
    tot = sum(s_["wall_s"] for s_ in steps)
    t_mmoc = sum(s_["temperature"]["ms_mmoc"] for s_ in steps) * 1e-3
    t_temp = sum(s_["temperature"]["ms_rhs"] + s_["temperature"]["ms_solve"] for s_ in steps) * 1e-3
    t_stokes = sum(s_["stokes"]["seconds"] for s_ in steps)
    out = {"workload": f"shell {args.n_tan}x{args.n_rad} level {args.level}, N_u={Nu}, N_p={Np}, "
                       f"temperature nodes {Nu // 3}",
           "tau": tau, "initial_solve": {k: rep0[k] for k in ("iterations", "seconds", "abs_residual")},
           "steps": steps, "total_step_s": tot,
           "shares": {"stokes": t_stokes / tot, "mmoc": t_mmoc / tot, "temperature_solve": t_temp / tot}}
    print(json.dumps({"time_loop_study": out}), flush=True)


def schur_study(args, sc, dev, Nu, Np):
    """Block preconditioners x Schur approximations on one synthetic shell
    problem (the comparison of Sec. 7.4, Fig. SchurCompInit): FGMRES stopped at
    an absolute residual of 1e-8, A-block tolerance 1e-2 for the symmetric
    Uzawa and 1e-4 for the inexact and adjoint ones, Uzawa omega 0.0125 for
    the weighted BFBT (the paper's best value in that test), a_r = 10, a_l = 1
    for its asymmetric scaling; FP32 preconditioner inside FP64 FGMRES."""
    import numpy as np
    import torch

    import inputs
    from paper_2506_04157_amd import default_params
    from paper_2506_04157_amd._lib import (SCHUR_MASS, SCHUR_VBFBT, SCHUR_WBFBT, UZAWA_ADJOINT, UZAWA_INEXACT,
                                           UZAWA_SYMMETRIC)
    field = inputs.SHField(2)
    X1 = torch.tensor(sc.coords(which=1)[0], device=dev)
    X2 = torch.tensor(sc.coords(which=2)[0], device=dev)
    mlog = (float(np.log(1e4)) * (0.5 - field.temperature_torch(X1))).contiguous()
    lnrho = (0.5 * (1.0 - torch.linalg.norm(X1, dim=1))).contiguous()
    T2 = field.temperature_torch(X2).contiguous()
    del X1, X2
    schurs = [("vbfbt", dict(schur=SCHUR_VBFBT)), ("mass", dict(schur=SCHUR_MASS)),
              ("wbfbt", dict(schur=SCHUR_WBFBT, omega=0.0125)),
              ("wbfbt_asym", dict(schur=SCHUR_WBFBT, omega=0.0125, a_r=10.0, a_l=1.0))]
    uzawas = [("symmetric", dict(uzawa=UZAWA_SYMMETRIC, tol_A=1e-2)),
              ("inexact", dict(uzawa=UZAWA_INEXACT, tol_A=1e-4)),
              ("adjoint", dict(uzawa=UZAWA_ADJOINT, tol_A=1e-4))]
    out = {"workload": f"shell {args.n_tan}x{args.n_rad} level {args.level}, N_u={Nu}, N_p={Np}, contrast 1e4",
           "stop": "absolute residual 1e-8 or 100 FGMRES iterations", "runs": {}}
    t0 = time.perf_counter()
    f = None
    for sname, skw in schurs:
        for uname, ukw in uzawas:
            kw = dict(precision=32, tol_rel=1e-30, tol_abs=1e-8, max_outer=100)
            kw.update(skw)
            kw.update(ukw)
            prm = default_params(**kw)
            sc.set_log_viscosity(mlog, lnrho, prm)
            if f is None:
                f = sc.rhs_buoyancy(T2)
            u, p, rep = sc.solve(f, params=prm, allow_noconv=True)
            torch.cuda.synchronize()
            key = f"{uname}+{sname}"
            out["runs"][key] = {k: rep[k] for k in ("iterations", "rel_residual", "abs_residual", "seconds",
                                                    "a_cg_its", "s_cg_its", "mass_its")}
            out["runs"][key]["history"] = rep["history"]
            log(f"{key}: {rep['iterations']} its, abs {rep['abs_residual']:.2e}, {rep['seconds']:.1f}s")
            if time.perf_counter() - t0 > args.budget:
                out["stopped_early"] = True
                print(json.dumps({"schur_study": out}), flush=True)
                return
    print(json.dumps({"schur_study": out}), flush=True)


if __name__ == "__main__":
    main()
