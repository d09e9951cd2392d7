"""Benchmark: eigenpairs/s of the rIGA shift-and-invert eigensolver on one MI355X.

Workload (one step): the 2D unit-square problem with p = 3 B-splines on
256 x 256 elements, rIGA separators every 16 elements (82,369 DOFs),
log-normal(0, 0.3) per-element coefficients already resident in HBM;
the step re-assembles K and M on the device from them and computes the 200
lowest eigenpairs (shift-and-invert Lanczos over spectrum slices, every
pair checked against residual <= 1e-9).  value = 200 * steps / wall time.

Also reported: the same step for maximum-continuity IGA on the same mesh
(66,049 DOFs), the roofline of the dominant kernel (measured live with HIP
events on the library's stream), and the CPU oracle timed on a bounded
sample of the same problem.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_steps(pr, kappa_d, rho_d, nev, steps, warmup, precision, torch):
    stats = None
    for _ in range(warmup):
        pr.update_coefficients(kappa_d, rho_d)
        pr.eigs(nev, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam = res = None
    for _ in range(steps):
        pr.update_coefficients(kappa_d, rho_d)
        lam, U, res, stats = pr.eigs(nev, precision=precision)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert len(lam) == nev, "only %d of %d pairs returned" % (len(lam), nev)
    assert float(max(res)) <= 1e-9, "residual %.3e above 1e-9" % max(res)
    return dt, lam, res, stats


def time_solves(pr, sigma, precision, reps, torch):
    """Average duration of one forward/backward elimination and of one
    factorisation, bracketed by events on the stream the library uses."""
    import numpy as np
    pr.factor(sigma, precision)
    b = torch.randn(pr.n_dof, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    pr.solve(b)  # warm
    # the sweeps queued back to back (no host synchronisation between them)
    B = b.unsqueeze(0).repeat(reps, 1).contiguous()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pr.solve_multi(B)
    e1.record(stream)
    torch.cuda.synchronize()
    t_fb = e0.elapsed_time(e1) / 1e3 / reps
    f0 = torch.cuda.Event(enable_timing=True)
    f1 = torch.cuda.Event(enable_timing=True)
    nf = 3
    f0.record(stream)
    for _ in range(nf):
        pr.factor(sigma, precision)
    f1.record(stream)
    torch.cuda.synchronize()
    t_fact = f0.elapsed_time(f1) / 1e3 / nf
    del np
    return t_fb, t_fact


MALL_BYTES = 256 * 1024 * 1024   # Infinity Cache of an MI355X


def event_time(fn, reps, torch):
    """Average duration of fn() queued `reps` times back to back on torch's
    current stream (the stream the library is handed), between two events."""
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def secondary_rooflines(riga, pr, t_fact, info, torch):
    """Event-timed rates of the other kernels of a Lanczos step on the main
    workload: the SpMV with M (CSR: nnz (8 + 4) + 2 N 8 bytes), one
    Gram-Schmidt pass over m = 256 columns (riga_project_noalloc: W and B
    read once, x read twice and written once: 2 N m 8 + 3 N 8 bytes), and the
    factorisation on its exact-fill flops (sum over the columns of L of
    c (c + 1))."""
    N, nnz = pr.n_dof, info["nnz"]
    x = torch.randn(N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    t_mv = event_time(lambda: pr.spmv(riga.RIGA_MAT_M, x, y=y), 50, torch)
    b_mv = nnz * 12.0 + 2.0 * N * 8
    m = 256
    W = torch.randn(m, N, dtype=torch.float64, device="cuda")
    B = torch.randn(m, N, dtype=torch.float64, device="cuda")
    c = torch.empty(m, dtype=torch.float64, device="cuda")
    t_gs = event_time(lambda: riga.project(W, B, x, c=c, noalloc=True), 20, torch)
    b_gs = 2.0 * N * m * 8 + 3.0 * N * 8
    f_ex = info["flops_fact_exact"]
    del W, B
    return {
        "spmv_M": {"bound": "hbm", "achieved": b_mv / t_mv / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": b_mv / t_mv / 1e9 / HBM_PEAK_GBS, "bytes": b_mv, "seconds": t_mv,
                   "mall_fits": b_mv <= MALL_BYTES},
        "gram_schmidt_pass_m256": {"bound": "hbm", "achieved": b_gs / t_gs / 1e9, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": b_gs / t_gs / 1e9 / HBM_PEAK_GBS, "bytes": b_gs,
                                   "seconds": t_gs, "mall_fits": b_gs <= MALL_BYTES},
        "factorisation": {"bound": "mfma", "achieved": f_ex / t_fact / 1e12, "peak": FP64_PEAK_TFLOPS,
                          "unit": "TFLOP/s", "frac": f_ex / t_fact / 1e12 / FP64_PEAK_TFLOPS,
                          "flops_exact": f_ex, "flops_supernodal": info["flops_fact"], "seconds": t_fact},
    }


def timed_eigs(pr, nev, precision, torch, reps=1):
    """Wall time of pr.eigs (after one untimed run) with the results on the
    device and synchronised."""
    pr.eigs(nev, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lam, U, res, st = pr.eigs(nev, precision=precision)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, lam, U, res, st


def secondary_lines(riga, workloads, torch, np):
    """The other workloads the metric is quoted for: 3D rIGA FP64 vs mixed
    precision (and the IGA twin), 64 uneven instances batched, and the
    adjoint gradient with its finite-difference check."""
    out = {}
    # 3D, 32^3, p = 2: rIGA (blocks of 8) FP64 vs FP32 fronts + FP64 refinement
    w3 = workloads.c3(True)
    log("assemble", w3.name)
    pr3 = riga.assemble(w3.dim, w3.ne, w3.p, w3.s)
    t64, l64, _, r64, s64 = timed_eigs(pr3, w3.nev, riga.RIGA_FP64, torch)
    tmx, lmx, _, rmx, smx = timed_eigs(pr3, w3.nev, riga.RIGA_MIXED, torch)
    rel = np.abs(lmx - l64) / l64
    out["3d_riga_fp64_vs_mixed"] = {
        "workload": w3.name, "n_dof": pr3.n_dof, "nev": w3.nev,
        "fp64": {"value": w3.nev / t64, "seconds": t64, "n_fact": s64["n_fact"], "n_fb": s64["n_fb"],
                 "max_residual": float(r64.max())},
        "mixed": {"value": w3.nev / tmx, "seconds": tmx, "n_fact": smx["n_fact"], "n_fb": smx["n_fb"],
                  "n_ir": smx["n_ir"], "max_residual": float(rmx.max())},
        "mixed_speedup": t64 / tmx,
        "max_rel_diff_per_pair": float(rel.max()), "median_rel_diff_per_pair": float(np.median(rel)),
        "flops_fact": pr3.info["flops_fact"], "nnz_l": pr3.info["nnz_l"]}
    log("3d riga: fp64 %.1f/s, mixed %.1f/s, max pair diff %.2e" % (w3.nev / t64, w3.nev / tmx, rel.max()))
    del pr3
    w3i = workloads.c3(False)
    log("assemble", w3i.name)
    pr3i = riga.assemble(w3i.dim, w3i.ne, w3i.p, w3i.s)
    ti, li, _, ri, si = timed_eigs(pr3i, w3i.nev, riga.RIGA_FP64, torch)
    out["3d_iga_fp64"] = {"workload": w3i.name, "n_dof": pr3i.n_dof, "value": w3i.nev / ti,
                          "seconds": ti, "n_fact": si["n_fact"], "n_fb": si["n_fb"],
                          "max_residual": float(ri.max()), "flops_fact": pr3i.info["flops_fact"],
                          "nnz_l": pr3i.info["nnz_l"]}
    out["3d_riga_over_iga_fp64"] = (w3.nev / t64) / (w3i.nev / ti)
    log("3d iga: fp64 %.1f/s" % (w3i.nev / ti))
    del pr3i
    # 64 uneven 2D rIGA instances, 20 pairs each, one stream per worker
    ws = workloads.c4()
    log("assemble %d batch instances" % len(ws))
    probs = []
    for w in ws:
        kap, rh = w.coefficients()
        probs.append(riga.assemble(w.dim, w.ne, w.p, w.s, kap, rh))
    total_dof = sum(p.n_dof for p in probs)
    bat = {"instances": len(ws), "total_dof": total_dof, "nev_each": ws[0].nev}
    for name, prec in (("mixed", riga.RIGA_MIXED), ("fp64", riga.RIGA_FP64)):
        riga.eigs_batched(probs, ws[0].nev, precision=prec, vectors=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = riga.eigs_batched(probs, ws[0].nev, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        npairs = sum(len(r[0]) for r in res)
        bat[name] = {"value": npairs / dt, "seconds": dt, "pairs": npairs,
                     "max_residual": float(max(r[2].max() for r in res))}
        log("batch %s: %.1f eigenpairs/s" % (name, npairs / dt))
    # the 64 first factorisations (sigma = 0) in one batched call against a
    # loop of single factorisations
    fac = {}
    for name, prec in (("fp64", riga.RIGA_FP64), ("mixed", riga.RIGA_MIXED)):
        sig = [0.0] * len(probs)
        riga.factor_batched(probs, sig, precision=prec)
        t0 = time.perf_counter()
        riga.factor_batched(probs, sig, precision=prec)
        tb = time.perf_counter() - t0
        for pr in probs:
            pr.factor(0.0, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pr in probs:
            pr.factor(0.0, precision=prec)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t0
        fac[name] = {"batched_ms": tb * 1e3, "single_loop_ms": tl * 1e3}
        log("batch factorisation %s: %.1f ms batched, %.1f ms one by one" % (name, tb * 1e3, tl * 1e3))
    bat["first_factorisations"] = fac
    out["batched_64_riga"] = bat
    del probs
    # adjoint gradient of sum w_i lambda_i, 20 pairs, with central FD on 50
    # elements x {kappa, rho}
    w5 = workloads.c5()
    kap, rh = w5.coefficients()
    kd = torch.tensor(kap, dtype=torch.float64, device="cuda")
    rd = torch.tensor(rh, dtype=torch.float64, device="cuda")
    pr5 = riga.assemble(w5.dim, w5.ne, w5.p, w5.s, kd, rd)
    wts = w5.extra["weights"]
    te, lam5, U5, r5, _ = timed_eigs(pr5, w5.nev, riga.RIGA_FP64, torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gk, gr = pr5.eig_grad(lam5, U5, wts)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    gk, gr = gk.cpu().numpy(), gr.cpu().numpy()
    h = 1e-6
    t0 = time.perf_counter()
    worst = 0.0
    for e in w5.extra["fd_elements"]:
        for which in (0, 1):
            vals = []
            for sgn in (1, -1):
                kp, rp = kd.clone(), rd.clone()
                (kp if which == 0 else rp)[e] *= 1 + sgn * h
                pr5.update_coefficients(kp, rp)
                vals.append(wts @ pr5.eigs(w5.nev, vectors=False)[0])
            base = kap[e] if which == 0 else rh[e]
            fd = (vals[0] - vals[1]) / (2 * h * base)
            adj = gk[e] if which == 0 else gr[e]
            worst = max(worst, abs(adj - fd) / max(abs(fd), 1e-300))
    tfd = time.perf_counter() - t0
    pr5.update_coefficients(kd, rd)
    out["gradient_2d_128_p3_riga16"] = {
        "workload": w5.name, "n_dof": pr5.n_dof, "n_elem": w5.n_elem, "nev": w5.nev,
        "eigs_seconds": te, "grad_seconds": tg, "value": w5.nev / te,
        "fd_checks": 2 * len(w5.extra["fd_elements"]), "fd_seconds": tfd,
        "fd_max_rel_dev": worst}
    log("gradient: eigs %.3f s, adjoint %.2f ms, FD max rel dev %.2e" % (te, tg * 1e3, worst))
    return out


def calibrate_copy(torch, mib=256, reps=3):
    """Plain device copies of known size (256 MiB read, 256 MiB written), for
    scaling HBM counters: the runtime's copy kernel, then an elementwise
    kernel (dst = src + 0)."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    for _ in range(reps):
        torch.add(src, 0.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


SWEEP_SOURCES = ("paper_2009_08167_amd/csrc/k_solve.hip", "paper_2009_08167_amd/csrc/k_inverse.hip",
                 "paper_2009_08167_amd/csrc/k_top.hip", "paper_2009_08167_amd/csrc/problem.h",
                 "paper_2009_08167_amd/csrc/runtime.cpp")


def sweep_kernel(name):
    """The kernels of one forward/backward sweep pair: the fused launches of
    the bottom heights, the per-level kernels above them and below the top
    block, and the three of the top block."""
    return any(t in name for t in ("::fwd_kernel<", "::bwd_kernel<", "::fwd_subtree_kernel<",
                                   "::bwd_subtree_kernel<", "top_rhs_kernel", "top_fwd_kernel",
                                   "top_bwd_kernel"))


def forward_kernel(name):
    return "::fwd_kernel<" in name or "::fwd_subtree_kernel<" in name


def sweep_pairs(rows):
    """Sweep pairs in dispatch-ordered rocprofv3 rows: on each queue, a pair
    starts with the lowest forward kernel after a kernel that is not a
    forward one (the queues separate the sweeps from a concurrent
    factorisation)."""
    pairs, prev = 0, {}
    for r in rows:
        q, cur = r["Queue_Id"], forward_kernel(r["Kernel_Name"])
        if cur and not prev.get(q, False):
            pairs += 1
        prev[q] = cur
    return pairs


def trace_summary(trace_csv, stats_csv):
    """Markdown summary of a rocprofv3 kernel trace of the main bench line:
    sweep pairs, summed sweep-kernel duration per pair, and the kernel table."""
    import csv
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    pairs = sweep_pairs(rows)
    dur = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows if sweep_kernel(r["Kernel_Name"]))
    n_sw = sum(1 for r in rows if sweep_kernel(r["Kernel_Name"]))
    # the sweeps that bench.py times with events: the last 30 sweep pairs
    # (riga_solve_multi, queued back to back after a factorisation)
    sw = [r for r in rows if sweep_kernel(r["Kernel_Name"])]
    starts = [i for i, r in enumerate(sw) if forward_kernel(r["Kernel_Name"])
              and (i == 0 or not forward_kernel(sw[i - 1]["Kernel_Name"]))]
    last = sw[starts[-30]:] if len(starts) >= 30 else []
    print("| quantity | value |\n|---|---|")
    print("| sweep pairs in the trace | %d (%d sweep-kernel launches) |" % (pairs, n_sw))
    print("| summed sweep-kernel durations / sweep pairs (all, incl. those beside a factorisation) | %.1f us |"
          % (dur / 1e3 / max(pairs, 1)))
    if last:
        span = (max(int(r["End_Timestamp"]) for r in last) - int(last[0]["Start_Timestamp"])) / 1e3 / 30
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in last) / 1e3 / 30
        print("| the 30 timed sweep pairs: span / 30 | %.1f us |" % span)
        print("| the 30 timed sweep pairs: summed kernel durations / 30 | %.1f us |" % busy)
    st = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in st)
    print("\n## All kernels (kernel_stats.csv, total %.1f ms)\n" % (tot / 1e6))
    print("| kernel | calls | total ms | avg us | % |\n|---|---|---|---|---|")
    for r in st[:30]:
        n = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        print("| `%s` | %s | %.2f | %.1f | %.2f |" % (n, r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                  float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fb_traffic.json")


def sweep_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_summary(fetch_csv, write_csv):
    """HBM bytes of one forward/backward sweep pair from two rocprofv3 --pmc
    runs of `bench.py --calibrate-copy` (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch).  Each counter is scaled by known bytes / reading of the
    256 MiB device copy at the start of the run; writes profiles/fb_traffic.json."""
    import csv

    def load(path):
        rows = list(csv.DictReader(open(path)))
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    out = {"source_sha256": sweep_source_hash(), "unit": "bytes per sweep pair"}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = load(path)
        # the elementwise copy of the calibration (3 dispatches of 256 MiB)
        # sets the scale; the runtime copy kernel's reading is kept beside it
        ew = [float(r["Counter_Value"]) for r in rows[:32]
              if "elementwise" in r["Kernel_Name"] and "Fill" not in r["Kernel_Name"]]
        cb = [float(r["Counter_Value"]) for r in rows[:32] if "copyBuffer" in r["Kernel_Name"]]
        cb = [c for c in cb if c > 0.25 * max(cb)] if cb else []
        calib = ew if ew else cb
        scale = 256 * 1024 / (sum(calib) / len(calib))   # KiB known / KiB read
        if cb:
            out[name + "_scale_runtime_copy"] = 256 * 1024 / (sum(cb) / len(cb))
        tot = sum(float(r["Counter_Value"]) for r in rows if sweep_kernel(r["Kernel_Name"]))
        pairs = sweep_pairs(rows)
        out[name] = tot * 1024.0 * scale / pairs
        out[name + "_scale"] = scale
        out["sweep_pairs"] = pairs
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def sweep_traffic():
    """Measured HBM bytes per sweep pair, if taken on the current sweep
    kernels (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != sweep_source_hash():
        return None
    return t["fetch"] + t["write"]


def cpu_baseline():
    """The oracle as it stands, on a bounded sample: NumPy element assembly of
    the same problem plus ARPACK/SuperLU shift-and-invert for its 20 lowest
    pairs; the median of 3 runs with the host's BLAS threads, and one run
    with a single thread."""
    import numpy as np
    import workloads
    from oracle import assembly, eigen
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    w = workloads.c2(True)
    kappa, rho = w.coefficients()
    k = 20

    def once():
        t0 = time.perf_counter()
        K, M = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
        lam, U = eigen.sparse_eigs(K, M, k, sigma=0.0)
        dt = time.perf_counter() - t0
        assert eigen.residual(K, M, lam, U).max() <= 1e-9
        return dt, lam

    runs = [once() for _ in range(3)]
    dts = sorted(r[0] for r in runs)
    with threadpool_limits(limits=1):
        dt1, _ = once()
    med = dts[1]
    return {"value": k / med, "unit": "eigenpairs/s", "cores": int(cores), "kind": "oracle",
            "value_1_thread": k / dt1,
            "sample": "%s: oracle assembly + eigsh shift-invert (sigma=0) for the %d lowest pairs; "
                      "median of 3 runs %.1f s (runs %s s), 1 thread %.1f s"
                      % (w.name, k, med, ", ".join("%.1f" % d for d in dts), dt1)}, runs[0][1]


# Separator-spacing study (the blocksize study of Sec. 7: total time and the
# times of the costly operations against the macroelement size BS = 2^(s-l),
# l = 0 ... s).  kappa = rho = 1 (the Laplace problem of the study); FP64.
SPACING_GRID = {2: (256, (2, 3, 4, 5), (256, 128, 64, 32, 16, 8, 4, 2, 1), 200),
                3: (32, (2, 3), (32, 16, 8, 4, 2, 1), 100)}
SPACING_MAX_FRONT = 6000   # larger fronts are left out of the sweep
SPACING_MAX_DOF = 2000000


def time_spmv(pr, reps, torch):
    """Average duration of y = M x on the library's default stream."""
    x = torch.randn(pr.n_dof, dtype=torch.float64, device="cuda")
    pr.spmv(1, x)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        pr.spmv(1, x)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def spacing_sweep(riga, torch, out_path):
    """One JSON line per (dim, p, BS): whole-solve wall time, operation
    counts, and the event-timed cost of one factorisation, one sweep pair
    and one M product; BS = ne is IGA (no separators)."""
    fout = open(out_path, "w") if out_path else None
    for dim in (2, 3):
        ne, degrees, sizes, nev = SPACING_GRID[dim]
        for p in degrees:
            for bs in sizes:
                s = 0 if bs >= ne else bs
                rec = {"dim": dim, "ne": ne, "p": p, "bs": bs, "sep_spacing": s, "nev": nev}
                an = riga.analyze(dim, ne, p, s)
                inf = an.info
                rec.update(n_dof=inf["n_dof"], max_front=inf["max_front"], nnz_l=inf["nnz_l"],
                           flops_fact=inf["flops_fact"])
                del an
                if inf["max_front"] > SPACING_MAX_FRONT or inf["n_dof"] > SPACING_MAX_DOF:
                    rec["skipped"] = "front or size above the sweep's limits"
                else:
                    try:
                        pr = riga.assemble(dim, ne, p, s)
                        wall, lam, U, res, st = timed_eigs(pr, nev, riga.RIGA_FP64, torch)
                        del U
                        sigma_mid = 0.5 * (lam[nev // 2] + lam[nev // 2 + 1])
                        t_fb, t_fact = time_solves(pr, sigma_mid, riga.RIGA_FP64, 10, torch)
                        t_mv = time_spmv(pr, 20, torch)
                        rec.update(wall=wall, rate=nev / wall, max_res=float(max(res)),
                                   n_fact=st["n_fact"], n_fb=st["n_fb"], n_mv=st["n_mv"],
                                   n_shift=st["n_shift"], t_fact=t_fact, t_fb=t_fb, t_mv=t_mv,
                                   T_fact=st["n_fact"] * t_fact, T_fb=st["n_fb"] * t_fb,
                                   T_mv=st["n_mv"] * t_mv)
                        del pr
                    except riga.RigaError as e:
                        rec["error"] = str(e)
                    torch.cuda.empty_cache()
                line = json.dumps(rec)
                print(line, flush=True)
                if fout:
                    fout.write(line + "\n")
                    fout.flush()
    if fout:
        fout.close()


def spacing_summary(path):
    """Markdown tables of a spacing sweep's JSON lines."""
    recs = [json.loads(l) for l in open(path) if l.strip()]
    for dim in (2, 3):
        rs = [r for r in recs if r["dim"] == dim]
        if not rs:
            continue
        print("\n### %dD, %d^%d elements, %d lowest eigenpairs\n" % (dim, rs[0]["ne"], dim, rs[0]["nev"]))
        print("| p | BS | N | max front | nnz(L) | eigenpairs/s | N_fa | N_fb | N_mv | "
              "t_fa ms | t_fb us | t_mv us | T_fa s | T_fb s | T_mv s | wall s |")
        print("|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|")
        for r in rs:
            bs = "%d (IGA)" % r["bs"] if r["sep_spacing"] == 0 else str(r["bs"])
            head = "| %d | %s | %d | %d | %.1fM |" % (r["p"], bs, r["n_dof"], r["max_front"], r["nnz_l"] / 1e6)
            if "wall" not in r:
                print(head + " %s |" % r.get("skipped", r.get("error")) + " |" * 10)
                continue
            print(head + " %.0f | %d | %d | %d | %.2f | %.0f | %.1f | %.3f | %.3f | %.3f | %.3f |" % (
                r["rate"], r["n_fact"], r["n_fb"], r["n_mv"], r["t_fact"] * 1e3, r["t_fb"] * 1e6,
                r["t_mv"] * 1e6, r["T_fact"], r["T_fb"], r["T_mv"], r["wall"]))
        print("\nFastest BS per degree (whole solve): " + ", ".join(
            "p=%d: %s" % (p, min((r for r in rs if r["p"] == p and "wall" in r), key=lambda r: r["wall"])["bs"])
            for p in sorted({r["p"] for r in rs if "wall" in r})))


# Accuracy study (Sec. 8, Eq. eigerrors): 2D 64^2, p = 2..5, IGA against rIGA
# of several macroelement sizes, the first N0 = N_IGA eigenpairs of each;
# EVerr over all of them against the sorted exact spectrum, EFerr_L2 and
# EFerr_E of the diagonal modes.  kappa = rho = 1, FP64.
ACCURACY_NE = 64
ACCURACY_DEGREES = (2, 3, 4, 5)
ACCURACY_SPACINGS = (0, 16, 8, 4)


def accuracy_study(riga, torch, out_path):
    import numpy as np
    fout = open(out_path, "w") if out_path else None
    ne = ACCURACY_NE
    for p in ACCURACY_DEGREES:
        n_iga = (ne + p - 2) ** 2
        for s in ACCURACY_SPACINGS:
            pr = riga.assemble(2, ne, p, s)
            t0 = time.perf_counter()
            lam, U, res, st = pr.eigs(n_iga, allow_partial=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            n = len(lam)
            exact = riga.exact_eigenvalues(2, n)
            ev = (lam - exact) / exact
            # diagonal modes (i, i) whose exact eigenvalue is among the first n
            top = exact[-1] / math.pi ** 2
            nd = int(math.floor(math.sqrt(top / 2.0)))
            modes = np.array([[i, i] for i in range(1, nd + 1)], dtype=np.int32)
            me = pr.mode_errors(lam, U, modes)
            rec = {"ne": ne, "p": p, "sep_spacing": s, "n_dof": pr.n_dof, "n0": n_iga, "found": n,
                   "wall": wall, "max_res": float(max(res)), "n_fb": st["n_fb"],
                   "everr": ev.tolist(),
                   "modes": modes[:, 0].tolist(), "mode_match": me["match"].tolist(),
                   "mode_overlap": me["overlap"].tolist(), "mode_ev": me["ev"].tolist(),
                   "ef_l2": me["l2"].tolist(), "ef_e": me["energy"].tolist()}
            log("accuracy p=%d s=%d: %d of %d pairs in %.2f s, max EVerr %.3e, %d diagonal modes"
                % (p, s, n, n_iga, wall, ev.max(), nd))
            line = json.dumps(rec)
            print(json.dumps({k: rec[k] for k in ("ne", "p", "sep_spacing", "n_dof", "found", "wall")}),
                  flush=True)
            if fout:
                fout.write(line + "\n")
                fout.flush()
            del pr, U
            torch.cuda.empty_cache()
    if fout:
        fout.close()


def accuracy_summary(path):
    """Markdown tables of an accuracy study's JSON lines."""
    import numpy as np
    recs = [json.loads(l) for l in open(path) if l.strip()]
    fr = (0.1, 0.25, 0.5, 0.75, 0.9, 1.0)
    print("\n### EVerr against the sorted exact spectrum, at mode number i / N0\n")
    print("| p | discretisation | N | pairs | " + " | ".join("i/N0=%.2g" % f for f in fr) + " | max |")
    print("|---|---|---|---|" + "---|" * (len(fr) + 1))
    for r in recs:
        ev = np.array(r["everr"])
        name = "IGA" if r["sep_spacing"] == 0 else "rIGA BS=%d" % r["sep_spacing"]
        cells = " | ".join("%.2e" % ev[max(0, int(round(f * r["n0"])) - 1)] if int(round(f * r["n0"])) <= len(ev)
                           else "-" for f in fr)
        print("| %d | %s | %d | %d | %s | %.2e |" % (r["p"], name, r["n_dof"], r["found"], cells, ev.max()))
    print("\n### Diagonal modes (i, i): EFerr_L2 / EFerr_E\n")
    picks = (1, 4, 8, 16, 24, 32, 40)
    print("| p | discretisation | " + " | ".join("i=%d" % i for i in picks) + " |")
    print("|---|---|" + "---|" * len(picks))
    for r in recs:
        name = "IGA" if r["sep_spacing"] == 0 else "rIGA BS=%d" % r["sep_spacing"]
        cells = []
        for i in picks:
            if i <= len(r["modes"]):
                cells.append("%.1e / %.1e" % (r["ef_l2"][i - 1], r["ef_e"][i - 1]))
            else:
                cells.append("-")
        print("| %d | %s | %s |" % (r["p"], name, " | ".join(cells)))


# Large N0 (the operation counts of Sec. 7's tables for N0 = 4096 eigenpairs
# in 2D): per mesh, degree and method the solve's shifts, factorisations,
# sweeps and products, the event-timed cost of one of each, and the average
# time per eigenpair.  kappa = rho = 1, FP64, rIGA with BS = 16.
LARGE_N0 = 4096
LARGE_CASES = ([(2, 256, p, s, 4096) for p in (2, 3, 4, 5) for s in (0, 16)]
               + [(2, 512, p, s, 4096) for p in (2, 3, 4, 5) for s in (0, 16)]
               + [(2, 1024, 3, s, 4096) for s in (0, 16)])
# 3D: 64^3, N0 = 1024 (the paper's 3D table); rIGA only (64^3 IGA fronts reach 12,160)
LARGE_CASES_3D = [(3, 64, 2, s, 1024) for s in (16, 8)]


def large_n0(riga, torch, out_path, dims=(2,), mesh=0):
    fout = open(out_path, "w") if out_path else None
    cases = [c for c in LARGE_CASES + LARGE_CASES_3D if c[0] in dims and (mesh == 0 or c[1] == mesh)]
    for dim, ne, p, s, n0 in cases:
        rec = {"dim": dim, "ne": ne, "p": p, "sep_spacing": s, "n0": n0}
        try:
            pr = riga.assemble(dim, ne, p, s)
            rec.update(n_dof=pr.n_dof, nnz_l=pr.info["nnz_l"], max_front=pr.info["max_front"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam, U, res, st = pr.eigs(n0)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            del U
            torch.cuda.empty_cache()
            sigma_mid = 0.5 * (lam[len(lam) // 2] + lam[len(lam) // 2 + 1])
            t_fb, t_fact = time_solves(pr, sigma_mid, riga.RIGA_FP64, 10, torch)
            t_mv = time_spmv(pr, 20, torch)
            rec.update(wall=wall, t_av=wall / n0, max_res=float(max(res)),
                       n_shift=st["n_shift"], n_fact=st["n_fact"], n_fb=st["n_fb"], n_mv=st["n_mv"],
                       t_fact=t_fact, t_fb=t_fb, t_mv=t_mv)
            del pr
        except riga.RigaError as e:
            rec["error"] = str(e)
        torch.cuda.empty_cache()
        line = json.dumps(rec)
        print(line, flush=True)
        if fout:
            fout.write(line + "\n")
            fout.flush()
    if fout:
        fout.close()


def large_n0_summary(path):
    """Markdown table in the shape of the paper's large-N0 tables (T_av per
    eigenpair of each row's own N0): per
    operation its count and its time per eigenpair (count x event-timed
    cost / N0), and the measured average time per eigenpair."""
    recs = [json.loads(l) for l in open(path) if l.strip()]
    print("| mesh | p | method | N | N_sh | N_fa | t_fa/N0 ms | N_fb | t_fb/N0 ms | N_mv | t_mv/N0 ms | "
          "T_av ms (measured) | rIGA gain |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    by = {}
    for r in recs:
        by[(r.get("dim", 2), r["ne"], r["p"], r["sep_spacing"])] = r
    for r in recs:
        name = "IGA" if r["sep_spacing"] == 0 else (
            "rIGA" if r.get("dim", 2) == 2 else "rIGA BS=%d" % r["sep_spacing"])
        head = "| %d^%d | %d | %s |" % (r["ne"], r.get("dim", 2), r["p"], name)
        if "wall" not in r:
            print(head + " %s |" % r.get("error", "") + " |" * 9)
            continue
        n0 = r["n0"]
        gain = ""
        if r["sep_spacing"] != 0:
            iga = by.get((r.get("dim", 2), r["ne"], r["p"], 0))
            if iga and "wall" in iga:
                gain = "%.2f" % (iga["wall"] / r["wall"])
        print(head + " %d | %d | %d | %.4f | %d | %.4f | %d | %.4f | %.4f | %s |" % (
            r["n_dof"], r["n_shift"], r["n_fact"], r["n_fact"] * r["t_fact"] / n0 * 1e3,
            r["n_fb"], r["n_fb"] * r["t_fb"] / n0 * 1e3, r["n_mv"], r["n_mv"] * r["t_mv"] / n0 * 1e3,
            r["t_av"] * 1e3, gain))


# Factorisations only, for counter profiles of the fronts (rocprofv3 --pmc):
# 3D 32^3 p=2 rIGA (blocks of 8) and IGA, and 3D 64^3 p=2 rIGA (blocks of
# 8), kappa = rho = 1, three factorisations each in FP64 and in mixed
# precision at a shift inside the spectrum, one line of event times each.
FACTOR_PROFILE = ((3, 32, 2, 8), (3, 32, 2, 0), (3, 64, 2, 8))


def factor_profile(riga, torch):
    for dim, ne, p, s in FACTOR_PROFILE:
        pr = riga.assemble(dim, ne, p, s)
        inf = pr.info
        for name, prec in (("fp64", riga.RIGA_FP64), ("mixed", riga.RIGA_MIXED)):
            sigma = 600.0
            pr.factor(sigma, prec)
            t = event_time(lambda: pr.factor(sigma, prec), 3, torch)
            print(json.dumps({"case": "%dd_%d_p%d_s%d" % (dim, ne, p, s), "precision": name,
                              "n_dof": pr.n_dof, "max_front": inf["max_front"], "fact_ms": t * 1e3,
                              "flops_exact": inf["flops_fact_exact"], "flops_supernodal": inf["flops_fact"],
                              "tflops_exact": inf["flops_fact_exact"] / t / 1e12,
                              "tflops_supernodal": inf["flops_fact"] / t / 1e12}), flush=True)
        del pr


def stall_summary(counter_csv):
    """Markdown summary of `rocprofv3 --pmc SQ_WAVE_CYCLES SQ_BUSY_CYCLES
    SQ_WAIT_ANY SQ_WAIT_INST_LDS SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT
    SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_MFMA_MOPS_F64` over `bench.py
    --factor-profile`, per case (split at its assembly) and FP64 kernel:
    the kernel's share of the case's wave cycles, the share of its wave
    cycles spent waiting on anything (memory, LDS, barriers), LDS bank
    conflict cycles per LDS instruction, and its FP64 matrix-core flops per
    factorisation (MOPS x 512 over the five factorisations)."""
    import csv
    reps = 5
    rows = list(csv.DictReader(open(counter_csv)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))

    def short(name):
        n = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("riga::", "")
        return n.split("(")[0]

    cases, cur = [], None
    for r in rows:
        name = short(r["Kernel_Name"])
        if name == "assemble_kernel":
            if cur is None or cur["seen_other"]:
                cur = {"seen_other": False, "kern": {}}
                cases.append(cur)
            continue
        if cur is None:
            continue
        cur["seen_other"] = True
        kd = cur["kern"].setdefault(name, {})
        kd[r["Counter_Name"]] = kd.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    names = ["3d_32_p2_s8", "3d_32_p2_s0", "3d_64_p2_s8"]
    print("| case | kernel (FP64) | share of wave cycles | waiting | LDS bank conflict cycles per LDS instruction "
          "| FP64 matrix-core flops per factorisation |")
    print("|---|---|---|---|---|---|")
    for i, c in enumerate(cases):
        kern = {k: v for k, v in c["kern"].items() if "<float" not in k}
        tot = sum(v.get("SQ_WAVE_CYCLES", 0.0) for v in kern.values()) or 1.0
        top = sorted(kern.items(), key=lambda kv: -kv[1].get("SQ_WAVE_CYCLES", 0.0))[:6]
        for k, v in top:
            wc = v.get("SQ_WAVE_CYCLES", 0.0) or 1.0
            lds = v.get("SQ_INSTS_LDS", 0.0)
            print("| %s | `%s` | %.1f%% | %.0f%% | %s | %.3g |"
                  % (names[i] if i < len(names) else str(i), k, 100.0 * wc / tot,
                     100.0 * v.get("SQ_WAIT_ANY", 0.0) / wc,
                     "%.2f" % (v.get("SQ_LDS_BANK_CONFLICT", 0.0) / lds) if lds else "-",
                     v.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512 / reps))


def mfma_summary(counter_csv, fprof_log):
    """Markdown summary of `rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F64
    SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE` over
    `bench.py --factor-profile` (per case and precision: one factorisation,
    one warm-up, three timed: five).  The dispatches of each case (split at
    its assembly) are summed per counter: matrix-core flops = MOPS x 512
    (rocprofv3's own MFMA_FLOPS metrics), per factorisation; MFMA busy share
    as rocprofv3's MfmaUtil metric, busy cycles over (GRBM_GUI_ACTIVE summed
    over the dispatches and divided by the 8 XCDs it is summed over) x 1024
    SIMDs, i.e. over the kernels' active time; and the matrix-core rate over
    the event-timed factorisation of an unprofiled run (`fprof_log`, lines
    of `bench.py --factor-profile`: the profiler serialises the kernels)."""
    import csv
    reps = 5
    xcd, simd = 8, 256 * 4
    rows = list(csv.DictReader(open(counter_csv)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))

    def short(name):
        n = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("riga::", "")
        return n.split("(")[0]

    cases, cur = [], None
    for r in rows:
        name = short(r["Kernel_Name"])
        if name == "assemble_kernel":
            if cur is None or cur["seen_other"]:
                cur = {"seen_other": False, "c": {}, "kern": {}}
                cases.append(cur)
            continue
        if cur is None:
            continue
        cur["seen_other"] = True
        cn, v = r["Counter_Name"], float(r["Counter_Value"])
        cur["c"][cn] = cur["c"].get(cn, 0.0) + v
        kd = cur["kern"].setdefault(name, {})
        kd[cn] = kd.get(cn, 0.0) + v
    lines = [json.loads(l) for l in open(fprof_log) if l.startswith("{")]
    print("| case | FP64 factorisation (unprofiled) | exact flops | FP64 MFMA flops | FP64 MFMA rate "
          "| FP32 MFMA flops (mixed) | MFMA busy over kernel-active time (both precisions) |")
    print("|---|---|---|---|---|---|---|")
    for i, c in enumerate(cases):
        if 2 * i + 1 >= len(lines):
            break
        a, b = lines[2 * i], lines[2 * i + 1]
        f64 = c["c"].get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512 / reps
        f32 = c["c"].get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512 / reps
        busy = c["c"].get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        act = c["c"].get("GRBM_GUI_ACTIVE", 0.0) / xcd
        util = 100.0 * busy / (act * simd) if act else 0.0
        print("| %s | %.2f ms | %.3g | %.3g | %.2f TFLOP/s (%.1f%% of 78.6) | %.3g | %.2f%% |"
              % (a["case"], a["fact_ms"], a["flops_exact"], f64, f64 / (a["fact_ms"] * 1e-3) / 1e12,
                 100 * f64 / (a["fact_ms"] * 1e-3) / 78.6e12, f32, util))
    print("\n## MFMA work by kernel (per factorisation, FP64 and mixed runs together)\n")
    print("| case | kernel | FP64 MFMA flops | FP32 MFMA flops | MFMA busy, share of the case's |\n|---|---|---|---|---|")
    for i, c in enumerate(cases):
        tag = lines[2 * i]["case"] if 2 * i < len(lines) else str(i)
        tot = c["c"].get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) or 1.0
        for kname, kd in sorted(c["kern"].items(), key=lambda t: -t[1].get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)):
            if kd.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) <= 0:
                continue
            print("| %s | `%s` | %.3g | %.3g | %.1f%% |" % (
                tag, kname, kd.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512 / reps,
                kd.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512 / reps,
                100 * kd.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / tot))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-iga", action="store_true", help="skip the IGA comparison")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 3D, batched and gradient workloads")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a 256 MiB device copy (for scaling HBM counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 counter runs into profiles/fb_traffic.json and exit")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_CSV", "STATS_CSV"),
                    help="print a markdown summary of a rocprofv3 kernel trace and exit")
    ap.add_argument("--spacing-sweep", metavar="OUT_JSONL", nargs="?", const="",
                    help="time the solve over separator spacings (2D 256^2, 3D 32^3) and exit")
    ap.add_argument("--spacing-summary", metavar="JSONL",
                    help="print markdown tables of a spacing sweep and exit")
    ap.add_argument("--accuracy-study", metavar="OUT_JSONL", nargs="?", const="",
                    help="EVerr / EFerr of IGA and rIGA on 2D 64^2 (first N_IGA pairs) and exit")
    ap.add_argument("--accuracy-summary", metavar="JSONL",
                    help="print markdown tables of an accuracy study and exit")
    ap.add_argument("--large-n0", metavar="OUT_JSONL", nargs="?", const="",
                    help="4096 lowest eigenpairs of 2D 256^2-1024^2 IGA and rIGA, operation counts, and exit")
    ap.add_argument("--large-n0-dims", default="2",
                    help="dimensions for --large-n0: 2, 3 or 2,3 (3: 64^3 rIGA, N0 = 1024)")
    ap.add_argument("--large-n0-mesh", type=int, default=0,
                    help="with --large-n0: only the meshes with this many elements per direction")
    ap.add_argument("--mfma-summary", nargs=2, metavar=("COUNTER_CSV", "FPROF_LOG"),
                    help="summarise an MFMA counter run over --factor-profile and exit")
    ap.add_argument("--stall-summary", metavar="COUNTER_CSV",
                    help="markdown summary of wait and LDS counters over --factor-profile")
    ap.add_argument("--factor-profile", action="store_true",
                    help="factorisations only (3D 32^3 rIGA / IGA, 64^3 rIGA; FP64 and mixed) and exit")
    ap.add_argument("--large-n0-summary", metavar="JSONL",
                    help="print the markdown table of a --large-n0 run and exit")
    args = ap.parse_args()
    if args.large_n0_summary:
        large_n0_summary(args.large_n0_summary)
        return
    if args.accuracy_summary:
        accuracy_summary(args.accuracy_summary)
        return
    if args.spacing_summary:
        spacing_summary(args.spacing_summary)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(*args.trace_summary)
        return
    if args.mfma_summary:
        mfma_summary(*args.mfma_summary)
        return
    if args.stall_summary:
        stall_summary(args.stall_summary)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the spectral slices would shard across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    from paper_2009_08167_amd import riga

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    riga.lib()
    torch.cuda.set_device(0)
    if args.spacing_sweep is not None:
        spacing_sweep(riga, torch, args.spacing_sweep)
        return
    if args.accuracy_study is not None:
        accuracy_study(riga, torch, args.accuracy_study)
        return
    if args.large_n0 is not None:
        large_n0(riga, torch, args.large_n0, tuple(int(d) for d in args.large_n0_dims.split(",")),
                 args.large_n0_mesh)
        return
    if args.calibrate_copy:
        calibrate_copy(torch)
    if args.factor_profile:
        factor_profile(riga, torch)
        return

    w = workloads.c2(True)
    kappa, rho = w.coefficients()
    kd = torch.tensor(kappa, dtype=torch.float64, device="cuda")
    rd = torch.tensor(rho, dtype=torch.float64, device="cuda")
    log("assemble", w.name)
    pr = riga.assemble(w.dim, w.ne, w.p, w.s, kd, rd)
    info = pr.info
    log("info", info)
    dt, lam, res, st = run_steps(pr, kd, rd, w.nev, args.steps, args.warmup, riga.RIGA_FP64, torch)
    value = w.nev * args.steps / dt
    log("riga fp64: %.3f s/step, %.1f eigenpairs/s, stats %s" % (dt / args.steps, value, st))

    # dominant-kernel roofline, measured on the library's stream
    sigma_mid = 0.5 * (lam[len(lam) // 2] + lam[len(lam) // 2 + 1])
    t_fb, t_fact = time_solves(pr, sigma_mid, riga.RIGA_FP64, 30, torch)
    info = pr.refresh_info()
    N = pr.n_dof
    # the method's bytes: the exact fill of the elimination order, read once
    # forward and once backward, plus the vectors; the factor as stored (the
    # supernodal fronts, the top block's two copies of its inverse) beside it
    bytes_fb = 2.0 * info["nnz_l_exact"] * 8 + 6.0 * N * 8
    bytes_stored = info["sweep_bytes_stored"] + 6.0 * N * 8
    flops_fact = info["flops_fact_exact"]
    share_fb = st["n_fb"] * t_fb
    share_fact = st["n_fact"] * t_fact
    log("f/b %.1f us (%.0f GB/s), factorisation %.2f ms (%.2f TFLOP/s); per step: fb %.3f s, fact %.3f s"
        % (t_fb * 1e6, bytes_fb / t_fb / 1e9, t_fact * 1e3, flops_fact / t_fact / 1e12,
           share_fb, share_fact))
    if share_fb >= share_fact:
        ach = bytes_fb / t_fb / 1e9
        roof = {"kernel": "forward/backward elimination (fwd_subtree + bwd_subtree for the fused bottom "
                          "heights, fwd_kernel + bwd_kernel for further levels below the top block, "
                          "top_rhs + top_fwd + top_bwd for it)",
                "launch": {"top_cut": info["top_cut"], "fused_heights": info["fused_heights"],
                           "fused_subtrees": info["fused_subtrees"]},
                "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": sweep_traffic(),
                "per_launch": {"bytes": bytes_fb, "seconds": t_fb, "unit": "one sweep pair",
                               "bytes_basis": "2 nnz_exact(L) 8 + 6 N 8, nnz_exact(L) = %d"
                                              % info["nnz_l_exact"],
                               "bytes_stored": bytes_stored,
                               "stored_GBs": bytes_stored / t_fb / 1e9},
                "mall": {"bytes_algorithmic": bytes_fb, "bytes_stored": bytes_stored,
                         "capacity": MALL_BYTES, "fits": bytes_stored <= MALL_BYTES,
                         "note": "the factor a sweep pair reads fits the 256 MiB Infinity Cache, so "
                                 "repeated sweeps may be served from it; frac is against the HBM peak"}}
    else:
        ach = flops_fact / t_fact / 1e12
        roof = {"kernel": "numeric factorisation (front_assemble + front_factor, all levels)",
                "bound": "mfma", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_PEAK_TFLOPS, "traffic": None,
                "per_launch": {"flops": flops_fact, "seconds": t_fact}}

    extra = {}
    if not args.no_iga:
        wi = workloads.c2(False)
        log("assemble", wi.name)
        pri = riga.assemble(wi.dim, wi.ne, wi.p, wi.s, kd, rd)
        dti, lami, resi, sti = run_steps(pri, kd, rd, wi.nev, 1, 1, riga.RIGA_FP64, torch)
        extra["iga"] = {"workload": wi.name, "n_dof": pri.n_dof, "value": wi.nev / dti,
                        "ms_per_step": dti * 1e3, "n_fact": sti["n_fact"], "n_fb": sti["n_fb"],
                        "flops_fact": pri.info["flops_fact"], "nnz_l": pri.info["nnz_l"]}
        extra["riga_over_iga"] = value / (wi.nev / dti)
        log("iga: %.1f eigenpairs/s" % (wi.nev / dti))
        del pri

    out = {
        "metric": "eigenpairs/s at residual <=1e-9 (rIGA, FP64)",
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "ne": w.ne, "p": w.p, "sep_spacing": w.s,
                   "n_dof": N, "nev": w.nev, "coefficients": "log-normal(0, 0.3), seed %d" % w.seed,
                   "max_residual": float(max(res))},
        "stats": {k: st[k] for k in ("n_shift", "n_fact", "n_fb", "n_mv", "n_it",
                                     "n_2x2_pivots", "n_perturbed_pivots")},
        "roofline": roof,
        "roofline_other": secondary_rooflines(riga, pr, t_fact, info, torch),
        "secondary": {"fb_us": t_fb * 1e6, "fb_GBs": bytes_fb / t_fb / 1e9,
                      "fact_ms": t_fact * 1e3, "fact_TFLOPs": flops_fact / t_fact / 1e12},
    }
    out.update(extra)
    if not args.no_secondary:
        out["secondary_workloads"] = secondary_lines(riga, workloads, torch, np)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cb, lam_cpu = cpu_baseline()
        out["cpu_baseline"] = cb
        err = float(np.max(np.abs(lam[:20] - lam_cpu) / lam_cpu))
        out["oracle_check"] = {"pairs": 20, "against": "ARPACK shift-invert of the oracle's K, M",
                               "max_rel_err": err, "bar": 1e-10, "pass": err <= 1e-10}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
