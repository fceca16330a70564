"""Benchmark: ROM-based inexact FETI-DP solve on one MI355X.

One step = one full solve of the saddle system (16) to a relative residual of
1e-8: right-preconditioned FGMRES whose preconditioner (Algorithm 1) runs the
interface PCG on F̊ with M̊_D^-1, the reduced local solves K̊^-ROM and the Ů/Ůᵀ
transfers, plus the true operator; inputs (cell operators, principal bank,
coefficients, coarse inverse, f, d) are resident in HBM before the timed
region.  Workload: 2D 64x64-cell lattice, 16x16 quadratic elements per cell
(648 dof/cell), 12 principal cells, FP64, one load case.

value = cell local-solve applies per second over the timed steps, counting one
apply per cell per load case for each F̊, M̊_D^-1, Ů, Ůᵀ and K̊^-ROM application.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
PEAK_FP32_MATRIX_TFLOPS = 157.3  # MI355X dense FP32 (matrix)
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
CELL_OPS = ("F", "MD", "U", "Ut", "Kinv_rom")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def roofline_of(kstats: dict, families):
    """Roofline of the dominant kernel: the timed families (launches of one kernel under several
    tags) are pooled; achieved = algorithmic flops (or bytes) per launch / average launch time."""
    fams = [f for f in families if f in kstats and kstats[f]["total_ms"] > 0]
    if not fams:
        fams = [max(kstats.items(), key=lambda kv: kv[1]["total_ms"])[0]]
    launches = sum(kstats[f]["launches"] for f in fams)
    timed = sum(kstats[f]["timed"] for f in fams)
    total_ms = sum(kstats[f]["total_ms"] for f in fams)
    avg_s = total_ms / 1e3 / max(timed, 1)
    flops = sum(kstats[f]["flops"] for f in fams) / max(launches, 1)
    byts = sum(kstats[f]["bytes"] for f in fams) / max(launches, 1)
    name = " + ".join(fams)
    ai = flops / byts if byts > 0 else float("inf")
    common = dict(traffic=None, kernel=name, launches=launches, timed_launches=timed, avg_us=avg_s * 1e6,
                  flops_per_launch=flops, bytes_per_launch=byts)
    if ai > PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
        ach = flops / avg_s / 1e12
        return dict(bound="mfma", achieved=ach, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s", frac=ach / PEAK_FP64_TFLOPS,
                    **common)
    ach = byts / avg_s / 1e9
    return dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS, **common)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_pc64_MD_gemm_c2_fp64_hbm_counters.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2308_11371_amd", "csrc", "gemm.hip")


def kernel_source_hash():
    """sha256 of the dominant kernel's source text: its argument block, constants, device body and
    launch wrapper in gemm.hip (host-side edits elsewhere in the file do not invalidate the counters)."""
    import hashlib
    with open(KERNEL_SOURCE) as f:
        src = f.read()
    a = src.index("struct GemmArgsFrag {")
    end_marker = "pc64_tile<RT, CB, PF, NW>(g, blockIdx.x, blockIdx.y, Xs, Cs);\n}\n"
    e = src.index(end_marker, a) + len(end_marker)
    return hashlib.sha256(src[a:e].encode()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (copy-calibrated), or None when the kernel source changed since the counters were taken."""
    try:
        fields = {}
        with open(TRAFFIC_PROFILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        sha = kernel_source_hash()
        if fields.get("source_sha256") != sha:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _count_applies(m, counts):
    for op in CELL_OPS:
        fn = getattr(m, "apply_" + op)

        def wrapped(x, _fn=fn, _op=op):
            counts[_op] += 1
            return _fn(x)
        setattr(m, "apply_" + op, wrapped)


def cpu_worker(flag_dir: str):
    """The CPU oracle on the measured workload itself (c2), in a process of its own pinned to the cores
    the GPU process does not use: the oracle model and reduced basis are built while the GPU legs run
    (setup, not timed), then, once the parent signals that the GPU work is done, the bounded sample is
    timed on all the worker's cores and on one thread (the paper's serial setting).  Sample: one outer
    FGMRES iteration of the c2 solve with the interface PCG capped at 4 iterations; cell applies
    counted as on the GPU."""
    import numpy as np
    import latticegen
    from oracle import Model
    from threadpoolctl import threadpool_info, threadpool_limits
    t0 = time.perf_counter()
    p = latticegen.make("c2")
    m = Model(p)
    m.build_reduced_basis()
    setup_s = time.perf_counter() - t0
    open(os.path.join(flag_dir, "ready"), "w").close()
    go = os.path.join(flag_dir, "go")
    t1 = time.perf_counter()
    while not os.path.exists(go) and time.perf_counter() - t1 < 900:
        time.sleep(0.5)
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    out = {"setup_s": setup_s, "cores": int(cores)}
    for label, nthreads in (("all_cores", cores), ("one_thread", 1)):
        counts = dict.fromkeys(CELL_OPS, 0)
        _count_applies(m, counts)
        with threadpool_limits(limits=nthreads):
            ts = time.perf_counter()
            r = m.solve(tol=1e-8, maxit=1, inner_maxit=4)
            dt = time.perf_counter() - ts
        applies = sum(counts.values()) * p.N
        out[label] = {"value": applies / dt, "seconds": dt, "cell_applies": applies, "threads": nthreads,
                      "applies": dict(counts), "pcg_its": [int(x) for x in r["inner_its"]]}
        for op in CELL_OPS:  # the counting wrappers are instance attributes: drop them for the next pass
            delattr(m, "apply_" + op)
    print(json.dumps(out), flush=True)


class CpuBaseline:
    """Starts the oracle worker at once (its setup overlaps the GPU legs) and collects its sample."""

    def __init__(self):
        import subprocess
        import tempfile
        self.dir = tempfile.mkdtemp(prefix="ifeti_cpu_")
        # the process's CPU share: the affinity set, capped by the thread budget the box sets
        mine = sorted(os.sched_getaffinity(0))
        ncpu = min(len(mine), int(os.environ.get("OMP_NUM_THREADS", len(mine)) or len(mine)))
        mine = mine[:ncpu]
        # the GPU process keeps four cores (launches, polls); the oracle gets the rest
        self.gpu_cores, self.cpu_cores = mine[:4], (mine[4:] or mine)
        env = dict(os.environ)
        n = str(len(self.cpu_cores))
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = n
        env["HIP_VISIBLE_DEVICES"] = ""  # the worker never touches the GPU
        self.proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", self.dir],
                                     stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env, text=True,
                                     preexec_fn=lambda: os.sched_setaffinity(0, self.cpu_cores))
        os.sched_setaffinity(0, self.gpu_cores)
        self.ncpu = ncpu

    def collect(self, timeout_s: float = 420.0):
        open(os.path.join(self.dir, "go"), "w").close()
        try:
            out, err = self.proc.communicate(timeout=timeout_s)
        except Exception:
            self.proc.kill()
            return None
        finally:
            os.sched_setaffinity(0, set(self.gpu_cores) | set(self.cpu_cores))
        try:
            r = json.loads(out.strip().splitlines()[-1])
        except (ValueError, IndexError):
            log(f"cpu baseline worker failed: {err[-2000:]}")
            return None
        a, o = r["all_cores"], r["one_thread"]
        return dict(value=a["value"], unit="cell-applies/s", cores=a["threads"], kind="oracle",
                    sample=(f"c2 itself (4096 cells, 12 principal cells, FP64): one outer FGMRES iteration with the "
                            f"interface PCG capped at 4 iterations ({a['cell_applies']} cell applies: "
                            f"{a['applies']}) in {a['seconds']:.1f} s on {a['threads']} threads; oracle setup "
                            f"(model, greedy, bank, coefficients, coarse factor) {r['setup_s']:.0f} s, not timed, "
                            f"overlapping the GPU legs on cores of its own"),
                    one_thread={"value": o["value"], "seconds": o["seconds"], "cell_applies": o["cell_applies"]},
                    setup_s=r["setup_s"], box_cpus=self.ncpu)


def timed_solve(ctx, f, d, nrhs, tol, inner_tol, reps=1, maxit=200, check=True):
    """Mean wall time of `reps` solves after one untimed warm-up; returns (seconds, info, u of the last).
    check=False: a solve that stops at the iteration limit is timed and reported, not raised."""
    import torch
    ctx.solve(f, d, nrhs=nrhs, tol=tol, inner_tol=inner_tol, maxit=maxit, check=check)  # untimed warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        u, lam, info = ctx.solve(f, d, nrhs=nrhs, tol=tol, inner_tol=inner_tol, maxit=maxit, check=check)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, info, u


def rel_err(u, ref):
    import torch
    return float(torch.linalg.norm(u - ref) / torch.linalg.norm(ref))


def reference_solution(ctx, f, d, nrhs=1, maxit=200):
    """FP64 plain solve at the parity tolerances (outer 1e-12, interface PCG 1e-13): the reference every
    precision-form result is compared with."""
    ctx.reset_options(fgmres_restart=max(200, maxit), pcg_maxit=3000)
    u, lam, info = ctx.solve(f, d, nrhs=nrhs, tol=1e-12, inner_tol=1e-13, maxit=maxit, check=False)
    ctx.reset_options()
    return u.clone(), float(max(info["relres"]))


def op_rates(ctx, reps=20):
    """Each cell operator applied alone, back to back (one load case, FP64 unless the context's precision
    says otherwise): time per apply and cell local-solve applies per second (cells / time)."""
    import torch
    s = ctx.sizes
    g = torch.Generator("cuda").manual_seed(9)
    n_in = {"F": s.L, "MD": s.L, "Ut": s.L, "U": s.nU, "Kinv_rom": s.nU}
    out = {}
    for op in ("F", "MD", "Kinv_rom", "U", "Ut"):
        x = torch.randn(n_in[op], dtype=torch.float64, device="cuda", generator=g)
        fn = getattr(ctx, "apply_" + op)
        y = fn(x)
        for _ in range(2):
            fn(x, out=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(x, out=y)
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out[op] = {"us_per_apply": us, "cell_applies_per_s": s.N / us * 1e6}
    return out


def kernel_roofline(ctx, fam, peak, unit="TFLOP/s"):
    """Average HIP-event time of one kernel family (timed launches) and its algorithmic rate."""
    k = ctx.stats()["kernels"].get(fam)
    if not k or not k["timed"]:
        return None
    us = k["total_ms"] * 1e3 / k["timed"]
    fl = k["flops"] / max(k["launches"], 1)
    by = k["bytes"] / max(k["launches"], 1)
    ach = fl / us / 1e6
    return {"kernel": fam, "avg_us": us, "flops_per_launch": fl, "bytes_per_launch": by, "achieved": ach,
            "peak": peak, "unit": unit, "frac": ach / peak, "hbm_gb_s": by / us / 1e3}


def run_forms(ctx, f, d, t_fp64, args, u_ref):
    """Precision form (FP32 / BF16 local contractions, FP64 PCG, coarse solve and outer FGMRES), the
    approximate coarse solve, the interface-block and local-solve variants on the same lattice, each
    against the plain FP64 solve time and with ||u - u_FP64|| / ||u_FP64|| against the FP64 solve at
    the parity tolerances; then the c2 lattice with 40 principal cells and the block-RHS form c4."""
    import latticegen
    from paper_2308_11371_amd import ifeti
    res = {"fp64_plain": {"solve_time_s": t_fp64}}

    def leg(name, itol, maxit=200, check=True, **opts):
        ctx.reset_options(**opts)
        t, info, u = timed_solve(ctx, f, d, 1, args.tol, itol, reps=3, maxit=maxit, check=check)
        r = {"solve_time_s": t, "vs_fp64": t / t_fp64, "outer_its": int(info["outer_its"][0]),
             "pcg_its": int(info["inner_its"][0]), "relres": float(info["relres"][0]), "inner_tol": itol,
             "converged": int(info["status"]) == 0, "err_vs_fp64": rel_err(u, u_ref)}
        log(f"form {name}: {t:.3f}s outer={r['outer_its']} pcg={r['pcg_its']} relres={r['relres']:.1e} "
            f"err={r['err_vs_fp64']:.1e}")
        res[name] = r
        return r

    B16, F32 = ifeti.IFETI_BF16_LOCAL, ifeti.IFETI_FP32_LOCAL
    for name, prec, itol in (("fp32_local", F32, 1e-6), ("bf16_local", B16, 1e-3)):
        # FP64 at the same (looser) inner tolerance: separates the gain of the narrow contractions from
        # that of the looser inner solve
        t64 = leg(name + "_fp64_same_inner_tol", itol)["solve_time_s"]
        r = leg(name, itol, precision=prec)
        r["vs_fp64_same_inner_tol"] = r["solve_time_s"] / t64
    # BF16 Dirichlet preconditioner (49) under FP64 or FP32 operators (PCG needs only an SPD
    # preconditioner; the interface solve keeps the operators' accuracy)
    leg("fp64_bf16_preconditioner", 1e-11, md_precision=B16)
    leg("fp32_bf16_preconditioner", 1e-6, precision=F32, md_precision=B16)
    leg("fp32_bf16_preconditioner_inner_1e-3", 1e-3, precision=F32, md_precision=B16)
    # approximate coarse solve (Sec. 3.2.1): block Jacobi over blocks of B primal dofs; the outer FGMRES
    # corrects the inexact F̊ (a leg that stops at 200 outer iterations is reported as such)
    for B in (128, 1040):
        leg(f"coarse_block_jacobi_{B}", 1e-11, check=False, coarse_approx=B, fgmres_restart=200)
    # interface block of Alg. 1: one application of (49) or of (47) in place of the interface PCG
    leg("interface_md_once", 1e-11, interface_block=1, fgmres_restart=200)
    leg("interface_md_rom_once", 1e-11, interface_block=2, fgmres_restart=200)
    # K̊^-MPCG (Remark 6): multi-preconditioned CG local solves, two and three iterations each
    for it in (2, 3):
        leg(f"mpcg_local_{it}", 1e-11, local_iters=it)
    ctx.reset_options()
    res["true_operator"] = run_true_operator(ctx)
    res["c2_K40"] = run_k40(args)
    res["block_rhs_fp32_local"] = run_c4(args, t_fp64)
    if not args.no_3d:
        res["c3_3d"] = run_c3(args)
        res["c5_gradient"] = run_c5(args)
    return res


def run_k40(args):
    """c2 with the greedy capped at 40 principal cells (the configuration's "reduced basis 40 modes per
    cell"): same kernels with K = 40, FP64 solve to 1e-8, the principal contraction's roofline."""
    import torch
    import latticegen
    from paper_2308_11371_amd import ifeti
    prob = latticegen.make("c2", n_principal=40)
    t0 = time.perf_counter()
    ctx = ifeti.setup(prob)
    torch.cuda.synchronize()
    s = ctx.sizes
    f, d = ctx.get_rhs()
    out = {"workload": f"c2 with {s.K} principal cells (greedy capped at 40), FP64, 1 load case",
           "principal_cells": s.K, "setup_s": time.perf_counter() - t0}
    ctx.set_options(timing=1, timing_filter="MD_gemm", timing_every=8)
    ctx.reset_stats()
    t, info, u = timed_solve(ctx, f, d, 1, args.tol, args.inner_tol, reps=3)
    st = ctx.stats()
    out.update(solve_time_s=t, outer_its=int(info["outer_its"][0]), pcg_its=int(info["inner_its"][0]),
               relres=float(info["relres"][0]),
               cell_applies_per_s=sum(st["applies"][op] for op in CELL_OPS) * s.N / (4 * t),
               roofline_MD_gemm=kernel_roofline(ctx, "MD_gemm", PEAK_FP64_TFLOPS))
    ctx.reset_options()
    out["operators"] = op_rates(ctx)
    log(f"c2 K={s.K}: solve {t:.3f}s outer={out['outer_its']} pcg={out['pcg_its']}")
    ctx.close()
    return out


def run_c4(args, t_fp64):
    """c4: the c2 lattice with 32 seeded load cases in one batched solve (block PCG: 32 recurrences
    sharing every operator application), FP32 local contractions with FP64 PCG, coarse solve and outer
    FGMRES, tiles autotuned in the untimed warm-up; per-load-case time against the FP64 single solve,
    the contractions' rooflines against the FP32 matrix peak and the error of every load case against
    the FP64 block solve at the parity tolerances."""
    import torch
    import latticegen
    from paper_2308_11371_amd import ifeti
    prob = latticegen.make("c4")
    ctx = ifeti.setup(prob)
    s = ctx.sizes
    f, d = ctx.get_rhs()
    u_ref, _ = reference_solution(ctx, f, d, nrhs=s.nrhs)
    ctx.set_options(precision=ifeti.IFETI_FP32_LOCAL, autotune=1)
    ctx.solve(f, d, nrhs=s.nrhs, tol=args.tol, inner_tol=1e-6, maxit=200)  # tiles tuned here
    torch.cuda.synchronize()
    ctx.set_options(timing=1, timing_filter="F_gemm,MD_gemm,coarse_sep_rhs,coarse_sep_solve,coarse_interior,"
                    "F_restrict,F_prolong,rom_R_gemm,rom_local", timing_every=4)
    ctx.reset_stats()
    t, info, u = timed_solve(ctx, f, d, s.nrhs, args.tol, 1e-6)
    U, R = u.view(s.nrhs, -1), u_ref.view(s.nrhs, -1)
    errs = [rel_err(U[r], R[r]) for r in range(s.nrhs)]
    out = {"workload": f"c4: the c2 lattice with {s.nrhs} seeded right-edge load cases in one batched solve",
           "nrhs": int(s.nrhs), "solve_time_s": t, "per_load_case_s": t / s.nrhs,
           "vs_fp64_plain_per_load_case": t / s.nrhs / t_fp64, "autotuned_tiles": True,
           "max_outer_its": int(max(info["outer_its"])), "max_relres": float(max(info["relres"])),
           "max_err_vs_fp64": max(errs),
           "roofline_F_gemm_fp32": kernel_roofline(ctx, "F_gemm", PEAK_FP32_MATRIX_TFLOPS),
           "roofline_MD_gemm_fp32": kernel_roofline(ctx, "MD_gemm", PEAK_FP32_MATRIX_TFLOPS),
           "rom_R_gemm_fp32": kernel_roofline(ctx, "rom_R_gemm", PEAK_FP32_MATRIX_TFLOPS),
           "rom_local": kernel_roofline(ctx, "rom_local", PEAK_FP64_TFLOPS),
           # the coarse branch runs beside F_gemm on the other stream: its event times include the waits
           # for compute units the contraction holds
           "coarse_branch_beside_F_gemm": {k: kernel_roofline(ctx, k, PEAK_FP64_TFLOPS) for k in
                                           ("F_restrict", "coarse_sep_rhs", "coarse_sep_solve", "coarse_interior",
                                            "F_prolong")}}
    log(f"form block_rhs: {t:.3f}s for {s.nrhs} load cases, max err {max(errs):.1e}")
    # the same solve with one block PCG over all load cases inside the preconditioner (O'Leary): the
    # block space spans every load case's Krylov space, the tractions' two directions collapse
    ctx.set_options(block_cg=1, timing=0)
    tb, infob, ub = timed_solve(ctx, f, d, s.nrhs, args.tol, 1e-6)
    Ub = ub.view(s.nrhs, -1)
    errs_b = [rel_err(Ub[r], R[r]) for r in range(s.nrhs)]
    out["block_cg"] = {"solve_time_s": tb, "per_load_case_s": tb / s.nrhs, "speedup_vs_independent": t / tb,
                       "max_outer_its": int(max(infob["outer_its"])), "max_relres": float(max(infob["relres"])),
                       "inner_its_max": int(max(infob["inner_its"])),
                       "inner_its_max_independent": int(max(info["inner_its"])),
                       "max_err_vs_fp64": max(errs_b)}
    ctx.reset_options()
    log(f"form block_rhs with block PCG: {tb:.3f}s, max err {max(errs_b):.1e}")
    ctx.close()
    return out


def run_true_operator(ctx, reps=10):
    """The cell operator K^(s) inside the true operator (16): assembled stencil values against the
    matrix-free form (Remark 9: pulled-back tensor at the quadrature points and shared 1D tables), per
    apply of ifeti_apply_A on one load case; HIP-event time of the cell kernel and its HBM rate."""
    import torch
    s = ctx.sizes
    x = torch.randn(s.nU + s.L, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    out = {}
    for mode, tag in ((0, "true_K"), (1, "true_K_mf")):
        ctx.set_options(true_operator=mode)
        ctx.apply_A(x)  # untimed warm-up
        torch.cuda.synchronize()
        ctx.set_options(true_operator=mode, timing=1, timing_filter=tag)
        ctx.reset_stats()
        for _ in range(reps):
            ctx.apply_A(x)
        torch.cuda.synchronize()
        k = ctx.stats()["kernels"][tag]
        us = k["total_ms"] * 1e3 / k["timed"]
        gb = k["bytes"] / k["launches"] / 1e9
        out["stencil" if mode == 0 else "matrix_free"] = {"kernel": tag, "us_per_apply": us,
                                                          "algorithmic_gb": gb, "tb_per_s": gb / us * 1e3}
    ctx.reset_options()
    log(f"true operator: stencil {out['stencil']['us_per_apply']:.1f} us, "
        f"matrix-free {out['matrix_free']['us_per_apply']:.1f} us")
    return out


def run_exact(ctx, f, d, t_rom, args, maxit=2000,
              workload="c2: standard FETI-DP (every K_rr^(s) factorised), 1 load case"):
    """Standard (exact) FETI-DP on the same c2 lattice, the paper's comparator: every cell's K_rr
    factorised on the GPU (batched blocked Cholesky), then PCG on the exact F with the exact Dirichlet
    preconditioner to the same relative residual, and the displacement recovery.  Reported: the
    factorisation time, the solve time and iterations, the true residual of (16), the device memory of
    the exact form, and the per-apply time and HBM rate of the exact per-cell products."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.build_exact()
    torch.cuda.synchronize()
    out = {"workload": workload, "factorisation_s": time.perf_counter() - t0}
    _, _, _, _, nbytes = ctx.exact_cell_blocks(0)
    out["device_gb"] = nbytes / 1e9
    # The interface tolerance is relative to d-bar of (25).  With exact local solves the residual of
    # (16) is the interface residual over the norm of (f, d): in 2D d-bar is several hundred times that
    # norm and 1e-3 of the saddle tolerance suffices; in 3D the ratio is larger, so the tolerance is
    # tightened by the measured shortfall (at most twice) until (16) meets the ROM solve's tolerance,
    # and the solve that meets it is the one reported.
    itol = args.tol * 1e-3
    ctx.exact_solve(f, d, tol=itol, maxit=maxit)  # untimed warm-up
    torch.cuda.synchronize()
    from paper_2308_11371_amd import ifeti
    b = torch.cat([f, d])
    tried, best = [], None
    for attempt in range(3):
        ctx.set_options(timing=1, timing_filter="exact_F_cells,exact_MD_cells", timing_every=8)
        ctx.reset_stats()
        t0 = time.perf_counter()
        # a tightened tolerance the PCG cannot reach ends the search with the last solve that did
        u, lam, info = ctx.exact_solve(f, d, tol=itol, maxit=maxit, check=attempt == 0)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = ctx.stats()
        ctx.reset_options()
        rs = float(torch.linalg.norm(b - ctx.apply_A(torch.cat([u, lam]))) / torch.linalg.norm(b))
        rec = {"interface_tol": itol, "pcg_its": int(info["iters"][0]), "pcg_relres": float(info["relres"][0]),
               "relres_saddle": rs, "solve_time_s": t, "status": ifeti.STATUS_NAMES.get(info["status"])}
        tried.append(rec)
        if info["status"] != ifeti.IFETI_OK:
            break
        best = (rec, st)
        if rs <= args.tol:
            break
        itol *= 0.5 * args.tol / rs
    rec, st = best
    for k in ("interface_tol", "solve_time_s", "pcg_its", "pcg_relres", "relres_saddle"):
        out[k] = rec[k]
    if len(tried) > 1:
        out["interface_tol_tried"] = tried
    out["vs_rom_solve"] = out["solve_time_s"] / t_rom
    for fam in ("exact_F_cells", "exact_MD_cells"):
        k = st["kernels"].get(fam)
        if k and k["timed"]:
            us = k["total_ms"] * 1e3 / k["timed"]
            out[fam] = {"avg_us": us, "bytes_per_launch": k["bytes"] / max(k["launches"], 1),
                        "gb_s": k["bytes"] / max(k["launches"], 1) / us / 1e3}
    log(f"exact FETI-DP: factorisation {out['factorisation_s']:.2f}s, solve {out['solve_time_s']:.3f}s "
        f"({out['pcg_its']} PCG its), saddle relres {out['relres_saddle']:.1e}, {out['device_gb']:.1f} GB")
    return out


def run_c3(args):
    """3D lattice c3 (2048 cells, 1536 dof/cell, 16 principal cells): FP64 plain vs FP32 / BF16 local
    contractions, each solved to relres 1e-8 (interface PCG capped at 200 iterations in 3D; contraction
    tiles autotuned during the untimed warm-up solve)."""
    import torch
    import latticegen
    from paper_2308_11371_amd import ifeti
    t0 = time.perf_counter()
    prob = latticegen.make("c3")
    ctx = ifeti.setup(prob)
    torch.cuda.synchronize()
    s = ctx.sizes
    out = {"workload": "c3: 3D 16x16x8-cell lattice, 1536 dof/cell, 16 principal cells, 1 load case",
           "autotuned_tiles": True,
           "setup_s": time.perf_counter() - t0}
    f, d = ctx.get_rhs()
    f = f[:s.nU].contiguous()
    d = d[:s.L].contiguous()
    u_ref, rr = reference_solution(ctx, f, d)
    out["reference"] = {"tol": 1e-12, "inner_tol": 1e-13, "relres": rr}
    B16 = ifeti.IFETI_BF16_LOCAL
    for name, prec, itol, mdp in (("fp64_plain", ifeti.IFETI_FP64, 1e-11, -1),
                                  ("fp32_local", ifeti.IFETI_FP32_LOCAL, 1e-6, -1),
                                  ("bf16_local", B16, 1e-3, -1),
                                  ("fp64_bf16_preconditioner", ifeti.IFETI_FP64, 1e-11, B16),
                                  ("fp32_bf16_preconditioner", ifeti.IFETI_FP32_LOCAL, 1e-6, B16)):
        # tiles tuned in the untimed warm-up
        ctx.reset_options(precision=prec, md_precision=mdp, pcg_maxit=200, autotune=1)
        t, info, u = timed_solve(ctx, f, d, 1, args.tol, itol, reps=3)
        out[name] = {"solve_time_s": t, "outer_its": int(info["outer_its"][0]), "pcg_its": int(info["inner_its"][0]),
                     "relres": float(info["relres"][0]), "inner_tol": itol, "err_vs_fp64": rel_err(u, u_ref)}
        if name != "fp64_plain":
            out[name]["vs_fp64"] = t / out["fp64_plain"]["solve_time_s"]
        log(f"form c3 {name}: {t:.3f}s outer={info['outer_its'][0]} pcg={info['inner_its'][0]} "
            f"err={out[name]['err_vs_fp64']:.1e}")
    ctx.reset_options()
    out["true_operator"] = run_true_operator(ctx)
    if not args.no_exact:
        out["exact_fetidp"] = run_exact(ctx, f, d, out["fp64_plain"]["solve_time_s"], args, maxit=5000,
                                        workload="c3: standard FETI-DP (every K_rr^(s) factorised), 1 load case")
    ctx.close()
    return out


def run_c5(args):
    """Differentiation form on c5 (3D 12x12x12 cells, 1536 dof/cell, 16 principal cells, per-cell strut
    widths uniform in [0.15, 0.30]): compliance and its gradient with respect to all 1728 widths through
    the torch.autograd.Function (width update: cell operators rebuilt, which the true operator and the
    reduced local solves of (46b) use, while the principal bank, coefficients and coarse factor are
    kept; FP64 solve to relres 1e-8; adjoint gradient kernel), timed after one untimed evaluation; then
    each part timed on its own."""
    import torch
    import latticegen
    from paper_2308_11371_amd import ifeti
    t0 = time.perf_counter()
    prob = latticegen.make("c5")
    ctx = ifeti.setup(prob)
    torch.cuda.synchronize()
    s = ctx.sizes
    out = {"workload": f"c5: 3D 12x12x12-cell lattice, 1536 dof/cell, {s.K} principal cells, per-cell widths, "
                       f"gradient w.r.t. {s.N} widths", "setup_s": time.perf_counter() - t0}
    ctx.set_options(pcg_maxit=200)
    f, d = ctx.get_rhs()
    f = f[:s.nU].contiguous()
    d = d[:s.L].contiguous()
    w = torch.tensor(prob.widths, dtype=torch.float64, device="cuda", requires_grad=True)

    def evaluate():
        c = ifeti.compliance(w, ctx, f, d, tol=args.tol, inner_tol=1e-11)
        (g,) = torch.autograd.grad(c, w)
        return c, g

    evaluate()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c, g = evaluate()
    torch.cuda.synchronize()
    out["compliance_and_gradient_s"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    ctx.update_widths(w.detach())
    torch.cuda.synchronize()
    out["width_update_s"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    u, lam, info = ctx.solve(f, d, tol=args.tol, inner_tol=1e-11, maxit=200)
    torch.cuda.synchronize()
    out["solve_s"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    ctx.compliance_grad(f, u)
    torch.cuda.synchronize()
    out["gradient_kernel_s"] = time.perf_counter() - t1
    out.update(outer_its=int(info["outer_its"][0]), pcg_its=int(info["inner_its"][0]),
               relres=float(info["relres"][0]), compliance=float(c.detach()), grad_norm=float(torch.linalg.norm(g)))
    log(f"form c5 gradient: {out['compliance_and_gradient_s']:.3f}s (update {out['width_update_s']:.3f}, "
        f"solve {out['solve_s']:.3f}, gradient {out['gradient_kernel_s'] * 1e3:.2f} ms)")
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--n-principal", type=int, default=None)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--inner-tol", type=float, default=1e-11)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--roofline-kernel", default="MD_gemm",
                    help="kernel families (comma-separated, pooled) of the dominant kernel for the roofline")
    ap.add_argument("--also-time", default="F_gemm",
                    help="further kernel families timed with HIP events (reported under 'kernels')")
    ap.add_argument("--all-kernels", action="store_true", help="event-time every kernel family (slower)")
    ap.add_argument("--timing-every", type=int, default=8,
                    help="event-time one launch in this many of each timed family (keeps the timeline unperturbed)")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision, variant and block-RHS legs")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D (c3, c5) legs of the forms")
    ap.add_argument("--no-exact", action="store_true", help="skip the standard FETI-DP comparison leg")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MIB",
                    help="run one device-to-device copy of this many MiB first (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    # the CPU oracle's setup runs on cores of its own while the GPU legs run (no GPU use in that process)
    cpu = None if args.no_cpu_baseline else CpuBaseline()

    import torch
    import latticegen
    from paper_2308_11371_amd import ifeti

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 20)) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 8} bytes read, {n * 8} bytes written")
        del a, c
    prob = latticegen.make(args.config, n_principal=args.n_principal)
    t0 = time.perf_counter()
    ctx = ifeti.setup(prob)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    s = ctx.sizes
    log(f"setup {setup_s:.1f}s  N={s.N} n_r={s.n_r} n_d={s.n_d} L={s.L} nP={s.nP} K={s.K}")
    f, d = ctx.get_rhs()
    f = f[:s.nU].contiguous()
    d = d[:s.L].contiguous()
    for i in range(args.warmup):
        t1 = time.perf_counter()
        u, lam, info = ctx.solve(f, d, tol=args.tol, inner_tol=args.inner_tol, maxit=200)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t1:.3f}s outer={info['outer_its'][0]} "
            f"pcg={info['inner_its'][0]} relres={info['relres'][0]:.2e}")
    timed = ",".join(x for x in (args.roofline_kernel, args.also_time) if x)
    ctx.set_options(timing=1, timing_filter="" if args.all_kernels else timed,
                    timing_every=1 if args.all_kernels else args.timing_every)
    ctx.reset_stats()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    infos = []
    for i in range(args.steps):
        u, lam, info = ctx.solve(f, d, tol=args.tol, inner_tol=args.inner_tol, maxit=200)
        infos.append(info)
        log(f"step {i}: outer={info['outer_its'][0]} pcg={info['inner_its'][0]} relres={info['relres'][0]:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    st = ctx.stats()
    ctx.reset_options()
    applies = sum(st["applies"][op] for op in CELL_OPS) * s.N
    value = applies / elapsed
    roof = roofline_of(st["kernels"], args.roofline_kernel.split(","))
    if args.roofline_kernel == "MD_gemm":
        roof["traffic"] = measured_traffic()
    kernels = {k: dict(launches=v["launches"], timed=v["timed"], avg_us=v["total_ms"] * 1e3 / max(v["timed"], 1),
                       share=v["total_ms"] / max(v["timed"], 1) * v["launches"] / 1e3 / elapsed) for k, v in sorted(
                           st["kernels"].items(), key=lambda kv: -kv[1]["total_ms"])[:10] if v["total_ms"] > 0}
    per_solve = {k: v // args.steps for k, v in st["applies"].items()}
    pcg_its = int(infos[-1]["inner_its"][0])
    outer = int(infos[-1]["outer_its"][0])
    ops = op_rates(ctx)
    per_operator = {op: {"applies_per_solve": per_solve[op], "in_solve_cell_applies_per_s": per_solve[op] * s.N /
                         (elapsed / args.steps), **ops[op]} for op in CELL_OPS}
    # one F̊ per PCG iteration; the others come from the look-ahead of the convergence polls (iterations
    # that run past convergence before a poll sees it leave the iterate unchanged)
    past = {"F": per_solve["F"] - pcg_its, "MD": per_solve["MD"] - pcg_its - outer}
    forms = None
    if not args.no_forms:
        u_ref, _ = reference_solution(ctx, f, d)
        err_headline = rel_err(u, u_ref)  # the last timed solve against the parity-tolerance solve
        forms = run_forms(ctx, f, d, elapsed / args.steps, args, u_ref)
        forms["fp64_plain"]["err_vs_fp64"] = err_headline
        if not args.no_exact:
            forms["exact_fetidp"] = run_exact(ctx, f, d, elapsed / args.steps, args)
    lat = "2D 64x64-cell lattice, 648 dof/cell" if prob.dim == 2 else f"3D {'x'.join(map(str, prob.shape))}-cell lattice, {s.n_dof} dof/cell"
    out = {
        "metric": "cell local-solve applies/s; solve time to rel. residual 1e-8 vs FP64 plain",
        "value": value,
        "unit": "cell-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {lat}, {s.K} principal cells, FP64, {s.nrhs if s.nrhs > 1 else 1} "
                               f"load case{'s' if s.nrhs > 1 else ''} solved one at a time, FGMRES to relres {args.tol:g}",
                   "cells": s.N, "dof_torn": int(s.nU), "multipliers": s.L, "principal_cells": s.K,
                   "precision": "fp64", "nrhs": 1},
        "solve_time_s": elapsed / args.steps,
        "setup_s": setup_s,
        "outer_its": outer,
        "pcg_its_per_solve": pcg_its,
        "relres": float(infos[-1]["relres"][0]),
        "applies_per_solve": per_solve,
        "applies_past_convergence_per_solve": past,
        "value_definition": "cell applies of F̊, M̊_D^-1, Ů, Ůᵀ and K̊^-ROM (one per cell per load case) over the "
                            "timed solves, divided by their wall time; per_operator gives each operator alone",
        "per_operator": per_operator,
        "roofline": roof,
        "kernels": kernels,
    }
    if forms is not None:
        out["forms"] = forms
    ctx.close()
    if cpu is not None:
        log("cpu baseline (oracle on c2, bounded sample) ...")
        out["cpu_baseline"] = cpu.collect()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
