#!/usr/bin/env python3
"""Benchmark: MDOF/s of Q1 multigrid solves to 1e-8 relative residual on one
MI355X, with the dominant kernel's HBM roofline fraction and the CPU oracle
timed beside it.

A step is one complete solve (V(2,2) cycles from u = 0 until the relative
residual is <= 1e-8) of the 3D Poisson problem on 256^3 Q1 hexahedra
(16,974,593 nodes, the largest single-GPU configuration) with the matrix-free
27-point stencil, red-black smoothing, FP64, 8 levels, right-hand side
U[-1, 1] from seed 0 -- inputs resident in device memory before timing.
The same JSON line also carries the other workloads (2D 64^2 Jacobi,
3D 128^3 CSR FP64, 3D 256^3 FP32-inner refinement, 3D 192^3 variable kappa
FP64 and FP32-inner) as "extra" entries, each timed the same way.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _device_rhs(w):
    import torch
    from paper_1609_04809_amd import workloads as W
    b, kappa = W.workload_inputs(w)
    bd = torch.from_numpy(W.interior_to_full(w.dim, w.n, b)).to("cuda")
    return b, kappa, bd


def time_solves(S, bd, tol, steps, warmup):
    import torch
    u = torch.empty_like(bd)
    k = None
    hist = None
    for _ in range(warmup):
        _, k, hist, st = S.solve(bd, tol, u=u)
        assert st == "ok", st
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, k, hist, st = S.solve(bd, tol, u=u)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert st == "ok", st
    return (t1 - t0) / steps, k, hist, u


def solve_spread(S, bd, tol, steps):
    """Median and minimum of `steps` single solves, each bracketed by
    device synchronisations (after the timed loop, outside it)."""
    import torch
    u = torch.empty_like(bd)
    ts = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.solve(bd, tol, u=u)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), float(np.min(ts))


def reference_copy(mib):
    """Attainable bandwidth: a plain device-to-device copy of `mib` MiB
    (read + write bytes / time), 1 warm-up + up to 10 timed copies."""
    import torch
    if mib <= 0:
        return None
    x = torch.ones(mib * 131072, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    reps = 10 if mib >= 256 else 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del x, y
    return round(2 * mib * 1048576 / dt / 1e9, 1)


def csr_halfsweep_bytes(n):
    """Algorithmic bytes of one red-black half-sweep on the 3D 27-point CSR
    operator, averaged over the two colours.  Colour-c launch: its rows'
    values (8 B) and column indices (4 B), row pointers and row->node map
    (4 B each), b and the new x of its rows (8 B each), and x of every
    unknown (8 B, read as neighbours)."""
    i = np.arange(1, n)
    cnt = 1 + (i > 1) + (i < n - 1)
    L = cnt[None, None, :] * cnt[None, :, None] * cnt[:, None, None]
    col = (i[None, None, :] + i[None, :, None] + i[:, None, None]) % 2
    NI = (n - 1) ** 3
    out = []
    for c in (0, 1):
        rows = int(np.sum(col == c))
        nnz = int(np.sum(L[col == c]))
        out.append(12 * nnz + 4 * (rows + 1) + 4 * rows + 16 * rows + 8 * NI)
    return sum(out) / 2.0, out


def stencil_halfsweep_bytes(n, s, kappa=False):
    """Algorithmic bytes of one red-black half-sweep on the 3D matrix-free
    stencil (s = 8 FP64, 4 FP32): x of every unknown, b and new x of the
    colour's unknowns, and (kappa) every cell coefficient once."""
    NI = (n - 1) ** 3
    b = s * NI + 2 * s * NI / 2.0
    if kappa:
        b += s * n ** 3
    return b


def measured_traffic(name):
    """HBM bytes per launch of the workload's finest-level half-sweep from the
    committed FETCH_SIZE / WRITE_SIZE record (profiles/traffic.md), scaled by
    the copy-kernel factors; None when the record is missing or the kernel
    sources have changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "traffic.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)```", text, re.S).group(1)).get(name)
    except (OSError, AttributeError, ValueError):
        return None
    if rec is None:
        return None
    for src, digest in rec["sources"].items():
        try:
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != digest:
                return None
        except OSError:
            return None
    return int(rec["bytes_per_launch"])


def roofline_csr(S, w, bd):
    from paper_1609_04809_amd.mg import PROF_SMOOTH
    S.profile(PROF_SMOOTH, True)
    _, k, _, st = S.solve(bd, w.tol)
    launches, ms = S.profile_read()
    S.profile(PROF_SMOOTH, False)
    avg_s = ms / 1e3 / launches
    per_launch, _ = csr_halfsweep_bytes(w.n)
    achieved = per_launch / avg_s / 1e9
    return {"bound": "hbm", "kernel": "k_csr_rows (red-black half-sweep, finest level)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(w.name),
            "launches": launches, "avg_us": round(avg_s * 1e6, 2),
            "bytes_per_launch": int(per_launch)}


def stencil_pair_bytes(n, s, kappa=False):
    """Algorithmic bytes of two red-black half-sweeps in one pass: x, b and
    the result of every unknown once (and every cell coefficient once)."""
    NI = (n - 1) ** 3
    return 3 * s * NI + (s * n ** 3 if kappa else 0)


def roofline_stencil(S, w, bd, s):
    """Finest-level smoothing kernels of one eager solve: single red-black
    half-sweeps that read the iterate (a step from x = 0 reads no x and is
    not counted) and half-sweep pairs, each timed with HIP events."""
    from paper_1609_04809_amd.mg import PROF_PAIR, PROF_SMOOTH
    out = {}
    for key, kid, per in (("halfsweep", PROF_SMOOTH,
                           stencil_halfsweep_bytes(w.n, s, kappa=w.kappa != "none")),
                          ("pair", PROF_PAIR, stencil_pair_bytes(w.n, s, kappa=w.kappa != "none"))):
        S.profile(kid, True)
        S.solve(bd, w.tol)
        launches, ms = S.profile_read()
        S.profile(kid, False)
        if launches == 0:
            continue
        avg_s = ms / 1e3 / launches
        ach = per / avg_s / 1e9
        out[key] = {"launches": launches, "avg_us": round(avg_s * 1e6, 2),
                    "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                    "bytes_per_launch": int(per)}
        if key == "halfsweep":
            out[key]["traffic"] = measured_traffic(w.name)
    if w.precision == "fp32_ir":
        # the first and last FP32 steps of each refinement cycle (the scaled
        # cast of the residual and the update of u fused in): timing only
        from paper_1609_04809_amd.mg import PROF_SMOOTH_IR
        S.profile(PROF_SMOOTH_IR, True)
        S.solve(bd, w.tol)
        launches, ms = S.profile_read()
        S.profile(PROF_SMOOTH_IR, False)
        if launches:
            out["ir_fused_steps"] = {"launches": launches,
                                     "avg_us": round(ms * 1e3 / launches, 2)}
    return out


def run_workload(name, steps, warmup, with_roofline=False, pcg=False, cycle="V",
                 smoother=None):
    """Time `steps` solves of a workload: the plain cycle iteration, or with
    pcg conjugate gradients preconditioned by one cycle per iteration; cycle
    V (the workload's), W or F; smoother the workload's or another one
    ("gs": multicolour Gauss-Seidel)."""
    import torch
    from paper_1609_04809_amd import workloads as W
    from paper_1609_04809_amd.mg import FLAG_PCG, Solver
    w = W.WORKLOADS[name]
    b, kappa, bd = _device_rhs(w)
    t0 = time.perf_counter()
    sm = smoother or w.smoother
    S = Solver(w.dim, w.n, w.levels, kappa=kappa, op=w.op, smoother=sm,
               nu_pre=w.nu_pre, nu_post=w.nu_post, omega=w.omega, precision=w.precision,
               flags=FLAG_PCG if pcg else 0, cycle=cycle)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    t, k, hist, u = time_solves(S, bd, w.tol, steps, warmup)
    res = {"workload": name, "dofs": w.dofs, "unknowns": w.unknowns,
           "MDOF_per_s": round(w.dofs / t / 1e6, 1), "ms_per_solve": round(t * 1e3, 3),
           "cycles": k, "final_rel_residual": hist[-1], "setup_s": round(setup_s, 3),
           "precision": w.precision, "op": w.op, "method": "pcg" if pcg else "cycle",
           "cycle": cycle, "smoother": sm}
    if with_roofline:
        med, mn = solve_spread(S, bd, w.tol, steps)
        res["ms_per_solve_median"] = round(med * 1e3, 3)
        res["ms_per_solve_min"] = round(mn * 1e3, 3)
    roof = None
    if pcg or cycle != "V" or sm != w.smoother:
        pass
    elif w.op == "csr":
        if with_roofline:
            roof = roofline_csr(S, w, bd)
    elif w.dim == 3:
        prof = roofline_stencil(S, w, bd, 8 if w.precision == "fp64" else 4)
        res.update(prof)
        key = "pair" if "pair" in prof else "halfsweep"
        if with_roofline and key in prof:
            hs = prof[key]
            roof = {"bound": "hbm",
                    "kernel": ("k_sweep3_pair (two red-black half-sweeps, finest level)"
                               if key == "pair" else
                               "k_sweep3 (red-black half-sweep, finest level)"),
                    "achieved": hs["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hs["frac"], "traffic": measured_traffic(w.name),
                    "avg_us": hs["avg_us"], "launches": hs["launches"],
                    "bytes_per_launch": hs["bytes_per_launch"],
                    "bytes_per_launch_basis": "x of every unknown, b and the new x of "
                                              "the colour's unknowns: 2 s N_I"
                                              + (" + s n^3 (kappa)" if w.kappa != "none"
                                                 else ""),
                    "model_bytes_3s_per_sweep": int(
                        1.5 * (8 if w.precision == "fp64" else 4) * w.unknowns
                        + ((8 if w.precision == "fp64" else 4) * w.n ** 3
                           if w.kappa != "none" else 0)),
                    "frac_of_model_bytes": None}
            m = roof["model_bytes_3s_per_sweep"]
            roof["frac_of_model_bytes"] = round(m / (hs["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                                4)
    S.close()
    if w.precision == "fp32_ir":
        # error of the FP32-inner / FP64-outer result against the FP64 V-cycle
        # solution of the same system (the FP64 path is the one the tests hold
        # to the oracle)
        S64 = Solver(w.dim, w.n, w.levels, kappa=kappa, op=w.op, smoother=w.smoother,
                     nu_pre=w.nu_pre, nu_post=w.nu_post, omega=w.omega, precision="fp64")
        u64, k64, _, st = S64.solve(bd, w.tol)
        S64.close()
        res["err_vs_fp64"] = float(torch.linalg.vector_norm(u - u64) /
                                   torch.linalg.vector_norm(u64))
        res["fp64_cycles"] = k64
    return res, roof, (b, kappa, u, k)


def run_heat(name, steps=None, precision=None, extrapolate=False):
    """The Crank-Nicolson time loop of the heat-equation model problem:
    `steps` steps (default the workload's: T = 5 in steps of 0.01), each a
    right-hand side and a solve warm-started from the previous step, timed
    as a whole with every input resident; each solve starts from the last
    step's solution, or with `extrapolate` from the linear extrapolation of
    the last two.  Also the finest-level half-sweep of the face-coupled
    operator timed with HIP events over one eager step, and the nodal error
    against the paper's exact solution at the end."""
    import torch
    from paper_1609_04809_amd import workloads as W
    from paper_1609_04809_amd.heat import HeatRun
    from paper_1609_04809_amd.mg import PROF_SMOOTH, PROF_SMOOTH_PRO
    w = W.HEAT_WORKLOADS[name]
    steps = steps or w.steps
    t0 = time.perf_counter()
    R = HeatRun(w, precision=precision, extrapolate=extrapolate)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    R.reset()
    R.step()                       # warm-up (captures the cycle graphs)
    R.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = R.run(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    exact = W.heat_gamma(R.t) * R.u0
    err = float((R.u - exact).abs().max() / exact.abs().max())
    s = 8 if (precision or w.precision) == "fp64" else 4
    per = stencil_halfsweep_bytes(w.n, s)
    prof = {}
    for key, kid in (("halfsweep", PROF_SMOOTH), ("prolong_fused", PROF_SMOOTH_PRO)):
        R.S.profile(kid, True)
        R.step()
        launches, ms = R.S.profile_read()
        R.S.profile(kid, False)
        if launches:
            avg = ms / 1e3 / launches
            prof[key] = {"launches": launches, "avg_us": round(avg * 1e6, 2)}
    hs = prof.get("halfsweep")
    if hs:
        ach = per / (hs["avg_us"] * 1e-6) / 1e9
        hs.update({"achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                   "bytes_per_launch": int(per),
                   "traffic": measured_traffic(f"{name}_{precision or w.precision}")})
    R.close()
    return {"workload": name, "dofs": w.dofs, "steps": steps, "dt": w.dt,
            "t_end": round(steps * w.dt, 6), "seconds": round(t, 3),
            "ms_per_step": round(t * 1e3 / steps, 3),
            "MDOF_steps_per_s": round(w.dofs * steps / t / 1e6, 1),
            "cycles_total": int(sum(its)), "cycles_per_step_mean": round(sum(its) / steps, 3),
            "cycles_per_step_min": int(min(its)), "cycles_per_step_max": int(max(its)),
            "tol": w.tol, "smoother": f"{w.smoother} V({w.nu_pre},{w.nu_post})",
            "levels": w.levels, "precision": precision or w.precision,
            "start": "extrapolated" if extrapolate else "previous step",
            "max_nodal_error_vs_exact": err, "setup_s": round(setup_s, 3), **prof}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(name, gpu_cycles):
    """The oracle (test infrastructure) on the same workload, on one host
    thread.  Assembled (CSR) workloads: one full solve.  Matrix-free
    workloads (256^3, 192^3): the first two cycles of the matrix-free oracle
    with their stopping residuals (about 10 s), timed and scaled by the
    GPU's cycle count (a full solve takes most of a minute).  Setup excluded
    from the timed region.  Returns (record, u_oracle_full_or_None,
    cycles_timed)."""
    import oracle as O
    from oracle import matfree as MF
    from paper_1609_04809_amd import workloads as W
    from threadpoolctl import threadpool_limits
    w = W.WORKLOADS[name]
    b, kappa = W.workload_inputs(w)
    with threadpool_limits(limits=1):
        if w.op == "csr":
            t0 = time.perf_counter()
            H = O.build_hierarchy(w.dim, w.n, w.levels, kappa=kappa, smoother=w.smoother,
                                  nu_pre=w.nu_pre, nu_post=w.nu_post, omega=w.omega)
            t_build = time.perf_counter() - t0
            t0 = time.perf_counter()
            u, k, hist, st = O.solve(H, b, w.tol)
            t_solve = time.perf_counter() - t0
            sample = (f"one full solve of {name} ({k} cycles, SciPy CSR matvec, one thread); "
                      f"assembly {t_build:.1f} s excluded")
            u_full, timed = W.interior_to_full(w.dim, w.n, u), k
        else:
            fp32 = w.precision == "fp32_ir"
            t0 = time.perf_counter()
            H = MF.build(w.dim, w.n, w.levels, kappa=kappa, smoother=w.smoother,
                         nu_pre=w.nu_pre, nu_post=w.nu_post, omega=w.omega, fp32=fp32)
            t_build = time.perf_counter() - t0
            bf = W.interior_to_full(w.dim, w.n, b).reshape((w.n + 1,) * w.dim)
            timed = min(2, gpu_cycles)
            t0 = time.perf_counter()
            for _, u1, rho1 in MF.iterate(H, bf, fp32=fp32, max_iter=timed):
                pass
            t_cycles = time.perf_counter() - t0
            t_solve = t_cycles / timed * gpu_cycles
            k = gpu_cycles
            sample = (f"the first {timed} cycles of {name} with their stopping residuals "
                      f"(matrix-free NumPy oracle, one thread, {t_cycles:.1f} s) scaled to "
                      f"the {gpu_cycles} cycles of the solve; setup {t_build:.1f} s excluded")
            u_full = u1.ravel()
    return {"value": round(w.dofs / t_solve / 1e6, 3), "unit": "MDOF/s", "cores": 1,
            "kind": "oracle", "sample": sample, "solve_s": round(t_solve, 2), "cycles": k,
            "os_cpu_count": os.cpu_count(), "threads_used": 1,
            "cpu_model": _cpu_model()}, u_full, timed


def gpu_after_cycles(name, cycles):
    """The GPU iterate after exactly `cycles` cycles (device full-grid tensor)."""
    import torch
    from paper_1609_04809_amd import workloads as W
    from paper_1609_04809_amd.mg import Solver
    w = W.WORKLOADS[name]
    b, kappa, bd = _device_rhs(w)
    with Solver(w.dim, w.n, w.levels, kappa=kappa, op=w.op, smoother=w.smoother,
                nu_pre=w.nu_pre, nu_post=w.nu_post, omega=w.omega, precision=w.precision,
                max_iter=cycles) as S:
        u, k, _, st = S.solve(bd, 1e-300)
        torch.cuda.synchronize()
    assert k == cycles, (k, st)
    return u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving runs")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--workload", default="poisson3d_256_rbgs_fp64")
    ap.add_argument("--heat-steps", type=int, default=0,
                    help="Crank-Nicolson steps of the heat workload (0: all 500)")
    ap.add_argument("--no-heat", action="store_true", help="skip the heat-equation time loop")
    ap.add_argument("--heat-extrapolate", action="store_true",
                    help="with --heat-only: start each solve from the extrapolated guess")
    ap.add_argument("--heat-only", default="",
                    help="run only the heat time loop in this precision (fp64 or fp32_ir) "
                         "and print its result (for profiling)")
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the reference device copy (attainable bandwidth; "
                         "also the known-size kernel that scales PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1609_04809_amd import workloads as W
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    if args.heat_only:
        copy_gbs = reference_copy(args.copy_mib)
        r = run_heat("heat3d_512_cn", args.heat_steps or None, precision=args.heat_only,
                     extrapolate=args.heat_extrapolate)
        log(f"[bench] heat3d_512_cn ({args.heat_only}): {r}")
        print(json.dumps({"heat": r, "copy_reference_GBs": copy_gbs}), flush=True)
        return
    name = args.workload
    w = W.WORKLOADS[name]
    copy_gbs = reference_copy(args.copy_mib)
    log(f"[bench] reference copy of {args.copy_mib} MiB: {copy_gbs} GB/s (read + write)")
    log(f"[bench] headline {name}: {args.warmup} warmup + {args.steps} timed solves")
    res, roof, (b, kappa, u, k) = run_workload(name, args.steps, args.warmup,
                                               with_roofline=True)
    if roof is not None and copy_gbs:
        # the same rate against the copy this GPU attains (read + write)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    log(f"[bench] {name}: {res['MDOF_per_s']} MDOF/s, {res['cycles']} cycles, "
        f"{res['ms_per_solve']} ms/solve; roofline {roof}")
    extra = []
    if not args.no_extra:
        for other in W.WORKLOADS:
            if other == name:
                continue
            r, _, _ = run_workload(other, max(3, args.steps // 4), 1)
            log(f"[bench] {other}: {r['MDOF_per_s']} MDOF/s, {r['cycles']} cycles, "
                f"{r['ms_per_solve']} ms/solve")
            extra.append(r)
        # the next row of the method: CG preconditioned by one cycle per
        # iteration, on the 3D workloads
        for other in W.WORKLOADS:
            if W.WORKLOADS[other].dim != 3:
                continue
            r, _, _ = run_workload(other, max(3, args.steps // 4), 1, pcg=True)
            log(f"[bench] {other} (pcg): {r['MDOF_per_s']} MDOF/s, {r['cycles']} iterations, "
                f"{r['ms_per_solve']} ms/solve")
            extra.append(r)
        # other cycle shapes on the CSR and the variable-coefficient workloads
        for other in ("poisson3d_128_csr_rbgs", "kappa3d_192_rbgs_ir"):
            for kind in ("W", "F"):
                r, _, _ = run_workload(other, max(3, args.steps // 4), 1, cycle=kind)
                log(f"[bench] {other} ({kind}-cycle): {r['MDOF_per_s']} MDOF/s, "
                    f"{r['cycles']} cycles, {r['ms_per_solve']} ms/solve")
                extra.append(r)
        # multicolour Gauss-Seidel in place of the red-black smoother
        for other in ("poisson3d_128_csr_rbgs", "poisson3d_256_rbgs_fp64"):
            r, _, _ = run_workload(other, max(3, args.steps // 4), 1, smoother="gs")
            log(f"[bench] {other} (multicolour GS): {r['MDOF_per_s']} MDOF/s, "
                f"{r['cycles']} cycles, {r['ms_per_solve']} ms/solve")
            extra.append(r)
    heat = None
    if not args.no_extra and not args.no_heat:
        heat = []
        for prec, ex in (("fp64", False), ("fp64", True), ("fp32_ir", True)):
            r = run_heat("heat3d_512_cn", args.heat_steps or None, precision=prec, extrapolate=ex)
            log(f"[bench] heat3d_512_cn ({prec}, {r['start']}): {r['steps']} steps in "
                f"{r['seconds']} s, "
                f"{r['ms_per_step']} ms/step, {r['cycles_per_step_mean']} cycles/step, "
                f"error vs exact {r['max_nodal_error_vs_exact']:.3e}; {r.get('halfsweep')}")
            heat.append(r)
    serving = None
    if not args.no_serve:
        from paper_1609_04809_amd import serve_load
        nreq = args.serve_requests
        trace = W.serving_trace(num=nreq, rate=200.0, seed=0)
        log(f"[bench] serving: {nreq} requests, Poisson arrivals at 200/s")
        serving = {"poisson_arrivals_200_per_s": serve_load.run_trace(trace, 64 << 30, 64,
                                                                       log=log)}
        log(f"[bench] serving: {serving['poisson_arrivals_200_per_s']}")
        burst = W.serving_trace(num=nreq, rate=200.0, seed=0, burst=True)
        serving["burst_all_at_t0"] = serve_load.run_trace(burst, 64 << 30, 64, log=log)
        log(f"[bench] serving burst: {serving['burst_all_at_t0']}")
        serving["burst_2GiB_budget"] = serve_load.run_trace(burst[: max(1, nreq // 5)],
                                                            2 << 30, 64, log=log)
        log(f"[bench] serving small budget: {serving['burst_2GiB_budget']}")
        # the same arrivals with a quarter of the requests variable-coefficient
        mixed = W.serving_trace(num=nreq, rate=200.0, seed=0, kappa_frac=0.25)
        serving["poisson_arrivals_200_per_s_kappa_25pct"] = serve_load.run_trace(
            mixed, 64 << 30, 64, log=log)
        log(f"[bench] serving with kappa: {serving['poisson_arrivals_200_per_s_kappa_25pct']}")
    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        cpu, u_or, k_or = cpu_baseline(name, res["cycles"])
        ug = u.cpu().numpy() if k_or == res["cycles"] else \
            gpu_after_cycles(name, k_or).cpu().numpy()
        cpu["gpu_vs_oracle_rel_err"] = float(np.linalg.norm(ug - u_or) / np.linalg.norm(u_or))
        cpu["gpu_vs_oracle_after_cycles"] = k_or
        log(f"[bench] CPU oracle: {cpu}")
    out = {
        "metric": "MDOF/s solved to 1e-8 rel. residual",
        "value": res["MDOF_per_s"],
        "unit": "MDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_solve"],
        "ms_per_step_median_single": res.get("ms_per_solve_median"),
        "ms_per_step_min_single": res.get("ms_per_solve_min"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "dim": w.dim, "n": w.n, "levels": w.levels,
                   "dofs": w.dofs, "operator": w.op, "smoother": f"{w.smoother} V(2,2)",
                   "precision": w.precision, "tol": w.tol,
                   "rhs": {"uniform": f"U[-1,1] seed {w.seed}", "ones": "f = 1 (b = h^3)",
                           "manufactured": "exact load of u = sin(pi x) sin(pi y)"}[w.rhs],
                   "kappa": "exp(N(0,1)) per cell" if w.kappa != "none" else "1",
                   "cycles": res["cycles"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "copy_reference_GBs": copy_gbs,
        "extra": extra,
        "heat": heat,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
