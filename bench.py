#!/usr/bin/env python3
"""Benchmark of the space-time inexact Uzawa solver on one MI355X.

Workload: 2-D heat equation, 255 x 255 interior nodes, N_t = 256 steps, T = 1,
kappa = 1 + 0.5 sin(2 pi t) cos(pi x), source = 8 space-time Gaussians,
u0 = random sine modes (k <= 16); seeded synthetic data.  The GPU path runs
in float64 (the workload's precision); the float32-preconditioner variant is
reported next to it.

A step is one inexact Uzawa iteration (eq. (3.1)) over all N_t slabs: both
residuals, the A-tilde^{-1} V-cycles, the two DSTs and the H-tilde^{-1}
V-cycles.  K steps are timed as one solve with tol = 0 and max_iter = K (K
updates plus the final residual evaluation).  Inputs are resident in HBM
before the timed region starts.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# HBM traffic per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (calibrated
# against a plain copy) for (workload, dtype, kernel, level); valid only while the
# kernel sources hash to the recorded value (see the named profile).
MEASURED_TRAFFIC = {
    ("heat2d_255_N256", "f64", "k_mg_down", 0): dict(
        bytes=183612010, sources_sha256="16c5e93e3f193a1e500494084853e1943c9b70a17f046f3513e2a95b72c50181",
        profile="profiles/heat2d_255_N256_f64_mg_down_L0_traffic.md"),
}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("stp_kernels.h", "stp_tiles.h", "stp.hip"):
        with open(os.path.join(ROOT, "paper_1802_08126_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def algorithmic_bytes(kernel: str, level: int, dims, ts: int) -> float | None:
    """Minimum HBM bytes one launch of ``kernel`` must move (every input read
    once, every output written once), for the solver's level sizes.

    dims: dict with N (slabs), npts per level list, nnodes per level list, R.
    """
    N = dims["N"]
    npts = dims["npts"]
    nn = dims["nnodes"]
    R = dims["R"]
    tc = 8 if ts == 8 else 4
    n_l = npts[level] if level < len(npts) else None
    kap = lambda l, b: R * nn[l] * b  # noqa: E731
    k = kernel.split("<")[0]
    add64 = "add64" in kernel
    if k == "k_resid_tile":        # u, p, F in; r out (the other slab's u, p rows are the same arrays)
        return N * npts[0] * (3 * 8 + ts) + kap(0, 8)
    if k == "k_mg_down":           # b in (fine), bc out (coarse)
        return N * (n_l + npts[level + 1]) * ts + kap(level, tc)
    if k == "k_mg_up":
        if add64:                  # b, e in; float64 p read and written
            return N * (n_l + npts[level + 1]) * ts + N * n_l * 16 + kap(level, tc)
        return N * (2 * n_l + npts[level + 1]) * ts + kap(level, tc)
    if k == "k_apply_tile":
        return N * n_l * 2 * ts + kap(level, tc)
    if k in ("k_time_fft", "k_time_fft2", "k_time_dense"):   # one step-count group (level = group 0)
        if add64:                  # in (TS); float64 u read and written
            return N * npts[0] * (ts + 16)
        return N * npts[0] * 2 * ts
    return None


def gpu_run(args):
    import numpy as np
    import torch

    import paper_1802_08126_amd as stp
    import synth

    torch.cuda.set_device(0)
    prob = synth.CONFIG_BUILDERS[args.workload]()
    dev = "cuda:0"
    kf = torch.as_tensor(np.ascontiguousarray(prob.kfields), dtype=torch.float64, device=dev)
    F = torch.as_tensor(np.ascontiguousarray(prob.F), dtype=torch.float64, device=dev)
    u0 = torch.as_tensor(np.ascontiguousarray(prob.u0), dtype=torch.float64, device=dev)
    shape = (prob.N,) + (prob.n,) * prob.dim
    dofs = prob.N * prob.npts
    levels = []
    n = prob.n
    while True:
        levels.append(n)
        if n == 1 or prob.dim == 1:
            break
        n = (n - 1) // 2
    dims = dict(N=prob.N, R=prob.R, npts=[m ** prob.dim for m in levels] + [1],
                nnodes=[(m + 2) ** prob.dim for m in levels] + [1])
    results = {}
    for prec in (["f64", "f32"] if not args.only_f64 else ["f64"]):
        s = stp.SpaceTimeSolver(prob.dim, prob.n, prob.N, prob.tau, kf, prob.tcoef, F, u0,
                                precision=prec, omega=args.omega, tol=0.0, max_iter=args.warmup,
                                check_every=args.check_every)
        u = torch.zeros(shape, dtype=torch.float64, device=dev)
        p = torch.zeros(shape, dtype=torch.float64, device=dev)
        tune = None
        if not args.no_tune:
            # the library's autotuner picks slabs per block and the time-transform path
            heuristic = s.schedule()
            t0 = time.perf_counter()
            tune = s.autotune(reps=5, use_cache=False)
            tune.update(sec=time.perf_counter() - t0, schedule=s.schedule(), heuristic=heuristic)
        # warmup
        s.solve(u, p)
        torch.cuda.synchronize()
        # timed region: exactly --steps iterations (each replayed as a captured HIP graph)
        s.close()
        s = stp.SpaceTimeSolver(prob.dim, prob.n, prob.N, prob.tau, kf, prob.tcoef, F, u0,
                                precision=prec, omega=args.omega, tol=0.0, max_iter=args.steps,
                                check_every=args.check_every)
        if tune is not None:
            assert s.autotune(use_cache=True)["from_cache"]
        u.zero_()
        p.zero_()
        s.solve(u, p)                        # captures the iteration graph for (u, p)
        u.zero_()
        p.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = s.solve(u, p)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert info["iters"] == args.steps, info
        sec = t1 - t0
        results[prec] = dict(sec=sec, ms_per_step=1e3 * sec / args.steps, value=dofs * args.steps / sec,
                             device_ms=info["ms"], autotune=tune, omega=info["omega"])
        if prec == "f64":
            # per-kernel device times: a second timed region of the same --steps
            # iterations, launched eagerly with a HIP event pair around every launch
            u.zero_()
            p.zero_()
            s.timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve(u, p)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            results[prec]["kernels"] = s.timing_report()
            results[prec]["ms_per_step_eager_timed"] = 1e3 * (t1 - t0) / args.steps
            s.timing(False)
        s.close()
        # time to tolerance from a zero guess
        if not args.skip_tol:
            s = stp.SpaceTimeSolver(prob.dim, prob.n, prob.N, prob.tau, kf, prob.tcoef, F, u0,
                                    precision=prec, omega=args.omega, tol=args.tol, max_iter=2000,
                                    check_every=args.check_every)
            if tune is not None:
                s.autotune(use_cache=True)
            u.zero_()
            p.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = s.solve(u, p)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            results[prec]["tol"] = dict(tol=args.tol, iters=info["iters"], sec=t1 - t0, rel_res=info["rel_res"],
                                        status=info["status"])
            # the same stop test reached with GMRES(restart) around the Uzawa sweep
            # (workspace allocated outside the timed region; second of two runs)
            nb = stp.stp_gmres_workspace_bytes(s.ctx, args.gmres_restart)
            ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=dev)
            for _ in range(2):
                u.zero_()
                p.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, gi = s.gmres(u, p, restart=args.gmres_restart, workspace=ws)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
            results[prec]["gmres"] = dict(tol=args.tol, restart=args.gmres_restart, steps=gi["iters"],
                                          sec=t1 - t0, ms_per_step=1e3 * (t1 - t0) / max(gi["iters"], 1),
                                          rel_res=gi["rel_res"], status=gi["status"])
            progress(f"{prec}: gmres to tol", f"{gi['iters']} steps {t1 - t0:.3f}s")
            del ws
            s.close()
            # the same stop test with two V-cycles per H~_k^{-1} (nu_H = 2; second of two runs)
            s = stp.SpaceTimeSolver(prob.dim, prob.n, prob.N, prob.tau, kf, prob.tcoef, F, u0,
                                    precision=prec, omega=args.omega, tol=args.tol, max_iter=2000,
                                    check_every=args.check_every, nu_H=2)
            if tune is not None:
                s.autotune(use_cache=True)
            for _ in range(2):
                u.zero_()
                p.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, info = s.solve(u, p)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
            results[prec]["tol_nuH2"] = dict(tol=args.tol, nu_H=2, iters=info["iters"], sec=t1 - t0,
                                             rel_res=info["rel_res"], status=info["status"], omega=info["omega"])
            progress(f"{prec}: uzawa nu_H=2 to tol", f"{info['iters']} its {t1 - t0:.3f}s")
            s.close()
    return prob, dims, results


def progress(*a):
    """Progress lines go to stderr; stdout carries only the JSON result."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def batch_inputs(count, seed, device):
    """The mixed-size batch workload on the device.  Coefficients, initial data
    and the source's separable Gaussian factors come from the seeded generator;
    the source is assembled on the device from those factors in the
    generator's own operation order (identical values)."""
    import torch

    import synth

    specs = synth.batch2d(count=count, seed=seed)
    probs = []
    for sp in specs:
        kf, tc, factors, u0 = synth.batch2d_parts(sp)
        n, N = sp["side"], sp["N"]
        F = torch.zeros((N, n, n), dtype=torch.float64, device=device)
        for gt, (gx, gy) in factors:
            G = torch.as_tensor(gy, device=device)[:, None] * torch.as_tensor(gx, device=device)[None, :]
            F += torch.as_tensor(gt, device=device)[:, None, None] * G[None]
        probs.append(dict(dim=2, n=n, N=N, tau=1.0 / N, tcoef=tc, F=F,
                          kfields=torch.as_tensor(kf, dtype=torch.float64, device=device),
                          u0=torch.as_tensor(u0, dtype=torch.float64, device=device)))
    return specs, probs


def batch_run(args):
    """64 independent 2-D problems: one batched context (merged launches, one
    graph per iteration) against a loop of 64 single-problem contexts."""
    import torch

    import paper_1802_08126_amd as stp

    dev = "cuda:0"
    t0 = time.perf_counter()
    specs, probs = batch_inputs(64, 1004, dev)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    dofs = sum(q["N"] * q["n"] ** 2 for q in probs)
    shapes = [(q["N"], q["n"], q["n"]) for q in probs]
    us = [torch.zeros(sh, dtype=torch.float64, device=dev) for sh in shapes]
    ps = [torch.zeros(sh, dtype=torch.float64, device=dev) for sh in shapes]
    K = args.batch_steps
    out = dict(problems=len(probs), dofs=dofs, sides=sorted({q["n"] for q in probs}),
               N_range=[min(q["N"] for q in probs), max(q["N"] for q in probs)], steps=K,
               input_setup_s=setup_s)

    def zero():
        for t in us + ps:
            t.zero_()
        torch.cuda.synchronize()

    def timed_batch(b):
        zero()
        b.solve(us, ps)                        # captures the graph
        zero()
        t0 = time.perf_counter()
        _, _, infos, _ = b.solve(us, ps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos

    omegas = None
    for prec in ("f32", "f64"):
        # the damping is estimated once per problem (first context) and set on the others
        b = stp.BatchSolver(probs, precision=prec, omega=args.omega if omegas is None else 1.0, tol=0.0,
                            max_iter=K, check_every=K + 1)
        if omegas is None:
            omegas = b.omegas()
            out["omega"] = dict(min=min(omegas), max=max(omegas), source="estimated" if args.omega <= 0 else "given")
        else:
            b.set_omegas(omegas)
        sec, infos = timed_batch(b)
        assert all(i["iters"] == K for i in infos)
        r = dict(batch_heuristic=dict(sec=sec, value=dofs * K / sec))
        t0 = time.perf_counter()
        tune = b.autotune(reps=2, use_cache=False)
        tune["sec"] = time.perf_counter() - t0
        sec, _ = timed_batch(b)
        r["batch_tuned"] = dict(sec=sec, value=dofs * K / sec, autotune=tune)
        b.close()
        # loop of single-problem contexts, built-in schedule, graph replay each
        ss = [stp.SpaceTimeSolver(2, q["n"], q["N"], q["tau"], q["kfields"], q["tcoef"], q["F"], q["u0"],
                                  precision=prec, omega=omegas[i], tol=0.0, max_iter=K, check_every=K + 1)
              for i, q in enumerate(probs)]
        zero()
        for i, sv in enumerate(ss):
            sv.solve(us[i], ps[i])
        zero()
        t0 = time.perf_counter()
        for i, sv in enumerate(ss):
            sv.solve(us[i], ps[i])
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        r["loop_heuristic"] = dict(sec=sec, value=dofs * K / sec)
        for sv in ss:
            sv.close()
        r["batching_speedup"] = r["batch_heuristic"]["value"] / r["loop_heuristic"]["value"]
        out[prec] = r
        progress("batch:", prec, {k: round(v["value"] / 1e9, 3) for k, v in r.items() if isinstance(v, dict)})
    if not args.skip_tol:
        # time to a 1e-8 residual for every problem: mixed-precision batch (tuned)
        # against a loop of plain float64 single-problem solves
        b = stp.BatchSolver(probs, precision="f32", omega=1.0, tol=args.tol, max_iter=2000,
                            check_every=args.check_every)
        b.set_omegas(omegas)
        b.autotune(reps=2, use_cache=True)
        zero()
        t0 = time.perf_counter()
        _, _, infos, status = b.solve(us, ps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        b.close()
        its = [i["iters"] for i in infos]
        progress("batch: f32 batch to tol", f"{tb:.2f}s")
        ss = [stp.SpaceTimeSolver(2, q["n"], q["N"], q["tau"], q["kfields"], q["tcoef"], q["F"], q["u0"],
                                  precision="f64", omega=omegas[i], tol=args.tol, max_iter=2000,
                                  check_every=args.check_every) for i, q in enumerate(probs)]
        zero()
        t0 = time.perf_counter()
        its64 = []
        for i, sv in enumerate(ss):
            _, _, info = sv.solve(us[i], ps[i])
            its64.append(info["iters"])
        torch.cuda.synchronize()
        tl = time.perf_counter() - t0
        for sv in ss:
            sv.close()
        progress("batch: f64 loop to tol", f"{tl:.2f}s")
        out["time_to_tol"] = dict(tol=args.tol, batch_f32_sec=tb, batch_status=status,
                                  batch_iters=[min(its), max(its)], loop_f64_sec=tl,
                                  loop_f64_iters=[min(its64), max(its64)],
                                  speedup_vs_loop_f64=tl / tb)
        # the mixed-precision batch with two V-cycles per H~_k^{-1} (each problem's
        # damping estimated for that preconditioner at setup)
        b = stp.BatchSolver(probs, precision="f32", omega=0.0, tol=args.tol, max_iter=2000,
                            check_every=args.check_every, nu_H=2)
        b.autotune(reps=2, use_cache=True)
        zero()
        t0 = time.perf_counter()
        _, _, infos, status = b.solve(us, ps)
        torch.cuda.synchronize()
        tb2 = time.perf_counter() - t0
        b.close()
        its = [i["iters"] for i in infos]
        progress("batch: f32 nu_H=2 batch to tol", f"{tb2:.2f}s")
        out["time_to_tol"].update(batch_f32_nuH2_sec=tb2, batch_nuH2_status=status,
                                  batch_nuH2_iters=[min(its), max(its)], speedup_nuH2_vs_loop_f64=tl / tb2)
    return out


def heat3d_run(args):
    """3-D heat, 127^3 interior nodes, N_t = 128, lognormal kappa (contrast 1e2)
    times (1 + 0.3 t), Gaussian source: time to ||f - B u|| <= 1e-10 ||f|| from a
    zero guess, Uzawa and GMRES(restart), with float64, float32 and
    bfloat16-storage preconditioners (outer residuals and updates in float64),
    and the float32 preconditioner with two V-cycles per H~_k^{-1}.  Each solve
    runs twice; the second is reported."""
    import torch

    import paper_1802_08126_amd as stp
    import synth

    prob = synth.CONFIG_BUILDERS["heat3d_127_N128_lognormal"]()
    dofs = prob.N * prob.npts
    dev = "cuda:0"
    kf = torch.as_tensor(prob.kfields, dtype=torch.float64, device=dev)
    F = torch.as_tensor(prob.F, dtype=torch.float64, device=dev)
    u0 = torch.as_tensor(prob.u0, dtype=torch.float64, device=dev)
    shape = (prob.N,) + (prob.n,) * prob.dim
    u = torch.zeros(shape, dtype=torch.float64, device=dev)
    p = torch.zeros_like(u)
    out = dict(workload="heat3d_127_N128_lognormal", dofs=dofs, tol=args.tol3d, restart=args.gmres_restart)
    # f32_nuH2: float32 preconditioner with two V-cycles per H~_k^{-1} (nu_H = 2)
    for key in ("f64", "f32", "bf16", "f32_nuH2"):
        prec = key.split("_")[0]
        s = stp.SpaceTimeSolver(prob.dim, prob.n, prob.N, prob.tau, kf, prob.tcoef, F, u0, precision=prec,
                                omega=0.0, tol=args.tol3d, max_iter=3000, check_every=args.check_every,
                                nu_H=2 if key.endswith("nuH2") else 1)
        s.autotune(reps=3)
        r = dict(omega=s.omega_info()["omega"])
        for _ in range(2):
            u.zero_()
            p.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = s.solve(u, p)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        r["uzawa"] = dict(iters=info["iters"], sec=t1 - t0, rel_res=info["rel_res"], status=info["status"],
                          dof_it_per_s=dofs * info["iters"] / (t1 - t0))
        progress(f"3-D {key}: uzawa to tol", f"{info['iters']} its {t1 - t0:.2f}s")
        nb = stp.stp_gmres_workspace_bytes(s.ctx, args.gmres_restart)
        ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=dev)
        for _ in range(2):
            u.zero_()
            p.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, gi = s.gmres(u, p, restart=args.gmres_restart, workspace=ws)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        r["gmres"] = dict(steps=gi["iters"], sec=t1 - t0, rel_res=gi["rel_res"], status=gi["status"])
        progress(f"3-D {key}: gmres to tol", f"{gi['iters']} steps {t1 - t0:.2f}s")
        del ws
        s.close()
        out[key] = r
    for prec in ("f32", "bf16", "f32_nuH2"):
        out[prec]["uzawa_speedup_vs_f64"] = out["f64"]["uzawa"]["sec"] / out[prec]["uzawa"]["sec"]
        out[prec]["best_speedup_vs_f64_uzawa"] = out["f64"]["uzawa"]["sec"] / min(out[prec]["uzawa"]["sec"],
                                                                                   out[prec]["gmres"]["sec"])
    return out


def paper83_run(args):
    """The 3-D problem of the paper's time-parallel experiments (Section 8.3,
    Tables 3 and 4) in finite-difference form on one GPU: 15^3 interior nodes
    (the paper's 16^3-cell mesh), T = 0.1, kappa = 1, F = 0, u0 = sin sin sin
    (exact solution exp(-3 pi^2 t) sin sin sin); time to ||f - B u|| <= 1e-8 ||f||
    from zero with Uzawa and GMRES(restart) for growing N (the weak-scaling
    direction of Table 3), float64, and float32 preconditioners at the largest
    N.  The paper's numbers (Q1 elements, hypre AMG, GMRES-accelerated Uzawa,
    Vulcan BlueGene/Q) are context only."""
    import torch

    import paper_1802_08126_amd as stp
    import synth

    out = dict(workload="heat3d_sine_15", tol=1e-8, restart=args.gmres_restart,
               paper_context=dict(source="Tables 3-4", machine="Vulcan BlueGene/Q", procs=4096, N=65536,
                                  iters=22, sec_per_iter=1.87, total_sec=41.09,
                                  method="GMRES-accelerated inexact Uzawa, Q1 FEM, hypre AMG, FFTW3"),
               runs=[])
    for N, prec in ((1024, "f64"), (16384, "f64"), (65536, "f64"), (65536, "f32")):
        prob = synth.heat3d_sine(N=N)
        dev = "cuda:0"
        kf = torch.as_tensor(prob.kfields, dtype=torch.float64, device=dev)
        F = torch.zeros((N,) + (prob.n,) * 3, dtype=torch.float64, device=dev)
        u0 = torch.as_tensor(prob.u0, dtype=torch.float64, device=dev)
        s = stp.SpaceTimeSolver(3, prob.n, N, prob.tau, kf, prob.tcoef, F, u0, precision=prec, omega=0.0,
                                tol=1e-8, max_iter=2000, check_every=args.check_every)
        s.autotune(reps=3)
        r = dict(N=N, precision=prec, dofs=N * prob.npts, omega=s.omega_info()["omega"])
        u = torch.zeros((N,) + (prob.n,) * 3, dtype=torch.float64, device=dev)
        p = torch.zeros_like(u)
        for _ in range(2):
            u.zero_()
            p.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = s.solve(u, p)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        r["uzawa"] = dict(iters=info["iters"], sec=t1 - t0, sec_per_iter=(t1 - t0) / max(info["iters"], 1),
                          rel_res=info["rel_res"], status=info["status"])
        nb = stp.stp_gmres_workspace_bytes(s.ctx, args.gmres_restart)
        ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=dev)
        for _ in range(2):
            u.zero_()
            p.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, gi = s.gmres(u, p, restart=args.gmres_restart, workspace=ws)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        r["gmres"] = dict(steps=gi["iters"], sec=t1 - t0, sec_per_step=(t1 - t0) / max(gi["iters"], 1),
                          rel_res=gi["rel_res"], status=gi["status"])
        progress(f"sec8.3 N={N} {prec}", f"uzawa {r['uzawa']['iters']} its {r['uzawa']['sec']:.2f}s, "
                 f"gmres {gi['iters']} steps {t1 - t0:.2f}s")
        del ws, u, p, F
        s.close()
        out["runs"].append(r)
    return out


def roofline(rep, dims, ts, steps, workload="heat2d_255_N256", dtype="f64"):
    """Dominant kernel (largest summed device time) and its achieved HBM rate."""
    if not rep:
        return None, []
    rep = sorted(rep, key=lambda r: -r["total_ms"])
    total = sum(r["total_ms"] for r in rep)
    top = rep[0]
    b = algorithmic_bytes(top["kernel"], top["level"], dims, ts)
    table = [dict(kernel=r["kernel"], level=r["level"], launches=r["launches"], avg_us=1e3 * r["avg_ms"],
                  share=r["total_ms"] / total) for r in rep[:12]]
    if b is None:
        return None, table
    achieved = b / (top["avg_ms"] * 1e-3) / 1e9
    traffic, src = None, None
    m = MEASURED_TRAFFIC.get((workload, dtype, top["kernel"], top["level"]))
    if m is not None and m["sources_sha256"] == kernel_sources_sha256():
        traffic, src = m["bytes"], m["profile"]
    return dict(bound="hbm", kernel=top["kernel"], level=top["level"], achieved=achieved, peak=HBM_PEAK_GBS,
                unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=traffic, traffic_unit="bytes per launch",
                traffic_source=src, bytes_per_launch=b, avg_launch_us=1e3 * top["avg_ms"]), table


def cpu_baseline(workload, iters=3):
    """The oracle's inexact Uzawa iteration timed on the host (``iters``
    iterations after its setup, about 10 s on the 2-D workload)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import uzawa

    prob = synth.CONFIG_BUILDERS[workload]()
    stamps = []

    def cb(j, u, p, r):
        stamps.append(time.perf_counter())
    with threadpool_limits(limits=1):
        uzawa.uzawa(prob, omega=0.8, tol=0.0, max_iter=iters, callback=cb)
    sec = float(stamps[-1] - stamps[0])
    n_it = len(stamps) - 1
    return dict(value=prob.N * prob.npts * n_it / sec, unit="DoF-it/s", cores=1, kind="oracle",
                sample=f"{n_it} inexact Uzawa iterations of the CPU float64 oracle (numpy, 1 thread) on "
                       f"{workload}: {sec:.1f} s")


# ---------------------------------------------------------------------------
# hardware-counter profiles (rocprofv3 output of this script)
# ---------------------------------------------------------------------------
COPY_ELEMS = 16646400   # float64 values in one slab-vector of heat2d_255_N256


def copy_calibration():
    """A plain device copy of a known size, profiled with the same counters as
    the solver so that FETCH_SIZE / WRITE_SIZE can be scaled to bytes."""
    import torch
    a = torch.randn(COPY_ELEMS, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=COPY_ELEMS * 8, copies=3)), flush=True)


# launches that precede a level-0 multigrid down-sweep of the 2-D float64 solver:
# the r_p residual, the forward transform and the middle operator
_L0_PRED = ("k_resid_tile<2, double, 0,", "k_time_fft2<double, double, 0, 0,", "k_apply_tile<")


def _kname(r):
    return r["Kernel_Name"].split("(")[0].replace("void ", "").replace("stp::", "")


def summarize_profile(d, steps):
    """Markdown summary of rocprofv3 output of this script under d: the
    --stats table (trace/), the level-0 down-sweep launches of the two timed
    solves (graph replays, then eager launches; 3 steps + 1 each, picked by
    their predecessor), and, when the counter passes are there, their HBM bytes
    from FETCH_SIZE (p1/) and WRITE_SIZE (p2/) scaled by the copy calibration
    passes (c1/, c2/).  Every run was made with --steps `steps`, --only-f64,
    --skip-tol, --no-batch and --no-3d, so those solves are the last launches."""
    import csv

    def rows(sub, f):
        with open(os.path.join(d, sub, f)) as fh:
            return list(csv.DictReader(fh))

    def l0(seq):
        sel = [b for a, b in zip(seq, seq[1:]) if b[0].startswith("k_mg_down<") and a[0].startswith(_L0_PRED)]
        return sel[-2 * (3 * steps + 1):]

    avg = lambda v: sum(v) / len(v)
    print("## rocprofv3 --stats (run_kernel_stats.csv, all dispatches of the run)\n")
    print("| kernel | calls | avg us | min us | max us | % |\n|---|---|---|---|---|---|")
    for r in rows("trace", "run_kernel_stats.csv")[:18]:
        print(f"| `{r['Name'].split('(')[0].replace('void ', '')}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {r['Percentage']} |")
    tr = sorted(rows("trace", "run_kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    t = [x[1] for x in l0([(_kname(r), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3) for r in tr])]
    print("\n## Level-0 multigrid down-sweep\n")
    print("Launches of `k_mg_down` that directly follow the r_p residual, the forward time transform or")
    print("the middle operator (the level-0 down-sweeps of the three V-cycles of an iteration), in the")
    print(f"two timed solves of {steps} iterations with the tuned schedule:\n")
    print(f"| launches | avg us | min us | max us |\n|---|---|---|---|\n| {len(t)} | {avg(t):.1f} | {min(t):.1f} | "
          f"{max(t):.1f} |")
    if not os.path.isdir(os.path.join(d, "p1")):
        return
    res = {}
    for i, cn in ((1, "FETCH_SIZE"), (2, "WRITE_SIZE")):
        pm = sorted(rows(f"p{i}", "run_counter_collection.csv"), key=lambda r: int(r["Dispatch_Id"]))
        v = l0([(_kname(r), float(r["Counter_Value"])) for r in pm if r["Counter_Name"] == cn])
        cal = [float(r["Counter_Value"]) for r in rows(f"c{i}", "run_counter_collection.csv")
               if "copy" in r["Kernel_Name"].lower() and int(r["Grid_Size"]) > 100000 and r["Counter_Name"] == cn]
        factor = COPY_ELEMS * 8 / (avg(cal) * 1024)
        kib = avg([x[1] for x in v])
        res[cn] = (len(v), kib, avg(cal), factor, kib * 1024 * factor)
    f, w = res["FETCH_SIZE"], res["WRITE_SIZE"]
    print("\n## HBM traffic of the level-0 down-sweep\n")
    print(f"Calibration: a copy of {COPY_ELEMS * 8:,} bytes reads FETCH_SIZE = {f[2]:,.1f} KiB and WRITE_SIZE = "
          f"{w[2]:,.1f} KiB per dispatch, so bytes = FETCH_SIZE x 1024 x {f[3]:.3f} and WRITE_SIZE x 1024 x "
          f"{w[3]:.3f}.\n")
    print("| quantity | per launch |\n|---|---|")
    print(f"| dispatches selected | {f[0]} (FETCH_SIZE run), {w[0]} (WRITE_SIZE run) |")
    print(f"| FETCH_SIZE (KiB, raw) | {f[1]:,.1f} |\n| WRITE_SIZE (KiB, raw) | {w[1]:,.1f} |")
    print(f"| HBM bytes read | {f[4]:,.0f} |\n| HBM bytes written | {w[4]:,.0f} |")
    print(f"| traffic (read + written) | {f[4] + w[4]:,.0f} |")
    print(f"\nKernel sources at measurement (sha256 of stp_kernels.h + stp_tiles.h + stp.hip):\n"
          f"{kernel_sources_sha256()}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="heat2d_255_N256")
    ap.add_argument("--omega", type=float, default=0.0, help="Uzawa damping; <= 0: estimated by the library")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-tol", action="store_true")
    ap.add_argument("--only-f64", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in schedule heuristic")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batch workload")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--gmres-restart", type=int, default=10)
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D lognormal time-to-tolerance runs")
    ap.add_argument("--tol3d", type=float, default=1e-10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of one slab-vector (counter calibration)")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="only summarise rocprofv3 output under DIR (no GPU use)")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.steps)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; sharding the time slabs over several GPUs is a design, "
              "not an implementation.  Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    prob, dims, res = gpu_run(args)
    progress("workload done:", args.workload)
    r64 = res["f64"]
    roof, table = roofline(r64.get("kernels"), dims, 8, args.steps, args.workload, "f64")
    out = {
        "metric": "space-time DoF-iterations/sec + time to 1e-8 residual, mixed vs FP64, 1 GPU",
        "metric_note": "value: u DoFs x Uzawa iterations / s, float64; time to 1e-8: time_to_tol_f64 "
                       "and mixed_f32_precond.time_to_tol (one V-cycle per spatial solve, the default); "
                       "nuH2_time_to_tol_f64 and mixed_f32_precond.nuH2_time_to_tol with two per H-block",
        "value": r64["value"],
        "unit": "DoF-it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": prob.dim, "n_interior": prob.n, "N_t": prob.N,
                   "dofs": prob.N * prob.npts, "omega": r64["omega"],
                   "omega_source": "estimated" if args.omega <= 0 else "given", "spatial": "mg V(1,1) Jacobi",
                   "parallelism": "all time slabs batched in every launch"},
        "roofline": roof,
        "kernels_f64": table,
        "ms_per_step_eager_timed": r64.get("ms_per_step_eager_timed"),
        "autotune_f64": r64.get("autotune"),
    }
    if "tol" in r64:
        out["time_to_tol_f64"] = r64["tol"]
        out["gmres_time_to_tol_f64"] = r64["gmres"]
        out["nuH2_time_to_tol_f64"] = r64["tol_nuH2"]
    if "f32" in res:
        r32 = res["f32"]
        out["mixed_f32_precond"] = {"value": r32["value"], "ms_per_step": r32["ms_per_step"],
                                    "dtype": "f32 preconditioner / f64 outer",
                                    "speedup_vs_f64": r32["value"] / r64["value"]}
        if "tol" in r32:
            out["mixed_f32_precond"]["time_to_tol"] = r32["tol"]
            out["mixed_f32_precond"]["gmres_time_to_tol"] = r32["gmres"]
            out["mixed_f32_precond"]["nuH2_time_to_tol"] = r32["tol_nuH2"]
            if "tol" in r64:
                out["mixed_f32_precond"]["time_to_tol_speedup"] = r64["tol"]["sec"] / r32["tol"]["sec"]
    if not args.no_batch:
        out["batch64"] = batch_run(args)
    if not args.no_3d:
        out["heat3d_lognormal"] = heat3d_run(args)
        out["paper_sec8_3"] = paper83_run(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
