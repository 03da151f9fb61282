#!/usr/bin/env python
"""Benchmark of the SBM elasticity multigrid solve on one MI355X.

One step = one complete solve of the workload to a relative residual of
1e-10 from a zero initial guess: load assembly, psi hierarchy and every
iteration, with the inputs already resident in device memory.  The metric is
free DOF solved per second.  The default workload is the 257^3 near-singular
diffuse crack (its 407 MB vectors exceed the 256 MB Infinity Cache); it is
solved by V-cycle-preconditioned flexible CG, because the plain V-cycle
iteration contracts by about 0.996 per cycle there.  The FP64 solve gives
``value``; the mixed solve (FP32 cycles, FP64 residual / correction / bottom
refinement) is timed beside it and its relative L2 distance to the FP64
solution is reported.

The dominant kernel is the finest-level Gauss-Seidel half-sweep; its average
launch time is measured with HIP events around every finest-level launch of
a profiled solve and set against its algorithmic bytes (80 B per node in
FP64: u 24 + psi 8 + f 24 read, u 24 written), the 8 TB/s HBM peak and the
bandwidth a plain triad kernel of the library reaches in the same process.

The CPU baseline is the FP64 oracle (plain loops, OpenMP, not a tuned solver)
on the host cores: its setup and one iteration are timed on the same workload
and projected to the FP64 iteration count.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF/s solved to 1e-10 rel. residual, FP64 vs mixed; stencil HBM GB/s % peak"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per finest-level node and launch, FP64 (FP32 halves the vector parts)
ALGO_BYTES = {              # (FP64, FP32) bytes per finest-level node
    "smooth": (80.0, 40.0),    # u, psi, f read, u written
    "residual": (80.0, 40.0),  # u, psi, f read, r written
    "restrict": (27.0, 13.5),  # r read, coarse f written (1/8 of the nodes)
    "prolong": (51.0, 25.5),   # coarse e read, u read and written
    "norm": (56.0, 56.0),      # u, psi, f read (always FP64)
    "sweep0": (56.0, 28.0),    # one-launch sweep from zero: psi, f read, u written
}
# V-cycle iteration: the convergence-test pass also writes the next cycle's
# first half-sweep (FP64) or the residual the FP32 cycle casts (mixed): u,
# psi, f read, one vector written
NORM_SWEEP_BYTES = 80.0


def _workload(name):
    import sbm_inputs as si
    if name == "spherical_voids_129":
        return si.spherical_voids_3d(128), (
            "3D unit cube, 129^3 nodes (128^3 cells), E=1 nu=0.3, 20 seeded spherical voids "
            "(seed 0), psi floor 1e-6, z=0 clamped, u=(0,0,1e-3) on z=1; V(2,2) two-colour "
            "Gauss-Seidel, rtol 1e-10")
    if name == "diffuse_crack_257":
        return si.diffuse_crack_3d(256), (
            "3D unit cube, 257^3 nodes, diffuse disc crack in a 40% void field (seed 0), psi "
            "floor 1e-6, mode-I displacement loading; V(2,2) two-colour Gauss-Seidel, rtol 1e-10")
    if name == "cantilever_193x97x97":
        return si.cantilever_density_3d(), (
            "3D cantilever 193x97x97 nodes, psi = rho^3 (rho = sigmoid of a seeded Gaussian "
            "random field), floor 1e-4, x=0 clamped, smoothed corner load; V(2,2) two-colour "
            "Gauss-Seidel, rtol 1e-10")
    raise SystemExit(f"unknown workload {name}")


AMR_WORKLOAD = "ellipsoidal_voids_amr_64x3"
AMR_DESC = ("3D BSAMR composite solve: base 64^3 cells on the unit cube, 3 levels (refinement "
            "ratio 2, finest 256^3 cells), 32^3-cell blocks tagged where |grad psi| h > 0.05, "
            "10 seeded ellipsoidal voids (seed 0, semi-axes U[0.04,0.12], random orientations), "
            "psi floor 1e-5, z=0 clamped, u=(0,0,1e-3) on z=1; FAS composite V(2,2) two-colour "
            "Gauss-Seidel, rtol 1e-10")


def _bench_amr(args):
    """The adaptive workload: one step = set_problem (tags, blocks, classes,
    psi average-down, loads) + composite solve to 1e-10 on the FP64 outer
    loop.  value = composite unknowns / second."""
    import numpy as np
    import torch

    import sbm_inputs as si
    from paper_2212_02362_amd import AmrSolver

    t0 = time.perf_counter()
    p, psis = si.ellipsoidal_voids_amr(base=64, levels=3, block=32, seed=0)
    print(f"[bench] {AMR_WORKLOAD}: inputs generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    psi_dev = [torch.tensor(x, dtype=torch.float64, device="cuda") for x in psis]
    S = AmrSolver(p.ncell, p.h, 3, 32, rtol=1e-10, max_cycles=400)
    if args.cluster_eff > 0.0:
        S.set_clustering(args.cluster_eff)

    def one():
        S.set_problem(psi_dev, p.lam, p.mu, p.psi_floor, p.kind, p.val, thresh=0.05)
        return S.solve()

    runs = {}
    variants = [("fp64", 0), ("mixed", 1)]
    if args.no_mixed:
        variants = variants[:1]
    for name, prec in variants:
        S.set_options(precision=prec)
        for _ in range(args.warmup):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc, st, fin = [], [], []
        for _ in range(args.steps):
            u, hist, status = one()
            cyc.append(len(hist) - 1)
            st.append(int(status))
            fin.append(float(hist[-1]))
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        S.profile(True)
        one()
        prof = S.profile_read()
        S.profile(False)
        runs[name] = dict(t=t, cyc=cyc, st=st, fin=fin, prof=prof, prec=prec)
        print(f"[bench] {name}: {t * 1e3:.2f} ms/solve, cycles {cyc}", file=sys.stderr, flush=True)
    dof, fnorm = S.stats()
    blk1, _, _ = S.level_info(1)
    blk2, cls2, _ = S.level_info(2)
    n_active = int((cls2 == 1).sum().item())
    nodes2 = int(cls2.numel())
    r = runs["fp64"]
    ms_s, n_s = r["prof"]["smooth"]
    avg_ms = ms_s / max(n_s, 1)
    # algorithmic bytes of a finest-level half-sweep: the unknowns' rows only
    # (u, psi, f read, u written; 80 B per node in FP64)
    by = 80.0 * n_active
    achieved = by / (avg_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": dof / r["t"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["t"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": AMR_DESC + (f"; blocks regridded by Berger-Rigoutsos clustering "
                                           f"at efficiency {args.cluster_eff}"
                                           if args.cluster_eff > 0.0 else ""),
                   "composite_dof": dof,
                   "level1_block_fraction": float(blk1.mean()),
                   "level2_block_fraction": float(blk2.mean()),
                   "finest_unknown_nodes": n_active, "finest_dense_nodes": nodes2,
                   "precision": "fp64", "method": "FAS composite cycle, FP64 outer loop",
                   "cycles": r["cyc"], "final_rel_residual": max(r["fin"]), "status": r["st"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_rb_tile<double, CoefCubic<double>, true, false> (LDS-tiled class-masked half-sweep) over the "
                               "tiles of the finest adaptive level that hold unknowns",
                     "algo_bytes_per_launch": by, "avg_launch_us": avg_ms * 1e3,
                     "timing": "HIP events around each finest-level launch, one profiled solve "
                               "after the timed region"},
        "kernels_fp64": {k: {"launches": n, "avg_us": ms / n * 1e3}
                         for k, (ms, n) in r["prof"].items() if n},
        "variants": {name: {"value": dof / v["t"], "unit": "DOF/s", "ms_per_step": v["t"] * 1e3,
                            "iterations": v["cyc"], "final_rel_residual": max(v["fin"]),
                            "status": v["st"], "speedup_vs_headline": r["t"] / v["t"],
                            "kernels": {k: {"launches": n, "avg_us": ms / n * 1e3}
                                        for k, (ms, n) in v["prof"].items() if n}}
                     for name, v in runs.items()},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        m = oracle.AmrProblem(p.ncell, p.h, p.lam, p.mu, psis, p.psi_floor, p.kind, p.val,
                              block=32, thresh=0.05, cluster_eff=args.cluster_eff)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        m.solve(rtol=0.0, max_cycles=0)
        t_res = time.perf_counter() - t0
        t0 = time.perf_counter()
        m.solve(rtol=0.0, max_cycles=1)
        per_cycle = max(time.perf_counter() - t0 - t_res, 1e-9)
        ncyc = int(np.median(r["cyc"]))
        projected = t_setup + t_res + ncyc * per_cycle
        line["cpu_baseline"] = {
            "value": dof / projected, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle (plain C loops, OpenMP where the uniform kernels have it) on "
                       f"the same workload: setup ({t_setup:.1f} s) and one composite cycle "
                       f"({per_cycle:.1f} s) timed, projected to the {ncyc} cycles of the GPU "
                       f"solve ({projected:.1f} s per solve)"),
        }
    print(json.dumps(line), flush=True)


J2_WORKLOAD = "j2_void_tension_128"
J2_DESC = ("J2 plastic-void tension specimen (Sec. 3.1): cube [-16,16]^3 with 128^3 cells, "
           "ellipsoidal void r=(7.5,4.08,4.08) with tanh width 0.4, E=210 nu=0.3, psi floor 1e-4, "
           "x=-16 clamped, u_x prescribed on x=+16 rising in increments of 0.004; J2 with "
           "sigma_Y=0.2, Hbar=50, theta=1.  One step = plastic load, set_problem, V(2,2) solve to "
           "1e-10, radial return; timed steps follow 15 loading steps (plastic zone present)")


def _bench_j2(args):
    """The staggered elastic / plastic step of the J2 example.  value = free
    DOF / second of whole steps; roofline for the finest half-sweep of the
    solve (the dominant kernel), plus HIP-event timings of the two plastic
    kernels against their algorithmic bytes."""
    import numpy as np
    import torch

    import sbm_inputs as si
    from paper_2212_02362_amd import Solver

    p = si.j2_void_tension(128)
    j2 = p.extra
    free = _free_dof(p)
    nodes, cells = p.n_nodes, int(np.prod(p.ncell))
    shape = tuple(reversed(p.ncell))
    S = Solver(p.ncell, p.h, rtol=1e-10, max_cycles=400)
    psi_dev = torch.tensor(p.psi_raw, dtype=torch.float64, device="cuda")
    ep = torch.zeros((6,) + shape, dtype=torch.float64, device="cuda")
    al = torch.zeros(shape, dtype=torch.float64, device="cuda")
    bt = torch.zeros_like(ep)
    state = {"d": 0.0, "set": False}

    def one():
        state["d"] += 0.004
        b = S.plastic_source(ep) if state["set"] else None  # eps_p = 0 before the first step
        state["set"] = True
        val = p.val.copy()
        val[1, 0] = state["d"]
        S.set_problem(psi_dev, p.lam, p.mu, p.psi_floor, p.kind, val, b)
        u, hist, st = S.solve()
        n = S.return_map(u, ep, al, bt, j2["sigma_y"], j2["hbar"], j2["theta"], inplace=True)[3]
        return u, hist, st, n

    for _ in range(15 + args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc, st, fin, npl = [], [], [], []
    for _ in range(args.steps):
        u, hist, status, n = one()
        cyc.append(len(hist) - 1)
        st.append(int(status))
        fin.append(float(hist[-1]))
        npl.append(n)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    print(f"[bench] {J2_WORKLOAD}: {t * 1e3:.2f} ms/step, cycles {cyc}, yielding cells {npl}",
          file=sys.stderr, flush=True)
    # one more step outside the timed region: its solve is profiled (the
    # dominant kernel) and its plastic kernels are timed on the state before
    # its return map
    state["d"] += 0.004
    b = S.plastic_source(ep)
    val = p.val.copy()
    val[1, 0] = state["d"]
    S.set_problem(psi_dev, p.lam, p.mu, p.psi_floor, p.kind, val, b)
    S.profile(True)
    u, _, _ = S.solve()
    prof = S.profile_read()
    S.profile(False)
    ms_s, n_s = prof["smooth"]
    avg_ms = ms_s / max(n_s, 1)
    by = ALGO_BYTES["smooth"][0] * nodes
    achieved = by / (avg_ms * 1e-3) / 1e9

    def timed(make, reps=10):
        ts, out = [], None
        for _ in range(reps):
            fn = make()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            out = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.median(ts)), out

    fp = S.new_nodes()
    t_src, _ = timed(lambda: (lambda: S.plastic_source(ep, out=fp)))

    def rm():
        e2, a2, b2 = ep.clone(), al.clone(), bt.clone()
        return lambda: S.return_map(u, e2, a2, b2, j2["sigma_y"], j2["hbar"], j2["theta"],
                                    inplace=True)[3]
    t_rm, n_rm = timed(rm)
    by_src = 56.0 * cells + 24.0 * nodes           # psi, eps_p read; load written
    by_rm = 24.0 * nodes + 104.0 * cells + 104.0 * n_rm  # u, state read; yielded state written
    line = {
        "metric": METRIC,
        "value": free / t,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": J2_DESC, "nodes": nodes, "free_dof": free, "precision": "fp64",
                   "method": "staggered step: V-cycle iteration + radial return",
                   "cycles": cyc, "final_rel_residual": max(fin), "status": st,
                   "yielding_cells": npl, "applied_displacement": state["d"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_rb_tile<double, ..., false, false> (LDS-tiled finest-level "
                               "Gauss-Seidel half-sweep; 129 nodes in x)",
                     "algo_bytes_per_launch": by, "avg_launch_us": avg_ms * 1e3,
                     "timing": "HIP events around each finest-level launch, one profiled solve "
                               "after the timed steps"},
        "plastic_kernels": {
            "plastic_source": {"us": t_src * 1e6, "algo_bytes": by_src,
                               "algo_GBps": by_src / t_src / 1e9,
                               "frac_hbm_peak": by_src / t_src / 1e9 / HBM_PEAK_GBS},
            "return_map": {"us": t_rm * 1e6, "algo_bytes": by_rm, "yielding_cells": n_rm,
                           "algo_GBps": by_rm / t_rm / 1e9,
                           "frac_hbm_peak": by_rm / t_rm / 1e9 / HBM_PEAK_GBS},
            "timing": "HIP events around single launches, median of 10"},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        import oracle
        ep_h, al_h, bt_h = ep.cpu().numpy(), al.cpu().numpy(), bt.cpu().numpy()
        u_h = u.cpu().numpy()
        psi_f = oracle.floor_psi(p.psi_raw, p.psi_floor)
        t0 = time.perf_counter()
        b_h = oracle.plastic_source(p.ncell, p.h, p.lam, p.mu, psi_f, ep_h)
        oracle.return_map(p.ncell, p.h, p.lam, p.mu, j2["sigma_y"], j2["hbar"], j2["theta"], u_h,
                          ep_h, al_h, bt_h)
        t_pl = time.perf_counter() - t0
        val = p.val.copy()
        val[1, 0] = state["d"]
        q = si.Problem(p.name, p.ncell, p.h, p.lam, p.mu, p.psi_floor, p.psi_raw, p.kind, val, b=b_h)
        base = _cpu_baseline(q, int(np.median(cyc)), free)
        per_step = t_pl + free / base["value"]
        line["cpu_baseline"] = {
            "value": free / per_step, "unit": "DOF/s", "cores": base["cores"], "kind": "oracle",
            "sample": (f"FP64 oracle on the same step: plastic load and radial return timed "
                       f"({t_pl:.1f} s), solve " + base["sample"].split("on the same workload: ")[-1]),
        }
    print(json.dumps(line), flush=True)


PF_WORKLOAD = "pf_mode1_4096"
PF_DESC = ("Mode-I phase-field fracture (Sec. 3.2, hybrid model) on a uniform 4096^2-cell grid "
           "(the resolution of the finest of six refinement levels over a 64^2 base, everywhere): "
           "square [-0.01,0.01]^2, lambda=121.15e9 mu=80.77e9, notch of length 1.5e-4 from the "
           "centre of the left edge, c0 = 1 - exp(-d/xi), xi=1e-5, Gc=2700, M=1e-5, dt=1e-4, "
           "eta=1e-4 (psi = g(c) + eta, floor 1e-4), bottom clamped, u_y=1.5e-5 on the top.  One "
           "step = set_problem(psi), V(2,2)-preconditioned flexible CG solve to 1e-10 warm-started "
           "from the previous step, "
           "crack driving force, explicit Ginzburg-Landau step; timed steps follow 5 steps")


def _bench_pf(args):
    """The staggered phase-field fracture step.  value = free DOF / second of
    whole steps; roofline for the finest half-sweep of the solve (the
    dominant kernel), plus HIP-event timings of the two fracture kernels
    against their algorithmic bytes."""
    import numpy as np
    import torch

    import sbm_inputs as si
    from paper_2212_02362_amd import Solver

    p = si.pf_mode1_2d(4096)
    e = p.extra
    free = _free_dof(p)
    nodes, cells = p.n_nodes, int(np.prod(p.ncell))
    # the crack makes the operator near-singular: V-cycle-preconditioned CG
    S = Solver(p.ncell, p.h, rtol=1e-10, max_cycles=400, krylov=1)
    c0 = torch.tensor(e["c0"], device="cuda")
    z = torch.zeros_like(c0)
    # the initial indicator psi = g(c0) + eta: the library's crack step with dt = 0
    _, psi0 = S.phase_step(c0, z, z.to(torch.uint8), e["Gc"], e["xi"], e["M"], 0.0, e["eta"])
    st_ = {"c": c0, "psi": psi0,
           "H": torch.zeros(e["c0"].shape, dtype=torch.float64, device="cuda"),
           "u": None}

    def one():
        S.set_problem(st_["psi"], p.lam, p.mu, p.psi_floor, p.kind, p.val)
        u, hist, status = S.solve(u0=st_["u"])
        st_["u"] = u
        H, intact = S.crack_drive(u, st_["H"], inplace=True)
        st_["c"], st_["psi"] = S.phase_step(st_["c"], H, intact, e["Gc"], e["xi"], e["M"],
                                            e["dt"], e["eta"])
        return hist, status, intact

    print(f"[bench] {PF_WORKLOAD}: {nodes} nodes, {free} free DOF", file=sys.stderr, flush=True)
    first = None
    for k in range(5 + args.warmup):
        hist, _, _ = one()
        if first is None:
            first = len(hist) - 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc, sts, fin = [], [], []
    for _ in range(args.steps):
        hist, status, intact = one()
        cyc.append(len(hist) - 1)
        sts.append(int(status))
        fin.append(float(hist[-1]))
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    c = st_["c"]
    cmin, cmax = float(c.min()), float(c.max())
    cracked = int((c < 0.5).sum())
    n_intact = int(intact.sum())
    print(f"[bench] {PF_WORKLOAD}: {t * 1e3:.2f} ms/step, cycles {cyc} (first solve {first}), "
          f"c in [{cmin:.3g}, {cmax:.3g}], {cracked} cells c<0.5, {n_intact} held intact",
          file=sys.stderr, flush=True)
    # one more solve outside the timed region, profiled (the dominant kernel)
    S.set_problem(st_["psi"], p.lam, p.mu, p.psi_floor, p.kind, p.val)
    S.profile(True)
    u, _, _ = S.solve(u0=st_["u"])
    prof = S.profile_read()
    S.profile(False)
    ms_s, n_s = prof["smooth"]
    avg_ms = ms_s / max(n_s, 1)
    by = PF_SMOOTH_BYTES * nodes
    achieved = by / (avg_ms * 1e-3) / 1e9

    def timed(fn, reps=10):
        ts, out = [], None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            out = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.median(ts)), out

    Hs = st_["H"].clone()
    t_cd, (_, intact) = timed(lambda: S.crack_drive(u, Hs, inplace=True))
    c_out, psi_out = torch.empty_like(st_["c"]), torch.empty_like(st_["c"])
    t_ps, _ = timed(lambda: S.phase_step(st_["c"], Hs, intact, e["Gc"], e["xi"], e["M"], e["dt"],
                                         e["eta"], out=(c_out, psi_out)))
    by_cd = 16.0 * nodes + 17.0 * cells   # u read, H read and written, intact written
    by_ps = 33.0 * cells                  # c, H, intact read; c, psi written
    line = {
        "metric": METRIC,
        "value": free / t,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": PF_DESC, "nodes": nodes, "free_dof": free, "precision": "fp64",
                   "method": "staggered step: warm-started MG-preconditioned CG + crack update",
                   "cycles": cyc, "first_solve_cycles": first, "final_rel_residual": max(fin),
                   "status": sts, "crack_cells_c_below_half": cracked, "c_range": [cmin, cmax],
                   "intact_cells": n_intact},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_rb_half<double,2,false> (finest-level Gauss-Seidel half-sweep)",
                     "algo_bytes_per_launch": by, "avg_launch_us": avg_ms * 1e3,
                     "timing": "HIP events around each finest-level launch, one profiled solve "
                               "after the timed steps"},
        "fracture_kernels": {
            "crack_drive": {"us": t_cd * 1e6, "algo_bytes": by_cd,
                            "algo_GBps": by_cd / t_cd / 1e9,
                            "frac_hbm_peak": by_cd / t_cd / 1e9 / HBM_PEAK_GBS},
            "phase_step": {"us": t_ps * 1e6, "algo_bytes": by_ps,
                           "algo_GBps": by_ps / t_ps / 1e9,
                           "frac_hbm_peak": by_ps / t_ps / 1e9 / HBM_PEAK_GBS},
            "timing": "HIP events around single launches, median of 10"},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        import oracle
        u_h, H_h, c_h = u.cpu().numpy(), st_["H"].cpu().numpy(), st_["c"].cpu().numpy()
        psi_h = st_["psi"].cpu().numpy()
        t0 = time.perf_counter()
        H_h, i_h = oracle.crack_drive(p.ncell, p.h, p.lam, p.mu, u_h, H_h)
        oracle.phase_step(p.ncell, p.h, c_h, H_h, i_h, e["Gc"], e["xi"], e["M"], e["dt"], e["eta"])
        t_pf = time.perf_counter() - t0
        q = si.Problem(p.name, p.ncell, p.h, p.lam, p.mu, p.psi_floor, psi_h, p.kind, p.val)
        base = _cpu_baseline(q, int(np.median(cyc)), free, krylov=1)
        per_step = t_pf + free / base["value"]
        line["cpu_baseline"] = {
            "value": free / per_step, "unit": "DOF/s", "cores": base["cores"], "kind": "oracle",
            "sample": (f"FP64 oracle on the same step: crack driving force and Ginzburg-Landau "
                       f"step timed ({t_pf:.1f} s), solve " +
                       base["sample"].split("on the same workload: ")[-1] +
                       "; the oracle solve starts from zero, its per-iteration cost is used"),
        }
    print(json.dumps(line), flush=True)


PRESS_WORKLOAD = "pressurised_voids_129"
PRESS_DESC = ("3D unit cube, 129^3 nodes (128^3 cells), E=1 nu=0.3, the 20 seeded spherical voids of "
              "spherical_voids_129 (seed 0) under an internal pressure 1e-3 applied as the diffuse "
              "traction load p grad psi (Sec. 2.1), psi floor 1e-6, z=0 clamped, other faces free.  "
              "One step = diffuse traction load, set_problem, V(2,2) solve to 1e-10")


def _bench_pressure(args):
    """Solves loaded by a diffuse traction (a pressure in every void).  value
    = free DOF / second of whole steps (load, set-up, FP64 V-cycle solve);
    roofline for the finest half-sweep; the load kernel is timed apart."""
    import numpy as np
    import torch

    import sbm_inputs as si
    from paper_2212_02362_amd import Solver

    p = si.pressurised_voids_3d(128)
    pr = p.extra["pressure"]
    free = _free_dof(p)
    nodes, cells = p.n_nodes, int(np.prod(p.ncell))
    S = Solver(p.ncell, p.h, rtol=1e-10, max_cycles=400)
    psi_dev = torch.tensor(p.psi_raw, dtype=torch.float64, device="cuda")
    b = S.new_nodes()

    def one():
        S.diffuse_traction(psi_dev, p.psi_floor, pressure=pr, out=b)
        S.set_problem(psi_dev, p.lam, p.mu, p.psi_floor, p.kind, p.val, b)
        return S.solve()

    print(f"[bench] {PRESS_WORKLOAD}: {nodes} nodes, {free} free DOF", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc, sts, fin = [], [], []
    for _ in range(args.steps):
        u, hist, status = one()
        cyc.append(len(hist) - 1)
        sts.append(int(status))
        fin.append(float(hist[-1]))
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    print(f"[bench] {PRESS_WORKLOAD}: {t * 1e3:.2f} ms/step, cycles {cyc}, max |u| "
          f"{float(u.abs().max()):.3e}", file=sys.stderr, flush=True)
    S.profile(True)
    S.solve()
    prof = S.profile_read()
    S.profile(False)
    ms_s, n_s = prof["smooth"]
    avg_ms = ms_s / max(n_s, 1)
    by = ALGO_BYTES["smooth"][0] * nodes
    achieved = by / (avg_ms * 1e-3) / 1e9
    ts = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        S.diffuse_traction(psi_dev, p.psi_floor, pressure=pr, out=b)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    t_dt = float(np.median(ts))
    by_dt = 8.0 * cells + 24.0 * nodes   # psi read, load written
    line = {
        "metric": METRIC,
        "value": free / t,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": PRESS_DESC, "nodes": nodes, "free_dof": free, "precision": "fp64",
                   "method": "diffuse traction load + V-cycle iteration", "cycles": cyc,
                   "final_rel_residual": max(fin), "status": sts},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_rb_tile<double, ..., false, false> (LDS-tiled finest-level "
                               "Gauss-Seidel half-sweep; 129 nodes in x)",
                     "algo_bytes_per_launch": by, "avg_launch_us": avg_ms * 1e3,
                     "timing": "HIP events around each finest-level launch, one profiled solve "
                               "after the timed steps"},
        "traction_kernel": {"k_diffuse_traction": {
            "us": t_dt * 1e6, "algo_bytes": by_dt, "algo_GBps": by_dt / t_dt / 1e9,
            "frac_hbm_peak": by_dt / t_dt / 1e9 / HBM_PEAK_GBS},
            "timing": "HIP events around single launches, median of 10"},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        import oracle
        t0 = time.perf_counter()
        load = oracle.diffuse_traction(p.ncell, p.h, p.psi_raw, p.psi_floor, pressure=pr)
        t_ld = time.perf_counter() - t0
        q = si.Problem(p.name, p.ncell, p.h, p.lam, p.mu, p.psi_floor, p.psi_raw, p.kind, p.val,
                       b=load)
        base = _cpu_baseline(q, int(np.median(cyc)), free)
        per_step = t_ld + free / base["value"]
        line["cpu_baseline"] = {
            "value": free / per_step, "unit": "DOF/s", "cores": base["cores"], "kind": "oracle",
            "sample": (f"FP64 oracle on the same step: diffuse traction load timed ({t_ld:.2f} s), "
                       f"solve " + base["sample"].split("on the same workload: ")[-1]),
        }
    print(json.dumps(line), flush=True)


# 2D finest half-sweep: u (16), psi (8), f (16) read, u (16) written per node
PF_SMOOTH_BYTES = 56.0


def _free_dof(p):
    import numpy as np
    d = p.dim
    shp = p.node_shape
    free = 0
    for k in range(d):
        m = np.zeros(shp, bool)
        for F in range(2 * d):
            if p.kind[F, k] != 1:
                continue
            a = F // 2
            ax = d - 1 - a
            sl = [slice(None)] * d
            sl[ax] = 0 if F % 2 == 0 else shp[ax] - 1
            m[tuple(sl)] = True
        free += int((~m).sum())
    return free


def _kernel_hash(files=("sbm_device.h", "sbm_kernels.hip")):
    h = hashlib.sha256()
    for fn in files:
        with open(os.path.join(ROOT, "paper_2212_02362_amd", "csrc", fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel_key, nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(kernel_key)
    files = next((v[2] for v in COUNTER_KERNELS.values() if v[0] == kernel_key), None)
    if not ent or files is None or ent.get("kernel_hash") != _kernel_hash(files) or \
            ent.get("nodes") != nodes:
        return None
    return ent.get("hbm_bytes_per_launch")


TRAFFIC_KERNEL = "k_rb_half<double,3,false>"
# counter runs per workload: (key in traffic_counters.json, kernel name in the
# rocprofv3 trace, the sources whose hash keys the entry).  The 129^3 vectors
# fit the 256 MB Infinity Cache; the 257^3 ones do not.
COUNTER_KERNELS = {
    "spherical_voids_129": (TRAFFIC_KERNEL, "k_rb_half<double, 3, false>",
                            ("sbm_device.h", "sbm_kernels.hip")),
    "diffuse_crack_257": ("k_rb_tile<double,false>",
                          "k_rb_tile<double, sbm::CoefCubic<double>, false, false>",
                          ("sbm_device.h", "sbm_tiled.hip")),
}
COPY_BYTES = 400_000_000  # calibration copy: this many bytes read and written


def _counter_driver(workload="spherical_voids_129"):
    """Workload for the two rocprofv3 counter passes: the finest-level
    half-sweep of the workload, launched as inside its V-cycles (same kernel,
    level and launch shape), then a plain device copy of known size that
    calibrates FETCH_SIZE / WRITE_SIZE."""
    import torch

    from paper_2212_02362_amd import Solver

    if workload not in COUNTER_KERNELS:
        raise SystemExit(f"no counter run defined for {workload}")
    p, _ = _workload(workload)
    S = Solver(p.ncell, p.h)
    S.set_problem(torch.tensor(p.psi_raw, device="cuda"), p.lam, p.mu, p.psi_floor, p.kind, p.val)
    import ctypes

    from paper_2212_02362_amd._lib import check, lib
    u = torch.randn((p.dim,) + p.node_shape, dtype=torch.float64, device="cuda")
    f = torch.randn_like(u)
    v = torch.empty_like(u)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    # ping-pong between two resident buffers, as the V-cycle does
    for it in range(10):
        check(lib().sbm_level_smooth(S._ctx, 0, it % 2, 1.0, ptr(u), ptr(f), ptr(v)))
        u, v = v, u
    x = torch.randn(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("[counters] driver done", flush=True)


def _counter_summary(fetch_dir, write_dir, workload="spherical_voids_129"):
    """HBM bytes per launch of the dominant kernel from the two counter runs,
    each counter scaled by its reading for the calibration copy; writes
    profiles/traffic_counters.json (keyed by the kernel-source hash, so a
    changed kernel reports no traffic) and a text summary."""
    import csv

    if workload not in COUNTER_KERNELS:
        raise SystemExit(f"no counter run defined for {workload}")
    key, trace_name, files = COUNTER_KERNELS[workload]

    def read(d, counter):
        path = None
        for root, _, files in os.walk(d):
            for fn in files:
                if fn.endswith("counter_collection.csv"):
                    path = os.path.join(root, fn)
        if path is None:
            raise SystemExit(f"no counter_collection.csv under {d}")
        kern, copy = [], []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * 1024.0  # KiB -> bytes
                name = r["Kernel_Name"]
                if trace_name in name:
                    kern.append(v)
                elif "copyBuffer" in name and v > 0.25 * COPY_BYTES:
                    copy.append(v)
        if not kern or not copy:
            raise SystemExit(f"{counter}: kernel or calibration copy missing in {path}")
        return sum(kern) / len(kern), sum(copy) / len(copy), len(kern)

    fk, fc, nf = read(fetch_dir, "FETCH_SIZE")
    wk, wc, nw = read(write_dir, "WRITE_SIZE")
    ff, fw = COPY_BYTES / fc, COPY_BYTES / wc
    p, _ = _workload(workload)
    nodes = p.n_nodes
    fetch, write = fk * ff, wk * fw
    ent = {"kernel_hash": _kernel_hash(files), "nodes": nodes, "workload": workload,
           "hbm_bytes_per_launch": fetch + write,
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "fetch_factor": ff, "write_factor": fw, "launches": [nf, nw],
           "algo_bytes_per_launch": ALGO_BYTES["smooth"][0] * nodes}
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = ent
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    print(json.dumps(ent))


def _time_solves(S, p, psi_dev, b_dev, precision, steps, warmup, krylov=0, prof_steps=None,
                 fused_sweep=0):
    """Timed region: `steps` complete solves (V-cycles replayed from HIP
    graphs).  Then `prof_steps` solves (default: `steps`) with live kernel
    timing (HIP events around every finest-level launch; those solves run
    launch by launch) give the per-kernel durations.  Returns the timings and
    the last solution."""
    import torch
    S.set_options(precision=precision, krylov=krylov, fused_sweep=fused_sweep)
    if prof_steps is None:
        prof_steps = steps

    def one():
        S.set_problem(psi_dev, p.lam, p.mu, p.psi_floor, p.kind, p.val, b_dev)
        return S.solve()

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles, status, final = [], [], []
    u = None
    for _ in range(steps):
        u, hist, st = one()
        cycles.append(len(hist) - 1)
        status.append(int(st))
        final.append(float(hist[-1]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.profile(True)
    t2 = time.perf_counter()
    for _ in range(prof_steps):
        one()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = S.profile_read()
    S.profile(False)
    return (t1 - t0) / steps, cycles, status, final, prof, (t3 - t2) / prof_steps, u


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(p, cycles_fp64, free, krylov=0):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.solve(p.ncell, p.h, p.lam, p.mu, p.psi_raw, p.psi_floor, p.kind, p.val, p.b,
                 rtol=0.0, max_cycles=0, krylov=krylov)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve(p.ncell, p.h, p.lam, p.mu, p.psi_raw, p.psi_floor, p.kind, p.val, p.b,
                 rtol=0.0, max_cycles=1, krylov=krylov)
    t_one = time.perf_counter() - t0
    per_cycle = max(t_one - t_setup, 1e-9)
    projected = t_setup + cycles_fp64 * per_cycle
    return {
        "value": free / projected, "unit": "DOF/s", "cores": threads, "kind": "oracle",
        "sample": (f"FP64 oracle (plain C loops, OpenMP, not a tuned solver) on the same workload: "
                   f"setup + 1 iteration timed ({t_one:.1f} s), projected to the {cycles_fp64} "
                   f"iterations of the FP64 GPU solve (projected {projected:.1f} s per solve)"),
        "seconds_setup": t_setup, "seconds_per_cycle": per_cycle, "projected": True,
        "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffuse_crack_257",
                    choices=["spherical_voids_129", "diffuse_crack_257", "cantilever_193x97x97",
                             AMR_WORKLOAD, J2_WORKLOAD, PF_WORKLOAD, PRESS_WORKLOAD])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cluster-eff", type=float, default=0.0,
                    help="adaptive workload: Berger-Rigoutsos efficiency of the block boxes")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cache-variant", action="store_true",
                    help="257^3 workload: skip the 129^3 cache-resident variant")
    ap.add_argument("--counter-driver", action="store_true",
                    help="run the dominant kernel and a calibration copy (under rocprofv3 --pmc)")
    ap.add_argument("--counter-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 counter runs into profiles/traffic_counters.json")
    args = ap.parse_args()
    if args.counter_driver:
        return _counter_driver(args.workload)
    if args.counter_summary:
        return _counter_summary(*args.counter_summary, workload=args.workload)
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for "
              f"--gpus {args.gpus}).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == AMR_WORKLOAD:
        return _bench_amr(args)
    if args.workload == PRESS_WORKLOAD:
        return _bench_pressure(args)
    if args.workload == PF_WORKLOAD:
        return _bench_pf(args)
    if args.workload == J2_WORKLOAD:
        return _bench_j2(args)

    import numpy as np
    import torch

    from paper_2212_02362_amd import Solver

    p, desc = _workload(args.workload)
    free = _free_dof(p)
    nodes = p.n_nodes
    print(f"[bench] {args.workload}: {nodes} nodes, {free} free DOF", file=sys.stderr, flush=True)
    psi_dev = torch.tensor(p.psi_raw, dtype=torch.float64, device="cuda")
    b_dev = None if p.b is None else torch.tensor(p.b, dtype=torch.float64, device="cuda")
    S = Solver(p.ncell, p.h, rtol=1e-10, max_cycles=1000)

    # variants: (name, precision, krylov).  The headline is the plain FP64
    # V-cycle iteration, unless it cannot reach the tolerance on this workload
    # (the near-singular crack), where V-cycle-preconditioned CG is the FP64
    # method.
    stationary_ok = args.workload != "diffuse_crack_257"
    variants = [("fp64", 0, 0), ("mixed", 1, 0), ("fp64_krylov", 0, 1), ("mixed_krylov", 1, 1)]
    if not stationary_ok:
        variants = [v for v in variants if v[2] == 1]
    if args.no_mixed:
        variants = [v for v in variants if v[1] == 0]
    head = "fp64" if stationary_ok else "fp64_krylov"
    runs = {}
    for name, prec, kry in variants:
        t, cyc, st, fin, prof, tp, u = _time_solves(S, p, psi_dev, b_dev, prec, args.steps,
                                                    args.warmup, kry, prof_steps=1)
        runs[name] = dict(t=t, cyc=cyc, st=st, fin=fin, prof=prof, tp=tp, prec=prec, kry=kry,
                          u=u)
        print(f"[bench] {name}: {t * 1e3:.2f} ms/solve, iterations {cyc}", file=sys.stderr,
              flush=True)
    t64, cyc64, st64, fin64, prof64, tp64 = (runs[head][k] for k in
                                             ("t", "cyc", "st", "fin", "prof", "tp"))
    u64 = runs[head]["u"]
    # each variant's distance to the FP64 solution of the same method
    for name, r in runs.items():
        ref = runs["fp64" if r["kry"] == 0 else "fp64_krylov"]["u"] if r["prec"] == 1 else None
        r["err"] = (float(torch.linalg.vector_norm(r["u"] - ref) / torch.linalg.vector_norm(ref))
                    if ref is not None else 0.0)
    triad = _triad()
    print(f"[bench] triad: {triad['GBps']:.0f} GB/s", file=sys.stderr, flush=True)

    def kstats(prof, fp32, fused_norm=False):
        out = {}
        for k, (ms, n) in prof.items():
            if n == 0:
                continue
            avg = ms / n
            ent = {"launches": n, "avg_us": avg * 1e3}
            if k in ALGO_BYTES:
                by = ALGO_BYTES[k][1 if fp32 and k != "norm" else 0] * nodes
                if k == "norm" and fused_norm:
                    by = NORM_SWEEP_BYTES * nodes  # the norm pass also writes a half-sweep
                ent["algo_GBps"] = by / (avg * 1e-3) / 1e9
                ent["frac_hbm_peak"] = ent["algo_GBps"] / HBM_PEAK_GBS
                ent["frac_measured_triad"] = ent["algo_GBps"] / triad["GBps"]
            out[k] = ent
        return out

    def vstats(r):
        n_it = float(np.median(r["cyc"]))
        fin = max(r["fin"])
        return {"value": free / r["t"], "unit": "DOF/s", "ms_per_step": r["t"] * 1e3,
                "iterations": r["cyc"], "ms_per_iteration": r["t"] * 1e3 / max(n_it, 1.0),
                "contraction_per_iteration": fin ** (1.0 / n_it) if n_it > 0 else None,
                "final_rel_residual": fin, "status": r["st"],
                "rel_l2_vs_fp64_solution": r["err"], "speedup_vs_headline": t64 / r["t"],
                "kernels": kstats(r["prof"], r["prec"] == 1,
                                  fused_norm=(r["kry"] == 0 and not tiled))}

    ms_s, n_s = prof64["smooth"]
    avg_ms = ms_s / max(n_s, 1)
    by = ALGO_BYTES["smooth"][0] * nodes
    achieved = by / (avg_ms * 1e-3) / 1e9
    # the library's thresholds: half-sweeps go tiled from 97 nodes in x, the
    # other finest-level passes (and the fused r.z) from 193
    tiled = p.ncell[0] + 1 > 192 and p.dim == 3
    tiled_sweep = p.ncell[0] + 1 > 96 and p.dim == 3
    traffic = _traffic("k_rb_tile<double,false>" if tiled_sweep else TRAFFIC_KERNEL, nodes)
    line = {
        "metric": METRIC,
        "value": free / t64,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "nodes": nodes, "free_dof": free, "precision": "fp64",
                   "method": ("V-cycle iteration" if head == "fp64" else
                              "V-cycle-preconditioned flexible CG"),
                   "cycles": cyc64, "final_rel_residual": max(fin64), "status": st64,
                   "vectors_exceed_infinity_cache": nodes * 24 > 256e6},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "measured_triad_GBps": triad["GBps"],
                     "frac_of_measured_triad": achieved / triad["GBps"],
                     "kernel": (("k_rb_tile<double, CoefCubic<double>, false, false> (LDS-tiled "
                                 "finest-level Gauss-Seidel half-sweep" +
                                 ("; the cycle's last one, which also sums r.z, is timed apart as "
                                  "smooth_dot)" if tiled and head != "fp64" else ")"))
                                if tiled_sweep else
                                "k_rb_half<double,3,false> (finest-level Gauss-Seidel half-sweep)"),
                     "algo_bytes_per_launch": by, "avg_launch_us": avg_ms * 1e3,
                     "timing": "HIP events on the solver's stream around each finest-level launch "
                               "of one profiled solve after the timed region (launched one by "
                               "one: %.2f ms/solve)" % (tp64 * 1e3)},
        "triad": triad,
        "kernels_fp64": kstats(prof64, False, fused_norm=(head == "fp64" and not tiled)),
        "variants": {name: vstats(r) for name, r in runs.items()},
    }
    for r in runs.values():
        r["u"] = None
    if args.workload == "diffuse_crack_257" and not args.no_cache_variant:
        # the 129^3 voids, whose vectors stay in the Infinity Cache
        del S, u64
        torch.cuda.empty_cache()
        q, qdesc = _workload("spherical_voids_129")
        qfree = _free_dof(q)
        qpsi = torch.tensor(q.psi_raw, dtype=torch.float64, device="cuda")
        Q = Solver(q.ncell, q.h, rtol=1e-10, max_cycles=400)
        cache = {"workload": qdesc, "note": "u, f, psi (171 MB) fit the 256 MB Infinity Cache"}
        for name, prec in (("fp64_krylov", 0), ("mixed_krylov", 1)):
            t, cyc, st, fin, prof, tp, _ = _time_solves(Q, q, qpsi, None, prec, args.steps,
                                                        args.warmup, 1, prof_steps=1)
            cache[name] = {"value": qfree / t, "unit": "DOF/s", "ms_per_step": t * 1e3,
                           "iterations": cyc, "final_rel_residual": max(fin)}
            print(f"[bench] spherical_voids_129 {name}: {t * 1e3:.2f} ms/solve", file=sys.stderr,
                  flush=True)
        line["cache_resident_variant"] = cache
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        if args.workload == "diffuse_crack_257":
            line["cpu_baseline"] = _cpu_baseline_half(int(np.median(cyc64)), free)
        else:
            line["cpu_baseline"] = _cpu_baseline(p, int(np.median(cyc64)), free,
                                                 krylov=0 if head == "fp64" else 1)
    print(json.dumps(line), flush=True)


def _cpu_baseline_half(iters, free):
    """The oracle on the 257^3 crack takes minutes per iteration, so the timed
    sample is the same workload at half the resolution (129^3 nodes, same
    generator and seed): its setup and one steady iteration of the same
    method (the second iteration of a run, the first also builds the search
    direction), scaled by the DOF ratio to the 257^3 problem and the GPU's
    iteration count."""
    import sbm_inputs as si
    import oracle
    q = si.diffuse_crack_3d(128)
    qfree = _free_dof(q)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    ts = []
    for m in (0, 1, 2):
        t0 = time.perf_counter()
        oracle.solve(q.ncell, q.h, q.lam, q.mu, q.psi_raw, q.psi_floor, q.kind, q.val, q.b,
                     rtol=0.0, max_cycles=m, krylov=1)
        ts.append(time.perf_counter() - t0)
    t_setup, per_iter = ts[0], max(ts[2] - ts[1], 1e-9)
    scale = free / qfree
    projected = scale * (t_setup + iters * per_iter)
    return {
        "value": free / projected, "unit": "DOF/s", "cores": threads, "kind": "oracle",
        "sample": (f"FP64 oracle (plain C loops, OpenMP, not a tuned solver), V-cycle-"
                   f"preconditioned flexible CG on the same crack workload at 129^3 nodes (same "
                   f"generator and seed; {qfree} free DOF): setup {t_setup:.1f} s and one steady "
                   f"iteration {per_iter:.1f} s timed ({sum(ts):.1f} s in all), scaled by the DOF "
                   f"ratio {scale:.2f} to 257^3 and to the {iters} iterations of the GPU solve: "
                   f"projected {projected:.0f} s per solve.  At 257^3 the oracle's time per "
                   f"iteration grows faster than the DOF count (caches), so this projection "
                   f"flatters the CPU"),
        "seconds_setup_129": t_setup, "seconds_per_iteration_129": per_iter, "projected": True,
        "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
    }


def _triad(n=1 << 26, reps=10):
    """The library's triad kernel (a = b + s c, three arrays of 512 MiB)
    timed with events on the current stream: median GB/s at 24 B per
    element."""
    import numpy as np
    import torch

    from paper_2212_02362_amd.solver import stream_triad
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    for _ in range(2):
        stream_triad(a, b, c, 0.5)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        stream_triad(a, b, c, 0.5)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    t = float(np.median(ts))
    ok = bool(torch.allclose(a[:1024], b[:1024] + 0.5 * c[:1024]))
    del a, b, c
    torch.cuda.empty_cache()
    return {"GBps": 24.0 * n / t / 1e9, "bytes_per_launch": 24 * n, "median_us": t * 1e6,
            "launches": reps, "kernel": "k_triad (a = b + s c, 16-byte accesses)", "checked": ok}


if __name__ == "__main__":
    main()
