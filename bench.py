"""Benchmark of the fused matrix-free operator and the PCG solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--prec fp32|fp64] [--no-pcg] [--no-cpu-baseline]

Timed region: K applications of y = K_c(x) v on the 340x170x85 cantilever (4.9M
elements, 15.0M DOFs) with seeded x ~ U(0.01, 1), v ~ N(0, 1), rotating over enough
independent (x, v, y) buffer sets (>= 512 MB) that the 256 MB Infinity Cache cannot hold
them, bracketed by torch.cuda.synchronize().  `value` = DOFs processed per second
(GDOF/s).  Alongside, in the same JSON line:
  * roofline: algorithmic bytes per launch / measured launch time vs 8 TB/s,
  * kv_other_precision: the same measurement for the other operator precision,
  * kv_mfma: the BF16 / FP16 matrix-core contraction variant (FP32 storage),
  * kv_torsion_55x55x165: FP32 / FP64 on the torsion mesh,
  * pcg: wall time to ||r|| <= 1e-6 ||f|| for plain FP64 Jacobi-PCG, for FP64
    refinement around an FP32 inner Jacobi-PCG, and for CG preconditioned by the
    geometric-multigrid V-cycle (FP64, and FP32 inside FP64 refinement), with the
    compliance error of each against an FP64 solve to 1e-10,
  * learned_pcg: the learned preconditioner on the 200x100x50 cantilever (pairs
    harvested from the first 10 SIMP iterations, U-Net trained on the GPU, flexible CG
    against Jacobi-PCG on the next iteration's system),
  * cpu_baseline: the CPU oracle's element-by-element K v on a bounded sample.
Only one GPU is supported: --gpus N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one K v launch at 340x170x85 from two rocprofv3 --pmc passes
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, factors from a 1 GiB device copy in the same run),
# valid only for the kernel sources they were taken with (sha256 of kv.hip, dev.h,
# common.h); reported as null once those change.
KV_TRAFFIC = {
    "fp32": (2.0 * 49071.3 + 59171.4) * 1024,
    "fp64": (2.0 * 94440.2 + 118010.8) * 1024,
}
KV_TRAFFIC_SOURCES = {
    "kv.hip": "d2f1041226fdb8f15f2a23303016a4577d1384ff5e3a4ae62cc63f8888814d29",
    "dev.h": "4f632875059f48985c77a57385922168b780fadc82dea0f30fd122a0d3fb5beb",
    "common.h": "df30c16e1b3674dd02ea4ea4ba8d26a6be57acd103967395e33bfc1f6290c412",
}


def kv_traffic(prec: str):
    """Measured HBM bytes per launch if the kernel sources match the measurement."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2604_18020_amd", "csrc")
    for fn, h in KV_TRAFFIC_SOURCES.items():
        with open(os.path.join(csrc, fn), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != h:
                return None
    return KV_TRAFFIC[prec]


def kv_bytes(prec: str, n_node: int, n_elem: int) -> int:
    """Algorithmic HBM bytes of one K v launch: v read once and y written once (3 values
    per node), the density read once per element, the 1-byte BC mask once per node."""
    w = 8 if prec == "fp64" else 4
    return 2 * 3 * w * n_node + w * n_elem + n_node


def time_kv(t, nx, ny, nz, prec, steps, warmup, fixed, seed=42, resident=False,
            scatter="owner", graph=False):
    """Per-launch HIP-event timing of the operator as the CG iterations apply it.  Buffer
    sets are rotated so that >= 512 MB are touched (the 256 MB Infinity Cache cannot hold
    them); resident=True uses one set ("MALL-resident" figures).  scatter selects the
    deterministic default or an atomic-scatter form (whose launch is a clearing pass plus
    the scatter kernel).  graph=True times the `steps` launches replayed as one captured
    HIP graph, the way the solver's CG batches run the operator (the eager loop's time is
    kept beside it); if capture fails the eager loop is the timed region."""
    import numpy as np
    import torch

    import synth_inputs as si

    dt = torch.float64 if prec == "fp64" else torch.float32
    rho, v = si.random_density_and_vector(nx, ny, nz, seed)
    # the operand as the CG iterations apply it: zero on fixed DOFs (K_c acts on the free
    # block; fixed rows are identity), with the library told so
    v[fixed] = 0.0
    set_bytes = kv_bytes(prec, t.n_node, t.n_elem)
    nset = 1 if resident else max(2, -(-512 * 2 ** 20 // set_bytes))
    xs = [torch.tensor(rho, dtype=dt, device="cuda:0") for _ in range(nset)]
    vs = [torch.tensor(v, dtype=dt, device="cuda:0") for _ in range(nset)]
    ys = [torch.empty_like(vs[0]) for _ in range(nset)]
    del rho, v
    for i in range(warmup):
        t.apply_K(xs[i % nset], vs[i % nset], ys[i % nset], prec=prec, v_zero_on_fixed=True,
                  scatter=scatter)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()  # the library launches on the caller's stream
    # Timed region: `steps` launches back to back, bracketed by synchronisations (wall
    # clock) and by HIP events on the launch stream (average launch duration, gaps
    # included).
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        t.apply_K(xs[i % nset], vs[i % nset], ys[i % nset], prec=prec, v_zero_on_fixed=True,
                  scatter=scatter)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    batch_ms = e0.elapsed_time(e1) / steps
    eager_batch_ms, graph_used = batch_ms, False
    if graph:
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for i in range(steps):
                    t.apply_K(xs[i % nset], vs[i % nset], ys[i % nset], prec=prec,
                              v_zero_on_fixed=True, scatter=scatter)
            g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            g.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            batch_ms = e0.elapsed_time(e1) / steps
            graph_used = True
            del g
        except Exception as err:  # capture refused: keep the eager figures
            print(f"graph capture of the operator failed ({err}); eager timing kept",
                  file=sys.stderr)
        t._sync_stream()
    # Per-launch events (diagnostic: each launch's own duration incl. its event overhead).
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for i in range(steps):
        ev[2 * i].record(stream)
        t.apply_K(xs[i % nset], vs[i % nset], ys[i % nset], prec=prec, v_zero_on_fixed=True,
                  scatter=scatter)
        ev[2 * i + 1].record(stream)
    torch.cuda.synchronize()
    launch_ms = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)]
    avg_ms = float(np.mean(launch_ms))
    ok = bool(torch.isfinite(ys[(steps - 1) % nset]).all())
    del xs, vs, ys
    torch.cuda.empty_cache()
    return dict(wall_s=wall, avg_launch_ms=avg_ms, median_launch_ms=float(np.median(launch_ms)),
                batch_ms=batch_ms, eager_batch_ms=eager_batch_ms, graph=graph_used,
                bytes=set_bytes, buffer_sets=nset, finite=ok)


def _solve_timed(t, x, f, tol, **kw):
    import torch
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kw.setdefault("maxit", 60000)
    st = t.pcg_solve(x, f, u, tol=tol, **kw)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    c = float(torch.dot(f, u))
    return u, dict(seconds=sec, iterations=st["iterations"],
                   outer_iterations=st["outer_iterations"], fallbacks=st["fallbacks"],
                   restarts=st["restarts"], status=st["status"],
                   true_rel_residual=st["true_rel_residual"], compliance=c)


def time_pcg(t, nx, ny, nz, tol, volfrac=0.3):
    """Cold-start solves of K(x) u = f at uniform density to ||b - K u|| <= tol ||f||:
    plain FP64 Jacobi-PCG against FP64 refinement around an FP32 Jacobi-PCG, with the
    compliance of each against a plain FP64 solve to 1e-10."""
    import torch

    import synth_inputs as si

    f = torch.tensor(si.cantilever_load(nx, ny, nz), device="cuda:0")
    t.set_loads(f)
    return pcg_compare(t, f, tol, volfrac)


def pcg_compare(t, f, tol, volfrac=0.3):
    """The solves of time_pcg for a context whose BCs and loads are set (f on device)."""
    import torch

    x = torch.full((t.n_elem,), volfrac, dtype=torch.float64, device="cuda:0")
    _, ref = _solve_timed(t, x, f, 1e-10, mode="plain_fp64", check_every=64)
    out = {"reference_compliance_tol1e-10": ref["compliance"]}
    # the multigrid hierarchy is allocated on first use: one untimed solve first
    _solve_timed(t, x, f, 1e-2, mode="plain_fp64", precond="mg", check_every=4)
    for name, kw in SOLVERS:
        _, r = _solve_timed(t, x, f, tol, **kw)
        r["compliance_rel_err"] = abs(r["compliance"] - ref["compliance"]) / abs(ref["compliance"])
        out[name] = r
    out["speedup_ir_over_plain"] = out["plain_fp64"]["seconds"] / out["ir_fp32"]["seconds"]
    out["speedup_ir_mg_over_plain"] = out["plain_fp64"]["seconds"] / out["ir_fp32_mg"]["seconds"]
    return out


# Solvers compared on one system: Jacobi-PCG in FP64, FP64 refinement around FP32
# Jacobi-PCG, and CG preconditioned by the geometric-multigrid V-cycle (FP64, and FP32
# inside FP64 refinement).
SOLVERS = [("plain_fp64", dict(mode="plain_fp64", check_every=64)),
           ("ir_fp32", dict(mode="ir", inner_prec="fp32", inner_tol=1e-4, max_outer=30,
                            check_every=64)),
           ("plain_fp64_mg", dict(mode="plain_fp64", precond="mg", check_every=4)),
           ("ir_fp32_mg", dict(mode="ir", inner_prec="fp32", inner_tol=1e-4, max_outer=30,
                               precond="mg", check_every=4))]


def time_nn(workload="cantilever_200x100x50", simp_iters=10, per_solve=200, every=5,
            train_steps=400, batch=4, lr=1e-3, tol=1e-6, volfrac=0.3):
    """Learned preconditioner: harvest (r, e) pairs from the FP64 Jacobi-PCG solves of
    the first SIMP iterations, train the U-Net (BF16) on the GPU, then solve the next
    SIMP iteration's system to tol with plain FP64 Jacobi-PCG, FP32 Jacobi-PCG inside
    FP64 refinement, and flexible CG with the learned preconditioner inside FP64
    refinement."""
    import numpy as np
    import torch

    import synth_inputs as si
    from paper_2604_18020_amd import Tosimp, learned

    cfg = si.CONFIGS[workload]
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    t = Tosimp(0).set_mesh(nx, ny, nz)
    t.set_bcs(si.cantilever_fixed_dofs(nx, ny, nz))
    f = torch.tensor(si.cantilever_load(nx, ny, nz), device="cuda:0")
    t.set_loads(f)
    x = torch.full((t.n_elem,), volfrac, dtype=torch.float64, device="cuda:0")
    xp = x.clone()
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    ps, stats = learned.harvest(t, x, xp, u, iters=simp_iters, every=every, per_solve=per_solve,
                                f=f, volfrac=volfrac)
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    t.nn_create(16, bf16=True)
    t.nn_set_weights(learned.he_normal_weights(t, 0))
    t.nn_set_loss("mse")
    t0 = time.perf_counter()
    losses = learned.train(t, ps, train_steps, batch=batch, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del ps
    torch.cuda.empty_cache()
    out = {"workload": f"{workload}: pairs from SIMP iterations 1-{simp_iters}, solve of "
                       f"iteration {simp_iters + 1}, cold start, tol {tol:g}",
           "pairs": int(sum(s["solve"]["harvested"] for s in stats)),
           "harvest_s": t_harvest, "train_steps": train_steps, "batch": batch,
           "train_s": t_train, "loss": "relative MSE to the unit-RMS error",
           "loss_first50": float(np.mean(losses[:50])),
           "loss_last50": float(np.mean(losses[-50:]))}
    _solve_timed(t, xp, f, 1e-2, mode="plain_fp64", precond="mg", check_every=4)  # allocation
    nn = dict(mode="ir", inner_prec="fp32", inner_tol=1e-4, precond="nn", check_every=8)
    for name, kw in [("plain_fp64_jacobi", dict(mode="plain_fp64", check_every=64)),
                     ("ir_fp32_jacobi", dict(mode="ir", inner_prec="fp32", inner_tol=1e-4,
                                             check_every=64)),
                     ("ir_fp32_mg", dict(mode="ir", inner_prec="fp32", inner_tol=1e-4,
                                         precond="mg", check_every=4)),
                     # guarded: an inner solve without a new residual minimum for 50
                     # iterations is finished by Jacobi-PCG; unguarded: the network alone
                     ("ir_fp32_nn_fcg_guarded", dict(nn, maxit=20000)),
                     ("ir_fp32_nn_fcg_unguarded", dict(nn, maxit=12000, nn_stall=-1))]:
        _, r = _solve_timed(t, xp, f, tol, **kw)
        out[name] = r
    # ablation: the untrained (He-normal) network, guarded
    t.nn_set_weights(learned.he_normal_weights(t, 0))
    _, r = _solve_timed(t, xp, f, tol, **dict(nn, maxit=20000))
    out["ir_fp32_nn_fcg_untrained_guarded"] = r
    t.close()
    return out


def _problem(workload):
    import torch

    import synth_inputs as si
    from paper_2604_18020_amd import Tosimp

    cfg = si.CONFIGS[workload]
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    t = Tosimp(0).set_mesh(nx, ny, nz)
    fixed, f = si.bcs_and_load(cfg["kind"], nx, ny, nz)
    t.set_bcs(fixed)
    fd = torch.tensor(f, device="cuda:0")
    t.set_loads(fd)
    return t, cfg, fd, fixed


def precision_study(workload="cantilever_340x170x85", lanczos_steps=1500, tol=1e-6):
    """Condition estimate (Lanczos, FP64) at uniform density, the precision rule
    u_l kappa < 1 for each inner precision, and refinement solves with FP32, BF16-MFMA and
    FP16-MFMA inner operators (rule not enforced, to show the outcome), each compared with
    an FP64 solve to 1e-10 in compliance, displacement and sensitivity."""
    import numpy as np
    import torch

    from paper_2604_18020_amd import tridiag_extremes

    t, cfg, f, fixed = _problem(workload)
    x = torch.full((t.n_elem,), cfg["volfrac"], dtype=torch.float64, device="cuda:0")
    rng = np.random.default_rng(7)
    v = rng.standard_normal(t.n_dof)
    v[fixed] = 0.0  # the Krylov space stays in the free block
    v0 = torch.tensor(v, device="cuda:0")
    out = {"workload": workload, "density": cfg["volfrac"]}
    for scaled in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, b = t.lanczos(x, v0, lanczos_steps, jacobi_scaled=scaled)
        lo, hi = tridiag_extremes(a, b)
        out["lanczos_jacobi" if scaled else "lanczos"] = {
            "steps": int(len(a)), "lambda_min": lo, "lambda_max": hi, "kappa": hi / lo,
            "seconds": time.perf_counter() - t0}
    kappa = out["lanczos_jacobi"]["kappa"]
    u = {"fp32": 2.0 ** -24, "bf16_mfma": 2.0 ** -8, "fp16_mfma": 2.0 ** -11}
    out["rule"] = {k: {"unit_roundoff": v, "u_kappa": v * kappa, "allowed": v * kappa < 1}
                   for k, v in u.items()}
    u_ref, ref = _solve_timed(t, x, f, 1e-10, mode="plain_fp64", check_every=64)
    dc_ref, c_ref = t.sensitivity(x, u_ref)
    dcn = float(torch.max(torch.abs(dc_ref)))
    un = float(torch.linalg.vector_norm(u_ref))
    runs = [("plain_fp64", dict(mode="plain_fp64", check_every=64))]
    runs += [(f"ir_{p}", dict(mode="ir", inner_prec=p, inner_tol=1e-4, max_outer=12,
                              check_every=64)) for p in ("fp32", "bf16_mfma", "fp16_mfma")]
    for name, kw in runs:
        try:
            uu, r = _solve_timed(t, x, f, tol, **kw)
        except Exception as e:  # a refused or broken-down solve is a result too
            out[name] = {"error": str(e)}
            continue
        dc, c = t.sensitivity(x, uu)
        r["compliance_rel_err"] = abs(c - c_ref) / abs(c_ref)
        r["displacement_rel_err"] = float(torch.linalg.vector_norm(uu - u_ref)) / un
        r["sensitivity_max_rel_err"] = float(torch.max(torch.abs(dc - dc_ref))) / dcn
        out[name] = r
    out["reference"] = {"tol": 1e-10, "iterations": ref["iterations"], "compliance": c_ref}
    t.close()
    return out


def simp_study(workload, iters=None, tol=None):
    """SIMP iterations from uniform density with warm-started solves: plain FP64
    Jacobi-PCG against FP64 refinement around FP32 Jacobi-PCG (same tolerance)."""
    import torch

    t, cfg, f, _ = _problem(workload)
    iters = iters or cfg["simp_iters"]
    tol = tol or cfg["pcg_tol"]
    out = {"workload": workload, "iterations": iters, "tol": tol}
    finals = {}
    for name, kw in [("plain_fp64", dict(mode="plain_fp64")),
                     ("ir_fp32", dict(mode="ir", inner_prec="fp32", inner_tol=1e-4))]:
        x = torch.full((t.n_elem,), cfg["volfrac"], dtype=torch.float64, device="cuda:0")
        xp = x.clone()
        u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
        comp, its = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            st = t.simp_step(x, xp, u, volfrac=cfg["volfrac"], move=0.2, tol=tol, maxit=50000,
                             check_every=64, **kw)
            comp.append(st["compliance"])
            its.append(st["solve"]["iterations"])
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "compliance": comp,
                     "cg_iterations": its, "total_cg_iterations": int(sum(its))}
        finals[name] = xp.clone()
    out["speedup_ir_over_plain"] = out["plain_fp64"]["seconds"] / out["ir_fp32"]["seconds"]
    c0, c1 = out["plain_fp64"]["compliance"], out["ir_fp32"]["compliance"]
    out["max_compliance_rel_diff"] = max(abs(a - b) / abs(a) for a, b in zip(c0, c1))
    out["final_density_max_diff"] = float(torch.max(torch.abs(finals["plain_fp64"] -
                                                              finals["ir_fp32"])))
    t.close()
    return out


def kv_reps(n_elem):
    """Launches per K v timing: 5e7 / n_elem, at least 100 and at most 2,000."""
    return max(100, min(2000, int(5e7 // n_elem)))


def kv_study(workloads=("cantilever_120x60x30", "cantilever_340x170x85")):
    """K v in every precision, HBM-bound (rotated buffer sets) and MALL-resident (one
    set), on the K v microbenchmark inputs."""
    out = {}
    for w in workloads:
        t, cfg, _, fixed = _problem(w)
        nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
        reps = kv_reps(t.n_elem)
        res = {"launches": reps}
        for p in ("fp64", "fp32", "bf16_mfma", "fp16_mfma"):
            res[p] = {}
            for label, resident in (("hbm", False), ("mall_resident", True)):
                r = time_kv(t, nx, ny, nz, p, reps, 10, fixed, resident=resident)
                us = r["batch_ms"] * 1e3
                res[p][label] = {"avg_launch_us": us, "median_launch_us": r["median_launch_ms"] * 1e3,
                                 "gdof_s": t.n_dof / (us * 1e-6) / 1e9,
                                 "algorithmic_gbs": r["bytes"] / (us * 1e-6) / 1e9,
                                 "frac_of_8tbs": r["bytes"] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                 "buffer_sets": r["buffer_sets"], "finite": r["finite"]}
        out[w] = res
        t.close()
    return out


def projection_study(workload="cantilever_340x170x85", reps=200, sets=4):
    """The Heaviside projection kernel (and its chain-rule form) on one density field per
    element of the mesh: algorithmic bytes 16 (read xbar, write out) and 24 (also g) per
    element; buffer sets rotated so the 256 MB Infinity Cache cannot hold them."""
    import numpy as np
    import torch

    t, cfg, _, _ = _problem(workload)
    n = t.n_elem
    rng = np.random.default_rng(3)
    xs = [torch.tensor(rng.uniform(0.0, 1.0, n), device="cuda:0") for _ in range(sets)]
    gs = [torch.tensor(rng.standard_normal(n), device="cuda:0") for _ in range(sets)]
    outs = [torch.empty(n, dtype=torch.float64, device="cuda:0") for _ in range(sets)]
    res = {"workload": workload, "n_elem": n, "launches": reps}
    for label, chain, per in (("projection", False, 16), ("chain_rule", True, 24)):
        for k in range(8):
            t.project(xs[k % sets], 8.0, 0.5, g=gs[k % sets] if chain else None, out=outs[k % sets])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for k in range(reps):
            t.project(xs[k % sets], 8.0, 0.5, g=gs[k % sets] if chain else None, out=outs[k % sets])
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = per * n / (us * 1e-6) / 1e9
        res[label] = {"avg_launch_us": us, "bytes_per_launch": per * n, "algorithmic_gbs": gbs,
                      "frac_of_8tbs": gbs / HBM_PEAK_GBS}
    t.close()
    return res


def simp_kernels_study(workload="cantilever_340x170x85", reps=20, sets=4):
    """The SIMP pieces beside the solve, one density field per element of the mesh, buffer
    sets rotated (>= 4 x the Infinity Cache is not guaranteed for the element fields, so
    the per-kernel HBM bytes come from the profiler's counters): sensitivity (with the
    compliance, one host synchronisation per call), density filter forward and adjoint,
    OC update (bisection, synchronises), Heaviside projection.  Wall time per call."""
    import numpy as np
    import torch

    t, cfg, _, _ = _problem(workload)
    n = t.n_elem
    rng = np.random.default_rng(5)
    xs = [torch.tensor(rng.uniform(0.01, 1.0, n), device="cuda:0") for _ in range(sets)]
    us = [torch.tensor(rng.standard_normal(t.n_dof), device="cuda:0") for _ in range(sets)]
    dcs = [torch.tensor(-rng.uniform(0.1, 1.0, n), device="cuda:0") for _ in range(sets)]
    outs = [torch.empty(n, dtype=torch.float64, device="cuda:0") for _ in range(sets)]
    outs2 = [torch.empty(n, dtype=torch.float64, device="cuda:0") for _ in range(sets)]
    calls = {
        "sensitivity": lambda k: t.sensitivity(xs[k], us[k], outs[k]),
        "filter_forward": lambda k: t.filter(xs[k], "forward", outs[k]),
        "filter_adjoint": lambda k: t.filter(dcs[k], "adjoint", outs[k]),
        "oc_update": lambda k: t.oc_update(xs[k], dcs[k], 0.3, 0.2, outs[k], outs2[k]),
        "projection": lambda k: t.project(xs[k], 8.0, 0.5, out=outs[k]),
    }
    res = {"workload": workload, "n_elem": n, "calls": reps}
    for name, fn in calls.items():
        for k in range(4):
            fn(k % sets)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(reps):
            fn(k % sets)
        torch.cuda.synchronize()
        res[name] = {"wall_us_per_call": (time.perf_counter() - t0) * 1e6 / reps}
    t.close()
    return res


def scatter_study(workload="cantilever_340x170x85", steps=100, warmup=10):
    """The operator's scatter designs side by side on one mesh: owner-computes (the
    default: every node written once from registers, no atomics) against the atomic
    scatter of the paper's fused algorithm, as stated (one thread per element, 24 global
    atomic additions) and reduced per 8x8x4 brick in LDS (global atomics on brick faces
    only).  Same buffers, same byte count per launch: algorithmic GB/s over the average
    launch (the atomic forms include their clearing pass)."""
    t, cfg, _, fixed = _problem(workload)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    out = {"workload": workload, "n_elem": t.n_elem, "n_dof": t.n_dof}
    for prec in ("fp32", "fp64"):
        for scatter in ("owner", "atomic_brick", "atomic_element"):
            r = time_kv(t, nx, ny, nz, prec, steps, warmup, fixed, scatter=scatter)
            gbs = r["bytes"] / (r["batch_ms"] * 1e-3) / 1e9
            out[f"{prec}_{scatter}"] = {"us_per_launch": r["batch_ms"] * 1e3,
                                        "median_launch_us": r["median_launch_ms"] * 1e3,
                                        "algorithmic_gbs": gbs, "frac_of_8tbs": gbs / HBM_PEAK_GBS,
                                        "finite": r["finite"]}
    t.close()
    return out


def mg_study(workload="cantilever_340x170x85", reps=3, tol=1e-6, volfrac=0.3):
    """Cold-start multigrid-preconditioned CG at uniform density (the fastest solves of
    the PCG leg) repeated on one mesh: plain FP64 and FP64 refinement around FP32, best of
    `reps` wall times with iteration counts."""
    import torch

    t, cfg, f, _ = _problem(workload)
    x = torch.full((t.n_elem,), volfrac, dtype=torch.float64, device="cuda:0")
    out = {"workload": workload, "tol": tol, "density": volfrac}
    for mode in ("plain_fp64", "ir"):
        best = None
        for _ in range(reps):
            _, r = _solve_timed(t, x, f, tol, mode=mode, precond="mg", check_every=4)
            if best is None or r["seconds"] < best["seconds"]:
                best = r
        out[mode] = best
    t.close()
    return out


def unet_study(workload="cantilever_200x100x50", applies=20, train_steps=5, base=16):
    """The learned preconditioner's kernels on their own: the U-Net (BF16 storage, random
    He-scaled weights, uniform density 0.3) applied `applies` times to a random residual,
    then `train_steps` Adam steps on batches of four random pairs.  Per-call wall times
    (HIP synchronised) and the forward's matrix-core rate."""
    import numpy as np
    import torch

    t, cfg, f, _ = _problem(workload)
    t.nn_create(base, bf16=True)
    rng = np.random.default_rng(0)
    t.nn_set_weights(rng.standard_normal(t.nn_params).astype(np.float32) * 0.05)
    t.nn_set_density(torch.full((t.n_elem,), 0.3, dtype=torch.float64, device="cuda:0"))
    gen = torch.Generator(device="cuda:0").manual_seed(1)
    r = torch.randn(t.n_dof, dtype=torch.float32, device="cuda:0", generator=gen)
    z = torch.empty_like(r)
    for _ in range(3):
        t.nn_apply(r, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(applies):
        t.nn_apply(r, z)
    torch.cuda.synchronize()
    apply_s = (time.perf_counter() - t0) / applies
    rb = torch.randn(4, t.n_dof, dtype=torch.float32, device="cuda:0", generator=gen)
    eb = torch.randn(4, t.n_dof, dtype=torch.float32, device="cuda:0", generator=gen)
    t.nn_train_step(rb, eb, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(train_steps):
        t.nn_train_step(rb, eb, 1e-4)
    torch.cuda.synchronize()
    train_s = (time.perf_counter() - t0) / train_steps
    # matrix-core work of one forward: 2 x taps x cin x cout per output voxel and layer
    g = [(cfg["nx"] + 1, cfg["ny"] + 1, cfg["nz"] + 1)]
    for _ in range(2):
        g.append(tuple((d - 1) // 2 + 1 for d in g[-1]))
    nvox = [a * b * c for a, b, c in g]
    b = base
    layers = [(4, b, 27, 0), (b, b, 27, 0), (b, 2 * b, 27, 1), (2 * b, 2 * b, 27, 1),
              (2 * b, 4 * b, 27, 2), (4 * b, 4 * b, 27, 2), (4 * b, 4 * b, 27, 2),
              (6 * b, 2 * b, 27, 1), (2 * b, 2 * b, 27, 1), (3 * b, b, 27, 0), (b, b, 27, 0),
              (b, 3, 1, 0)]
    flop = sum(2.0 * taps * ci * co * nvox[lv] for ci, co, taps, lv in layers)
    t.close()
    return {"workload": workload, "base": base, "storage": "bf16", "apply_ms": apply_s * 1e3,
            "forward_gflop": flop / 1e9, "forward_tflops": flop / apply_s / 1e12,
            "frac_of_bf16_peak": flop / apply_s / 2.5e15, "train_step_ms_batch4": train_s * 1e3}


def pcg_cold_study(workloads=("cantilever_120x60x30", "torsion_55x55x165",
                              "cantilever_200x100x50"), tol=1e-6):
    """Cold-start PCG at uniform density on the other benchmark meshes (the main line
    covers 340x170x85): plain FP64 against FP32 refinement, compliance against 1e-10."""
    out = {}
    for w in workloads:
        t, cfg, f, _ = _problem(w)
        out[w] = pcg_compare(t, f, tol, cfg["volfrac"])
        t.close()
    return out


class PowerMeter:
    """Board power from the amdgpu hwmon sensor (power1_input, microwatts), polled by a
    thread every `period` s and integrated by the trapezoid rule over the measured
    window.  The sensor's own update cadence limits the resolution: windows are kept
    >= 1 s by repeating the measured work."""

    def __init__(self, period=0.02):
        import glob
        self.path = None
        for d in sorted(glob.glob("/sys/class/drm/card*/device/hwmon/hwmon*")):
            try:
                with open(os.path.join(d, "name")) as fh:
                    if fh.read().strip() == "amdgpu" and os.access(os.path.join(d, "power1_input"), os.R_OK):
                        self.path = os.path.join(d, "power1_input")
                        break
            except OSError:
                continue
        self.period = period
        self.samples = []

    def _read(self):
        with open(self.path) as fh:
            return float(fh.read()) * 1e-6

    def __enter__(self):
        import threading
        self.samples = []
        self._stop = threading.Event()

        def run():
            while not self._stop.is_set():
                try:
                    self.samples.append((time.perf_counter(), self._read()))
                except (OSError, ValueError):
                    pass
                self._stop.wait(self.period)

        if self.path:
            self._t = threading.Thread(target=run, daemon=True)
            self._t.start()
        return self

    def __exit__(self, *exc):
        if self.path:
            self._stop.set()
            self._t.join()

    def energy(self):
        """(joules, mean watts) over the samples, or (None, None) without a sensor."""
        if len(self.samples) < 2:
            return None, None
        e = sum(0.5 * (w0 + w1) * (t1 - t0)
                for (t0, w0), (t1, w1) in zip(self.samples, self.samples[1:]))
        span = self.samples[-1][0] - self.samples[0][0]
        return e, e / span


def _solve_energy(t, x, f, tol, min_window=1.5, **kw):
    """One timed solve (as _solve_timed), then the same solve repeated for >= min_window
    seconds under the power meter: energy per solve and mean board power."""
    import torch
    u, r = _solve_timed(t, x, f, tol, **kw)
    meter = PowerMeter()
    n, t0 = 0, time.perf_counter()
    with meter:
        while time.perf_counter() - t0 < min_window:
            u.zero_()
            t.pcg_solve(x, f, u, tol=tol, **kw)
            torch.cuda.synchronize()
            n += 1
    e, w = meter.energy()
    r["energy_J_per_solve"] = None if e is None else e / n
    r["mean_board_W"] = w
    return u, r


def presets_study(tol=1e-6):
    """Paper presets and reports: the cold-start FEA ladder of 4:2:1 cantilevers at uniform
    density 0.5 from 216 k to 8 M elements (time, iterations, energy per solve, VRAM), and
    the MBB and bridge stress tests at 150x50x25 (FEA-only cold start at uniform density
    volfrac, and 60 SIMP iterations with cold-start solves)."""
    import torch

    import synth_inputs as si
    from paper_2604_18020_amd import Tosimp

    gb = 1024.0 ** 3
    out = {"fea_ladder": [], "vram_note": "device memory in use (hipMemGetInfo) at the end of "
                                           "each ladder size, and the part the library's "
                                           "context holds (mesh workspace + multigrid hierarchy)"}
    solvers = [s for s in SOLVERS]
    for nx, ny, nz in si.FEA_LADDER:
        torch.cuda.empty_cache()
        free0, total = torch.cuda.mem_get_info()
        t = Tosimp(0).set_mesh(nx, ny, nz)
        fixed, f = si.bcs_and_load("cantilever", nx, ny, nz)
        t.set_bcs(fixed)
        fd = torch.tensor(f, device="cuda:0")
        t.set_loads(fd)
        x = torch.full((t.n_elem,), 0.5, dtype=torch.float64, device="cuda:0")
        row = {"mesh": f"{nx}x{ny}x{nz}", "n_elem": t.n_elem, "n_dof": t.n_dof}
        _solve_timed(t, x, fd, 1e-2, mode="plain_fp64", precond="mg", check_every=4)
        for name, kw in solvers:
            _, r = _solve_energy(t, x, fd, tol, **kw)
            row[name] = r
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        row["vram_in_use_GB"] = (total - free1) / gb
        row["vram_context_and_vectors_GB"] = (free0 - free1) / gb
        out["fea_ladder"].append(row)
        del x, fd
        t.close()
        print(json.dumps({"ladder": row["mesh"], **{k: (v["seconds"], v["iterations"])
                                                  for k, v in row.items() if isinstance(v, dict)}}),
              file=sys.stderr, flush=True)
    for name in ("mbb_150x50x25", "bridge_150x50x25"):
        cfg = si.CONFIGS[name]
        nx, ny, nz, vf = cfg["nx"], cfg["ny"], cfg["nz"], cfg["volfrac"]
        t = Tosimp(0).set_mesh(nx, ny, nz)
        fixed, f = si.bcs_and_load(cfg["kind"], nx, ny, nz)
        t.set_bcs(fixed)
        fd = torch.tensor(f, device="cuda:0")
        t.set_loads(fd)
        x = torch.full((t.n_elem,), vf, dtype=torch.float64, device="cuda:0")
        res = {"fea_cold_start": {}, "simp60_cold_start": {}}
        _solve_timed(t, x, fd, 1e-2, mode="plain_fp64", precond="mg", check_every=4)
        for sname, kw in solvers:
            res["fea_cold_start"][sname] = _solve_energy(t, x, fd, tol, **kw)[1]
        for sname, kw in (("plain_fp64_jacobi", dict(mode="plain_fp64", check_every=64)),
                          ("ir_fp32_mg", dict(mode="ir", inner_prec="fp32", inner_tol=1e-4,
                                              precond="mg", check_every=4))):
            xs = torch.full((t.n_elem,), vf, dtype=torch.float64, device="cuda:0")
            xp = xs.clone()
            u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
            cs, its = [], 0
            meter = PowerMeter()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with meter:
                for _ in range(cfg["simp_iters"]):
                    u.zero_()  # cold start
                    st = t.simp_step(xs, xp, u, volfrac=vf, move=0.2, tol=tol, maxit=60000, **kw)
                    cs.append(st["compliance"])
                    its += st["solve"]["iterations"]
                torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            e, w = meter.energy()
            res["simp60_cold_start"][sname] = {"seconds": sec, "cg_iterations": its,
                                               "final_compliance": cs[-1], "energy_J": e,
                                               "mean_board_W": w}
        a_, b_ = (res["simp60_cold_start"][k]["final_compliance"]
                  for k in ("plain_fp64_jacobi", "ir_fp32_mg"))
        res["simp60_cold_start"]["final_compliance_rel_diff"] = abs(a_ - b_) / abs(a_)
        res["simp60_cold_start"]["speedup"] = (res["simp60_cold_start"]["plain_fp64_jacobi"]["seconds"]
                                               / res["simp60_cold_start"]["ir_fp32_mg"]["seconds"])
        out[name] = res
        t.close()
        print(json.dumps({name: res["simp60_cold_start"]["speedup"]}), file=sys.stderr, flush=True)
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload="cantilever_340x170x85", kv_budget_s=10.0, pcg_iters=3,
                 pcg_iterations_to_tol=None):
    """The oracle on the host: its element-by-element K v (gather, dense 24x24 product,
    scatter-add) on the workload's mesh, repeated for ~kv_budget_s, and a few iterations
    of its Jacobi-PCG (same operator) on the workload's cold-start system (uniform
    density 0.3), whose time per iteration times the iterations the FP64 solve takes to
    1e-6 (pcg_iterations_to_tol, when given) estimates its time to 1e-6."""
    import numpy as np

    import synth_inputs as si
    from oracle import fem, solvers

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    cfg = si.CONFIGS[workload]
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    rho, v = si.random_density_and_vector(nx, ny, nz, 42)
    KE = fem.element_stiffness(0.3)
    E = fem.simp_modulus(rho, 1.0, 1e-9, 3.0)
    fixed = fem.fixed_mask(v.size, si.cantilever_fixed_dofs(nx, ny, nz))
    calls, t0 = 0, time.perf_counter()
    while True:
        fem.apply_K_elementwise(nx, ny, nz, E, KE, v, fixed)
        calls += 1
        el = time.perf_counter() - t0
        if el >= kv_budget_s:
            break
    # Jacobi-PCG: a bounded number of iterations on the cold-start system
    E3 = fem.simp_modulus(np.full(nx * ny * nz, 0.3), 1.0, 1e-9, 3.0)
    f = si.cantilever_load(nx, ny, nz)
    d = fem.diag_K(nx, ny, nz, E3, KE, fixed)
    t1 = time.perf_counter()
    _, its, _ = solvers.pcg_jacobi(lambda x: fem.apply_K_elementwise(nx, ny, nz, E3, KE, x, fixed),
                                   d, f, tol=1e-6, maxit=pcg_iters)
    per_it = (time.perf_counter() - t1) / max(its, 1)
    out = {"value": calls * v.size / el / 1e9, "unit": "GDOF/s", "cores": int(threads),
           "kind": "oracle",
           "sample": f"oracle element-by-element K v on {workload} ({v.size} DOFs), {calls} "
                     f"calls in {el:.1f} s; {its} oracle Jacobi-PCG iterations on its "
                     f"cold-start system (uniform density 0.3)",
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "blas_threads": int(threads),
           "pcg_seconds_per_iteration": per_it}
    if pcg_iterations_to_tol:
        out["pcg_seconds_to_1e-6_extrapolated"] = per_it * pcg_iterations_to_tol
        out["pcg_iterations_to_1e-6"] = int(pcg_iterations_to_tol)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cantilever_340x170x85")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--pcg-tol", type=float, default=1e-6)
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned-preconditioner leg")
    ap.add_argument("--suite", action="store_true",
                    help="instead of the benchmark line: precision study (340x170x85) and "
                         "SIMP runs (120x60x30, torsion 55x55x165), one JSON line each")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--presets", action="store_true",
                    help="paper presets and reports: FEA ladder to 8M elements with energy and "
                         "VRAM, MBB and bridge stress tests (prints that JSON only)")
    ap.add_argument("--simp-kernels", action="store_true",
                    help="time the SIMP kernels beside the solve on the workload (prints that "
                         "JSON only)")
    ap.add_argument("--mg-study", action="store_true",
                    help="time the multigrid-preconditioned CG solves on the workload (prints "
                         "that JSON only)")
    ap.add_argument("--unet-study", action="store_true",
                    help="time the U-Net preconditioner's forward application and training "
                         "step at 200x100x50 (prints that JSON only)")
    ap.add_argument("--scatter-study", action="store_true",
                    help="time the owner-computes operator against its atomic-scatter forms "
                         "on the workload (prints that JSON only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (for scaling profiler byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sharded design, one process per GPU, is documented with it).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth_inputs as si
    from paper_2604_18020_amd import Tosimp

    if a.presets:
        print(json.dumps({"presets_study": presets_study()}), flush=True)
        return
    if a.mg_study:
        print(json.dumps({"mg_study": mg_study(a.workload)}), flush=True)
        return
    if a.unet_study:
        print(json.dumps({"unet_study": unet_study()}), flush=True)
        return
    if a.simp_kernels or a.scatter_study:
        if a.copy_calibration:
            src = torch.empty(2 ** 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
        if a.scatter_study:
            print(json.dumps({"scatter_study": scatter_study(a.workload, a.steps, a.warmup)}),
                  flush=True)
        else:
            print(json.dumps({"simp_kernels_study": simp_kernels_study(a.workload)}), flush=True)
        return
    if a.suite:
        print(json.dumps({"kv_study": kv_study()}), flush=True)
        print(json.dumps({"projection_study": projection_study()}), flush=True)
        print(json.dumps({"pcg_cold_study": pcg_cold_study()}), flush=True)
        print(json.dumps({"precision_study": precision_study()}), flush=True)
        print(json.dumps({"simp_study": simp_study("cantilever_120x60x30")}), flush=True)
        print(json.dumps({"simp_study": simp_study("torsion_55x55x165")}), flush=True)
        return

    cfg = si.CONFIGS[a.workload]
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    t = Tosimp(0).set_mesh(nx, ny, nz)
    fixed = (si.cantilever_fixed_dofs if cfg["kind"] == "cantilever" else si.torsion_fixed_dofs)(nx, ny, nz)
    t.set_bcs(fixed)

    if a.copy_calibration:
        src = torch.empty(2 ** 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    main_kv = time_kv(t, nx, ny, nz, a.prec, a.steps, a.warmup, fixed, graph=True)
    other = "fp64" if a.prec == "fp32" else "fp32"
    other_kv = time_kv(t, nx, ny, nz, other, max(20, a.steps // 4), 5, fixed, graph=True)

    ms = main_kv["wall_s"] * 1e3 / a.steps
    value = t.n_dof / (ms * 1e-3) / 1e9
    # achieved: algorithmic bytes per launch over the average launch duration that the
    # HIP events around the timed region (one graph replay of the launches) give
    achieved = main_kv["bytes"] / (main_kv["batch_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": kv_traffic(a.prec),
                "bytes_per_launch": main_kv["bytes"],
                "avg_launch_us": main_kv["batch_ms"] * 1e3,
                "timed_as": "hip_graph" if main_kv["graph"] else "eager_launches",
                "eager_avg_launch_us": main_kv["eager_batch_ms"] * 1e3,
                "per_launch_event_avg_us": main_kv["avg_launch_ms"] * 1e3,
                "per_launch_event_median_us": main_kv["median_launch_ms"] * 1e3}
    line = {
        "metric": "K·v GDOF/s + PCG time-to-1e-6 residual: plain FP64 vs mixed/learned form",
        "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if a.prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": a.workload, "n_elem": t.n_elem, "n_dof": t.n_dof,
                   "operator_precision": a.prec, "buffer_sets": main_kv["buffer_sets"],
                   "inputs": "rho~U(0.01,1), v~N(0,1) zeroed on fixed DOFs, seed 42; "
                             "cantilever BCs"},
        "roofline": roofline,
        "kv_other_precision": {
            "precision": other,
            "gdof_s": t.n_dof / (other_kv["batch_ms"] * 1e-3) / 1e9,
            "achieved_gbs": other_kv["bytes"] / (other_kv["batch_ms"] * 1e-3) / 1e9,
            "frac": other_kv["bytes"] / (other_kv["batch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "avg_launch_us": other_kv["batch_ms"] * 1e3,
            "per_launch_event_avg_us": other_kv["avg_launch_ms"] * 1e3,
            "traffic": kv_traffic(other)},
    }
    def summary(r, prec):
        us = r["batch_ms"] * 1e3
        return {"gdof_s": t.n_dof / (us * 1e-6) / 1e9, "achieved_gbs": r["bytes"] / (us * 1e-6) / 1e9,
                "frac": r["bytes"] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "avg_launch_us": us}
    # low-precision contraction on the matrix cores (FP32 storage, FP32 accumulate)
    line["kv_mfma"] = {p: summary(time_kv(t, nx, ny, nz, p, 50, 5, fixed), p)
                       for p in ("bf16_mfma", "fp16_mfma")}
    if not a.no_pcg:
        line["pcg"] = dict(workload=f"{a.workload}, cold start, uniform density 0.3, "
                                    f"tol {a.pcg_tol:g}",
                           **time_pcg(t, nx, ny, nz, a.pcg_tol))
    t.close()
    # the torsion mesh (55x55x165, 499,125 elements)
    tor = Tosimp(0).set_mesh(55, 55, 165)
    tfix = si.torsion_fixed_dofs(55, 55, 165)
    tor.set_bcs(tfix)
    line["kv_torsion_55x55x165"] = {}
    for p in ("fp32", "fp64"):
        r = time_kv(tor, 55, 55, 165, p, 100, 10, tfix)
        us = r["batch_ms"] * 1e3
        line["kv_torsion_55x55x165"][p] = {
            "gdof_s": tor.n_dof / (us * 1e-6) / 1e9, "avg_launch_us": us,
            "frac": r["bytes"] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    tor.close()
    if not a.no_nn:
        line["learned_pcg"] = time_nn()
    if not a.no_cpu_baseline:
        its = line.get("pcg", {}).get("plain_fp64", {}).get("iterations")
        line["cpu_baseline"] = cpu_baseline(a.workload, pcg_iterations_to_tol=its)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
