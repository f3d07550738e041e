"""Training pipeline of the learned preconditioner (orchestration of library calls).

1. harvest: run SIMP iterations with plain FP64 Jacobi-PCG.  With the load vector given,
   each step's solution is refined to a tighter tolerance on the same system (ref_tol,
   default 1e-10) and the step's Jacobi-PCG run is replayed from its warm start (the
   library's CG is deterministic: the same iterates), copying r_k and e_k = u* - u_k
   (formed in FP64, then stored in FP32) every `every` iterations.  Snapshots are taken
   while the solve has not converged, so every harvested ||r_k|| exceeds tol ||b||, and
   K e_k - r_k = -r* with ||r*|| <= ref_tol ||b|| up to the FP32 storage of r_k and e_k
   (an FP32 u_k differenced afterwards would carry 2^-24 ||u*||, large against the late
   errors).  Without the load vector the pairs come from the step's own solve and the
   library forms e_k from the stored FP32 u_k.  All pairs stay resident in HBM.
2. train: Adam steps on batches of consecutive pairs of one SIMP iteration (the network's
   density input is that iteration's filtered density).
3. solve: flexible CG with the trained network inside FP64 iterative refinement.

Every numerical step runs in the library's kernels; this module only allocates device
buffers, picks batches and loops.
"""
from __future__ import annotations

import numpy as np
import torch


def he_normal_weights(t, seed: int = 0) -> np.ndarray:
    """He-normal initial weights (std sqrt(2 / fan_in)) in the library's master layout:
    layers in order, each [c_out][c_in][kz][ky][kx]."""
    b = t.nn_base
    layers = [(4, b, 3), (b, b, 3), (b, 2 * b, 3), (2 * b, 2 * b, 3), (2 * b, 4 * b, 3),
              (4 * b, 4 * b, 3), (4 * b, 4 * b, 3), (6 * b, 2 * b, 3), (2 * b, 2 * b, 3),
              (3 * b, b, 3), (b, b, 3), (b, 3, 1)]
    rng = np.random.default_rng(seed)
    out = [rng.standard_normal(co * ci * k ** 3) * np.sqrt(2.0 / (ci * k ** 3))
           for ci, co, k in layers]
    w = np.concatenate(out).astype(np.float32)
    assert w.size == t.nn_params
    return w


class PairSet:
    """Harvested (r, e) pairs on the device, grouped by the SIMP iteration (density)."""

    def __init__(self):
        self.R, self.E, self.density, self.groups = None, None, [], []

    @property
    def count(self):
        return sum(n for _, n in self.groups)


def harvest(t, x, xphys, u, iters: int, every: int, per_solve: int, f=None, volfrac=0.3,
            move=0.2, tol=1e-8, ref_tol=1e-10, maxit=50000, check_every=64
            ) -> tuple[PairSet, list]:
    """Run `iters` SIMP steps (FP64 Jacobi-PCG, warm start) harvesting pairs; with the
    load vector f given, each step's solution is refined to ref_tol before the targets
    are formed.  Returns the pairs and the per-step statistics."""
    dev = x.device
    cap = iters * per_solve
    ps = PairSet()
    ps.R = torch.empty(cap, t.n_dof, dtype=torch.float32, device=dev)
    ps.E = torch.empty(cap, t.n_dof, dtype=torch.float32, device=dev)
    stats = []
    start = 0
    for _ in range(iters):
        rho = xphys.clone()  # density of the system this step solves
        hr, hu = ps.R[start:start + per_solve], ps.E[start:start + per_solve]
        if f is None:
            st = t.simp_step(x, xphys, u, volfrac=volfrac, move=move, harvest=(hr, hu),
                             harvest_every=every, tol=tol, maxit=maxit,
                             check_every=check_every, mode="plain_fp64")
            n = st["solve"]["harvested"]
            t.nn_make_targets(u, hu, n)  # u holds this step's solution u*
        else:
            u0 = u.clone()  # the warm start of this step's solve
            st = t.simp_step(x, xphys, u, volfrac=volfrac, move=move, tol=tol, maxit=maxit,
                             check_every=check_every, mode="plain_fp64")
            # u* of this step's system (density rho) to the tighter tolerance
            t.pcg_solve(rho, f, u, tol=min(ref_tol, tol), maxit=maxit,
                        check_every=check_every, mode="plain_fp64")
            hst = t.pcg_solve(rho, f, u0, tol=tol, maxit=maxit, mode="plain_fp64",
                              harvest=(hr, hu), harvest_every=every, harvest_ustar=u)
            n = hst["harvested"]
            st["solve"]["harvested"] = n
        ps.density.append(rho)
        ps.groups.append((start, n))
        start += n
        stats.append(st)
    return ps, stats


def train(t, ps: PairSet, steps: int, batch: int = 4, lr: float = 1e-3, seed: int = 0,
          lr_final: float | None = None, log_every: int = 0):
    """Adam on random batches of `batch` consecutive pairs of one SIMP iteration.
    The learning rate decays geometrically to lr_final (default lr / 10)."""
    rng = np.random.default_rng(seed)
    lr_final = lr / 10 if lr_final is None else lr_final
    usable = [g for g, (s, n) in enumerate(ps.groups) if n >= 1]
    losses = []
    cur_group = -1
    for k in range(steps):
        g = usable[rng.integers(len(usable))]
        s, n = ps.groups[g]
        nb = min(batch, n)
        j = s + int(rng.integers(n - nb + 1))
        if g != cur_group:
            t.nn_set_density(ps.density[g])
            cur_group = g
        lr_k = lr * (lr_final / lr) ** (k / max(steps - 1, 1))
        loss = t.nn_train_step(ps.R[j:j + nb], ps.E[j:j + nb], lr=lr_k)
        losses.append(loss)
        if log_every and (k % log_every == 0 or k == steps - 1):
            print(f"  train step {k:5d}  loss {loss:.4f}  lr {lr_k:.2e}", flush=True)
    return losses
