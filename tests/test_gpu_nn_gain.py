"""What training buys the learned preconditioner, measured end to end on the GPU.

Pairs (r_k, e_k = u* - u_k) are harvested from the FP64 Jacobi-PCG solves of five SIMP
iterations on the 32x16x16 cantilever; the network is trained (Adam, relative MSE) on
the pairs of the first four iterations and judged on those of the fifth, which it has
not seen:

* held-out relative MSE of the correction against the unit-RMS error (the training
  loss), before training (He-normal weights) and after;
* held-out energy-norm error of the best multiple of the correction,
  1 - <n,r>^2 / (<n,K n> <e,r>), the quantity the two-stage step depends on;
* the fifth iteration's system solved to 1e-6 with FP32 Jacobi-PCG and with flexible CG
  around the untrained and the trained network (all inside FP64 refinement).

Measured on MI355X: MSE 2.41 -> 0.90, energy-norm error 0.9999 -> 0.989, and flexible
CG needs ~3-5x Jacobi's iterations with either network: the network learns the smooth
part of the error, but the high-frequency remainder of its output carries almost all of
the K-norm error (the Jacobi-scaled operator has condition number ~1e5-1e6 on these
meshes), so each application removes little of the error CG measures.  The test asserts
the gain in approximation (the held-out MSE at least drops to 0.6x), that the energy-norm
error does not grow, that every solve converges, and records the iteration counts."""
import numpy as np
import pytest
import torch

from tests.helpers import dev, gpu_problem

pytestmark = pytest.mark.gpu


def test_training_gain_on_held_out_pairs_and_in_the_solve(record_property):
    from paper_2604_18020_amd import learned

    nx, ny, nz = 32, 16, 16
    t, fixed, f = gpu_problem(nx, ny, nz)
    t.nn_create(16, bf16=True)
    w0 = learned.he_normal_weights(t, seed=0)
    t.nn_set_weights(w0)
    x = torch.full((t.n_elem,), 0.3, dtype=torch.float64, device="cuda:0")
    xphys = x.clone()
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    ps, _ = learned.harvest(t, x, xphys, u, iters=5, every=4, per_solve=80)
    assert len(ps.groups) == 5 and all(n >= 40 for _, n in ps.groups)

    held = len(ps.groups) - 1
    s0, n0 = ps.groups[held]

    def held_out(kind):
        t.nn_set_loss(kind)
        t.nn_set_density(ps.density[held])
        return float(np.mean([t.nn_sample_grad(ps.R[k], ps.E[k], want_grad=False)[0]
                              for k in range(s0, s0 + n0)]))

    before = {k: held_out(k) for k in ("mse", "energy")}
    train = learned.PairSet()
    train.R, train.E = ps.R, ps.E
    train.density, train.groups = ps.density[:held], ps.groups[:held]
    t.nn_set_loss("mse")
    losses = learned.train(t, train, steps=300, batch=4, lr=1e-3, seed=0)
    after = {k: held_out(k) for k in ("mse", "energy")}
    w_trained = t.nn_get_weights()

    def solve(**kw):
        uu = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
        r = t.pcg_solve(ps.density[held], dev(f), uu, tol=1e-6, mode="ir", inner_prec="fp32",
                        inner_tol=1e-4, check_every=8, maxit=20000, **kw)
        assert r["true_rel_residual"] <= 1e-6, (kw, r)
        return r["iterations"]

    it_jacobi = solve(precond="jacobi")
    it_trained = solve(precond="nn", fcg_window=1)
    t.nn_set_weights(w0)
    it_untrained = solve(precond="nn", fcg_window=1)
    t.nn_set_weights(w_trained)
    t.close()

    summary = {"held_out_mse_before": before["mse"], "held_out_mse_after": after["mse"],
               "held_out_energy_before": before["energy"],
               "held_out_energy_after": after["energy"],
               "train_loss_first20": float(np.mean(losses[:20])),
               "train_loss_last20": float(np.mean(losses[-20:])),
               "iterations_jacobi": it_jacobi, "iterations_fcg_untrained": it_untrained,
               "iterations_fcg_trained": it_trained}
    for k, v in summary.items():
        record_property(k, v)
    print(summary)

    assert all(np.isfinite(v) for v in summary.values())
    assert np.mean(losses[-20:]) < np.mean(losses[:20])
    assert after["mse"] <= 0.6 * before["mse"], summary
    assert after["energy"] <= before["energy"], summary
