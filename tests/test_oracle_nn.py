"""Pins of the oracle's network pieces: convolutions against a library convolution (torch,
CPU, float64, tests only), gradients against autograd and finite differences, adjoint
identities, Adam against its textbook formulas, and flexible CG against plain PCG."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import fem, nn, solvers

torch.set_default_dtype(torch.float64)


@pytest.mark.parametrize("stride,shape", [(1, (3, 5, 4, 6)), (2, (2, 7, 5, 4)), (2, (4, 6, 6, 6))])
def test_conv3d_matches_library(stride, shape):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(shape)
    w = rng.standard_normal((5, shape[0], 3, 3, 3))
    ref = torch.nn.functional.conv3d(torch.tensor(x)[None], torch.tensor(w), stride=stride,
                                     padding=1)[0].numpy()
    y = nn.conv3d(x, w, stride)
    assert y.shape == ref.shape
    assert np.max(np.abs(y - ref)) < 1e-12


def test_conv1x1_matches_library():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((6, 3, 4, 5))
    w = rng.standard_normal((3, 6, 1, 1, 1))
    ref = torch.nn.functional.conv3d(torch.tensor(x)[None], torch.tensor(w))[0].numpy()
    assert np.max(np.abs(nn.conv3d(x, w) - ref)) < 1e-12


@pytest.mark.parametrize("stride,shape,k", [(1, (3, 5, 4, 6), 3), (2, (2, 7, 5, 4), 3),
                                            (1, (4, 3, 3, 3), 1)])
def test_conv3d_gradients_match_autograd(stride, shape, k):
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.standard_normal(shape), requires_grad=True)
    w = torch.tensor(rng.standard_normal((3, shape[0], k, k, k)), requires_grad=True)
    y = torch.nn.functional.conv3d(x[None], w, stride=stride, padding=k // 2)[0]
    g = torch.tensor(rng.standard_normal(y.shape))
    (y * g).sum().backward()
    dx = nn.conv3d_bwd_data(g.numpy(), w.detach().numpy(), shape, stride)
    dw = nn.conv3d_bwd_weight(x.detach().numpy(), g.numpy(), k, stride)
    assert np.max(np.abs(dx - x.grad.numpy())) < 1e-12
    assert np.max(np.abs(dw - w.grad.numpy())) < 1e-12


def test_upsample_and_adjoint():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 2))
    up = nn.upsample(x, (5, 7, 4))
    assert up.shape == (2, 5, 7, 4)
    assert up[1, 4, 6, 3] == x[1, 2, 3, 1]
    g = rng.standard_normal(up.shape)
    assert abs(np.sum(up * g) - np.sum(x * nn.upsample_adjoint(g, x.shape[1:]))) < 1e-12


def test_unet_gradient_finite_difference():
    base = 2
    rng = np.random.default_rng(4)
    params = nn.unet_init(base, 4, 3, seed=1)
    x = rng.standard_normal((4, 5, 4, 6))
    target = rng.standard_normal((3, 5, 4, 6))
    mask = (rng.uniform(size=(3, 5, 4, 6)) > 0.1).astype(float)
    out, cache = nn.unet_forward(params, x, base)
    assert out.shape == (3, 5, 4, 6)
    loss, dout = nn.rel_mse_loss(out, target, mask)
    grads = nn.unet_backward(params, cache, dout, base)
    h = 1e-6
    for name in ["e0a", "d1", "m2b", "u1a", "u0a", "head"]:
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in params[name].shape)
            p_ = {k: v.copy() for k, v in params.items()}
            p_[name][idx] += h
            lp = nn.rel_mse_loss(nn.unet_forward(p_, x, base)[0], target, mask)[0]
            p_[name][idx] -= 2 * h
            lm = nn.rel_mse_loss(nn.unet_forward(p_, x, base)[0], target, mask)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[name][idx]) <= 1e-6 * max(1e-3, abs(fd)), (name, idx)


def test_adam_step_textbook():
    p = {"a": np.array([1.0, -2.0])}
    g = {"a": np.array([0.5, 0.25])}
    st = {}
    nn.adam_step(p, g, st, lr=0.1)
    # first step: m = 0.1 g, v = 0.001 g^2, bias-corrected mhat = g, vhat = g^2
    assert np.allclose(p["a"], [1.0 - 0.1 * 0.5 / (0.5 + 1e-8), -2.0 - 0.1 * 0.25 / (0.25 + 1e-8)],
                       rtol=0, atol=1e-15)


def test_fcg_equals_pcg_with_fixed_preconditioner():
    nx, ny, nz = 6, 3, 3
    rho = np.random.default_rng(5).uniform(0.2, 1, nx * ny * nz)
    E = fem.simp_modulus(rho, 1.0, 1e-9, 3.0)
    K = fem.assemble_K(nx, ny, nz, E, fem.element_stiffness(0.3))
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    Kc = fem.constrain(K, fixed)
    f = si.cantilever_load(nx, ny, nz)
    d = Kc.diagonal()
    _, it_p, h_p = solvers.pcg_jacobi(lambda v: Kc @ v, d, f, None, 1e-10)
    _, it_f, h_f = nn.fcg(lambda v: Kc @ v, lambda r: r / d, f, None, 1e-10)
    # identical in exact arithmetic: the first iterates agree to rounding, the counts
    # agree up to rounding drift late in the run
    assert abs(it_p - it_f) <= 2
    hp, hf = np.array(h_p[:30]), np.array(h_f[:30])
    assert np.max(np.abs(hf / hp - 1.0)) < 1e-8


def test_node_density():
    x = np.random.default_rng(6).uniform(0, 1, 24)
    rn = nn.node_density(x, 4, 3, 2)
    assert rn.shape == (3, 4, 5)
    assert rn[0, 0, 0] == x[0]
    e = x.reshape(2, 3, 4)
    assert abs(rn[1, 1, 1] - e[0:2, 0:2, 0:2].mean()) < 1e-15
    assert np.allclose(nn.node_density(np.full(24, 0.3), 4, 3, 2), 0.3)


def test_nn_preconditioner_masks_and_scales():
    nx, ny, nz = 4, 3, 2
    params = nn.unet_init(2, 4, 3, seed=2)
    rho = nn.node_density(np.full(nx * ny * nz, 0.5), nx, ny, nz)
    fixed = fem.fixed_mask(3 * 60, si.cantilever_fixed_dofs(nx, ny, nz))
    r = np.random.default_rng(7).standard_normal(180)
    z1 = nn.nn_precondition(params, r, rho, fixed, base=2)
    z2 = nn.nn_precondition(params, 3.0 * r, rho, fixed, base=2)
    assert np.all(z1[fixed] == 0)
    assert np.allclose(z2, 3.0 * z1, rtol=1e-12, atol=0)  # homogeneous in ||r||


def _small_system(seed=8):
    nx, ny, nz = 5, 3, 3
    rho = np.random.default_rng(seed).uniform(0.2, 1, nx * ny * nz)
    K = fem.assemble_K(nx, ny, nz, fem.simp_modulus(rho, 1.0, 1e-9, 3.0), fem.element_stiffness(0.3))
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    Kc = fem.constrain(K, fixed)
    r = np.random.default_rng(seed + 1).standard_normal(K.shape[0])
    r[fixed] = 0.0
    return Kc, fixed, r


def test_two_stage_exact_correction_returns_solution():
    Kc, fixed, r = _small_system()
    e = np.linalg.solve(Kc.toarray(), r)
    z = nn.two_stage(r, e, lambda v: Kc @ v, Kc.diagonal())
    assert np.max(np.abs(z - e)) <= 1e-10 * np.max(np.abs(e))


def test_two_stage_zero_correction_is_jacobi():
    Kc, fixed, r = _small_system()
    d = Kc.diagonal()
    z = nn.two_stage(r, np.zeros_like(r), lambda v: Kc @ v, d)
    assert np.array_equal(z, r / d)


def test_two_stage_scale_invariant_and_energy_optimal():
    Kc, fixed, r = _small_system()
    rng = np.random.default_rng(3)
    n = np.linalg.solve(Kc.toarray(), r) + 0.3 * rng.standard_normal(r.size)
    n[fixed] = 0.0
    A = lambda v: Kc @ v
    z1 = nn.two_stage(r, n, A, Kc.diagonal())
    z2 = nn.two_stage(r, 7.5 * n, A, Kc.diagonal())
    assert np.allclose(z1, z2, rtol=1e-12, atol=1e-14)
    # s minimises the energy norm of e - s n
    e = np.linalg.solve(Kc.toarray(), r)
    s = (r @ n) / (n @ (Kc @ n))
    en = lambda c: (e - c * n) @ (Kc @ (e - c * n))
    assert en(s) <= min(en(0.99 * s), en(1.01 * s))


def test_energy_loss_definition_gradient_and_exact_case():
    Kc, fixed, r = _small_system(11)
    free = (~fixed).astype(float)
    A = lambda v: Kc @ v
    e = np.linalg.solve(Kc.toarray(), r)
    rng = np.random.default_rng(12)
    n = e + 0.5 * rng.standard_normal(r.size)
    L, g = nn.energy_loss(n, r, e, A, free)
    # the definition: best multiple of the masked correction, energy norm, relative
    nm = n * free
    s = (nm @ r) / (nm @ (Kc @ nm))
    d = s * nm - e
    assert abs(L - (d @ (Kc @ d)) / (e @ (Kc @ e))) <= 1e-12
    # exact direction: zero loss (any positive multiple)
    assert abs(nn.energy_loss(3.0 * e, r, e, A, free)[0]) <= 1e-12
    # gradient against central differences
    h = 1e-6
    for i in rng.choice(np.flatnonzero(free), 6, replace=False):
        dp = np.zeros_like(n)
        dp[i] = h
        fd = (nn.energy_loss(n + dp, r, e, A, free)[0] - nn.energy_loss(n - dp, r, e, A, free)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd))
    assert np.all(g[fixed] == 0)


def test_fcg_window_equals_pcg_with_fixed_preconditioner_and_helps_variable_one():
    nx, ny, nz = 6, 3, 3
    rho = np.random.default_rng(15).uniform(0.2, 1, nx * ny * nz)
    K = fem.assemble_K(nx, ny, nz, fem.simp_modulus(rho, 1.0, 1e-9, 3.0), fem.element_stiffness(0.3))
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    Kc = fem.constrain(K, fixed)
    f = si.cantilever_load(nx, ny, nz)
    d = Kc.diagonal()
    _, it_p, h_p = solvers.pcg_jacobi(lambda v: Kc @ v, d, f, None, 1e-10)
    for m in (1, 3, 8):
        _, it_f, h_f = nn.fcg(lambda v: Kc @ v, lambda r: r / d, f, None, 1e-10, window=m)
        assert abs(it_p - it_f) <= 2
        assert np.max(np.abs(np.array(h_f[:30]) / np.array(h_p[:30]) - 1.0)) < 1e-8
    # a preconditioner that changes every step: a longer window converges no slower
    rng = np.random.default_rng(16)
    noisy = lambda r: (r / d) * rng.uniform(0.5, 1.5, r.size)
    its = [nn.fcg(lambda v: Kc @ v, noisy, f, None, 1e-8, window=m)[1] for m in (1, 8)]
    assert its[1] <= its[0]



def _fcg_system(seed=5):
    nx, ny, nz = 6, 3, 3
    rho = np.random.default_rng(seed).uniform(0.2, 1, nx * ny * nz)
    K = fem.assemble_K(nx, ny, nz, fem.simp_modulus(rho, 1.0, 1e-9, 3.0), fem.element_stiffness(0.3))
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    Kc = fem.constrain(K, fixed)
    return Kc, si.cantilever_load(nx, ny, nz), Kc.diagonal()


@pytest.mark.parametrize("bad", ["nan", "negative"])
@pytest.mark.parametrize("window", [1, 4])
def test_fcg_fallback_reproduces_jacobi_pcg(bad, window):
    """A preconditioner whose output is not finite, or points uphill (<r, z> < 0), is
    replaced by the Jacobi step at every iteration, so flexible CG becomes Jacobi-PCG
    (identical in exact arithmetic) and every iteration counts one fallback."""
    Kc, f, d = _fcg_system()
    pre = (lambda r: np.full_like(r, np.nan)) if bad == "nan" else (lambda r: -r)
    info = {}
    x, it, h = nn.fcg(lambda v: Kc @ v, pre, f, None, 1e-10, window=window, d=d, info=info)
    _, it_p, h_p = solvers.pcg_jacobi(lambda v: Kc @ v, d, f, None, 1e-10)
    assert info["fallbacks"] == it and not info["restarted"]
    assert abs(it - it_p) <= 2
    assert np.max(np.abs(np.array(h[:30]) / np.array(h_p[:30]) - 1.0)) < 1e-8
    u = solvers.solve_direct(Kc, f)
    assert np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)


def test_fcg_without_fallback_diagonal_fails_on_nan():
    """Without the Jacobi diagonal a non-finite preconditioner output propagates (the
    fallback is what keeps the solve alive)."""
    Kc, f, _ = _fcg_system()
    x, it, h = nn.fcg(lambda v: Kc @ v, lambda r: np.full_like(r, np.nan), f, None, 1e-10, maxit=3)
    assert not np.all(np.isfinite(x))


def test_fcg_stall_restarts_into_jacobi_pcg():
    """Stagnation guard: when ||r|| makes no new minimum for `stall` iterations, flexible
    CG stops at the first such iteration and plain Jacobi-PCG continues from its iterate."""
    Kc, f, d = _fcg_system(seed=8)
    A = lambda v: Kc @ v
    pre = lambda r: (r / d) * (1.0 + 0.5 * np.sign(r))  # changes with r: not a fixed SPD M
    stall = 2
    info = {}
    x, it, h = nn.fcg(A, pre, f, None, 1e-10, 5000, d=d, stall=stall, info=info)
    assert info["restarted"] and info["fallbacks"] == 0
    k = info["fcg_iterations"]
    # the same iterations without the guard give the same history up to k ...
    xk, _, hk = nn.fcg(A, pre, f, None, 1e-10, k, d=d)
    assert hk == h[:k + 1]
    # ... and k is the first iteration that is `stall` past the running minimum
    first = next(j for j in range(1, k + 1) if j - int(np.argmin(hk[:j + 1])) >= stall)
    assert first == k
    # then plain Jacobi-PCG from the k-th iterate with the iterations left
    x2, it2, _ = solvers.pcg_jacobi(A, d, f, xk, 1e-10, 5000 - k)
    assert np.array_equal(x, x2) and it == k + it2
    u = solvers.solve_direct(Kc, f)
    assert np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)
