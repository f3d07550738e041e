"""GPU parity of the learned preconditioner against the oracle: U-Net forward and weight
gradients (FP32 and BF16 storage), the preconditioner application, an Adam step, the
harvesting of (r_k, u_k) pairs from FP64 PCG, and flexible CG with the Jacobi fallback.

Tolerances: FP32 storage runs the convolutions on v_mfma_f32_16x16x4f32 with FP32
accumulation over at most 27 x 96 products per output, so relative errors stay near
1e-6; 1e-4 is asserted.  BF16 storage rounds weights and every activation to 8
mantissa bits (relative 2^-9 per rounding, 12 layers deep): 5e-2 is asserted on the
output and on each layer's gradient as a whole (relative L2)."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import fem, nn, solvers
from tests.helpers import dev, gpu_problem, rel

pytestmark = pytest.mark.gpu

BASE = 16


def _flat(params, base=BASE):
    return np.concatenate([params[name].reshape(-1) for name, *_ in nn.unet_layers(base)])


def _unflat(vec, base=BASE):
    out, o = {}, 0
    for name, ci, co, k, _ in nn.unet_layers(base):
        n = co * ci * k ** 3
        out[name] = vec[o:o + n].reshape(co, ci, k, k, k)
        o += n
    return out


def _to_oracle(a, grid, c):
    X, Y, Z = grid
    return np.asarray(a, dtype=np.float64).reshape(Z, Y, X, c).transpose(3, 0, 1, 2)


def _from_oracle(a):
    return np.ascontiguousarray(a.transpose(1, 2, 3, 0)).reshape(-1)


def _net(nx, ny, nz, bf16, seed=1, kind="cantilever"):
    t, fixed, f = gpu_problem(nx, ny, nz, kind)
    t.nn_create(BASE, bf16=bf16)
    params = nn.unet_init(BASE, 4, 3, seed=seed)
    w = _flat(params)
    assert t.nn_params == w.size
    t.nn_set_weights(w.astype(np.float32))
    # the oracle runs the FP32-rounded weights the library holds
    params32 = _unflat(w.astype(np.float32).astype(np.float64))
    return t, fixed, f, params32


def _inputs(nx, ny, nz, seed=3):
    rng = np.random.default_rng(seed)
    grid = (nx + 1, ny + 1, nz + 1)
    x4 = rng.standard_normal((grid[2], grid[1], grid[0], 4)).astype(np.float32)
    x4[..., 3] = rng.uniform(0.0, 1.0, x4.shape[:3])
    return grid, x4


@pytest.mark.parametrize("dims", [(8, 6, 5), (19, 12, 9)])
def test_forward_fp32_matches_oracle(dims):
    nx, ny, nz = dims
    t, _, _, params = _net(nx, ny, nz, bf16=False)
    grid, x4 = _inputs(nx, ny, nz)
    out = t.nn_forward(dev(x4.reshape(-1))).cpu().numpy()
    ref, _ = nn.unet_forward(params, _to_oracle(x4, grid, 4), BASE)
    err = rel(_to_oracle(out, grid, 3), ref)
    t.close()
    assert err <= 1e-4, err


# (8, 6, 5): one result tile per layer.  (40, 20, 18) and (31, 9, 23): the BF16 z-sweep
# convolutions of levels 0 and 1 span several 16 x 8 tiles with ragged x and y edges and
# several z chunks per tile column (K channel counts 8, 16, 32, 48 forward; 16, 32 in
# the data gradient).
BF16_DIMS = [(8, 6, 5), (40, 20, 18), (31, 9, 23)]


@pytest.mark.parametrize("dims", BF16_DIMS)
def test_forward_bf16_close_to_oracle(dims):
    """Relative L2 error <= 5e-2, and no voxel off by more than 10% of the output's largest
    magnitude (a mis-addressed tap, row or plane of a tile would exceed both)."""
    nx, ny, nz = dims
    t, _, _, params = _net(nx, ny, nz, bf16=True)
    grid, x4 = _inputs(nx, ny, nz)
    out = t.nn_forward(dev(x4.reshape(-1))).cpu().numpy()
    ref, _ = nn.unet_forward(params, _to_oracle(x4, grid, 4), BASE)
    got = _to_oracle(out, grid, 3)
    err = rel(got, ref)
    worst = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    t.close()
    assert err <= 5e-2, err
    assert worst <= 0.1, worst


@pytest.mark.parametrize("bf16,tol,gtol,dims", [(False, 1e-4, 1e-4, (8, 6, 5))] +
                         [(True, 5e-2, 0.15, d) for d in BF16_DIMS])
def test_loss_and_gradients_match_oracle(bf16, tol, gtol, dims):
    """The weight gradient is a signed sum over every voxel, so its relative error is the
    storage rounding times the cancellation ratio sum|terms| / |sum|; in BF16 the first
    layers also see the rounding of every gradient tensor of the backward chain.  BF16
    asserts 15% (relative L2) and a direction within 8 degrees (cosine >= 0.99)."""
    nx, ny, nz = dims
    t, fixed, _, params = _net(nx, ny, nz, bf16=bf16)
    grid, x4 = _inputs(nx, ny, nz)
    target = np.random.default_rng(9).standard_normal(3 * t.n_node).astype(np.float32)
    loss, g = t.nn_loss_grad(dev(x4.reshape(-1)), dev(target))
    xo = _to_oracle(x4, grid, 4)
    out, cache = nn.unet_forward(params, xo, BASE)
    free = np.ones(3 * t.n_node)
    free[fixed] = 0.0
    lo, dout = nn.rel_mse_loss(out, _to_oracle(target, grid, 3), _to_oracle(free, grid, 3))
    grads = nn.unet_backward(params, cache, dout, BASE)
    t.close()
    assert abs(loss - lo) <= tol * lo
    gg = _unflat(g.astype(np.float64))
    errs = {name: rel(gg[name], grads[name]) for name, *_ in nn.unet_layers(BASE)}
    cos = {name: float(np.sum(gg[name] * grads[name]) /
                       (np.linalg.norm(gg[name]) * np.linalg.norm(grads[name])))
           for name in errs}
    assert max(errs.values()) <= gtol, errs
    assert min(cos.values()) >= (0.99 if bf16 else 1 - 1e-8), cos


@pytest.mark.parametrize("bf16,tol,dims", [(False, 1e-4, (8, 6, 5))] +
                         [(True, 5e-2, d) for d in BF16_DIMS])
def test_apply_matches_oracle_preconditioner(bf16, tol, dims):
    """The preconditioner application: its own forward (in BF16 the level-0 up-sampling
    concatenation is read in place by the z-sweep convolution) and the head fused into
    the output scaling."""
    nx, ny, nz = dims
    t, fixed, _, params = _net(nx, ny, nz, bf16=bf16)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.05, 1.0, t.n_elem).astype(np.float32)
    r = rng.standard_normal(t.n_dof).astype(np.float32)
    r[fixed] = 0.0
    t.nn_set_density(dev(x))
    z = t.nn_apply(dev(r)).cpu().numpy()
    rho = nn.node_density(x.astype(np.float64), nx, ny, nz)
    fm = fem.fixed_mask(t.n_dof, fixed)
    zo = nn.nn_precondition(params, r.astype(np.float64), rho, fm, base=BASE)
    t.close()
    assert np.all(z[fixed] == 0.0)
    assert rel(z, zo) <= tol


def test_train_step_is_adam_on_mean_gradient():
    nx, ny, nz = 8, 6, 5
    t, fixed, _, params = _net(nx, ny, nz, bf16=False)
    rng = np.random.default_rng(5)
    x = np.full(t.n_elem, 0.5, dtype=np.float32)
    t.nn_set_density(dev(x))
    nb = 2
    R = rng.standard_normal((nb, t.n_dof)).astype(np.float32)
    E = rng.standard_normal((nb, t.n_dof)).astype(np.float32)
    R[:, fixed] = 0.0
    lr = 1e-3
    loss = t.nn_train_step(dev(R), dev(E), lr=lr)
    w1 = t.nn_get_weights().astype(np.float64)
    # oracle: mean loss and mean gradient over the batch, then one Adam step
    rho = nn.node_density(x.astype(np.float64), nx, ny, nz)
    grid = (nx + 1, ny + 1, nz + 1)
    free = np.ones(t.n_dof)
    free[fixed] = 0.0
    gsum = {k: np.zeros_like(v) for k, v in params.items()}
    lsum = 0.0
    for s in range(nb):
        g = np.sqrt(t.n_dof) / np.linalg.norm(R[s].astype(np.float64))
        inp = np.concatenate([_to_oracle(R[s] * g, grid, 3), rho[None]], axis=0)
        out, cache = nn.unet_forward(params, inp, BASE)
        ge = np.sqrt(t.n_dof) / np.linalg.norm(E[s].astype(np.float64))
        lo, dout = nn.rel_mse_loss(out, _to_oracle(E[s] * ge, grid, 3), _to_oracle(free, grid, 3))
        lsum += lo
        for k, v in nn.unet_backward(params, cache, dout, BASE).items():
            gsum[k] += v
    gmean = {k: v / nb for k, v in gsum.items()}
    p_new = {k: v.copy() for k, v in params.items()}
    nn.adam_step(p_new, gmean, {}, lr=lr)
    w_ref = _flat(p_new)
    w0 = _flat(params)
    t.close()
    assert abs(loss - lsum / nb) <= 1e-4 * lsum / nb
    # the first Adam step moves each weight by lr * g / (|g| + eps): compare the moves
    d_gpu, d_ref = w1 - w0, w_ref - w0
    # The move is lr * sign(g) up to eps: it is exact only where FP32 settles the sign of
    # the gradient, a signed sum over all voxels.  Gradients above 1% of the largest must
    # all agree, and the weights that disagree carry under 1% of the gradient's l1 mass.
    g_flat = np.abs(_flat(gmean))
    big = g_flat > 1e-2 * np.max(g_flat)
    match = np.abs(d_gpu - d_ref) <= 1e-3 * lr
    assert np.all(match[big])
    assert np.sum(g_flat[~match]) <= 1e-2 * np.sum(g_flat)
    # no weight moves by more than lr (plus the FP32 rounding of the stored weight)
    assert np.all(np.abs(d_gpu) <= lr * (1 + 1e-6) + 2.0 ** -23 * np.abs(w0))


def test_weights_roundtrip_and_errors():
    from paper_2604_18020_amd import TosimpError
    t, _, _ = gpu_problem(6, 4, 4)
    with pytest.raises(TosimpError):
        t.nn_create(base=12)
    t.nn_create(16, bf16=True)
    w = np.random.default_rng(0).standard_normal(t.nn_params).astype(np.float32)
    t.nn_set_weights(w)
    assert np.array_equal(t.nn_get_weights(), w)
    with pytest.raises(TosimpError):
        t.nn_set_weights(w[:-1])
    t.close()


def test_harvest_pairs_from_fp64_pcg():
    nx, ny, nz = 12, 6, 6
    t, fixed, f = gpu_problem(nx, ny, nz)
    rng = np.random.default_rng(6)
    xd = dev(rng.uniform(0.1, 1.0, t.n_elem))
    b = dev(f)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    cap, every = 6, 5
    hr = torch.zeros(cap, t.n_dof, dtype=torch.float32, device="cuda:0")
    hu = torch.zeros(cap, t.n_dof, dtype=torch.float32, device="cuda:0")
    st = t.pcg_solve(xd, b, u, tol=1e-10, harvest=(hr, hu), harvest_every=every)
    assert st["harvested"] == min(cap, (st["iterations"] - 1) // every + 1)
    # pair k is (r, u) after k * every iterations of the same Jacobi-PCG run in the oracle
    xo = xd.cpu().numpy()
    K = fem.constrain(fem.assemble_K(nx, ny, nz, fem.simp_modulus(xo, 1.0, 1e-9, 3.0),
                                     fem.element_stiffness(0.3)), fem.fixed_mask(t.n_dof, fixed))
    d = K.diagonal()
    for k in range(st["harvested"]):
        uk, _, _ = solvers.pcg_jacobi(lambda v: K @ v, d, f, None, 1e-30, maxit=k * every)
        rk = f - K @ uk
        assert rel(hu[k].cpu().numpy(), uk) <= 1e-6 or k == 0
        assert rel(hr[k].cpu().numpy(), rk) <= 1e-5
    assert np.all(hu[0].cpu().numpy() == 0.0)  # zero initial guess
    n = st["harvested"]
    t.nn_make_targets(u, hu, n)
    e0 = hu[0].cpu().numpy()
    assert rel(e0, u.cpu().numpy()) <= 1e-7
    t.close()


def _fcg_problem(nx=12, ny=6, nz=6, seed=7):
    t, fixed, f = gpu_problem(nx, ny, nz)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.1, 1.0, t.n_elem)
    return t, fixed, f, x


@pytest.mark.parametrize("window", [1, 8])
def test_fcg_zero_network_is_jacobi_pcg(window):
    t, fixed, f, x = _fcg_problem()
    t.nn_create(16, bf16=True)
    t.nn_set_weights(np.zeros(t.nn_params, dtype=np.float32))
    kw = dict(tol=1e-8, mode="ir", inner_prec="fp32", inner_tol=1e-5, check_every=1)
    u1 = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    s_nn = t.pcg_solve(dev(x), dev(f), u1, precond="nn", fcg_window=window, **kw)
    u2 = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    s_j = t.pcg_solve(dev(x), dev(f), u2, precond="jacobi", **kw)
    t.close()
    # n = N(r) = 0 gives s = 0 and z = D^-1 r: flexible CG with the Jacobi preconditioner,
    # which is PCG in exact arithmetic.  FCG's beta = -<z, q_prev> / <p_prev, q_prev> and
    # PCG's <r, z> ratio round differently in FP32, so the counts drift apart a little.
    assert s_nn["fallbacks"] == 0 and s_nn["rc"] == 0
    assert abs(s_nn["iterations"] - s_j["iterations"]) <= 0.15 * s_j["iterations"]
    assert s_nn["true_rel_residual"] <= 1e-8


@pytest.mark.parametrize("bf16,tol", [(False, 1e-4), (True, 5e-2)])
def test_two_stage_preconditioner_matches_oracle(bf16, tol):
    nx, ny, nz = 8, 6, 5
    t, fixed, _, params = _net(nx, ny, nz, bf16=bf16)
    rng = np.random.default_rng(12)
    x = rng.uniform(0.05, 1.0, t.n_elem).astype(np.float32)
    r = rng.standard_normal(t.n_dof).astype(np.float32)
    r[fixed] = 0.0
    z = t.nn_precondition(dev(x), dev(r)).cpu().numpy()
    x64 = x.astype(np.float64)
    fm = fem.fixed_mask(t.n_dof, fixed)
    Kc = fem.constrain(fem.assemble_K(nx, ny, nz, fem.simp_modulus(x64, 1.0, 1e-9, 3.0),
                                      fem.element_stiffness(0.3)), fm)
    zo = nn.nn_two_stage_precondition(params, r.astype(np.float64), nn.node_density(x64, nx, ny, nz),
                                      fm, lambda v: Kc @ v, Kc.diagonal(), base=BASE)
    t.close()
    assert rel(z, zo) <= tol


@pytest.mark.parametrize("window", [1, 16])
def test_fcg_random_network_converges_to_direct_solution(window):
    t, fixed, f, x = _fcg_problem()
    t.nn_create(16, bf16=True)
    t.nn_set_weights(_flat(nn.unet_init(BASE, 4, 3, seed=2)).astype(np.float32))
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    s = t.pcg_solve(dev(x), dev(f), u, precond="nn", tol=1e-9, mode="ir", inner_prec="fp32",
                    inner_tol=1e-5, check_every=1, maxit=5000, fcg_window=window)
    nx, ny, nz = t.dims
    t.close()
    assert s["rc"] in (0, 2)
    assert s["true_rel_residual"] <= 1e-9
    E = fem.simp_modulus(x, 1.0, 1e-9, 3.0)
    u_ref = solvers.solve_direct(fem.constrain(fem.assemble_K(nx, ny, nz, E, fem.element_stiffness(0.3)),
                                               fem.fixed_mask(3 * (nx + 1) * (ny + 1) * (nz + 1), fixed)), f)
    assert rel(u.cpu().numpy(), u_ref) <= 1e-6


def test_fcg_window_out_of_range_is_rejected():
    from paper_2604_18020_amd import TosimpError
    t, fixed, f, x = _fcg_problem()
    t.nn_create(16, bf16=True)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    with pytest.raises(TosimpError):
        t.pcg_solve(dev(x), dev(f), u, precond="nn", mode="ir", tol=1e-8, fcg_window=17)
    t.close()


def test_nn_precond_without_network_is_rejected():
    from paper_2604_18020_amd import TosimpError
    t, fixed, f, x = _fcg_problem()
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    with pytest.raises(TosimpError):
        t.pcg_solve(dev(x), dev(f), u, precond="nn", mode="ir", tol=1e-8)
    t.close()


@pytest.mark.parametrize("bf16,tol", [(False, 1e-4), (True, 0.15)])
def test_energy_loss_gradient_matches_oracle(bf16, tol):
    nx, ny, nz = 8, 6, 5
    t, fixed, _, params = _net(nx, ny, nz, bf16=bf16)
    t.nn_set_loss("energy")
    rng = np.random.default_rng(21)
    x = rng.uniform(0.1, 1.0, t.n_elem).astype(np.float32)
    x64 = x.astype(np.float64)
    fm = fem.fixed_mask(t.n_dof, fixed)
    Kc = fem.constrain(fem.assemble_K(nx, ny, nz, fem.simp_modulus(x64, 1.0, 1e-9, 3.0),
                                      fem.element_stiffness(0.3)), fm)
    r = rng.standard_normal(t.n_dof)
    r[fm] = 0.0
    r = r.astype(np.float32).astype(np.float64)
    e = np.linalg.solve(Kc.toarray(), r).astype(np.float32).astype(np.float64)
    t.nn_set_density(dev(x))
    loss, g = t.nn_sample_grad(dev(r, torch.float32), dev(e, torch.float32))
    # oracle: unit-RMS input, correction on free DOFs, energy loss, back through the net
    grid = (nx + 1, ny + 1, nz + 1)
    gsc = np.sqrt(t.n_dof) / np.linalg.norm(r)
    inp = np.concatenate([_to_oracle(r * gsc, grid, 3), nn.node_density(x64, nx, ny, nz)[None]], axis=0)
    out, cache = nn.unet_forward(params, inp, BASE)
    n = out.transpose(1, 2, 3, 0).reshape(-1)
    free = (~fm).astype(float)
    lo, gd = nn.energy_loss(n, r, e, lambda v: Kc @ v, free)
    grads = nn.unet_backward(params, cache, _to_oracle(gd, grid, 3), BASE)
    t.close()
    assert abs(loss - lo) <= tol * max(lo, 1e-3)
    gg = _unflat(g.astype(np.float64))
    errs = {name: rel(gg[name], grads[name]) for name, *_ in nn.unet_layers(BASE)}
    assert max(errs.values()) <= tol, errs



@pytest.mark.parametrize("bf16,tol", [(False, 1e-4), (True, 5e-2)])
@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 3)])
def test_forward_on_degenerate_grids_matches_oracle(dims, bf16, tol):
    """Level grids of one or two nodes per axis (stride-2 convolutions down to 1 x 1 x 1;
    in BF16 the z-sweeps with single-plane chunks and one partial tile); the BF16 case
    also applies the preconditioner (its in-place concatenations and fused head)."""
    nx, ny, nz = dims
    t, fixed, _, params = _net(nx, ny, nz, bf16=bf16)
    grid, x4 = _inputs(nx, ny, nz, seed=8)
    out = t.nn_forward(dev(x4.reshape(-1))).cpu().numpy()
    ref, _ = nn.unet_forward(params, _to_oracle(x4, grid, 4), BASE)
    assert rel(_to_oracle(out, grid, 3), ref) <= tol
    if bf16:
        rng = np.random.default_rng(5)
        x = rng.uniform(0.05, 1.0, t.n_elem).astype(np.float32)
        r = rng.standard_normal(t.n_dof).astype(np.float32)
        r[fixed] = 0.0
        t.nn_set_density(dev(x))
        z = t.nn_apply(dev(r)).cpu().numpy()
        zo = nn.nn_precondition(params, r.astype(np.float64),
                                nn.node_density(x.astype(np.float64), nx, ny, nz),
                                fem.fixed_mask(t.n_dof, fixed), base=BASE)
        assert np.all(z[fixed] == 0.0)
        assert rel(z, zo) <= tol
    t.close()


def _oracle_fcg_system(nx, ny, nz, x, fixed, f):
    E = fem.simp_modulus(np.asarray(x, dtype=np.float64), 1.0, 1e-9, 3.0)
    Kc = fem.constrain(fem.assemble_K(nx, ny, nz, E, fem.element_stiffness(0.3)),
                       fem.fixed_mask(f.size, fixed))
    return Kc, Kc.diagonal()


def test_fcg_nan_network_takes_the_jacobi_step_every_iteration():
    """Host-forced fallback: with NaN weights the network output is not finite, so every
    flexible-CG iteration takes the Jacobi step (the guard the oracle's flexible CG pins);
    the solve is then Jacobi-PCG and converges to the direct solution."""
    from paper_2604_18020_amd import FALLBACK_USED
    t, fixed, f, x = _fcg_problem()
    nx, ny, nz = t.dims
    t.nn_create(16, bf16=True)
    t.nn_set_weights(np.full(t.nn_params, np.nan, dtype=np.float32))
    kw = dict(tol=1e-8, mode="ir", inner_prec="fp32", inner_tol=1e-5, check_every=1)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    s = t.pcg_solve(dev(x), dev(f), u, precond="nn", nn_stall=-1, **kw)
    u2 = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    s_j = t.pcg_solve(dev(x), dev(f), u2, precond="jacobi", **kw)
    t.close()
    assert s["rc"] == FALLBACK_USED and s["restarts"] == 0
    assert s["fallbacks"] == s["iterations"] > 0
    assert abs(s["iterations"] - s_j["iterations"]) <= 0.15 * s_j["iterations"]
    assert s["true_rel_residual"] <= 1e-8
    Kc, d = _oracle_fcg_system(nx, ny, nz, x, fixed, f)
    u_ref = solvers.solve_direct(Kc, f)
    assert rel(u.cpu().numpy(), u_ref) <= 1e-6
    # the oracle's guarded flexible CG with the same forced preconditioner
    info = {}
    _, it_o, _ = nn.fcg(lambda v: Kc @ v, lambda r: np.full_like(r, np.nan), f, None, 1e-5,
                        d=d, info=info)
    assert info["fallbacks"] == it_o


def test_fcg_stagnation_restarts_with_jacobi_pcg():
    """The solve-level fallback: an inner flexible-CG solve whose residual makes no new
    minimum for nn_stall iterations is finished by plain Jacobi-PCG from its iterate.
    Forced from the host with nn_stall = 1 (the first iteration that does not lower
    ||r||) and NaN weights; the oracle's guarded flexible CG restarts at the same point."""
    from paper_2604_18020_amd import FALLBACK_USED
    t, fixed, f, x = _fcg_problem()
    nx, ny, nz = t.dims
    Kc, d = _oracle_fcg_system(nx, ny, nz, x, fixed, f)
    info = {}
    _, _, h = nn.fcg(lambda v: Kc @ v, lambda r: np.full_like(r, np.nan), f, None, 1e-5,
                     d=d, stall=1, info=info)
    k = info["fcg_iterations"]
    assert info["restarted"] and k >= 1
    # every step up to k is decided with a margin FP32 rounding cannot flip
    steps = np.array(h[1:k + 1]) / np.minimum.accumulate(np.array(h[:k]))
    assert np.all(np.abs(steps - 1.0) > 1e-3)
    t.nn_create(16, bf16=True)
    t.nn_set_weights(np.full(t.nn_params, np.nan, dtype=np.float32))
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    s = t.pcg_solve(dev(x), dev(f), u, precond="nn", nn_stall=1, tol=1e-8, mode="ir",
                    inner_prec="fp32", inner_tol=1e-5, check_every=1)
    t.close()
    assert s["rc"] == FALLBACK_USED and s["restarts"] >= 1
    # the first inner solve (right-hand side f / ||f||) took k flexible-CG iterations
    assert s["fallbacks"] >= k
    assert s["true_rel_residual"] <= 1e-8
    assert rel(u.cpu().numpy(), solvers.solve_direct(Kc, f)) <= 1e-6


def test_harvested_targets_are_consistent():
    """learned.harvest with the reference solve refined to 1e-10: the refined solution
    has ||b - K u*|| <= 1e-10 ||b|| (FP64); every harvested residual is above the
    harvesting tolerance (taken before convergence); each stored pair satisfies
    K e_k - r_k = -r* up to its FP32 storage: ||K e_k - r_k|| <= 1e-8 ||b|| +
    2^-23 (||r_k|| + ||K|| ||e_k||) with ||K|| <= 8 lambda_max(K_E) max E (each node lies
    in at most eight elements)."""
    from paper_2604_18020_amd import learned
    nx, ny, nz = 12, 6, 6
    t, fixed, f = gpu_problem(nx, ny, nz)
    x = torch.full((t.n_elem,), 0.3, dtype=torch.float64, device="cuda:0")
    xp = x.clone()
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    b = dev(f)
    ps, stats = learned.harvest(t, x, xp, u, iters=2, every=7, per_solve=8, f=b, tol=1e-8,
                                ref_tol=1e-10)
    bn = float(torch.linalg.norm(b))
    # the last group's refined solution: u holds u* of its density
    rstar = b - t.apply_K(ps.density[-1], u)
    assert float(torch.linalg.norm(rstar)) <= 1.5e-10 * bn
    knorm = 8.0 * float(np.linalg.eigvalsh(fem.element_stiffness(0.3))[-1])  # E <= 1
    assert ps.count >= 8
    for g, (s0, n) in enumerate(ps.groups):
        rho = ps.density[g]
        for k in range(s0, s0 + n):
            r = ps.R[k].double()
            e = ps.E[k].double()
            rn, en = float(torch.linalg.norm(r)), float(torch.linalg.norm(e))
            assert rn > 1e-8 * bn
            err = float(torch.linalg.norm(t.apply_K(rho, e) - r))
            assert err <= 1e-8 * bn + 2.0 ** -23 * (rn + knorm * en), (g, k, err)
    t.close()
