"""GPU parity of the geometric-multigrid preconditioner (Sec. "Path to Geometric
Multigrid Integration") against the oracle (oracle/mg.py): the hierarchy, one V-cycle
element by element in FP64 and FP32, and CG preconditioned by it (plain FP64 and FP32
inner solves in refinement) against the oracle's iteration counts and the direct
solution."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import fem, mg, solvers
from tests.helpers import dev, gpu_problem

pytestmark = pytest.mark.gpu

KE = fem.element_stiffness(0.3)
LAM = mg.chebyshev_bound(KE)


def _oracle_levels(nx, ny, nz, x, kind="cantilever"):
    fixed_ids = si.cantilever_fixed_dofs(nx, ny, nz) if kind == "cantilever" else \
        si.torsion_fixed_dofs(nx, ny, nz)
    fixed = fem.fixed_mask(3 * (nx + 1) * (ny + 1) * (nz + 1), fixed_ids)
    E = fem.simp_modulus(x, 1.0, 1e-9, 3.0)
    return mg.build_hierarchy(nx, ny, nz, E, KE, fixed), fixed


@pytest.mark.parametrize("dims", [(16, 8, 8), (13, 7, 5), (55, 55, 165), (340, 170, 85)])
def test_hierarchy_matches_oracle(dims):
    nx, ny, nz = dims
    t, _, _ = gpu_problem(nx, ny, nz)
    got = t.mg_levels()
    t.close()
    want = [dims]
    while min(want[-1]) >= 2 and len(want) < 12:
        want.append(mg.coarse_dims(*want[-1]))
    assert got == want


@pytest.mark.parametrize("dims,kind,seed", [((12, 6, 6), "cantilever", 1),
                                            ((13, 7, 5), "cantilever", 2),
                                            ((9, 9, 14), "torsion", 3),
                                            ((40, 20, 10), "cantilever", 4),
                                            # whole V-cycle in the single-workgroup tail,
                                            # its LDS arena ~112 KB in FP64
                                            ((11, 6, 5), "cantilever", 5)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vcycle_matches_oracle(dims, kind, seed, prec):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.01, 1.0, nx * ny * nz)
    levels, fixed = _oracle_levels(nx, ny, nz, x, kind)
    r = rng.standard_normal(fixed.size)
    r[fixed] = 0.0
    z_o = mg.vcycle(levels, r, LAM)
    t, _, _ = gpu_problem(nx, ny, nz, kind=kind)
    dt = torch.float64 if prec == "fp64" else torch.float32
    z = t.mg_apply(dev(x), dev(r, dt)).double().cpu().numpy()
    t.close()
    err = np.max(np.abs(z - z_o)) / np.max(np.abs(z_o))
    assert err <= (1e-11 if prec == "fp64" else 2e-4), err
    assert np.all(z[fixed] == 0.0)


def test_vcycle_degree_and_alpha_match_oracle():
    nx, ny, nz = 10, 6, 4
    rng = np.random.default_rng(9)
    x = rng.uniform(0.01, 1.0, nx * ny * nz)
    levels, fixed = _oracle_levels(nx, ny, nz, x)
    r = rng.standard_normal(fixed.size)
    r[fixed] = 0.0
    t, _, _ = gpu_problem(nx, ny, nz)
    for degree, alpha in ((1, 20.0), (3, 10.0), (4, 30.0)):
        z_o = mg.vcycle(levels, r, LAM, degree=degree, alpha=alpha)
        z = t.mg_apply(dev(x), dev(r), degree=degree, alpha=alpha).cpu().numpy()
        assert np.max(np.abs(z - z_o)) <= 1e-11 * np.max(np.abs(z_o)), (degree, alpha)
    t.close()


@pytest.mark.parametrize("dims,seed", [((16, 8, 8), 4), ((13, 7, 5), 4), ((48, 24, 24), 6)])
def test_mg_pcg_matches_oracle(dims, seed):
    """Plain FP64 CG with the FP64 V-cycle: the oracle's iteration count (+-1) and the
    direct solution."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.01, 1.0, nx * ny * nz)
    levels, fixed = _oracle_levels(nx, ny, nz, x)
    f = si.cantilever_load(nx, ny, nz)
    u_o, it_o, _ = mg.pcg_mg(levels, f, LAM, tol=1e-10)
    t, _, _ = gpu_problem(nx, ny, nz)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    st = t.pcg_solve(dev(x), dev(f), u, tol=1e-10, precond="mg", check_every=4)
    t.close()
    assert st["rc"] == 0 and abs(st["iterations"] - it_o) <= 1, (st["iterations"], it_o)
    assert st["true_rel_residual"] <= 1e-9
    u = u.cpu().numpy()
    assert np.linalg.norm(u - u_o) <= 1e-8 * np.linalg.norm(u_o)
    if nx <= 16:
        ud = solvers.solve_direct(levels[0].K, f)
        assert np.linalg.norm(u - ud) <= 1e-8 * np.linalg.norm(ud)


def test_mg_refinement_fp32_inner():
    """FP64 refinement around FP32 CG with the FP32 V-cycle reaches the FP64 tolerance;
    compliance matches the direct solve."""
    nx, ny, nz = 24, 12, 12
    rng = np.random.default_rng(8)
    x = rng.uniform(0.01, 1.0, nx * ny * nz)
    levels, fixed = _oracle_levels(nx, ny, nz, x)
    f = si.cantilever_load(nx, ny, nz)
    ud = solvers.solve_direct(levels[0].K, f)
    t, _, _ = gpu_problem(nx, ny, nz)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    st = t.pcg_solve(dev(x), dev(f), u, tol=1e-9, mode="ir", precond="mg", inner_tol=1e-4,
                     check_every=4)
    t.close()
    assert st["rc"] == 0 and st["true_rel_residual"] <= 1e-9
    c, cd = f @ u.cpu().numpy(), f @ ud
    assert abs(c - cd) <= 1e-8 * cd
    assert st["iterations"] < 60


def test_mg_arguments_refused():
    from paper_2604_18020_amd import TosimpError
    nx, ny, nz = 8, 4, 4
    t, _, f = gpu_problem(nx, ny, nz)
    x = dev(np.full(nx * ny * nz, 0.5))
    r = dev(np.zeros(t.n_dof))
    with pytest.raises(TosimpError):
        t.mg_apply(x, r, degree=17)
    with pytest.raises(TosimpError):
        t.mg_apply(x, r, alpha=0.5)
    with pytest.raises(TosimpError):
        t.mg_apply(x, r, z=r)  # z overlaps r
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    with pytest.raises(TosimpError):
        t.pcg_solve(x, dev(f), u, mode="ir", precond="mg", inner_prec="bf16_mfma")
    t.close()


@pytest.mark.parametrize("mode", ["plain_fp64", "ir"])
def test_mg_graph_replay_matches_eager_bitwise(mode):
    """Batches of MG-CG iterations replayed as a HIP graph (many replays, with the host's
    polls between them) give bit-identical iterates to direct launches."""
    nx, ny, nz = 20, 10, 10
    rng = np.random.default_rng(12)
    x = dev(rng.uniform(0.01, 1.0, nx * ny * nz))
    t, _, f = gpu_problem(nx, ny, nz)
    out = []
    for eager in (True, False):
        u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
        kw = dict(tol=1e-10, precond="mg", check_every=2, eager=eager)
        if mode == "ir":
            kw.update(mode="ir", inner_tol=1e-4)
        st = t.pcg_solve(x, dev(f), u, **kw)
        assert st["rc"] == 0
        out.append((st["iterations"], u.cpu().numpy()))
    t.close()
    assert out[0][0] == out[1][0] and out[0][0] > 4
    assert np.array_equal(out[0][1], out[1][1])


def test_mg_graph_cache_reuse_and_penalty_change():
    """Repeated solves with the same buffers replay the cached batch graphs and give the
    eager solve's iterates bit for bit; after the SIMP exponent changes, no graph of the
    old exponent is replayed (graph and eager solves agree again, and the solution moves)."""
    nx, ny, nz = 20, 10, 10
    rng = np.random.default_rng(13)
    x = dev(rng.uniform(0.05, 1.0, nx * ny * nz))
    t, _, f = gpu_problem(nx, ny, nz)
    b = dev(f)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")

    def solve(eager):
        u.zero_()
        st = t.pcg_solve(x, b, u, tol=1e-10, precond="mg", mode="ir", inner_tol=1e-4,
                         check_every=4, eager=eager)
        assert st["rc"] == 0
        return st["iterations"], u.cpu().numpy().copy()

    ref = solve(True)
    for _ in range(3):
        it, got = solve(False)
        assert it == ref[0] and np.array_equal(got, ref[1])
    t.set_params(2.5, 1.5)
    ref25 = solve(True)
    it, got = solve(False)
    t.close()
    assert it == ref25[0] and np.array_equal(got, ref25[1])
    assert not np.array_equal(ref25[1], ref[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vcycle_degrees_through_the_per_level_kernels(prec):
    """Degrees 1, 3 and 4 on a mesh whose two finest levels run the per-level kernels
    (degree 1: no fused first-two-steps pass; degree >= 3: extra fused passes) and whose
    coarser levels run the single-workgroup tail, against the oracle's V-cycle."""
    nx, ny, nz = 40, 20, 10
    rng = np.random.default_rng(21)
    x = rng.uniform(0.01, 1.0, nx * ny * nz)
    levels, fixed = _oracle_levels(nx, ny, nz, x)
    r = rng.standard_normal(fixed.size)
    r[fixed] = 0.0
    t, _, _ = gpu_problem(nx, ny, nz)
    dt = torch.float64 if prec == "fp64" else torch.float32
    for degree, alpha in ((1, 20.0), (3, 10.0), (4, 30.0)):
        z_o = mg.vcycle(levels, r, LAM, degree=degree, alpha=alpha)
        z = t.mg_apply(dev(x), dev(r, dt), degree=degree, alpha=alpha).double().cpu().numpy()
        err = np.max(np.abs(z - z_o)) / np.max(np.abs(z_o))
        assert err <= (1e-11 if prec == "fp64" else 2e-4), (degree, alpha, err)
        assert np.all(z[fixed] == 0.0)
    t.close()
