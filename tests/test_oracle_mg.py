"""Pins of the oracle's geometric multigrid (oracle/mg.py) against what the mathematics
fixes: interpolation reproduces affine fields, the re-discretised coarse operator equals
the Galerkin product on uniform fields, moduli and constraints restrict as defined, the
Chebyshev bound is attained on one element and holds on random fields, the smoother is
the closed-form Chebyshev polynomial, the V-cycle is symmetric, and MG-preconditioned CG
reaches the direct solution in far fewer iterations than Jacobi-PCG."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest
import scipy.sparse as sp

import synth_inputs as si
from oracle import fem, mg, solvers

KE = fem.element_stiffness(0.3)


def _nodes(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


@pytest.mark.parametrize("dims", [(4, 2, 2), (5, 3, 1), (7, 4, 3)])
def test_prolongation_reproduces_affine_fields(dims):
    """Trilinear interpolation is exact for affine functions: coarse node (I, J, K) sits at
    fine coordinates (2I, 2J, 2K) (also past an odd mesh end)."""
    nx, ny, nz = dims
    cx, cy, cz = mg.coarse_dims(nx, ny, nz)
    P = mg.prolongation(nx, ny, nz)
    assert P.shape == (3 * (nx + 1) * (ny + 1) * (nz + 1), 3 * (cx + 1) * (cy + 1) * (cz + 1))
    I, J, K = _nodes(cx, cy, cz)
    i, j, k = _nodes(nx, ny, nz)
    coef = np.array([[0.3, -1.1, 2.0, 0.7], [1.5, 0.2, -0.4, -2.0], [-0.6, 0.9, 1.3, 0.1]])
    vc = np.zeros((I.size, 3))
    vf = np.zeros((i.size, 3))
    for c in range(3):
        a0, a1, a2, a3 = coef[c]
        vc[:, c] = a0 + a1 * 2 * I + a2 * 2 * J + a3 * 2 * K
        vf[:, c] = a0 + a1 * i + a2 * j + a3 * k
    assert np.max(np.abs(P @ vc.ravel() - vf.ravel())) <= 1e-12


@pytest.mark.parametrize("dims", [(4, 2, 2), (6, 4, 2)])
def test_rediscretised_coarse_operator_is_galerkin_on_uniform_fields(dims):
    """Nested trilinear spaces: with a uniform modulus and even element counts the coarse
    operator of edge 2h (K_E scaled by 2) equals P^T K_h P exactly (no constraints)."""
    nx, ny, nz = dims
    E = np.full(nx * ny * nz, 0.7)
    Kf = fem.assemble_K(nx, ny, nz, E, KE)
    P = mg.prolongation(nx, ny, nz)
    cx, cy, cz = mg.coarse_dims(nx, ny, nz)
    Ec = mg.restrict_modulus(E, nx, ny, nz)
    assert np.allclose(Ec, 0.7, rtol=0, atol=1e-15)
    Kc = fem.assemble_K(cx, cy, cz, Ec, 2.0 * KE)
    G = (P.T @ Kf @ P).toarray()
    assert np.max(np.abs(G - Kc.toarray())) <= 1e-12 * np.max(np.abs(G))


def test_restrict_modulus_sums_children():
    rng = np.random.default_rng(3)
    nx, ny, nz = 6, 4, 2
    E = rng.uniform(0.01, 1.0, nx * ny * nz)
    Ec = mg.restrict_modulus(E, nx, ny, nz)
    assert abs(8.0 * Ec.sum() - E.sum()) <= 1e-12 * E.sum()
    # odd counts: the last coarse element holds the existing children only
    nx, ny, nz = 5, 3, 1
    E = np.ones(nx * ny * nz)
    Ec = mg.restrict_modulus(E, nx, ny, nz).reshape(1, 2, 3)
    assert Ec[0, 0, 0] == 4 / 8 and Ec[0, 0, 2] == 2 / 8 and Ec[0, 1, 2] == 1 / 8


@pytest.mark.parametrize("kind", ["cantilever", "torsion"])
def test_coarse_constraints_keep_the_clamped_face(kind):
    """The support rule maps a clamped face onto exactly the coarse clamped face on every
    level (odd counts included) and every level's operator is positive definite."""
    nx, ny, nz = 11, 5, 7
    fixed_ids = si.cantilever_fixed_dofs(nx, ny, nz) if kind == "cantilever" else \
        si.torsion_fixed_dofs(nx, ny, nz)
    fixed = fem.fixed_mask(3 * (nx + 1) * (ny + 1) * (nz + 1), fixed_ids)
    levels = mg.build_hierarchy(nx, ny, nz, np.full(nx * ny * nz, 0.5), KE, fixed)
    assert len(levels) >= 3
    for lev in levels:
        lx, ly, lz = lev.dims
        i, j, k = _nodes(lx, ly, lz)
        face = (i == 0) if kind == "cantilever" else (k == 0)
        want = np.repeat(face, 3)
        assert np.array_equal(lev.fixed, want), lev.dims
    C = levels[-1].K.toarray()
    assert np.linalg.eigvalsh(C)[0] > 0


def test_chebyshev_bound():
    """lambda_max(K_E) / K_E[0,0] equals lambda_max(D^-1 K) on one unconstrained element
    and bounds it on constrained random-density meshes."""
    lam = mg.chebyshev_bound(KE)
    assert abs(np.linalg.eigvalsh(KE / KE[0, 0])[-1] - lam) <= 1e-12 * lam
    rng = np.random.default_rng(0)
    nx, ny, nz = 6, 3, 3
    fixed = fem.fixed_mask(3 * (nx + 1) * (ny + 1) * (nz + 1), si.cantilever_fixed_dofs(nx, ny, nz))
    for _ in range(3):
        E = fem.simp_modulus(rng.uniform(0.01, 1, nx * ny * nz), 1.0, 1e-9, 3.0)
        K = fem.constrain(fem.assemble_K(nx, ny, nz, E, KE), fixed).toarray()
        d = np.sqrt(np.diag(K))
        assert np.linalg.eigvalsh(K / np.outer(d, d))[-1] <= lam * (1 + 1e-12)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_chebyshev_smoother_is_the_chebyshev_polynomial(degree):
    """From x0 = 0 on A = diag(lambda), d = 1: x = (1 - p(A)) A^-1 b with
    p(l) = T_k((theta - l) / delta) / T_k(theta / delta) over [lam / alpha, lam]."""
    lam, alpha = 5.0, 20.0
    lo, hi = lam / alpha, lam
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    ev = np.linspace(0.01, lam, 37)
    A = sp.diags(ev)
    b = np.random.default_rng(1).standard_normal(ev.size)
    x = mg.chebyshev_smooth(A, np.ones(ev.size), b, np.zeros(ev.size), degree, lam, alpha)
    Tk = npc.Chebyshev.basis(degree)
    p = Tk((theta - ev) / delta) / Tk(theta / delta)
    assert np.max(np.abs(x - (1 - p) * b / ev)) <= 1e-12 * np.max(np.abs(b / ev))


def _problem(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    E = fem.simp_modulus(rng.uniform(0.01, 1, nx * ny * nz), 1.0, 1e-9, 3.0)
    fixed = fem.fixed_mask(3 * (nx + 1) * (ny + 1) * (nz + 1), si.cantilever_fixed_dofs(nx, ny, nz))
    return E, fixed, si.cantilever_load(nx, ny, nz)


def test_vcycle_is_symmetric():
    nx, ny, nz = 9, 5, 4
    E, fixed, _ = _problem(nx, ny, nz, 2)
    levels = mg.build_hierarchy(nx, ny, nz, E, KE, fixed)
    lam = mg.chebyshev_bound(KE)
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, fixed.size))
    a[fixed] = b[fixed] = 0.0
    Va, Vb = mg.vcycle(levels, a, lam), mg.vcycle(levels, b, lam)
    assert abs(b @ Va - a @ Vb) <= 1e-10 * abs(b @ Va)
    assert a @ Va > 0 and b @ Vb > 0  # positive definite


@pytest.mark.parametrize("dims", [(16, 8, 8), (13, 7, 5)])
def test_mg_pcg_reaches_the_direct_solution(dims):
    nx, ny, nz = dims
    E, fixed, f = _problem(nx, ny, nz, 4)
    levels = mg.build_hierarchy(nx, ny, nz, E, KE, fixed)
    lam = mg.chebyshev_bound(KE)
    u, it, hist = mg.pcg_mg(levels, f, lam, tol=1e-10)
    ud = solvers.solve_direct(levels[0].K, f)
    assert np.linalg.norm(u - ud) <= 1e-8 * np.linalg.norm(ud)
    K = levels[0].K
    _, itj, _ = solvers.pcg_jacobi(lambda v: K @ v, levels[0].d, f, tol=1e-10)
    assert it <= itj / 5, (it, itj)
