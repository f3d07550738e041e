"""Pins of the oracle's solvers: direct vs PCG, the paper's iteration counts, Lanczos vs
a dense eigensolver, and the precision-admissibility rule."""
import json
import os

import numpy as np
import pytest

import synth_inputs as si
from oracle import fem, solvers

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _system(nx, ny, nz, seed=0, uniform=None):
    KE = fem.element_stiffness(0.3)
    n = nx * ny * nz
    x = (np.full(n, uniform) if uniform is not None
         else np.random.default_rng(seed).uniform(0.2, 1.0, n))
    E = fem.simp_modulus(x, 1.0, 1e-9, 3.0)
    K = fem.assemble_K(nx, ny, nz, E, KE)
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    return fem.constrain(K, fixed), fixed, si.cantilever_load(nx, ny, nz)


@pytest.mark.parametrize("dims", [(2, 1, 1), (4, 2, 2), (16, 8, 8)])
def test_pcg_matches_direct(dims):
    Kc, fixed, f = _system(*dims)
    u_d = solvers.solve_direct(Kc, f)
    assert np.linalg.norm(Kc @ u_d - f) <= 1e-12 * np.linalg.norm(f)
    u, it, hist = solvers.pcg_jacobi(lambda v: Kc @ v, Kc.diagonal(), f, None, 1e-13, 50000)
    assert hist[-1] <= 1e-13
    assert np.linalg.norm(u - u_d) <= 1e-9 * np.linalg.norm(u_d)
    # compliance identity f^T u = u^T K u at the solution
    assert abs(f @ u_d - u_d @ (Kc @ u_d)) <= 1e-12 * abs(f @ u_d)
    assert np.all(u_d[fixed] == 0.0) or np.max(np.abs(u_d[fixed])) < 1e-14


def test_pcg_warm_start_and_zero_rhs():
    Kc, fixed, f = _system(4, 2, 2)
    u, it, _ = solvers.pcg_jacobi(lambda v: Kc @ v, Kc.diagonal(), f, None, 1e-10)
    u2, it2, _ = solvers.pcg_jacobi(lambda v: Kc @ v, Kc.diagonal(), f, u, 1e-10)
    assert it2 == 0
    z, itz, _ = solvers.pcg_jacobi(lambda v: Kc @ v, Kc.diagonal(), 0 * f, None, 1e-10)
    assert itz == 0 and np.all(z == 0)


@pytest.mark.slow
def test_paper_iteration_count_64k():
    """Cold-start Jacobi-PCG iterations on the paper's 80x40x20 cantilever (golden)."""
    case = json.load(open(os.path.join(GOLDEN, "paper_pcg_iterations.json")))["cases"][0]
    nx, ny, nz = case["nx"], case["ny"], case["nz"]
    KE = fem.element_stiffness(0.3)
    E = fem.simp_modulus(np.full(nx * ny * nz, 0.5), 1.0, 1e-9, 3.0)
    K = fem.assemble_K(nx, ny, nz, E, KE)
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    Kc = fem.constrain(K, fixed)
    f = si.cantilever_midpoint_load(nx, ny, nz)
    _, it, _ = solvers.pcg_jacobi(lambda v: Kc @ v, Kc.diagonal(), f, None, 1e-5, 5000)
    assert abs(it - case["iterations"]) <= case["tolerance_iterations"]


def test_lanczos_matches_dense_eig():
    nx, ny, nz = 8, 4, 4
    Kc, fixed, _ = _system(nx, ny, nz, uniform=0.5)
    Kff = solvers.free_block(Kc, fixed)
    lo, hi = solvers.kappa_dense(Kff)
    v0 = np.random.default_rng(42).standard_normal(Kff.shape[0])
    a, b = solvers.lanczos_tridiagonal(lambda v: Kff @ v, v0, 600, reorthogonalize=True)
    lmin, lmax = solvers.tridiagonal_extremes(a, b)
    assert abs(lmax - hi) <= 1e-10 * hi
    assert abs(lmin - lo) <= 1e-8 * hi
    # Jacobi-scaled spectrum is computed as well and is better conditioned
    slo, shi = solvers.kappa_dense(Kff, jacobi_scaled=True)
    assert shi / slo < hi / lo


def test_jacobi_scaled_kappa_is_the_generalized_problem():
    """The spectrum of D^-1/2 K D^-1/2 is that of the pencil K x = lambda D x (D the
    diagonal of K), solved here by the library's generalized symmetric eigensolver."""
    import scipy.linalg as sla
    Kc, fixed, _ = _system(6, 3, 3, uniform=0.4)
    Kff = solvers.free_block(Kc, fixed)
    A = Kff.toarray()
    ev = sla.eigh(A, np.diag(np.diag(A)), eigvals_only=True)
    slo, shi = solvers.kappa_dense(Kff, jacobi_scaled=True)
    assert abs(slo - ev[0]) <= 1e-10 * ev[-1] and abs(shi - ev[-1]) <= 1e-12 * ev[-1]
    # a non-uniform density: the diagonal varies, so a wrong scaling would show
    Kc2, fixed2, _ = _system(6, 3, 3, uniform=None)
    A2 = solvers.free_block(Kc2, fixed2).toarray()
    ev2 = sla.eigh(A2, np.diag(np.diag(A2)), eigvals_only=True)
    slo2, shi2 = solvers.kappa_dense(solvers.free_block(Kc2, fixed2), jacobi_scaled=True)
    assert abs(slo2 - ev2[0]) <= 1e-8 * ev2[-1] and abs(shi2 - ev2[-1]) <= 1e-12 * ev2[-1]


def test_lanczos_on_constrained_operator_stays_free():
    """A start vector that is zero on fixed DOFs keeps K_c's Krylov space in the free
    subspace, so Lanczos on K_c returns K_ff's extremes (identity rows never enter)."""
    nx, ny, nz = 6, 3, 3
    Kc, fixed, _ = _system(nx, ny, nz, uniform=0.3)
    v0 = np.random.default_rng(42).standard_normal(Kc.shape[0])
    v0[fixed] = 0.0
    a, b = solvers.lanczos_tridiagonal(lambda v: Kc @ v, v0, 400, reorthogonalize=True)
    lmin, lmax = solvers.tridiagonal_extremes(a, b)
    lo, hi = solvers.kappa_dense(solvers.free_block(Kc, fixed))
    assert abs(lmax - hi) <= 1e-10 * hi and abs(lmin - lo) <= 1e-8 * hi


def test_kappa_independent_of_uniform_density():
    """At uniform density K = E K_1, so kappa does not depend on rho or p."""
    k = []
    for rho, p in [(0.5, 3.0), (0.5, 5.0), (0.9, 3.0)]:
        KE = fem.element_stiffness(0.3)
        E = fem.simp_modulus(np.full(32, rho), 1.0, 1e-9, p)
        K = fem.assemble_K(4, 4, 2, E, KE)
        fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(4, 4, 2))
        lo, hi = solvers.kappa_dense(solvers.free_block(fem.constrain(K, fixed), fixed))
        k.append(hi / lo)
    assert np.ptp(k) <= 1e-9 * k[0]


def test_precision_rule():
    assert solvers.precision_allowed(255.0, "bf16")
    assert not solvers.precision_allowed(256.0, "bf16")
    assert solvers.precision_allowed(1e7, "fp32")
    assert not solvers.precision_allowed(1e4, "fp16")


def test_lanczos_stopping_rule():
    """The stopping rule ends the run at the first multiple of the window where the
    smallest Ritz value moved by less than rtol over the last window; the extremes then
    bound the dense spectrum from inside and are close to it."""
    Kc, fixed, _ = _system(8, 4, 4, uniform=0.5)
    Kff = solvers.free_block(Kc, fixed)
    lo, hi = solvers.kappa_dense(Kff, jacobi_scaled=True)
    d = Kff.diagonal()
    s = 1.0 / np.sqrt(d)
    A = lambda v: s * (Kff @ (s * v))
    v0 = np.random.default_rng(42).standard_normal(Kff.shape[0])
    lmin, lmax, steps, conv = solvers.lanczos_extremes(A, v0, 2000, rtol=1e-3, window=50)
    assert conv and steps % 50 == 0 and steps < 2000
    assert lmin >= lo * (1 - 1e-10) and lmax <= hi * (1 + 1e-10)
    assert lmax >= hi * (1 - 1e-6) and lmin <= lo * (1 + 2e-3)
    # the rule, restated on the same coefficients: it did not fire one window earlier
    a, b = solvers.lanczos_tridiagonal(A, v0, steps)
    th = [solvers.tridiagonal_extremes(a[:j], b[:j - 1])[0] for j in range(50, steps + 1, 50)]
    assert abs(th[-1] - th[-2]) <= 1e-3 * th[-1]
    assert all(abs(th[i] - th[i - 1]) > 1e-3 * th[i] for i in range(1, len(th) - 1))
    # a cap below the convergence point reports "not converged"
    lmin2, _, steps2, conv2 = solvers.lanczos_extremes(A, v0, 60, rtol=1e-3, window=50)
    assert not conv2 and steps2 == 60 and lmin2 >= lmin * (1 - 1e-12)
