"""Pins of the oracle's compliance, sensitivities, density filter, OC update and SIMP
loop: finite differences, stencil weights from the cone definition, adjointness,
bracketing by an independent root finder, and mirror/rotation symmetry of designs."""
import numpy as np
import pytest
from scipy.optimize import brentq

import synth_inputs as si
from oracle import fem, solvers, topopt


def test_filter_weights_and_invariants():
    nx, ny, nz = 5, 4, 3
    H, Hs = topopt.filter_matrix(nx, ny, nz, 1.5)
    Hd = H.toarray()
    assert np.array_equal(Hd, Hd.T)
    e = 1 + nx * (1 + ny * 1)  # interior element (1,1,1)
    row = Hd[e]
    assert abs(row[e] - 1.5) < 1e-15
    assert np.count_nonzero(row) == 19
    assert abs(row[e + 1] - 0.5) < 1e-15
    assert abs(row[e + 1 + nx] - (1.5 - np.sqrt(2))) < 1e-15
    assert row[e + 1 + nx + nx * ny] == 0.0  # corner neighbour excluded (sqrt 3 > 1.5)
    assert abs(Hs[e] - (22.5 - 12 * np.sqrt(2))) < 1e-14  # 1.5 + 6*0.5 + 12*(1.5 - sqrt 2)
    assert abs(Hs[0] - (1.5 + 3 * 0.5 + 3 * (1.5 - np.sqrt(2)))) < 1e-14
    x = np.full(nx * ny * nz, 0.37)
    assert np.max(np.abs(topopt.filter_forward(H, Hs, x) - 0.37)) < 1e-15
    rng = np.random.default_rng(1)
    a, g = rng.standard_normal(x.size), rng.standard_normal(x.size)
    lhs = topopt.filter_forward(H, Hs, a) @ g
    rhs = a @ topopt.filter_adjoint(H, Hs, g)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_filter_radius_two():
    H, Hs = topopt.filter_matrix(6, 6, 6, 2.0)
    e = 3 + 6 * (3 + 6 * 3)
    # offsets with |d| < 2: 1 + 6 + 12 + 8 = 27 (distance-2 points get weight 0)
    assert np.count_nonzero(H[e].toarray()) == 27


def _small_problem(nx=3, ny=2, nz=2):
    fixed = si.cantilever_fixed_dofs(nx, ny, nz)
    f = si.cantilever_load(nx, ny, nz)
    return topopt.Problem(nx, ny, nz, fixed, f, volfrac=0.3)


def test_sensitivity_finite_difference():
    prob = _small_problem()
    rng = np.random.default_rng(7)
    xphys = rng.uniform(0.2, 1.0, prob.n_elem)
    u, _ = prob.solve(xphys, direct=True)
    dc = prob.sensitivity(xphys, u)
    c0 = topopt.compliance(prob.f, u)
    h = 1e-6
    for e in range(prob.n_elem):
        xp, xm = xphys.copy(), xphys.copy()
        xp[e] += h
        xm[e] -= h
        cp = topopt.compliance(prob.f, prob.solve(xp, direct=True)[0])
        cm = topopt.compliance(prob.f, prob.solve(xm, direct=True)[0])
        fd = (cp - cm) / (2 * h)
        assert abs(fd - dc[e]) <= 1e-6 * max(abs(dc[e]), 1e-3 * c0)
    # sum_e E_e ce_e = u^T K u = f^T u
    ce = topopt.element_energy(prob.nx, prob.ny, prob.nz, u, prob.KE)
    assert abs(np.sum(prob.modulus(xphys) * ce) - c0) < 1e-11 * c0
    assert np.all(dc <= 0)


def test_oc_bracket_contains_root_and_limits():
    prob = _small_problem(6, 3, 3)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.1, 0.6, prob.n_elem)
    dc = -rng.uniform(0.01, 2.0, prob.n_elem)
    dv = prob.dv
    xnew, xphys, change, steps = topopt.oc_update(x, dc, dv, prob.H, prob.Hs, 0.3, 0.2)
    assert np.all(xnew >= 0) and np.all(xnew <= 1)
    assert np.all(np.abs(xnew - x) <= 0.2 + 1e-15)
    assert abs(change - np.max(np.abs(xnew - x))) == 0.0
    assert np.allclose(xphys, topopt.filter_forward(prob.H, prob.Hs, xnew), rtol=0,
                       atol=1e-15)

    def excess(lam):
        xn = np.clip(np.sqrt(-dc / (dv * lam)) * x, np.maximum(x - 0.2, 0),
                     np.minimum(x + 0.2, 1))
        return topopt.filter_forward(prob.H, prob.Hs, xn).sum() - 0.3 * x.size

    root = brentq(excess, 1e-9, 1e9, xtol=1e-14, rtol=1e-15)
    # the final midpoint is within the bisection's relative bracket of the root
    lam = (np.sqrt(-dc / dv) * x)  # recover the multiplier from an unclipped element
    free = (xnew > np.maximum(x - 0.2, 0) + 1e-12) & (xnew < np.minimum(x + 0.2, 1) - 1e-12)
    lam_used = np.median((lam[free] / xnew[free]) ** 2)
    assert abs(lam_used - root) / root <= 2e-3
    assert abs(xphys.sum() - 0.3 * x.size) / (0.3 * x.size) < 2e-3
    assert steps > 10


def test_simp_z_mirror_symmetry_cantilever():
    nx, ny, nz = 8, 4, 4
    prob = topopt.Problem(nx, ny, nz, si.cantilever_fixed_dofs(nx, ny, nz),
                          si.cantilever_load(nx, ny, nz), volfrac=0.3)
    hist, x, xphys, u = topopt.simp_run(prob, 4, direct=True)
    g = x.reshape(nz, ny, nx)
    assert np.max(np.abs(g - g[::-1])) < 1e-10
    cs = [h["c"] for h in hist]
    assert cs[-1] < cs[0]
    assert all(abs(h["vol"] - 0.3) < 2e-3 for h in hist)


def test_simp_torsion_rotation_symmetry():
    n, nz = 6, 6
    prob = topopt.Problem(n, n, nz, si.torsion_fixed_dofs(n, n, nz),
                          si.torsion_load(n, n, nz), volfrac=0.3)
    hist, x, xphys, u = topopt.simp_run(prob, 3, direct=True)
    g = x.reshape(nz, n, n)  # [z, y, x]
    rot = np.rot90(g, k=1, axes=(1, 2))
    assert np.max(np.abs(g - rot)) < 1e-9


def test_simp_pcg_equals_direct_path():
    prob = _small_problem(8, 4, 4)
    h1, x1, _, _ = topopt.simp_run(prob, 3, direct=True)
    h2, x2, _, _ = topopt.simp_run(prob, 3, tol=1e-12)
    for a, b in zip(h1, h2):
        assert abs(a["c"] - b["c"]) <= 1e-9 * a["c"]
    assert np.max(np.abs(x1 - x2)) < 1e-8


# ---- smoothed Heaviside projection (pins independent of the formula's own form) ----
@pytest.mark.parametrize("beta,eta", [(1.0, 0.5), (8.0, 0.5), (32.0, 0.3), (4.0, 0.7)])
def test_projection_fixes_the_ends_and_increases(beta, eta):
    x = np.linspace(0.0, 1.0, 1001)
    h = topopt.heaviside_project(x, beta, eta)
    assert abs(h[0]) <= 1e-15 and abs(h[-1] - 1.0) <= 1e-15
    assert np.all(np.diff(h) >= 0)  # tanh saturates to 1.0 in double far from eta
    assert np.all(np.diff(h)[np.abs(x[:-1] - eta) < 0.1] > 0)


def test_projection_limits_identity_and_step():
    x = np.linspace(0.0, 1.0, 201)
    for eta in (0.5, 0.3):
        # beta -> 0: tanh is linear, the projection is the identity (error O(beta^2))
        assert np.max(np.abs(topopt.heaviside_project(x, 1e-4, eta) - x)) <= 1e-8
        # beta -> infinity: a unit step at eta
        big = topopt.heaviside_project(np.array([eta - 0.05, eta + 0.05]), 400.0, eta)
        assert big[0] <= 1e-6 and big[1] >= 1.0 - 1e-6


@pytest.mark.parametrize("beta", [1.0, 16.0])
def test_projection_at_half_is_odd_about_the_threshold(beta):
    t = np.linspace(0.0, 0.5, 101)
    a = topopt.heaviside_project(0.5 + t, beta, 0.5)
    b = topopt.heaviside_project(0.5 - t, beta, 0.5)
    assert np.max(np.abs(a + b - 1.0)) <= 1e-15
    # eta = 1/2: the same map written as 1/2 + tanh(beta (x - 1/2)) / (2 tanh(beta / 2))
    alt = 0.5 + np.tanh(beta * t) / (2.0 * np.tanh(beta / 2.0))
    assert np.max(np.abs(a - alt)) <= 1e-15


@pytest.mark.parametrize("beta,eta", [(2.0, 0.5), (16.0, 0.5), (8.0, 0.35)])
def test_projection_derivative_against_differences_and_its_integral(beta, eta):
    from scipy.integrate import quad
    x = np.linspace(0.01, 0.99, 99)
    h = 1e-6
    fd = (topopt.heaviside_project(x + h, beta, eta) -
          topopt.heaviside_project(x - h, beta, eta)) / (2 * h)
    d = topopt.heaviside_derivative(x, beta, eta)
    assert np.max(np.abs(fd - d)) <= 1e-7 * np.max(d)
    total, _ = quad(lambda s: float(topopt.heaviside_derivative(s, beta, eta)), 0.0, 1.0,
                    epsabs=1e-13, epsrel=1e-13, limit=200)
    assert abs(total - 1.0) <= 1e-10


def test_three_field_sensitivity_is_the_derivative_of_compliance():
    """Central differences of c(x) = f^T u(x), u from a direct solve at the projected
    filtered density, against the chained sensitivity (filter, projection, SIMP)."""
    nx, ny, nz = 4, 2, 2
    prob = topopt.Problem(nx, ny, nz, si.cantilever_fixed_dofs(nx, ny, nz),
                          si.cantilever_load(nx, ny, nz), volfrac=0.3)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.2, 0.8, prob.n_elem)
    beta, eta = 4.0, 0.5

    def comp(xx):
        xphys = topopt.heaviside_project(topopt.filter_forward(prob.H, prob.Hs, xx), beta, eta)
        u = solvers.solve_direct(prob.stiffness(xphys), prob.f)
        return float(prob.f @ u)

    xphys = topopt.heaviside_project(topopt.filter_forward(prob.H, prob.Hs, x), beta, eta)
    u = solvers.solve_direct(prob.stiffness(xphys), prob.f)
    _, dc = topopt.three_field_sensitivity(prob, x, u, beta, eta)
    h = 1e-6
    for e in range(prob.n_elem):
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        fd = (comp(xp) - comp(xm)) / (2 * h)
        assert abs(fd - dc[e]) <= 1e-5 * np.max(np.abs(dc)), (e, fd, dc[e])
