"""Pins of the oracle's element stiffness, assembly and constrained operator.

Each check comes from the mathematics of linear elasticity on a unit cube, not from the
oracle's own formulas: an analytic construction of K_E from one-dimensional integrals
(a different route from the Gauss-point B^T D B sum), constant-strain energies, the
rigid-body null space, the patch test, and two independent routes for K v.
"""
import itertools

import numpy as np
import pytest

import synth_inputs as si
from oracle import fem

NU = 0.3
LAM = NU / ((1 + NU) * (1 - 2 * NU))
MU = 1.0 / (2 * (1 + NU))


def _ke_analytic(lam, mu):
    """K_E from K[(a,c),(b,d)] = int lam dcNa ddNb + mu ddNa dcNb + mu delta_cd gradNa.gradNb,
    with every integral over the unit cube written as a product of 1D integrals of the
    linear hat functions phi0 = 1 - t, phi1 = t (derivative signs -1, +1)."""
    def one_d(sa, sb, da, db):
        # integral over [0,1] of phi_sa^(da) * phi_sb^(db), da/db = derivative flags
        s = lambda bit: 1.0 if bit else -1.0
        if da and db:
            return s(sa) * s(sb)
        if da:
            return s(sa) * 0.5
        if db:
            return s(sb) * 0.5
        return 1.0 / 3.0 if sa == sb else 1.0 / 6.0

    def grad_int(a, b, p, q):
        # integral of d_p N_a * d_q N_b
        out = 1.0
        for t in range(3):
            out *= one_d((a >> t) & 1, (b >> t) & 1, t == p, t == q)
        return out

    K = np.zeros((24, 24))
    for a, b, c, d in itertools.product(range(8), range(8), range(3), range(3)):
        v = lam * grad_int(a, b, c, d) + mu * grad_int(a, b, d, c)
        if c == d:
            v += mu * sum(grad_int(a, b, t, t) for t in range(3))
        K[3 * a + c, 3 * b + d] = v
    return K


def test_ke_matches_analytic_integrals():
    KE = fem.element_stiffness(NU)
    assert np.max(np.abs(KE - _ke_analytic(LAM, MU))) < 1e-14


@pytest.mark.parametrize("nu", [0.2, 0.3, 0.4])
def test_ke_matches_analytic_integrals_other_nu(nu):
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    assert np.max(np.abs(fem.element_stiffness(nu) - _ke_analytic(lam, mu))) < 1e-14


def test_ke_closed_form_entries():
    KE = fem.element_stiffness(NU)
    # every diagonal entry (lam + 4 mu) / 9 = (2 - 3nu) / (9 (1+nu)(1-2nu))
    assert np.allclose(np.diag(KE), (2 - 3 * NU) / (9 * (1 + NU) * (1 - 2 * NU)), rtol=0,
                       atol=1e-15)
    assert abs(KE[0, 0] - 0.2350427350427350) < 1e-15
    # same-node x-y coupling (lam + mu) / 12
    assert abs(KE[0, 1] - 1.0 / (24 * (1 + NU) * (1 - 2 * NU))) < 1e-15
    # x-edge neighbour (local node 0 and 1): xx -(lam+mu)/9, xy (lam-mu)/12, zz (lam+mu)/18
    assert abs(KE[0, 3] + (LAM + MU) / 9) < 1e-15
    assert abs(KE[0, 4] - (LAM - MU) / 12) < 1e-15
    assert abs(KE[2, 5] - (LAM + MU) / 18) < 1e-15


def test_ke_symmetry_spectrum_rowsums():
    KE = fem.element_stiffness(NU)
    assert np.array_equal(KE, KE.T) or np.max(np.abs(KE - KE.T)) < 1e-16
    ev = np.sort(np.linalg.eigvalsh(KE))
    expect = np.sort(np.array(
        [0.0] * 6 + [MU / 6] * 2 + [(LAM + 4 * MU) / 18] * 3 + [MU / 2] * 3 + [2 * MU / 3]
        + [MU] * 8 + [1.0 / (2 * (1 - 2 * NU))]))
    assert np.max(np.abs(ev - expect)) < 1e-14
    assert abs(np.trace(KE) - 5.641025641025641) < 1e-13
    # translations are in the null space: each row sums to zero per component
    for c in range(3):
        assert np.max(np.abs(KE[:, c::3].sum(axis=1))) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ke_constant_strain_energy(seed):
    """u_a = A X_a with symmetric A: u^T K_E u = eps : D : eps * volume (Q1 is exact on
    linear fields), eps in Voigt form with engineering shear."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3))
    A = 0.5 * (A + A.T)
    X = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float)
    u = (X @ A.T).ravel()
    eps = A
    tr = np.trace(eps)
    energy = LAM * tr * tr + 2 * MU * np.sum(eps * eps)
    KE = fem.element_stiffness(NU)
    assert abs(u @ KE @ u - energy) < 1e-13 * max(1.0, energy)


def test_edof_layout():
    ed = fem.edof_table(2, 1, 1)
    # element 0 local node 7 is node (1,1,1) = 1 + 3*(1 + 2*1) = 10
    assert list(ed[0, 21:24]) == [30, 31, 32]
    assert list(ed[1, 0:3]) == [3, 4, 5]


def _small(nx, ny, nz, seed=0):
    rng = np.random.default_rng(seed)
    E = rng.uniform(0.1, 1.0, nx * ny * nz)
    KE = fem.element_stiffness(NU)
    return E, KE, fem.assemble_K(nx, ny, nz, E, KE)


def test_global_K_symmetric_psd_nullspace():
    nx, ny, nz = 3, 2, 2
    E, KE, K = _small(nx, ny, nz)
    Kd = K.toarray()
    assert np.max(np.abs(Kd - Kd.T)) < 1e-15
    ev = np.linalg.eigvalsh(Kd)
    assert ev[0] > -1e-13
    assert np.sum(ev < 1e-10 * ev[-1]) == 6  # exactly the rigid-body modes
    R = fem.rigid_body_modes(nx, ny, nz)
    assert np.linalg.norm(Kd @ R) <= 1e-13 * np.linalg.norm(Kd) * np.linalg.norm(R)


def test_patch_test_uniform_E():
    """Uniform E, u = A X: zero force at every interior node; on a face-interior node
    the force equals the traction sigma n times the node's tributary area (1)."""
    nx, ny, nz = 4, 3, 3
    KE = fem.element_stiffness(NU)
    K = fem.assemble_K(nx, ny, nz, np.ones(nx * ny * nz), KE)
    X = si.node_coords(nx, ny, nz).astype(float)
    A = np.array([[0.3, -0.2, 0.1], [0.5, 0.7, -0.4], [0.2, 0.6, -0.1]])
    u = (X @ A.T).ravel()
    F = (K @ u).reshape(-1, 3)
    eps = 0.5 * (A + A.T)
    sigma = LAM * np.trace(eps) * np.eye(3) + 2 * MU * eps
    i, j, k = X[:, 0], X[:, 1], X[:, 2]
    on = [(i == 0), (i == nx), (j == 0), (j == ny), (k == 0), (k == nz)]
    normals = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    nfaces = sum(o.astype(int) for o in on)
    interior = nfaces == 0
    assert np.max(np.abs(F[interior])) < 1e-13
    for o, nrm in zip(on, normals):
        sel = o & (nfaces == 1)
        assert np.max(np.abs(F[sel] - sigma @ np.array(nrm, float))) < 1e-13


def test_two_routes_for_Kv_agree():
    nx, ny, nz = 5, 4, 3
    E, KE, K = _small(nx, ny, nz, seed=3)
    n_dof = K.shape[0]
    fixed = fem.fixed_mask(n_dof, si.cantilever_fixed_dofs(nx, ny, nz))
    Kc = fem.constrain(K, fixed)
    v = np.random.default_rng(4).standard_normal(n_dof)
    y1 = Kc @ v
    y2 = fem.apply_K_elementwise(nx, ny, nz, E, KE, v, fixed, chunk=7)
    assert np.linalg.norm(y1 - y2) <= 1e-14 * np.linalg.norm(y1)
    assert np.array_equal(y2[fixed], v[fixed])


@pytest.mark.parametrize("dims", [(5, 4, 3), (1, 1, 1), (7, 2, 5)])
def test_grid_route_for_Kv_agrees_with_assembly(dims):
    """The grid-slice route (used for full-size checks) against the assembled CSR and
    the element-by-element route, with and without Dirichlet rows; a permuted local-node
    offset or a transposed K_E would break it (K_E is symmetric, but the offsets are
    not)."""
    nx, ny, nz = dims
    E, KE, K = _small(nx, ny, nz, seed=11)
    n_dof = K.shape[0]
    v = np.random.default_rng(12).standard_normal(n_dof)
    assert np.linalg.norm(fem.apply_K_grid(nx, ny, nz, E, KE, v) - K @ v) <= 1e-14 * np.linalg.norm(K @ v)
    fixed = fem.fixed_mask(n_dof, si.cantilever_fixed_dofs(nx, ny, nz))
    y1 = fem.constrain(K, fixed) @ v
    y3 = fem.apply_K_grid(nx, ny, nz, E, KE, v, fixed)
    assert np.linalg.norm(y1 - y3) <= 1e-14 * np.linalg.norm(y1)
    assert np.array_equal(y3[fixed], v[fixed])


def test_grid_diagonal_agrees_with_element_route():
    nx, ny, nz = 6, 3, 4
    E, KE, K = _small(nx, ny, nz, seed=13)
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    d1 = fem.diag_K(nx, ny, nz, E, KE, fixed)
    d2 = fem.diag_K_grid(nx, ny, nz, E, KE, fixed)
    assert np.max(np.abs(d1 - d2)) <= 1e-15 * np.max(d1)
    assert np.array_equal(d2, fem.constrain(K, fixed).diagonal()) or \
        np.max(np.abs(d2 - fem.constrain(K, fixed).diagonal())) <= 1e-15 * np.max(d1)


def test_constrained_operator_rows():
    nx, ny, nz = 3, 2, 2
    E, KE, K = _small(nx, ny, nz)
    fixed = fem.fixed_mask(K.shape[0], si.cantilever_fixed_dofs(nx, ny, nz))
    Kc = fem.constrain(K, fixed).toarray()
    Kd = K.toarray()
    fr = ~fixed
    assert np.array_equal(Kc[np.ix_(fixed, fixed)], np.eye(fixed.sum()))
    assert np.all(Kc[np.ix_(fixed, fr)] == 0) and np.all(Kc[np.ix_(fr, fixed)] == 0)
    assert np.array_equal(Kc[np.ix_(fr, fr)], Kd[np.ix_(fr, fr)])
    assert np.linalg.eigvalsh(Kc)[0] > 0  # clamped face removes the null space


def test_diag_closed_form():
    """diag(K) at node n, component c = K_E,d * sum of E over the elements at n."""
    nx, ny, nz = 3, 3, 3
    E, KE, K = _small(nx, ny, nz, seed=5)
    d = fem.diag_K(nx, ny, nz, E, KE)
    assert np.max(np.abs(d - K.diagonal())) < 1e-15
    n_int = int(si.node_id(1, 1, 1, nx, ny))
    Eg = E.reshape(nz, ny, nx)
    s = Eg[0:2, 0:2, 0:2].sum()
    kd = (2 - 3 * NU) / (9 * (1 + NU) * (1 - 2 * NU))
    assert abs(d[3 * n_int] - kd * s) < 1e-15
    dun = fem.diag_K(nx, ny, nz, np.ones(nx * ny * nz), KE)
    assert abs(dun[3 * n_int] - 1.8803418803418803) < 1e-14


def test_problem_inputs():
    for name in ["cantilever_16x8x8", "torsion_55x55x165"]:
        cfg, fixed, f = si.problem(name)
        nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
        assert f.size == 3 * (nx + 1) * (ny + 1) * (nz + 1)
        assert np.all(f[fixed] == 0.0)
        F = f.reshape(-1, 3)
        # zero net force for torsion, -(nz+1) in y for the cantilever
        if cfg["kind"] == "torsion":
            assert np.max(np.abs(F.sum(axis=0))) < 1e-12
            X = si.node_coords(nx, ny, nz).astype(float) - [nx / 2, ny / 2, 0]
            Mz = np.sum(X[:, 0] * F[:, 1] - X[:, 1] * F[:, 0])
            assert Mz > 0 and np.count_nonzero(F[:, 0] ** 2 + F[:, 1] ** 2) == 220
        else:
            assert F[:, 1].sum() == -(nz + 1)
    c = si.counts(16, 8, 8)
    assert (c["n_node"], c["n_dof"]) == (1377, 4131)
    assert si.cantilever_fixed_dofs(16, 8, 8).size == 243


@pytest.mark.parametrize("kind,dims", [("mbb", (12, 4, 3)), ("mbb", (12, 4, 2)),
                                       ("bridge", (12, 4, 3)), ("bridge", (9, 3, 2))])
def test_stress_test_presets_are_well_posed(kind, dims):
    """MBB and bridge (Sec. "Experimental Setup", hard-problem stress tests): the
    constrained operator is positive definite (no rigid mode survives the supports), the
    load is a unit downward total applied only on free DOFs."""
    nx, ny, nz = dims
    fixed_ids, f = si.bcs_and_load(kind, nx, ny, nz)
    fixed = fem.fixed_mask(f.size, fixed_ids)
    K = fem.constrain(fem.assemble_K(nx, ny, nz, np.full(nx * ny * nz, 0.5),
                                     fem.element_stiffness(0.3)), fixed).toarray()
    assert np.linalg.eigvalsh(K)[0] > 1e-6
    F = f.reshape(-1, 3)
    assert abs(F[:, 1].sum() + 1.0) <= 1e-12 and np.all(F[:, [0, 2]] == 0.0)
    assert np.all(f[fixed] == 0.0)
    # the reading of the MBB supports: x = 0 face holds u_x only; the far bottom edge
    # holds u_y over the depth and u_z at mid-depth
    if kind == "mbb":
        c = si.node_coords(nx, ny, nz)
        fx = fixed.reshape(-1, 3)
        assert np.array_equal(fx[:, 0], c[:, 0] == 0)
        edge = (c[:, 0] == nx) & (c[:, 1] == 0)
        mid = np.isin(c[:, 2], [nz // 2] if nz % 2 == 0 else [nz // 2, nz // 2 + 1])
        assert np.array_equal(fx[:, 1], edge) and np.array_equal(fx[:, 2], edge & mid)
