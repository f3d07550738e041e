"""Geometric multigrid preconditioner for K_c(rho) (oracle, float64, CPU; test
infrastructure only: the library never calls it).

Paper: Sec. "Path to Geometric Multigrid Integration" names the pieces a V-cycle needs on
the structured mesh: the fused operator as the fine-grid smoother (a fixed number of
matvec-plus-update steps per pre/post smoothing), a restriction R between grids,
the prolongation P = R^T, and a direct solve on the coarsest grid.  It leaves open how
the coarse operators are formed and which smoother is used; the readings taken here:

* Hierarchy.  Level l + 1 halves the element count of level l per axis, rounding up
  (n -> ceil(n / 2)); its elements have twice the edge.  An odd count leaves the last
  coarse element half outside the mesh.  Coarsening stops once an axis has one element
  (or after a level cap); the last level is solved exactly.
* Coarse operators by re-discretisation: the element stiffness scales with the edge
  (K_E(2h) = 2 K_E(h) for 3D linear elasticity) and a coarse element's modulus is the
  sum of its (up to eight) children's moduli divided by eight, so a coarse element's
  energy under a uniform strain equals its children's.  On a uniform field and even
  element counts this equals the Galerkin product P^T K P (nested trilinear spaces).
* Transfer: P is trilinear interpolation of nodal values (per displacement component;
  fine node 2i takes coarse node i, node 2i + 1 the mean of i and i + 1), R = P^T.
* Boundary conditions: a coarse DOF is fixed when any fine DOF it interpolates to
  (P weight > 0: fine nodes 2I - 1 .. 2I + 1 per axis, same component) is fixed, so no
  constraint is lost on odd grids (matching only the fine node 2I drops the nodes that
  fall past the mesh and can leave a rigid mode on coarse levels); a clamped face stays
  exactly the clamped face.  Every level's operator keeps fixed rows as identity
  (K_c = P K P + (I - P)); restricted residuals and prolonged corrections are zeroed on
  fixed DOFs.
* Smoother: Chebyshev iteration of degree k on D^-1 K (D the level's diagonal) over the
  interval [lam / alpha, lam] with lam = lambda_max(K_E) / K_E[0, 0], an upper bound of
  lambda_max(D^-1 K) for every density field (the Rayleigh quotient of K against its
  diagonal is a modulus-weighted mean of element quotients, and every diagonal entry of
  K_E is the same).  Pre- and post-smoothing use the same polynomial, so the V-cycle is
  a symmetric preconditioner.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle import fem, solvers


def coarse_dims(nx: int, ny: int, nz: int):
    """Element counts of the next coarser level: ceil(n / 2) per axis."""
    return (nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2


def interpolation_1d(n: int) -> sp.csr_matrix:
    """Nodal linear interpolation from the ceil(n/2) + 1 coarse nodes of an axis of n
    fine elements to its n + 1 fine nodes."""
    nc = (n + 1) // 2
    rows, cols, vals = [], [], []
    for i in range(n + 1):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [i // 2, i // 2 + 1]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, nc + 1))


def prolongation(nx: int, ny: int, nz: int) -> sp.csr_matrix:
    """P (fine DOFs x coarse DOFs): trilinear interpolation of each displacement
    component.  Node ids i + (nx+1)(j + (ny+1)k), DOF 3 node + c, on both grids."""
    Pn = sp.kron(interpolation_1d(nz), sp.kron(interpolation_1d(ny), interpolation_1d(nx)))
    return sp.kron(Pn, sp.identity(3), format="csr")


def restrict_modulus(E: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Coarse element moduli: the sum of the existing children's moduli over eight."""
    cx, cy, cz = coarse_dims(nx, ny, nz)
    Ef = E.reshape(nz, ny, nx)
    Ec = np.zeros((cz, cy, cx))
    for a in range(2):
        for b in range(2):
            for c in range(2):
                sub = Ef[c::2, b::2, a::2]
                Ec[:sub.shape[0], :sub.shape[1], :sub.shape[2]] += sub
    return (Ec / 8.0).ravel()


def coarse_fixed(fixed: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Fixed-DOF mask of the coarser level: a coarse DOF is fixed when a fine DOF in its
    interpolation support is."""
    P = prolongation(nx, ny, nz)
    return (P.T @ fixed.astype(np.float64)) > 0.0


def chebyshev_bound(KE: np.ndarray) -> float:
    """lambda_max(K_E) / K_E[0,0]: an upper bound of lambda_max(D^-1 K) on any mesh."""
    assert np.allclose(np.diag(KE), KE[0, 0])
    return float(np.linalg.eigvalsh(KE)[-1] / KE[0, 0])


class Level:
    """One grid of the hierarchy: dims, moduli, constrained operator, diagonal, fixed
    mask, and (below the finest) the prolongation from this level to the one above."""

    def __init__(self, nx, ny, nz, E, KE, fixed):
        self.dims = (nx, ny, nz)
        self.E = E
        self.fixed = fixed
        self.K = fem.constrain(fem.assemble_K(nx, ny, nz, E, KE), fixed)
        self.d = self.K.diagonal().copy()
        self.P = None  # set on coarse levels: fine-of-parent x this level


def build_hierarchy(nx, ny, nz, E, KE, fixed, max_levels=8):
    """Levels 0 (finest) .. L-1, coarsening while every axis has at least two elements
    and fewer than max_levels levels exist."""
    levels = [Level(nx, ny, nz, E, KE, fixed)]
    scale = 1.0
    while len(levels) < max_levels and min(levels[-1].dims) >= 2:
        fx, fy, fz = levels[-1].dims
        cx, cy, cz = coarse_dims(fx, fy, fz)
        scale *= 2.0
        Ec = restrict_modulus(levels[-1].E, fx, fy, fz)
        fc = coarse_fixed(levels[-1].fixed, fx, fy, fz)
        lev = Level(cx, cy, cz, Ec, scale * KE, fc)
        lev.P = prolongation(fx, fy, fz)
        levels.append(lev)
    return levels


def chebyshev_smooth(K, d, b, x, degree, lam, alpha):
    """`degree` Chebyshev steps for K x = b preconditioned by diag d, eigenvalues of
    D^-1 K taken in [lam / alpha, lam] (three-term recurrence of the shifted and scaled
    Chebyshev polynomials)."""
    lo, hi = lam / alpha, lam
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b - K @ x
    dd = (r / d) / theta
    x = x + dd
    for _ in range(degree - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        r = b - K @ x
        dd = rho_new * rho * dd + (2.0 * rho_new / delta) * (r / d)
        x = x + dd
        rho = rho_new
    return x


def vcycle(levels, b, lam, degree=2, alpha=20.0, l=0):
    """Approximate solve of K_l x = b: pre-smooth from zero, restrict the residual,
    recurse (exact solve on the coarsest level), prolong and add, post-smooth."""
    lev = levels[l]
    if l == len(levels) - 1:
        return solvers.solve_direct(lev.K, b)
    x = chebyshev_smooth(lev.K, lev.d, b, np.zeros_like(b), degree, lam, alpha)
    r = b - lev.K @ x
    nxt = levels[l + 1]
    rc = nxt.P.T @ r
    rc[nxt.fixed] = 0.0
    ec = vcycle(levels, rc, lam, degree, alpha, l + 1)
    e = nxt.P @ ec
    e[lev.fixed] = 0.0
    x = x + e
    return chebyshev_smooth(lev.K, lev.d, b, x, degree, lam, alpha)


def pcg_mg(levels, b, lam, x0=None, tol=1e-8, maxit=1000, degree=2, alpha=20.0):
    """CG on the finest level preconditioned by one V-cycle per iteration; stops on the
    recursive ||r|| <= tol ||b||.  Returns (x, iterations, history ||r_k|| / ||b||)."""
    K = levels[0].K
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0]
    r = b - K @ x
    hist = [np.linalg.norm(r) / bnorm]
    if hist[-1] <= tol:
        return x, 0, hist
    z = vcycle(levels, r, lam, degree, alpha)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = K @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            break
        z = vcycle(levels, r, lam, degree, alpha)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist
