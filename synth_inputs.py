"""Seeded synthetic workloads shared by the CPU oracle, the tests and the benchmark.

This module holds problem *inputs* only: mesh sizes and material constants of the
benchmark problems, the node/DOF numbering convention, the Dirichlet sets and load
vectors of the cantilever and torsion cases, and seeded random fields.  It holds none
of the method's arithmetic (no stiffness, no solver, no filter, no update rule), so the
oracle and the GPU library can both consume it without sharing any computation.

Numbering convention (structured grid of unit cubes):
  node (i, j, k), 0 <= i <= nx, 0 <= j <= ny, 0 <= k <= nz,
  node id n = i + (nx+1) * (j + (ny+1) * k),
  DOF id 3*n + c with c in {0: x, 1: y, 2: z} (interleaved),
  element (ex, ey, ez) has id ex + nx * (ey + ny * ez).
"""
from __future__ import annotations

import numpy as np

# Material and optimisation constants of the benchmark problems (unit-cube elements,
# E0 = 1, Emin = 1e-9, nu = 0.3, p = 3, rmin = 1.5, volume fraction 0.3).
MATERIAL = dict(E0=1.0, Emin=1e-9, nu=0.3, penal=3.0, rmin=1.5, h=1.0)

CONFIGS = {
    # small parity case: 1,024 elements, 1,377 nodes, 4,131 DOFs
    "cantilever_16x8x8": dict(kind="cantilever", nx=16, ny=8, nz=8, volfrac=0.3,
                              simp_iters=5, pcg_tol=1e-8),
    # 216,000 elements, 686,433 DOFs
    "cantilever_120x60x30": dict(kind="cantilever", nx=120, ny=60, nz=30, volfrac=0.3,
                                 simp_iters=20, pcg_tol=1e-6),
    # 4,913,000 elements, 15,044,238 DOFs
    "cantilever_340x170x85": dict(kind="cantilever", nx=340, ny=170, nz=85, volfrac=0.3,
                                  simp_iters=0, pcg_tol=1e-6),
    # 499,125 elements, 1,561,728 DOFs
    "torsion_55x55x165": dict(kind="torsion", nx=55, ny=55, nz=165, volfrac=0.3,
                              simp_iters=30, pcg_tol=1e-6),
    # 1,000,000 elements, 3,106,053 DOFs
    "cantilever_200x100x50": dict(kind="cantilever", nx=200, ny=100, nz=50, volfrac=0.3,
                                  simp_iters=20, pcg_tol=1e-6),
}


def counts(nx: int, ny: int, nz: int) -> dict:
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    return dict(n_elem=nx * ny * nz, n_node=nodes, n_dof=3 * nodes)


def node_id(i, j, k, nx: int, ny: int):
    return np.asarray(i) + (nx + 1) * (np.asarray(j) + (ny + 1) * np.asarray(k))


def node_coords(nx: int, ny: int, nz: int) -> np.ndarray:
    """(n_node, 3) integer coordinates (i, j, k) in node-id order."""
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def cantilever_fixed_dofs(nx: int, ny: int, nz: int) -> np.ndarray:
    """All three DOFs of every node on the x = 0 face are clamped."""
    j, k = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    n = node_id(0, j.ravel(), k.ravel(), nx, ny)
    return np.sort((3 * n[:, None] + np.arange(3)[None, :]).ravel()).astype(np.int64)


def cantilever_load(nx: int, ny: int, nz: int) -> np.ndarray:
    """Unit -y point load on every node of the free-end bottom edge (x = nx, y = 0)."""
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    n = node_id(nx, 0, np.arange(nz + 1), nx, ny)
    f[3 * n + 1] = -1.0
    return f


def cantilever_midpoint_load(nx: int, ny: int, nz: int) -> np.ndarray:
    """Unit -y point load at the centre node of the x = nx face (needs even ny, nz)."""
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    f[3 * int(node_id(nx, ny // 2, nz // 2, nx, ny)) + 1] = -1.0
    return f


def torsion_fixed_dofs(nx: int, ny: int, nz: int) -> np.ndarray:
    """All three DOFs of every node on the z = 0 face are clamped."""
    i, j = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    n = node_id(i.ravel(), j.ravel(), 0, nx, ny)
    return np.sort((3 * n[:, None] + np.arange(3)[None, :]).ravel()).astype(np.int64)


def torsion_load(nx: int, ny: int, nz: int) -> np.ndarray:
    """Unit tangential forces on the perimeter ring of the z = nz face.

    Each perimeter node p gets the unit vector z_hat x (p - c) / |p - c| with
    c = (nx/2, ny/2) the face centre, i.e. a pure torque about the z axis.
    """
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    i, j = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    i, j = i.ravel(), j.ravel()
    ring = (i == 0) | (i == nx) | (j == 0) | (j == ny)
    i, j = i[ring], j[ring]
    dx, dy = i - nx / 2.0, j - ny / 2.0
    r = np.hypot(dx, dy)
    n = node_id(i, j, nz, nx, ny)
    f[3 * n + 0] = -dy / r
    f[3 * n + 1] = dx / r
    return f


def problem(name: str):
    """(config dict, fixed DOF ids, load vector) of a named benchmark problem."""
    cfg = dict(CONFIGS[name])
    cfg.update(MATERIAL)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    if cfg["kind"] == "cantilever":
        return cfg, cantilever_fixed_dofs(nx, ny, nz), cantilever_load(nx, ny, nz)
    if cfg["kind"] == "torsion":
        return cfg, torsion_fixed_dofs(nx, ny, nz), torsion_load(nx, ny, nz)
    raise KeyError(name)


def random_density_and_vector(nx: int, ny: int, nz: int, seed: int = 42):
    """rho ~ U(0.01, 1) per element, then v ~ N(0, 1) per DOF, from one generator."""
    c = counts(nx, ny, nz)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.01, 1.0, c["n_elem"])
    v = rng.standard_normal(c["n_dof"])
    return rho, v


def random_field(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)
