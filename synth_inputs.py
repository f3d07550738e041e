"""Seeded synthetic workloads shared by the CPU oracle, the tests and the benchmark.

This module holds problem *inputs* only: mesh sizes and material constants of the
benchmark problems, the node/DOF numbering convention, the Dirichlet sets and load
vectors of the cantilever, torsion, MBB and bridge cases, and seeded random fields.  It holds none
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
    # hard-problem stress tests: 187,500 elements each (domain 3 x 1 x 0.5)
    "mbb_150x50x25": dict(kind="mbb", nx=150, ny=50, nz=25, volfrac=0.5, simp_iters=60,
                          pcg_tol=1e-6),
    "bridge_150x50x25": dict(kind="bridge", nx=150, ny=50, nz=25, volfrac=0.3, simp_iters=60,
                             pcg_tol=1e-6),
}

# Cold-start FEA scaling ladder (4:2:1 cantilevers, uniform density 0.5):
# 216 k, 512 k, 1 M, 2.0 M, 4.9 M and 8 M elements.
FEA_LADDER = [(120, 60, 30), (160, 80, 40), (200, 100, 50), (252, 126, 63), (340, 170, 85),
              (400, 200, 100)]


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


def _mid_nodes(n: int):
    """The node(s) at the middle of an axis of n elements: one for even n, the two
    nearest for odd n."""
    return [n // 2] if n % 2 == 0 else [n // 2, n // 2 + 1]


def mbb_fixed_dofs(nx: int, ny: int, nz: int) -> np.ndarray:
    """MBB stress test on the domain 3 x 1 x 0.5 (x, y, z; y up): u_x = 0 on every node of
    the x = 0 face (the symmetry plane of the half beam); u_y = 0 along the bottom edge of
    the far end, (x, y) = (nx, 0), over the whole depth (the support point, extended so
    that no rotation about the x axis survives); u_z = 0 at its mid-depth node(s) (the z
    translation)."""
    j, k = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    face = 3 * node_id(0, j.ravel(), k.ravel(), nx, ny)
    edge = node_id(nx, 0, np.arange(nz + 1), nx, ny)
    mid = node_id(nx, 0, np.array(_mid_nodes(nz)), nx, ny)
    ids = np.concatenate([face, 3 * edge + 1, 3 * mid + 2])
    return np.unique(ids).astype(np.int64)


def mbb_load(nx: int, ny: int, nz: int) -> np.ndarray:
    """Unit downward (-y) load at the top of the symmetry plane, (x, y) = (0, ny) at
    mid-depth, split evenly over the mid-depth node(s)."""
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    ks = _mid_nodes(nz)
    n = node_id(0, ny, np.array(ks), nx, ny)
    f[3 * n + 1] = -1.0 / len(ks)
    return f


def bridge_fixed_dofs(nx: int, ny: int, nz: int) -> np.ndarray:
    """Bridge stress test: the left lower edge (x = 0, y = 0, every z) fixed in all three
    components; the right lower edge (x = nx, y = 0) a roller in x (u_y = u_z = 0)."""
    k = np.arange(nz + 1)
    left = node_id(0, 0, k, nx, ny)
    right = node_id(nx, 0, k, nx, ny)
    ids = np.concatenate([3 * left, 3 * left + 1, 3 * left + 2, 3 * right + 1, 3 * right + 2])
    return np.unique(ids).astype(np.int64)


def bridge_load(nx: int, ny: int, nz: int) -> np.ndarray:
    """Distributed downward load on the top (y = ny face), total magnitude 1, equal on
    every node of the face."""
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    i, k = np.meshgrid(np.arange(nx + 1), np.arange(nz + 1), indexing="ij")
    n = node_id(i.ravel(), ny, k.ravel(), nx, ny)
    f[3 * n + 1] = -1.0 / n.size
    return f


def bcs_and_load(kind: str, nx: int, ny: int, nz: int):
    """(fixed DOF ids, load vector) of a problem kind on an nx x ny x nz mesh."""
    table = {"cantilever": (cantilever_fixed_dofs, cantilever_load),
             "torsion": (torsion_fixed_dofs, torsion_load),
             "mbb": (mbb_fixed_dofs, mbb_load),
             "bridge": (bridge_fixed_dofs, bridge_load)}
    fixed, load = table[kind]
    return fixed(nx, ny, nz), load(nx, ny, nz)


def problem(name: str):
    """(config dict, fixed DOF ids, load vector) of a named benchmark problem."""
    cfg = dict(CONFIGS[name])
    cfg.update(MATERIAL)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    return (cfg, *bcs_and_load(cfg["kind"], nx, ny, nz))


def random_density_and_vector(nx: int, ny: int, nz: int, seed: int = 42):
    """rho ~ U(0.01, 1) per element, then v ~ N(0, 1) per DOF, from one generator."""
    c = counts(nx, ny, nz)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.01, 1.0, c["n_elem"])
    v = rng.standard_normal(c["n_dof"])
    return rho, v


def random_field(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)
