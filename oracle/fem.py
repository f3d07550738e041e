"""Finite-element definitions of the operator K(rho) (oracle, float64, CPU).

Paper: Sec. "Three-Dimensional SIMP Topology Optimization", Eq. (simp): the global
stiffness is the sum over elements of B_e^T E_e K_E B_e with B_e the Boolean gather of
the element's 24 DOFs, E_e = Emin + rho_e^p (E0 - Emin), and K_E the 24x24 stiffness of
a unit-modulus isotropic trilinear hexahedron.  Eq. (matfree) applies the same sum to a
vector without forming K.

Readings where the paper is silent: Poisson ratio 0.3; unit-cube elements; local node
a = ax + 2*ay + 4*az at offset (ax, ay, az); local DOF 3*a + c; Dirichlet rows handled
as K_c = P K P + (I - P) with P the free-DOF mask.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------- geometry
def element_node_ids(nx: int, ny: int, nz: int) -> np.ndarray:
    """(n_elem, 8) global node ids of each element, local node a = ax + 2ay + 4az."""
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    out = np.empty((ex.size, 8), dtype=np.int64)
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        out[:, a] = (ex + ax) + (nx + 1) * ((ey + ay) + (ny + 1) * (ez + az))
    return out


def edof_table(nx: int, ny: int, nz: int) -> np.ndarray:
    """(n_elem, 24) element-to-DOF table (the paper's `edof`), local DOF 3a + c."""
    nodes = element_node_ids(nx, ny, nz)
    return (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 24)


# ------------------------------------------------------------------ element stiffness
def isotropic_D(E: float, nu: float) -> np.ndarray:
    """6x6 isotropic elasticity matrix, Voigt order (xx, yy, zz, xy, yz, zx),
    engineering shear strains."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def shape_gradients(xi: np.ndarray) -> np.ndarray:
    """(8, 3) gradients of the trilinear shape functions on the unit cube at point xi.

    N_a(x) = prod_d (x_d if bit_d(a) else 1 - x_d)."""
    g = np.zeros((8, 3))
    for a in range(8):
        bits = [(a >> d) & 1 for d in range(3)]
        f = [xi[d] if bits[d] else 1.0 - xi[d] for d in range(3)]
        df = [1.0 if bits[d] else -1.0 for d in range(3)]
        g[a, 0] = df[0] * f[1] * f[2]
        g[a, 1] = f[0] * df[1] * f[2]
        g[a, 2] = f[0] * f[1] * df[2]
    return g


def strain_displacement(xi: np.ndarray) -> np.ndarray:
    """6x24 strain-displacement matrix B at xi (unit cube, Jacobian = identity)."""
    g = shape_gradients(xi)
    B = np.zeros((6, 24))
    for a in range(8):
        cx, cy, cz = 3 * a, 3 * a + 1, 3 * a + 2
        B[0, cx] = g[a, 0]
        B[1, cy] = g[a, 1]
        B[2, cz] = g[a, 2]
        B[3, cx], B[3, cy] = g[a, 1], g[a, 0]
        B[4, cy], B[4, cz] = g[a, 2], g[a, 1]
        B[5, cx], B[5, cz] = g[a, 2], g[a, 0]
    return B


def element_stiffness(nu: float = 0.3, E: float = 1.0) -> np.ndarray:
    """K_E = sum over the 2x2x2 Gauss points of B^T D B w (exact for Q1 on a cube).

    Points (1 +- 1/sqrt(3))/2 per axis in [0,1]^3, weight 1/8 each."""
    D = isotropic_D(E, nu)
    gp = [(1.0 - 1.0 / np.sqrt(3.0)) / 2.0, (1.0 + 1.0 / np.sqrt(3.0)) / 2.0]
    KE = np.zeros((24, 24))
    for z in gp:
        for y in gp:
            for x in gp:
                B = strain_displacement(np.array([x, y, z]))
                KE += B.T @ D @ B * 0.125
    return KE


# -------------------------------------------------------------------------- material
def simp_modulus(xphys: np.ndarray, E0: float, Emin: float, penal: float) -> np.ndarray:
    """E_e = Emin + xphys_e^p (E0 - Emin)   (Eq. simp with rho_min = Emin, E0 = 1)."""
    return Emin + np.power(xphys, penal) * (E0 - Emin)


# -------------------------------------------------------------------------- assembly
def assemble_K(nx: int, ny: int, nz: int, E: np.ndarray, KE: np.ndarray) -> sp.csr_matrix:
    """Global K = sum_e B_e^T E_e K_E B_e as CSR (COO triplets, duplicates summed)."""
    edof = edof_table(nx, ny, nz)
    n_dof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    rows = np.repeat(edof, 24, axis=1).ravel()
    cols = np.tile(edof, (1, 24)).ravel()
    vals = (E[:, None] * KE.ravel()[None, :]).ravel()
    return sp.coo_matrix((vals, (rows, cols)), shape=(n_dof, n_dof)).tocsr()


def fixed_mask(n_dof: int, fixed_dofs: np.ndarray) -> np.ndarray:
    m = np.zeros(n_dof, dtype=bool)
    m[np.asarray(fixed_dofs, dtype=np.int64)] = True
    return m


def constrain(K: sp.spmatrix, fixed: np.ndarray) -> sp.csr_matrix:
    """K_c = P K P + (I - P): free block kept, fixed rows/columns replaced by identity."""
    p = (~fixed).astype(np.float64)
    P = sp.diags(p)
    return (P @ K @ P + sp.diags(1.0 - p)).tocsr()


def apply_K_elementwise(nx, ny, nz, E, KE, v, fixed=None, chunk=65536):
    """y = K_c v element by element (Eq. matfree): gather 24 values, multiply by
    E_e K_E, scatter-add; a second route independent of the CSR assembly."""
    edof = edof_table(nx, ny, nz)
    vin = v.copy()
    if fixed is not None:
        vin[fixed] = 0.0
    y = np.zeros_like(v)
    for s in range(0, edof.shape[0], chunk):
        ed = edof[s:s + chunk]
        fe = (vin[ed] @ KE.T) * E[s:s + chunk, None]
        np.add.at(y, ed.ravel(), fe.ravel())
    if fixed is not None:
        y[fixed] = v[fixed]
    return y


def apply_K_grid(nx, ny, nz, E, KE, v, fixed=None):
    """y = K_c v on the structured grid (Eq. matfree), a third route for full-size
    checks: the 24 element DOFs of every element are gathered at once as shifted
    node-grid slices (local node a at offset (ax, ay, az), one slice per component),
    multiplied by E_e K_E in one matrix product, and each local DOF's results are added
    back into the slice it came from (within one local node, elements map to distinct
    nodes).  Components are held as separate grids so that every slice is row-contiguous."""
    vin = np.array(v, dtype=np.float64, copy=True)
    if fixed is not None:
        vin[fixed] = 0.0
    g = np.ascontiguousarray(vin.reshape(nz + 1, ny + 1, nx + 1, 3).transpose(3, 0, 1, 2))
    offs = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]
    ve = np.empty((24, nz, ny, nx))
    for a, (ax, ay, az) in enumerate(offs):
        for c in range(3):
            ve[3 * a + c] = g[c, az:az + nz, ay:ay + ny, ax:ax + nx]
    fe = KE @ ve.reshape(24, -1)
    fe *= np.asarray(E, dtype=np.float64)[None, :]
    fe = fe.reshape(24, nz, ny, nx)
    y = np.zeros((3, nz + 1, ny + 1, nx + 1))
    for a, (ax, ay, az) in enumerate(offs):
        for c in range(3):
            y[c, az:az + nz, ay:ay + ny, ax:ax + nx] += fe[3 * a + c]
    y = np.ascontiguousarray(y.transpose(1, 2, 3, 0)).reshape(-1)
    if fixed is not None:
        y[fixed] = np.asarray(v, dtype=np.float64)[fixed]
    return y


def diag_K(nx, ny, nz, E, KE, fixed=None) -> np.ndarray:
    """Jacobi diagonal of K_c, accumulated element by element (1 on fixed DOFs)."""
    edof = edof_table(nx, ny, nz)
    d = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    np.add.at(d, edof.ravel(), (E[:, None] * np.diag(KE)[None, :]).ravel())
    if fixed is not None:
        d[fixed] = 1.0
    return d


def diag_K_grid(nx, ny, nz, E, KE, fixed=None) -> np.ndarray:
    """diag_K on the structured grid: each local node a adds E_e diag(K_E)[3a:3a+3] to
    the node-grid slice it occupies (the full-size companion of apply_K_grid)."""
    Eg = np.asarray(E, dtype=np.float64).reshape(nz, ny, nx)
    dk = np.diag(KE)
    d = np.zeros((nz + 1, ny + 1, nx + 1, 3))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        d[az:az + nz, ay:ay + ny, ax:ax + nx, :] += Eg[..., None] * dk[3 * a:3 * a + 3]
    d = d.reshape(-1)
    if fixed is not None:
        d[fixed] = 1.0
    return d


def rigid_body_modes(nx: int, ny: int, nz: int) -> np.ndarray:
    """(n_dof, 6): three translations and three infinitesimal rotations w x X."""
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    n = X.shape[0]
    R = np.zeros((3 * n, 6))
    for c in range(3):
        R[c::3, c] = 1.0
    for w in range(3):
        omega = np.zeros(3)
        omega[w] = 1.0
        R[:, 3 + w] = np.cross(omega[None, :], X).ravel()
    return R


def apply_K_rows(nx, ny, nz, xphys, v, fixed_dofs, dofs, KE, E0=1.0, Emin=1e-9, penal=3.0):
    """(K_c v)[d] for selected DOFs only, summing the contributions of the (at most
    eight) elements around each DOF's node; for checking full-size runs one row at a
    time.  xphys, v may be huge arrays: only the touched entries are read."""
    fixed = np.zeros(0, dtype=np.int64) if fixed_dofs is None else np.asarray(fixed_dofs)
    fixed_set = set(int(x) for x in fixed)
    out = np.zeros(len(dofs))
    for t, d in enumerate(dofs):
        d = int(d)
        if d in fixed_set:
            out[t] = v[d]
            continue
        n, c = divmod(d, 3)
        i = n % (nx + 1)
        j = (n // (nx + 1)) % (ny + 1)
        k = n // ((nx + 1) * (ny + 1))
        s = 0.0
        for ez in (k - 1, k):
            for ey in (j - 1, j):
                for ex in (i - 1, i):
                    if not (0 <= ex < nx and 0 <= ey < ny and 0 <= ez < nz):
                        continue
                    e = ex + nx * (ey + ny * ez)
                    a = (i - ex) + 2 * (j - ey) + 4 * (k - ez)
                    Ee = Emin + xphys[e] ** penal * (E0 - Emin)
                    ed = np.empty(24, dtype=np.int64)
                    for b in range(8):
                        nb = (ex + (b & 1)) + (nx + 1) * ((ey + ((b >> 1) & 1))
                                                          + (ny + 1) * (ez + ((b >> 2) & 1)))
                        ed[3 * b:3 * b + 3] = 3 * nb + np.arange(3)
                    ve = v[ed].astype(np.float64)
                    for q in range(24):
                        if int(ed[q]) in fixed_set:
                            ve[q] = 0.0
                    s += Ee * (KE[3 * a + c] @ ve)
        out[t] = s
    return out
