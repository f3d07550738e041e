"""SIMP compliance minimisation pieces (oracle, float64, CPU).

Paper: Sec. "Three-Dimensional SIMP Topology Optimization": problem Eq. (tomin)
(minimise f^T u subject to K u = f and a volume fraction), the SIMP interpolation
Eq. (simp), a cone density filter of radius rmin, analytic sensitivities and the
optimality-criteria (OC) update with bisection on the volume multiplier.

Readings where the paper is silent (all textbook density-filter SIMP):
  * the density entering K is the filtered field xphys = H x / Hs (no projection);
  * cone weights H_ej = max(0, rmin - |c_e - c_j|) over element centroids, the
    neighbourhood truncated at the domain boundary, Hs_e = sum_j H_ej;
  * sensitivities are chained through the filter: dc <- H (dc / Hs), dv <- H (1 / Hs);
  * OC: lambda bracketed in [0, 1e9], bisection until (l2 - l1) / (l1 + l2) <= 1e-3,
    x_new = clip(x * sqrt(-dc / (dv * lambda)), max(0, x - m), min(1, x + m)), and the
    volume test filters x_new and compares its sum with volfrac * n_elem
    ("greater" moves the lower bracket up);
  * initial design x = volfrac everywhere, initial displacement 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem, solvers


# ------------------------------------------------------------------------ filter
def filter_matrix(nx: int, ny: int, nz: int, rmin: float):
    """Explicit sparse H (n_elem x n_elem) and Hs = H 1 from centroid distances."""
    R = int(np.ceil(rmin)) - 1
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    rows, cols, vals = [], [], []
    for dk in range(-R, R + 1):
        for dj in range(-R, R + 1):
            for di in range(-R, R + 1):
                w = rmin - np.sqrt(di * di + dj * dj + dk * dk)
                if w <= 0.0:
                    continue
                jx, jy, jz = ex + di, ey + dj, ez + dk
                ok = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny) & (jz >= 0) & (jz < nz)
                rows.append((ex + nx * (ey + ny * ez))[ok])
                cols.append((jx + nx * (jy + ny * jz))[ok])
                vals.append(np.full(ok.sum(), w))
    n = nx * ny * nz
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    Hs = np.asarray(H.sum(axis=1)).ravel()
    return H, Hs


def filter_forward(H, Hs, x):
    """xphys = H x / Hs."""
    return (H @ x) / Hs


def filter_adjoint(H, Hs, g):
    """Chain rule through the density filter: H^T (g / Hs) (H is symmetric)."""
    return H.T @ (g / Hs)


# ------------------------------------------------------------------- projection
def heaviside_project(xbar, beta, eta=0.5):
    """Smoothed Heaviside projection of the filtered density (Sec. "Three-Dimensional
    SIMP Topology Optimization", the projection equation of the three-field scheme):
    (tanh(beta eta) + tanh(beta (xbar - eta))) / (tanh(beta eta) + tanh(beta (1 - eta)))."""
    xbar = np.asarray(xbar, dtype=np.float64)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (np.tanh(beta * eta) + np.tanh(beta * (xbar - eta))) / den


def heaviside_derivative(xbar, beta, eta=0.5):
    """d(projection)/d(xbar) of heaviside_project: beta (1 - tanh^2(beta (xbar - eta)))
    over the same denominator (the chain-rule factor of the sensitivities)."""
    xbar = np.asarray(xbar, dtype=np.float64)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    t = np.tanh(beta * (xbar - eta))
    return beta * (1.0 - t * t) / den


# ------------------------------------------------------------ compliance, sensitivity
def compliance(f, u):
    """c = f^T u (Eq. tomin objective)."""
    return float(f @ u)


def element_energy(nx, ny, nz, u, KE):
    """ce_e = u_e^T K_E u_e for every element."""
    ue = u[fem.edof_table(nx, ny, nz)]
    return np.einsum("ei,ij,ej->e", ue, KE, ue)


def sensitivity(nx, ny, nz, xphys, u, KE, E0, Emin, penal):
    """dc_e = d(f^T u)/d xphys_e = -p xphys_e^(p-1) (E0 - Emin) ce_e  (adjoint-free)."""
    ce = element_energy(nx, ny, nz, u, KE)
    return -penal * np.power(xphys, penal - 1.0) * (E0 - Emin) * ce


# ---------------------------------------------------------------------------- OC
def oc_update(x, dc, dv, H, Hs, volfrac, move=0.2, l1=0.0, l2=1e9, rel_tol=1e-3,
              max_steps=256):
    """Optimality-criteria update with bisection on the volume multiplier.

    Returns (x_new, xphys_new, change, number_of_bisection_steps).  Raises if the
    bracket has not closed after max_steps (e.g. all sensitivities zero)."""
    n = x.size
    target = volfrac * n
    steps = 0
    while (l2 - l1) / (l1 + l2) > rel_tol:
        if steps >= max_steps:
            raise RuntimeError("OC bisection did not terminate")
        lmid = 0.5 * (l2 + l1)
        xnew = np.sqrt(-dc / (dv * lmid)) * x
        xnew = np.minimum(np.minimum(xnew, x + move), 1.0)
        xnew = np.maximum(np.maximum(xnew, x - move), 0.0)
        xphys = filter_forward(H, Hs, xnew)
        if xphys.sum() > target:
            l1 = lmid
        else:
            l2 = lmid
        steps += 1
    change = float(np.max(np.abs(xnew - x)))
    return xnew, xphys, change, steps


# --------------------------------------------------------------------------- SIMP
class Problem:
    """Everything the oracle needs for one mesh: K_E, edof, filter, BCs, loads."""

    def __init__(self, nx, ny, nz, fixed_dofs, f, E0=1.0, Emin=1e-9, nu=0.3, penal=3.0,
                 rmin=1.5, volfrac=0.3, **_):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.E0, self.Emin, self.nu, self.penal, self.rmin = E0, Emin, nu, penal, rmin
        self.volfrac = volfrac
        self.n_elem = nx * ny * nz
        self.n_dof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
        self.KE = fem.element_stiffness(nu)
        self.fixed = fem.fixed_mask(self.n_dof, fixed_dofs)
        self.f = np.asarray(f, dtype=np.float64).copy()
        self.H, self.Hs = filter_matrix(nx, ny, nz, rmin)
        self.dv = filter_adjoint(self.H, self.Hs, np.ones(self.n_elem))

    def modulus(self, xphys):
        return fem.simp_modulus(xphys, self.E0, self.Emin, self.penal)

    def stiffness(self, xphys):
        K = fem.assemble_K(self.nx, self.ny, self.nz, self.modulus(xphys), self.KE)
        return fem.constrain(K, self.fixed)

    def diag(self, xphys):
        return fem.diag_K(self.nx, self.ny, self.nz, self.modulus(xphys), self.KE,
                          self.fixed)

    def solve(self, xphys, u0=None, tol=1e-8, maxit=20000, direct=False):
        Kc = self.stiffness(xphys)
        if direct:
            return solvers.solve_direct(Kc, self.f), 0
        u, it, _ = solvers.pcg_jacobi(lambda v: Kc @ v, self.diag(xphys), self.f, u0,
                                      tol, maxit)
        return u, it

    def sensitivity(self, xphys, u):
        return sensitivity(self.nx, self.ny, self.nz, xphys, u, self.KE, self.E0,
                           self.Emin, self.penal)


def three_field_sensitivity(prob: Problem, x, u, beta, eta=0.5):
    """Three-field chain (Sec. "Three-Dimensional SIMP Topology Optimization": raw x,
    filtered xbar = H x / Hs, projected xphys = heaviside_project(xbar)): returns xphys
    and dc/dx = H^T ((dc/dxphys * d xphys / d xbar) / Hs) for the displacement u of
    K(xphys) u = f."""
    xbar = filter_forward(prob.H, prob.Hs, x)
    xphys = heaviside_project(xbar, beta, eta)
    dc_phys = prob.sensitivity(xphys, u)
    return xphys, filter_adjoint(prob.H, prob.Hs, dc_phys * heaviside_derivative(xbar, beta, eta))


def simp_run(prob: Problem, iters: int, tol=1e-8, move=0.2, direct=False, maxit=20000):
    """Plain SIMP loop: x = volfrac; each iteration solves K(xphys) u = f (warm start),
    takes c and dc, filters dc, runs OC and refilters.  Returns per-iteration history
    and the final (x, xphys, u)."""
    x = np.full(prob.n_elem, prob.volfrac)
    xphys = filter_forward(prob.H, prob.Hs, x)
    u = np.zeros(prob.n_dof)
    hist = []
    for _ in range(iters):
        u, its = prob.solve(xphys, u, tol=tol, maxit=maxit, direct=direct)
        c = compliance(prob.f, u)
        dc = prob.sensitivity(xphys, u)
        dc_f = filter_adjoint(prob.H, prob.Hs, dc)
        xnew, xphys_new, change, steps = oc_update(x, dc_f, prob.dv, prob.H, prob.Hs,
                                                   prob.volfrac, move)
        hist.append(dict(c=c, cg_iters=its, change=change, bisect=steps,
                         vol=float(xphys_new.mean())))
        x, xphys = xnew, xphys_new
    return hist, x, xphys, u


# ----------------------------------------------------------- three-field SIMP protocol
def grayness(rho):
    """g = 4/n sum_e rho_e (1 - rho_e) (Sec. "Experimental Setup"): 0 for a 0/1 design,
    1 for a uniform 0.5 field."""
    rho = np.asarray(rho, dtype=np.float64)
    return float(4.0 * np.sum(rho * (1.0 - rho)) / rho.size)


def projected_volume_gradient(H, Hs, xbar, beta, eta=0.5):
    """d/dx of sum_e project(filter(x))_e: H^T (project'(xbar) / Hs)."""
    return filter_adjoint(H, Hs, heaviside_derivative(xbar, beta, eta))


def oc_update_projected(x, dc, dv, H, Hs, beta, eta, volfrac, move=0.2, l1=0.0, l2=1e9,
                        rel_tol=1e-3, max_steps=256):
    """OC update of the three-field scheme: the same bisection and update rule as
    oc_update, with the volume of the projected density, sum(project(filter(x_new))),
    tested against volfrac * n (dc and dv are derivatives with respect to x).  Returns
    (x_new, xphys_new (projected), change, steps)."""
    n = x.size
    target = volfrac * n
    steps = 0
    while (l2 - l1) / (l1 + l2) > rel_tol:
        if steps >= max_steps:
            raise RuntimeError("OC bisection did not terminate")
        lmid = 0.5 * (l2 + l1)
        xnew = np.sqrt(-dc / (dv * lmid)) * x
        xnew = np.minimum(np.minimum(xnew, x + move), 1.0)
        xnew = np.maximum(np.maximum(xnew, x - move), 0.0)
        xphys = heaviside_project(filter_forward(H, Hs, xnew), beta, eta)
        if xphys.sum() > target:
            l1 = lmid
        else:
            l2 = lmid
        steps += 1
    change = float(np.max(np.abs(xnew - x)))
    return xnew, xphys, change, steps


# The four-phase continuation of the SIMP-120 protocol (Sec. "Experimental Setup"):
# (last iteration of the phase, penalty p, projection sharpness beta, OC move limit,
#  filter radius reached at the end of the phase; None = unchanged).
CONTINUATION = ((15, 1.5, 1.0, 0.20, None),
                (40, 3.5, 4.0, 0.15, 1.35),
                (65, 4.5, 16.0, 0.08, 1.25),
                (120, 4.5, 32.0, 0.05, 1.20))


def continuation(it, rmin0=1.5, phases=CONTINUATION):
    """(p, beta, move, rmin) of 1-based iteration `it`.  Within a phase with a radius
    target, rmin moves linearly from the previous phase's final value to the target,
    reaching it on the phase's last iteration; iterations past the last phase keep the
    last phase's values."""
    start, r_prev = 1, rmin0
    for last, p, beta, move, r_end in phases:
        if r_end is None:
            r_end_v = r_prev
        else:
            r_end_v = r_end
        if it <= last:
            frac = (it - start + 1) / (last - start + 1)
            return p, beta, move, r_prev + (r_end_v - r_prev) * frac
        start, r_prev = last + 1, r_end_v
    last, p, beta, move, r_end = phases[-1]
    return p, beta, move, r_prev


def simp_protocol(prob: Problem, iters=120, eta=0.5, tol=1e-8, maxit=20000, direct=False,
                  restart_factor=1.12, eligible_penal=3.0, eligible_gray=0.25,
                  phases=CONTINUATION):
    """Three-field SIMP with the continuation schedule, the restart rule and the
    selected iterate (Sec. "Experimental Setup").  Iteration it = 1..iters:
      (p, beta, m, rmin) = continuation(it); xbar = filter_rmin(x); xphys = project(xbar);
      solve K_p(xphys) u = f (warm start); c = f^T u; g = grayness(xphys);
      restart: if a selected iterate exists and c > restart_factor * c_selected, the next
        design is the selected design field (no update this iteration);
      otherwise the iterate is eligible when p >= eligible_penal and g < eligible_gray, and
        becomes the selected one when its c is the lowest eligible so far; then the OC
        update with the projected volume gives the next design.
    The problem's own rmin is the initial filter radius.  Returns (history, selected, x, u)
    with selected = dict(it, c, g, x, xphys) or None; x is the design after the last
    iteration and u the last displacement."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    x = np.full(prob.n_elem, prob.volfrac)
    u = np.zeros(prob.n_dof)
    hist, sel = [], None
    for it in range(1, iters + 1):
        p, beta, move, rmin = continuation(it, prob.rmin, phases)
        H, Hs = filter_matrix(nx, ny, nz, rmin)
        xbar = filter_forward(H, Hs, x)
        xphys = heaviside_project(xbar, beta, eta)
        E = fem.simp_modulus(xphys, prob.E0, prob.Emin, p)
        Kc = fem.constrain(fem.assemble_K(nx, ny, nz, E, prob.KE), prob.fixed)
        if direct:
            u, its = solvers.solve_direct(Kc, prob.f), 0
        else:
            d = fem.diag_K(nx, ny, nz, E, prob.KE, prob.fixed)
            u, its, _ = solvers.pcg_jacobi(lambda v: Kc @ v, d, prob.f, u, tol, maxit)
        c = compliance(prob.f, u)
        g = grayness(xphys)
        rec = dict(it=it, penal=p, beta=beta, move=move, rmin=rmin, c=c, gray=g,
                   cg_iters=its, restart=False, eligible=False)
        if sel is not None and c > restart_factor * sel["c"]:
            rec["restart"] = True
            hist.append(rec)
            x = sel["x"].copy()
            continue
        if p >= eligible_penal and g < eligible_gray:
            rec["eligible"] = True
            if sel is None or c < sel["c"]:
                sel = dict(it=it, c=c, g=g, x=x.copy(), xphys=xphys.copy())
        dc_phys = sensitivity(nx, ny, nz, xphys, u, prob.KE, prob.E0, prob.Emin, p)
        dc = filter_adjoint(H, Hs, dc_phys * heaviside_derivative(xbar, beta, eta))
        dv = projected_volume_gradient(H, Hs, xbar, beta, eta)
        x, _, change, steps = oc_update_projected(x, dc, dv, H, Hs, beta, eta, prob.volfrac,
                                                  move)
        rec.update(change=change, bisect=steps)
        hist.append(rec)
    return hist, sel, x, u
