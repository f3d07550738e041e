"""Linear solvers and spectral estimates (oracle, float64, CPU).

Paper: Sec. "Preconditioned Conjugate Gradient and Warm-Start Strategy" (Jacobi-PCG
with the exact diagonal, warm start, stop on the unpreconditioned relative residual
||r_k|| / ||f|| <= tol or an iteration cap) and Sec. "BF16 Arithmetic in the Conjugate
Gradient Solver" (residual-correction refinement r = f - K u, e ~ K^{-1} r, u += e; the
unit-roundoff rule u_l * kappa(K) < 1, Eq. bf16barrier).  The paper estimates kappa by
power and inverse iteration; here the extremes come from Lanczos and, on small meshes,
from a dense symmetric eigensolver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Unit roundoffs (Carson-Higham convention: 2^-t with t the stored significand bits).
UNIT_ROUNDOFF = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp32": 2.0 ** -24, "fp64": 2.0 ** -53}


def solve_direct(Kc: sp.spmatrix, b: np.ndarray, dense_limit: int = 20000) -> np.ndarray:
    """Exact solve of K_c u = b: dense Cholesky when small, sparse LU otherwise."""
    n = Kc.shape[0]
    if n <= dense_limit:
        c = sla.cho_factor(Kc.toarray(), lower=True)
        return sla.cho_solve(c, b)
    return spla.spsolve(Kc.tocsc(), b)


def pcg_jacobi(apply_K, diag: np.ndarray, b: np.ndarray, x0: np.ndarray | None = None,
               tol: float = 1e-8, maxit: int = 20000):
    """Jacobi-preconditioned CG with the paper's stopping rule.

    Stops when the recursively updated residual satisfies ||r|| <= tol * ||b|| (checked
    before the first iteration and after every update) or after `maxit` iterations.
    Returns (x, iterations, residual history ||r_k|| / ||b||)."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0]
    r = b - apply_K(x)
    hist = [np.linalg.norm(r) / bnorm]
    if hist[-1] <= tol:
        return x, 0, hist
    z = r / diag
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = apply_K(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            break
        z = r / diag
        rz_new = r @ z
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    return x, it, hist


def lanczos_tridiagonal(apply_A, v0: np.ndarray, k: int, reorthogonalize: bool = False):
    """k steps of symmetric Lanczos from v0.  Returns (alpha[k'], beta[k'-1]) with
    k' <= k (early stop on an invariant subspace)."""
    n = v0.size
    q = v0 / np.linalg.norm(v0)
    q_prev = np.zeros(n)
    beta_prev = 0.0
    alphas, betas = [], []
    Q = [q] if reorthogonalize else None
    for j in range(k):
        w = apply_A(q) - beta_prev * q_prev
        a = q @ w
        w -= a * q
        if reorthogonalize:
            for qq in Q:
                w -= (qq @ w) * qq
        alphas.append(a)
        b = np.linalg.norm(w)
        if j == k - 1 or b == 0.0:
            break
        betas.append(b)
        q_prev, q = q, w / b
        beta_prev = b
        if reorthogonalize:
            Q.append(q)
    return np.array(alphas), np.array(betas)


def lanczos_extremes(apply_A, v0: np.ndarray, kmax: int, rtol: float = 1e-3, window: int = 50):
    """Lanczos with the precision study's stopping rule: after every `window` steps the
    smallest Ritz value (smallest eigenvalue of the tridiagonal T_j of the steps so far)
    is compared with its value `window` steps earlier; the run stops at the first j with
    |theta_j - theta_{j - window}| <= rtol * theta_j, or after kmax steps.  The
    coefficients of the first j steps do not depend on later ones, so this is evaluated
    on prefixes of one kmax-step run.  Returns (lmin, lmax, steps, converged): lmin is an
    upper bound of the smallest eigenvalue, lmax a lower bound of the largest."""
    a, b = lanczos_tridiagonal(apply_A, v0, kmax)
    m = a.size
    prev = None
    for j in range(window, m + 1, window):
        lo, hi = tridiagonal_extremes(a[:j], b[:j - 1])
        if prev is not None and abs(lo - prev) <= rtol * abs(lo):
            return lo, hi, j, True
        prev = lo
    lo, hi = tridiagonal_extremes(a, b[:m - 1])
    return lo, hi, m, m < kmax


def tridiagonal_extremes(alpha: np.ndarray, beta: np.ndarray):
    """Smallest and largest eigenvalue of the symmetric tridiagonal (alpha, beta)."""
    ev = sla.eigh_tridiagonal(alpha, beta, eigvals_only=True)
    return float(ev[0]), float(ev[-1])


def free_block(Kc: sp.spmatrix, fixed: np.ndarray) -> sp.csr_matrix:
    free = np.flatnonzero(~fixed)
    return Kc.tocsr()[free][:, free]


def kappa_dense(Kff: sp.spmatrix, jacobi_scaled: bool = False):
    """(lambda_min, lambda_max) of K_ff (or D^-1/2 K_ff D^-1/2) by a dense eigensolver."""
    A = Kff.toarray()
    if jacobi_scaled:
        s = 1.0 / np.sqrt(np.diag(A))
        A = A * s[:, None] * s[None, :]
    ev = np.linalg.eigvalsh(A)
    return float(ev[0]), float(ev[-1])


def precision_allowed(kappa: float, precision: str) -> bool:
    """Admissibility rule u_l * kappa < 1 (Eq. bf16barrier, extended to fp16/fp32)."""
    return UNIT_ROUNDOFF[precision] * kappa < 1.0
