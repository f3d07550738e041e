"""GPU parity on the code paths that full-size runs take.

The SIMP kernels (sensitivity, filter in both modes, OC with its bisection, projection)
use grid-stride loops over fixed grids: at 200x100x50 (1,000,000 elements) every loop
makes several passes, unlike the small parity meshes.  The solvers' reductions sum one
partial per operator tile or vector block: at 340x170x85 (4,913,000 elements) those are
thousands of partials, which takes the unrolled branch of the finalize kernel.  Each case
is compared with the oracle element by element (the oracle's grid-slice operator route
keeps the CPU side to seconds per product).
"""
import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import fem, topopt
from tests.helpers import dev

pytestmark = pytest.mark.gpu
KE = fem.element_stiffness(0.3)


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_simp_kernels_match_oracle_at_one_million_elements():
    from tests.helpers import gpu_problem
    nx, ny, nz = 200, 100, 50
    rng = np.random.default_rng(21)
    x = rng.uniform(0.05, 1.0, nx * ny * nz)
    u = rng.standard_normal(3 * (nx + 1) * (ny + 1) * (nz + 1))
    fixed = si.cantilever_fixed_dofs(nx, ny, nz)
    u[fixed] = 0.0
    t, _, _ = gpu_problem(nx, ny, nz)
    print(f"[fullsize] SIMP kernels at {nx}x{ny}x{nz}", flush=True)
    xd, ud = dev(x), dev(u)
    # sensitivity
    dc, _ = t.sensitivity(xd, ud)
    dc_o = topopt.sensitivity(nx, ny, nz, x, u, KE, 1.0, 1e-9, 3.0)
    assert _maxrel(dc.cpu().numpy(), dc_o) <= 1e-12
    # filter, both modes
    H, Hs = topopt.filter_matrix(nx, ny, nz, 1.5)
    xf = t.filter(xd, "forward").cpu().numpy()
    assert _maxrel(xf, topopt.filter_forward(H, Hs, x)) <= 1e-13
    dcf = t.filter(dc, "adjoint")
    dcf_o = topopt.filter_adjoint(H, Hs, dc_o)
    assert _maxrel(dcf.cpu().numpy(), dcf_o) <= 1e-12
    # OC on the filtered sensitivity: the same multiplier steps, design and filtered design
    dv_o = topopt.filter_adjoint(H, Hs, np.ones_like(x))
    dcf64 = dcf.cpu().numpy()
    xn, xpn, ch, steps = t.oc_update(xd, dcf, 0.3, 0.2)
    xn_o, xpn_o, ch_o, steps_o = topopt.oc_update(x, dcf64, dv_o, H, Hs, 0.3, 0.2)
    assert steps == steps_o
    assert np.max(np.abs(xn.cpu().numpy() - xn_o)) <= 1e-12
    assert np.max(np.abs(xpn.cpu().numpy() - xpn_o)) <= 1e-12
    assert abs(ch - ch_o) <= 1e-12
    # projection and its chain rule
    for beta in (1.0, 16.0):
        p = t.project(xd, beta, 0.5).cpu().numpy()
        assert np.max(np.abs(p - topopt.heaviside_project(x, beta, 0.5))) <= 2e-15
        g = t.project(xd, beta, 0.5, g=dc).cpu().numpy()
        go = dc_o * topopt.heaviside_derivative(x, beta, 0.5)
        assert _maxrel(g, go) <= 1e-12
    t.close()


def _c3_system():
    nx, ny, nz = 340, 170, 85
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=42)
    fixed = fem.fixed_mask(v.size, si.cantilever_fixed_dofs(nx, ny, nz))
    b = v.copy()
    b[fixed] = 0.0
    E = fem.simp_modulus(rho, 1.0, 1e-9, 3.0)
    return nx, ny, nz, rho, b, fixed, E


def test_pcg_iterates_match_oracle_at_340x170x85():
    """A fixed number of Jacobi-PCG iterations on the 15M-DOF system (random density and
    right-hand side, cantilever clamp), FP64 and, in one refinement step, FP32: the
    iterate after k iterations against the oracle's FP64 iterate.  FP64: both sides take
    the same steps and differ only in summation order (bound 1e-12).  FP32 inner solve:
    each iteration rounds its vectors and operator products to FP32 (u_32 = 6e-8), and k
    iterations of CG compound that to a few 1e-7 .. 1e-6 (bound 1e-5)."""
    from tests.helpers import gpu_problem
    k = 8
    nx, ny, nz, rho, b, fixed, E = _c3_system()
    print(f"[fullsize] PCG iterates at {nx}x{ny}x{nz}, {k} iterations", flush=True)
    t, _, _ = gpu_problem(nx, ny, nz)
    xd, bd = dev(rho), dev(b)
    u64 = torch.zeros(b.size, dtype=torch.float64, device="cuda:0")
    s64 = t.pcg_solve(xd, bd, u64, tol=1e-30, maxit=k, check_every=4)
    assert s64["rc"] == 1 and s64["iterations"] == k
    u32 = torch.zeros(b.size, dtype=torch.float64, device="cuda:0")
    s32 = t.pcg_solve(xd, bd, u32, tol=1e-30, maxit=k, mode="ir", inner_prec="fp32",
                      inner_tol=1e-12, max_outer=1, check_every=4)
    assert s32["iterations"] == k and s32["outer_iterations"] == 1
    g64, g32 = u64.cpu().numpy(), u32.cpu().numpy()
    t.close()
    A = lambda w: fem.apply_K_grid(nx, ny, nz, E, KE, w, fixed)
    d = fem.diag_K_grid(nx, ny, nz, E, KE, fixed)
    from oracle import solvers
    uo, ito, _ = solvers.pcg_jacobi(A, d, b, None, 1e-30, maxit=k)
    assert ito == k
    e64 = float(np.linalg.norm(g64 - uo) / np.linalg.norm(uo))
    print(f"[fullsize] FP64 iterate rel. difference {e64:.2e}", flush=True)
    assert e64 <= 1e-12
    bn = np.linalg.norm(b)
    bhat = (b * (1.0 / bn)).astype(np.float32).astype(np.float64)
    eo, _, _ = solvers.pcg_jacobi(A, d, bhat, None, 1e-30, maxit=k)
    e32 = float(np.linalg.norm(g32 - bn * eo) / np.linalg.norm(bn * eo))
    print(f"[fullsize] FP32 inner iterate rel. difference {e32:.2e}", flush=True)
    assert e32 <= 1e-5
    assert np.all(g64[fixed] == 0.0) and np.all(g32[fixed] == 0.0)
