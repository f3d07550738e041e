"""GPU parity of the three-field SIMP scheme and the SIMP-120 protocol machinery (Sec.
"Experimental Setup"; projection equation of Sec. "Three-Dimensional SIMP Topology
Optimization"): the three-field step (stiffness and OC volume on the projected
density) and a 20-iteration continuation run with restarts and selection, against the
oracle."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import fem, solvers, topopt
from tests.helpers import dev, gpu_problem

pytestmark = pytest.mark.gpu


def _prob(nx, ny, nz, rmin=1.5):
    return topopt.Problem(nx, ny, nz, si.cantilever_fixed_dofs(nx, ny, nz),
                          si.cantilever_load(nx, ny, nz), volfrac=0.3, rmin=rmin)


@pytest.mark.parametrize("beta", [2.0, 8.0])
def test_three_field_steps_match_oracle(beta):
    """Three steps of the three-field scheme: K and the OC volume on the projected
    density.  Solves to 1e-10 on both sides (direct in the oracle), so each step's
    compliance agrees to ~1e-9 and the designs to the bisection's rounding."""
    nx, ny, nz = 16, 8, 8
    prob = _prob(nx, ny, nz)
    eta = 0.5
    x = np.full(prob.n_elem, 0.3)
    xo = x.copy()
    t, _, f = gpu_problem(nx, ny, nz)
    xd = dev(x)
    xp = t.project(t.filter(xd), beta, eta)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    for k in range(3):
        xp_in = xp.cpu().numpy()
        st = t.simp_step(xd, xp, u, volfrac=0.3, move=0.2, beta=beta, eta=eta, tol=1e-11)
        xbar = topopt.filter_forward(prob.H, prob.Hs, xo)
        xpo = topopt.heaviside_project(xbar, beta, eta)
        uo = solvers.solve_direct(prob.stiffness(xpo), prob.f)
        co = float(prob.f @ uo)
        assert abs(st["compliance"] - co) <= 1e-8 * co, k
        # grayness 4/n sum rho(1 - rho) has |d/drho| <= 4: after the first step the two
        # designs differ by the bisection's rounding, which bounds the grayness gap.
        gbound = 4.0 * np.max(np.abs(xp_in - xpo)) + 1e-13
        assert abs(st["grayness"] - topopt.grayness(xpo)) <= gbound, k
        dc_phys = prob.sensitivity(xpo, uo)
        dc = topopt.filter_adjoint(prob.H, prob.Hs, dc_phys * topopt.heaviside_derivative(xbar, beta, eta))
        dv = topopt.projected_volume_gradient(prob.H, prob.Hs, xbar, beta, eta)
        xo, xpo_new, ch, steps = topopt.oc_update_projected(xo, dc, dv, prob.H, prob.Hs, beta, eta,
                                                            0.3, 0.2)
        assert st["bisection_steps"] == steps
        assert np.max(np.abs(xd.cpu().numpy() - xo)) <= 1e-7, k
        assert np.max(np.abs(xp.cpu().numpy() - xpo_new)) <= 1e-6, k
        assert abs(st["volume"] - xpo_new.mean()) <= 1e-6
    t.close()


def test_protocol_twenty_iterations_match_oracle():
    """A 20-iteration continuation (penalty 1.5 -> 3 -> 3.5 -> 4, beta 1 -> 1 -> 4 -> 8,
    radius 1.5 -> 1.45 -> 1.4) with the restart and selection rules active: the jump of
    penalty and beta after iteration 10 raises the compliance above 1.001 x the selected
    one, so the rule restarts from the selected design (every later iteration, the
    parameters staying above those of the selection): iteration by iteration the
    compliance, grayness and the eligible / restart / selected decisions of the GPU run
    equal the oracle's."""
    nx, ny, nz = 16, 8, 8
    prob = _prob(nx, ny, nz)
    phases = ((3, 1.5, 1.0, 0.2, None), (10, 3.0, 1.0, 0.2, 1.45), (14, 3.5, 4.0, 0.15, 1.4),
              (20, 4.0, 8.0, 0.1, 1.4))
    kw = dict(restart_factor=1.001, eligible_gray=0.9)
    hist, sel, xo, _ = topopt.simp_protocol(prob, 20, direct=True, phases=phases, **kw)
    t, _, _ = gpu_problem(nx, ny, nz)
    x = torch.full((prob.n_elem,), 0.3, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    rec, it_sel, c_sel, x_sel, _ = t.simp_protocol(x, u, iters=20, phases=phases, tol=1e-11, **kw)
    t.close()
    for r, h in zip(rec, hist):
        assert r["it"] == h["it"]
        assert (r["penal"], r["beta"], r["move"]) == (h["penal"], h["beta"], h["move"])
        assert r["rmin"] == h["rmin"]
        assert abs(r["compliance"] - h["c"]) <= 1e-6 * h["c"], r["it"]
        assert abs(r["grayness"] - h["gray"]) <= 1e-7, r["it"]
        assert bool(r["restart"]) == h["restart"] and bool(r["eligible"]) == h["eligible"], r["it"]
    assert any(h["restart"] for h in hist) and sel is not None
    assert it_sel == sel["it"] and abs(c_sel - sel["c"]) <= 1e-6 * sel["c"]
    assert np.max(np.abs(x_sel.cpu().numpy() - sel["x"])) <= 1e-6
    assert np.max(np.abs(x.cpu().numpy() - xo)) <= 1e-6


def test_set_params_rebuilds_the_filter():
    """A new radius through tosimp_set_params filters exactly as a context created with
    that radius; the penalty enters the operator."""
    nx, ny, nz = 9, 5, 4
    rng = np.random.default_rng(2)
    x = rng.uniform(0.1, 1.0, nx * ny * nz)
    t, _, _ = gpu_problem(nx, ny, nz)
    t.set_params(4.0, 1.3)
    a = t.filter(dev(x)).cpu().numpy()
    H, Hs = topopt.filter_matrix(nx, ny, nz, 1.3)
    assert np.max(np.abs(a - topopt.filter_forward(H, Hs, x))) <= 1e-15
    v = rng.standard_normal(t.n_dof)
    y = t.apply_K(dev(x), dev(v)).cpu().numpy()
    E = fem.simp_modulus(x, 1.0, 1e-9, 4.0)
    fixed = fem.fixed_mask(t.n_dof, si.cantilever_fixed_dofs(nx, ny, nz))
    yo = fem.constrain(fem.assemble_K(nx, ny, nz, E, fem.element_stiffness(0.3)), fixed) @ v
    assert np.linalg.norm(y - yo) <= 1e-12 * np.linalg.norm(yo)
    t.close()
