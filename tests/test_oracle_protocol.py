"""Pins of the oracle's three-field SIMP protocol pieces (Sec. "Experimental Setup" and
the projection equation of Sec. "Three-Dimensional SIMP Topology Optimization"): the
continuation schedule against the values the paper prints, grayness closed forms, the
projected-volume gradient against finite differences, the projected-volume OC against an
independent root finder and, for a vanishing projection sharpness, against the
density-filter OC."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import synth_inputs as si
from oracle import topopt

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "continuation_schedule.json")))


def test_continuation_schedule_matches_the_paper():
    r_prev = GOLDEN["initial_rmin"]
    for ph in GOLDEN["phases"]:
        for it in range(ph["first"], ph["last"] + 1):
            p, beta, move, rmin = topopt.continuation(it, GOLDEN["initial_rmin"])
            assert (p, beta, move) == (ph["penal"], ph["beta"], ph["move"])
            target = r_prev if ph["rmin_end"] is None else ph["rmin_end"]
            lo, hi = min(r_prev, target), max(r_prev, target)
            assert lo - 1e-15 <= rmin <= hi + 1e-15
        # the radius reaches the phase's target on its last iteration
        assert abs(topopt.continuation(ph["last"], GOLDEN["initial_rmin"])[3] -
                   (r_prev if ph["rmin_end"] is None else ph["rmin_end"])) <= 1e-15
        if ph["rmin_end"] is not None:
            r_prev = ph["rmin_end"]
    radii = [topopt.continuation(it)[3] for it in range(1, 121)]
    assert all(b <= a for a, b in zip(radii, radii[1:]))  # never grows
    # linear within a phase: equal steps
    steps = np.diff(radii[15:40])
    assert np.ptp(steps) <= 1e-15


def test_grayness_closed_forms():
    assert topopt.grayness(np.array([0.0, 1.0, 1.0, 0.0])) == 0.0
    assert topopt.grayness(np.full(7, 0.5)) == 1.0
    assert abs(topopt.grayness(np.array([0.1, 0.9])) - 0.36) <= 1e-15


def _small(nx=8, ny=4, nz=4, rmin=1.5, seed=3):
    H, Hs = topopt.filter_matrix(nx, ny, nz, rmin)
    x = np.random.default_rng(seed).uniform(0.05, 0.95, nx * ny * nz)
    return H, Hs, x


@pytest.mark.parametrize("beta", [1.0, 8.0])
def test_projected_volume_gradient_finite_difference(beta):
    H, Hs, x = _small()
    vol = lambda z: topopt.heaviside_project(topopt.filter_forward(H, Hs, z), beta).sum()
    g = topopt.projected_volume_gradient(H, Hs, topopt.filter_forward(H, Hs, x), beta)
    h = 1e-6
    for e in (0, 17, 63, x.size - 1):
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        fd = (vol(xp) - vol(xm)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("beta", [2.0, 16.0])
def test_oc_projected_volume_against_root_finder(beta):
    H, Hs, x = _small(seed=5)
    rng = np.random.default_rng(6)
    dc = -rng.uniform(0.1, 2.0, x.size)
    xbar = topopt.filter_forward(H, Hs, x)
    dv = topopt.projected_volume_gradient(H, Hs, xbar, beta)
    vf, move = 0.4, 0.2
    xn, xp, change, steps = topopt.oc_update_projected(x, dc, dv, H, Hs, beta, 0.5, vf, move)

    def excess(lam):
        z = np.clip(np.sqrt(-dc / (dv * lam)) * x, np.maximum(x - move, 0), np.minimum(x + move, 1))
        return topopt.heaviside_project(topopt.filter_forward(H, Hs, z), beta).sum() - vf * x.size

    lam_star = brentq(excess, 1e-9, 1e9, xtol=1e-14, rtol=1e-14)
    xs = np.clip(np.sqrt(-dc / (dv * lam_star)) * x, np.maximum(x - move, 0), np.minimum(x + move, 1))
    # the bisection stops within 1e-3 (relative) of the multiplier: the design moves
    # by at most about half that relative change of sqrt(1 / lambda)
    assert np.max(np.abs(xn - xs)) <= 2e-3
    assert np.all(xn >= np.maximum(x - move, 0) - 1e-15) and np.all(xn <= np.minimum(x + move, 1) + 1e-15)
    assert np.allclose(xp, topopt.heaviside_project(topopt.filter_forward(H, Hs, xn), beta), rtol=0, atol=1e-15)
    assert abs(xp.sum() - vf * x.size) <= 2e-3 * vf * x.size
    assert change == np.max(np.abs(xn - x))


def test_oc_projected_reduces_to_density_filter_oc_for_vanishing_beta():
    """As beta -> 0 the projection tends to the identity (tanh(b t) / b -> t), so the
    projected volume is the filtered volume and the update is the density-filter OC."""
    H, Hs, x = _small(seed=8)
    dc = -np.random.default_rng(9).uniform(0.1, 2.0, x.size)
    beta = 1e-5
    dv_p = topopt.projected_volume_gradient(H, Hs, topopt.filter_forward(H, Hs, x), beta)
    dv = topopt.filter_adjoint(H, Hs, np.ones_like(x))
    assert np.max(np.abs(dv_p - dv)) <= 1e-8
    a = topopt.oc_update_projected(x, dc, dv, H, Hs, beta, 0.5, 0.3, 0.2)
    b = topopt.oc_update(x, dc, dv, H, Hs, 0.3, 0.2)
    assert a[3] == b[3] and np.max(np.abs(a[0] - b[0])) <= 1e-12


def test_protocol_selection_and_restart_rules():
    """A short schedule on a small cantilever: the selected iterate is the lowest-compliance
    eligible one, an iteration whose compliance exceeds restart_factor x the selected one
    hands the selected design to the next iteration, and the design stays mirror
    symmetric about the mid-plane z = nz / 2 (the load and the clamp are)."""
    nx, ny, nz = 12, 4, 4
    prob = topopt.Problem(nx, ny, nz, si.cantilever_fixed_dofs(nx, ny, nz),
                          si.cantilever_load(nx, ny, nz), volfrac=0.3)
    phases = ((3, 1.5, 1.0, 0.2, None), (8, 3.5, 4.0, 0.15, 1.35), (14, 4.5, 16.0, 0.08, 1.25))
    hist, sel, x, u = topopt.simp_protocol(prob, 14, direct=True, eligible_gray=0.9,
                                           restart_factor=1.0005, phases=phases)
    el = [h for h in hist if h["eligible"]]
    assert el and sel is not None
    assert sel["c"] == min(h["c"] for h in el)
    assert all(h["penal"] >= 3.0 and h["gray"] < 0.9 for h in el)
    restarts = [h for h in hist if h["restart"]]
    for h in restarts:
        prior = [e["c"] for e in el if e["it"] < h["it"]]
        assert h["c"] > 1.0005 * min(prior)
    g = x.reshape(nz, ny, nx)
    assert np.max(np.abs(g - g[::-1])) <= 1e-10
