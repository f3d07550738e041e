"""tosimp_lanczos_noalloc (the allocation-free variant of tosimp_lanczos, whose alpha and
beta live in a fixed device array of the library) against tosimp_lanczos through the C
ABI: the same kernels in the same order, so the coefficients are bit-identical.  Two
calls in a row share the device array, the second on a smaller mesh with fewer steps;
an invariant subspace (more steps than free DOFs) and the size limit are covered."""
import numpy as np
import pytest

import synth_inputs as si
from tests.helpers import dev, gpu_problem

pytestmark = pytest.mark.gpu


def _start(nx, ny, nz, seed):
    n_dof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    v0 = np.random.default_rng(seed).standard_normal(n_dof)
    v0[si.cantilever_fixed_dofs(nx, ny, nz)] = 0.0
    return v0


def _case(nx, ny, nz, k, jacobi, seed):
    rho = np.random.default_rng(seed).uniform(0.01, 1.0, nx * ny * nz)
    v0 = _start(nx, ny, nz, seed + 1)
    t, _, _ = gpu_problem(nx, ny, nz)
    an, bn = t.lanczos_noalloc(dev(rho), dev(v0), k, jacobi_scaled=jacobi)
    a, b = t.lanczos(dev(rho), dev(v0), k, jacobi_scaled=jacobi)
    an2, bn2 = t.lanczos_noalloc(dev(rho), dev(v0), k, jacobi_scaled=jacobi)
    t.close()
    return a, b, an, bn, an2, bn2


def test_noalloc_lanczos_equals_lanczos_twice_in_a_row():
    # first call: 12 x 6 x 6, 120 Jacobi-scaled steps
    a, b, an, bn, an2, bn2 = _case(12, 6, 6, 120, True, 7)
    assert len(a) == 120 and len(b) == 119
    assert np.array_equal(an, a) and np.array_equal(bn, b)
    assert np.array_equal(an2, a) and np.array_equal(bn2, b)
    # second call, smaller input: 6 x 3 x 3, 40 unscaled steps (the array keeps the first
    # call's longer contents past step 40)
    a, b, an, bn, an2, bn2 = _case(6, 3, 3, 40, False, 11)
    assert len(a) == 40
    assert np.array_equal(an, a) and np.array_equal(bn, b)
    assert np.array_equal(an2, a) and np.array_equal(bn2, b)


def test_noalloc_lanczos_invariant_subspace():
    """2 x 1 x 1 has 24 free DOFs; 60 steps end early on both entry points alike."""
    a, b, an, bn, _, _ = _case(2, 1, 1, 60, True, 3)
    assert 1 <= len(a) <= 60 and len(an) == len(a)
    assert np.array_equal(an, a) and np.array_equal(bn, b)


def test_noalloc_lanczos_refuses_more_steps_than_its_storage():
    from paper_2604_18020_amd import TosimpError
    nx, ny, nz = 4, 2, 2
    t, _, _ = gpu_problem(nx, ny, nz)
    rho = np.full(nx * ny * nz, 0.5)
    with pytest.raises(TosimpError, match="exceeds"):
        t.lanczos_noalloc(dev(rho), dev(_start(nx, ny, nz, 1)), 16384)
    # the largest admitted run still works after the refusal, as tosimp_lanczos does
    v0 = dev(_start(nx, ny, nz, 1))
    an, bn = t.lanczos_noalloc(dev(rho), v0, 16383)
    a, b = t.lanczos(dev(rho), v0, 16383)
    t.close()
    assert 1 <= len(a) <= 16383 and len(an) == len(a)
    assert np.array_equal(an, a, equal_nan=True) and np.array_equal(bn, b, equal_nan=True)
