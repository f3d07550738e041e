"""The per-row oracle route agrees with the assembled operator (pins apply_K_rows)."""
import numpy as np

import synth_inputs as si
from oracle import fem


def test_rows_match_assembled():
    nx, ny, nz = 6, 4, 5
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=11)
    fixed = si.cantilever_fixed_dofs(nx, ny, nz)
    KE = fem.element_stiffness(0.3)
    E = fem.simp_modulus(rho, 1.0, 1e-9, 3.0)
    Kc = fem.constrain(fem.assemble_K(nx, ny, nz, E, KE), fem.fixed_mask(v.size, fixed))
    y = Kc @ v
    dofs = np.random.default_rng(0).choice(v.size, 60, replace=False)
    dofs = np.concatenate([dofs, fixed[:3], [v.size - 1, 0]])
    yr = fem.apply_K_rows(nx, ny, nz, rho, v, fixed, dofs, KE)
    assert np.max(np.abs(yr - y[dofs])) <= 1e-14 * np.max(np.abs(y))
