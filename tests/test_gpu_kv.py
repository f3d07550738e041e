"""GPU parity of the fused operator y = K_c(x) v and the Jacobi diagonal against the CPU
oracle (assembled CSR), element by element.

Tolerances: FP64 <= 1e-12 relative (2-norm and max-norm), FP32 <= 1e-5 relative
(2-norm); the FP32 max-norm bound 2e-5 follows from ~150 rounded operations of unit
roundoff 6e-8 on values of the size of max|y|."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import fem
from tests.helpers import dev, gpu_problem, maxrel, rel

pytestmark = pytest.mark.gpu
KE = fem.element_stiffness(0.3)


def _oracle_y(nx, ny, nz, rho, v, fixed, penal=3.0, nu=0.3, h=1.0):
    KEl = fem.element_stiffness(nu) * h
    E = fem.simp_modulus(rho, 1.0, 1e-9, penal)
    K = fem.assemble_K(nx, ny, nz, E, KEl)
    return fem.constrain(K, fem.fixed_mask(v.size, fixed)) @ v


SIZES = [(16, 8, 8), (37, 19, 23), (31, 16, 9), (1, 1, 1), (2, 1, 3), (15, 14, 40),
         (29, 29, 3), (45, 2, 17), (3, 47, 2)]


@pytest.mark.parametrize("dims", SIZES)
def test_apply_K_fp64_matches_oracle(dims):
    nx, ny, nz = dims
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=42)
    y = t.apply_K(dev(rho), dev(v)).cpu().numpy()
    y_ref = _oracle_y(nx, ny, nz, rho, v, fixed)
    assert rel(y, y_ref) <= 1e-12
    assert maxrel(y, y_ref) <= 1e-12
    assert np.array_equal(y[fixed], v[fixed])


@pytest.mark.parametrize("dims", [(16, 8, 8), (37, 19, 23), (15, 14, 40)])
def test_apply_K_fp32_matches_oracle(dims):
    nx, ny, nz = dims
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=7)
    y_ref = _oracle_y(nx, ny, nz, rho, v, fixed)
    for xdt in (torch.float32, torch.float64):
        y = t.apply_K(dev(rho, xdt), dev(v, torch.float32), prec="fp32").double().cpu().numpy()
        assert rel(y, y_ref) <= 1e-5
        assert maxrel(y, y_ref) <= 2e-5


def test_apply_K_torsion_bcs_and_general_penal_nu_h():
    nx, ny, nz = 12, 12, 20
    t, fixed, _ = gpu_problem(nx, ny, nz, kind="torsion", penal=2.5, nu=0.25, h=0.5)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=3)
    y = t.apply_K(dev(rho), dev(v)).cpu().numpy()
    y_ref = _oracle_y(nx, ny, nz, rho, v, fixed, penal=2.5, nu=0.25, h=0.5)
    assert maxrel(y, y_ref) <= 1e-12


def test_apply_K_rigid_modes_in_null_space():
    nx, ny, nz = 20, 17, 9
    t, _, _ = gpu_problem(nx, ny, nz, kind="free")
    rho = np.random.default_rng(1).uniform(0.01, 1, nx * ny * nz)
    R = fem.rigid_body_modes(nx, ny, nz)
    x = dev(rho)
    scale = np.linalg.norm(t.apply_K(x, dev(np.random.default_rng(2).standard_normal(R.shape[0]))).cpu().numpy())
    for k in range(6):
        y = t.apply_K(x, dev(R[:, k])).cpu().numpy()
        assert np.linalg.norm(y) <= 1e-13 * scale * np.linalg.norm(R[:, k])


def test_apply_K_bitwise_reproducible():
    nx, ny, nz = 40, 21, 33
    t, _, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=5)
    x, vd = dev(rho), dev(v)
    y0 = t.apply_K(x, vd)
    for _ in range(5):
        assert torch.equal(t.apply_K(x, vd), y0)
    x32, v32 = x.float(), vd.float()
    z0 = t.apply_K(x32, v32, prec="fp32")
    for _ in range(3):
        assert torch.equal(t.apply_K(x32, v32, prec="fp32"), z0)


@pytest.mark.parametrize("dims", [(16, 8, 8), (23, 9, 31)])
def test_diag_matches_oracle(dims):
    nx, ny, nz = dims
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho = np.random.default_rng(9).uniform(0.01, 1, nx * ny * nz)
    d = t.diag_K(dev(rho)).cpu().numpy()
    E = fem.simp_modulus(rho, 1.0, 1e-9, 3.0)
    d_ref = fem.diag_K(nx, ny, nz, E, KE, fem.fixed_mask(d.size, fixed))
    assert maxrel(d, d_ref) <= 1e-14
    d32 = t.diag_K(dev(rho), dtype=torch.float32).double().cpu().numpy()
    assert maxrel(d32, d_ref) <= 1e-6


def test_bad_arguments_raise():
    from paper_2604_18020_amd import TosimpError
    t, _, _ = gpu_problem(4, 3, 2)
    x = torch.zeros(24, dtype=torch.float64, device="cuda:0")
    v = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    with pytest.raises(TosimpError):
        t.apply_K(x, v, y=v)
    with pytest.raises(ValueError):
        t.apply_K(x, v[:-1])
    with pytest.raises(TypeError):
        t.apply_K(x, v.float(), prec="fp64")
    # partial overlaps are refused; adjacent ranges are fine
    n = t.n_dof
    buf = torch.zeros(2 * n + 32, dtype=torch.float64, device="cuda:0")
    with pytest.raises(TosimpError, match="overlap"):
        t.apply_K(x, buf[:n], y=buf[8:8 + n])
    with pytest.raises(TosimpError, match="overlap"):
        t.apply_K(buf[n - 4:n - 4 + t.n_elem], buf[:n], y=buf[n:2 * n])
    with pytest.raises(TosimpError, match="overlap"):
        t.sensitivity(x, buf[:n], dc=buf[n - 4:n - 4 + t.n_elem])
    y = t.apply_K(x + 0.5, buf[:n], y=buf[n:2 * n])
    dc, _ = t.sensitivity(x + 0.5, buf[:n], dc=buf[n:n + t.n_elem])
    torch.cuda.synchronize()
    assert torch.equal(y, torch.zeros_like(y)) and torch.equal(dc, torch.zeros_like(dc))


def _samples(nx, ny, nz, rng, n=1500):
    """Sample DOFs uniformly plus on tile seams (blocks own 31 x 7 node columns) and z
    chunk seams (chunks of 9-13 planes at the benchmark size) and the last planes."""
    NX1, NY1 = nx + 1, ny + 1
    pick = list(rng.integers(0, 3 * NX1 * NY1 * (nz + 1), n))
    for _ in range(300):
        i = int(rng.choice([0, 1, 30, 31, 61, 62, nx - 1, nx]))
        j = int(rng.choice([0, 1, 6, 7, 13, 14, ny - 1, ny]))
        k = int(rng.choice([0, 1, 9, 10, 11, 12, 13, 21, 22, nz - 1, nz]))
        pick.append(3 * (min(i, nx) + NX1 * (min(j, ny) + NY1 * min(k, nz))) + int(rng.integers(0, 3)))
    return np.array(pick, dtype=np.int64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_K_full_size_4p9M_sampled(prec):
    """340x170x85 (4.9M elements, 15M DOFs), the benchmark's launch configuration,
    checked on ~1,800 sampled outputs computed one by one by the oracle."""
    nx, ny, nz = 340, 170, 85
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=42)
    if prec == "fp64":
        y = t.apply_K(dev(rho), dev(v)).cpu().numpy()
        tol = 1e-12
    else:
        y = t.apply_K(dev(rho, torch.float32), dev(v, torch.float32), prec="fp32").double().cpu().numpy()
        tol = 2e-5
    dofs = _samples(nx, ny, nz, np.random.default_rng(0))
    y_ref = fem.apply_K_rows(nx, ny, nz, rho, v, fixed, dofs, KE)
    scale = np.max(np.abs(y_ref))
    assert np.max(np.abs(y[dofs] - y_ref)) <= tol * scale
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_K_full_size_repeatable(prec):
    """Every output of every call is identical at 4.9M elements (deterministic owner
    writes, no atomics).  Regression test for a store whose data registers were
    overwritten before the store read them: a few outputs per call, at random places,
    took the value of the next instruction."""
    nx, ny, nz = 340, 170, 85
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=42)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x, vd = dev(rho, dt), dev(v, dt)
    y0 = t.apply_K(x, vd, prec=prec)
    y = torch.empty_like(y0)
    bad = []
    for _ in range(12):
        t.apply_K(x, vd, y, prec=prec)
        bad.append(int((y != y0).sum()))
    assert not any(bad), bad


@pytest.mark.parametrize("prec,u", [("bf16_mfma", 2.0 ** -9), ("fp16_mfma", 2.0 ** -11)])
@pytest.mark.parametrize("dims", [(16, 8, 8), (37, 19, 23), (2, 1, 3), (15, 14, 40)])
def test_apply_K_mfma_within_rounding_bound(prec, u, dims):
    """Low-precision contraction: K_E and the element DOFs are rounded to the MFMA input
    type (unit roundoff u), products and sums are FP32.  Per free DOF the error is then
    at most (2u + u^2 + ~50 * 2^-24) (|K| |v|)_i, with |K| |v| = sum_e E_e |K_E| |v_e|
    computed by the oracle; 2.5u is asserted, plus 1e-6 max(|K||v|) for FP16 values
    below its normal range (the per-element power-of-two scaling keeps the rest exact)."""
    nx, ny, nz = dims
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=11)
    v32 = v.astype(np.float32).astype(np.float64)
    rho32 = rho.astype(np.float32).astype(np.float64)
    E = fem.simp_modulus(rho32, 1.0, 1e-9, 3.0)
    y_ref = fem.apply_K_elementwise(nx, ny, nz, E, KE, v32, fixed)
    bound = fem.apply_K_elementwise(nx, ny, nz, E, np.abs(KE), np.abs(v32), fixed)
    free = ~fem.fixed_mask(v.size, fixed)
    for xdt in (torch.float32, torch.float64):
        y = t.apply_K(dev(rho32, xdt), dev(v32, torch.float32), prec=prec).double().cpu().numpy()
        err = np.abs(y - y_ref)
        lim = 2.5 * u * bound + 1e-6 * bound[free].max()
        assert np.all(err[free] <= lim[free]), float(np.max(err[free] / lim[free]))
        assert np.array_equal(y[~free], v32[~free])
        # the bound is not vacuous: the error is of the size the rounding predicts
        assert rel(y, y_ref) <= 4 * u


@pytest.mark.parametrize("dims", [(16, 8, 8), (37, 19, 23), (2, 1, 3), (70, 9, 13)])
def test_apply_K_zero_on_fixed_flag_is_bit_identical(dims):
    """The path the CG iterations use (v known to be zero on fixed DOFs, BC bytes of the
    planes not read) gives bit-identical results to the general path."""
    nx, ny, nz = dims
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=13)
    v[fixed] = 0.0
    for dt, prec in [(torch.float64, "fp64"), (torch.float32, "fp32")]:
        x, vd = dev(rho, dt), dev(v, dt)
        y0 = t.apply_K(x, vd, prec=prec)
        y1 = t.apply_K(x, vd, prec=prec, v_zero_on_fixed=True)
        assert torch.equal(y0, y1), prec
        assert torch.all(y1[torch.as_tensor(fixed, device="cuda:0")] == 0)



def test_apply_K_smooth_displacement_within_rounding_bound(record_property):
    """K applied to a displacement u (the FP64 solution of K u = f on the 120x60x30
    cantilever at rho = 0.3), where K u = f is tiny next to |K| |u|: the cancellation
    case.  Per free DOF every precision stays within 2.5 u_p (|K| |u|)_i of the oracle's
    exact product of the same (rounded) input, u_p its unit roundoff (measured worst
    ratios err / (u_p |K||u|): 1.4 FP64, 0.75 FP32, 1.2 BF16, 0.53 FP16).  Relative to
    ||K u|| that is 3e-13 (FP64), 1e-4 (FP32), 6.1 (BF16) and 0.78 (FP16): a low-precision
    product of a converged displacement is mostly rounding error, which is why such inner
    solves stagnate.  These relative errors are recorded, not asserted."""
    nx, ny, nz = 120, 60, 30
    t, fixed, f = gpu_problem(nx, ny, nz)
    rho = np.full(nx * ny * nz, 0.3)
    u = torch.zeros(t.n_dof, dtype=torch.float64, device="cuda:0")
    st = t.pcg_solve(dev(rho), dev(f), u, tol=1e-10)
    assert st["true_rel_residual"] <= 1e-10
    u64 = u.cpu().numpy()
    E = fem.simp_modulus(rho, 1.0, 1e-9, 3.0)
    free = ~fem.fixed_mask(u64.size, fixed)
    cases = [("fp64", 2.0 ** -53, torch.float64), ("fp32", 2.0 ** -24, torch.float32),
             ("bf16_mfma", 2.0 ** -9, torch.float32), ("fp16_mfma", 2.0 ** -11, torch.float32)]
    for prec, up, dt in cases:
        v = u64.astype(np.float32).astype(np.float64) if dt == torch.float32 else u64
        y_ref = fem.apply_K_elementwise(nx, ny, nz, E, KE, v, fixed)
        bound = fem.apply_K_elementwise(nx, ny, nz, E, np.abs(KE), np.abs(v), fixed)
        y = t.apply_K(dev(rho, dt), dev(v, dt), prec=prec).double().cpu().numpy()
        err = np.abs(y - y_ref)
        lim = 2.5 * up * bound + (1e-6 * bound[free].max() if prec == "fp16_mfma" else 0.0)
        ratio = float(np.max(err[free] / (up * bound[free] + 1e-300)))
        record_property(f"{prec}_max_err_over_u_absK_absu", ratio)
        record_property(f"{prec}_rel_err", rel(y, y_ref))
        assert np.all(err[free] <= lim[free]), (prec, ratio)
        assert np.array_equal(y[~free], v[~free])
    # the cancellation is real: |K| |u| exceeds |K u| by orders of magnitude
    assert np.linalg.norm(bound[free]) > 1e3 * np.linalg.norm(y_ref[free])
    t.close()


def test_set_mesh_rejects_meshes_beyond_the_offset_limit():
    """126 x 112 x 6234 elements have 127 * 113 * 6235 = 89,478,485 nodes: an FP64 DOF
    vector would span 2,147,483,640 bytes, past the operator's out-of-range offset
    0x7FFFFFF0, so the mesh is refused before anything is allocated."""
    from paper_2604_18020_amd import Tosimp, TosimpError
    t = Tosimp(0)
    with pytest.raises(TosimpError):
        t.set_mesh(126, 112, 6234)
    t.set_mesh(2, 2, 2)  # the context stays usable
    t.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_K_near_the_size_limit_sampled(prec):
    """126 x 112 x 6233 elements (89,464,134 nodes, 99.98% of the limit): plane offsets
    reach 2^31 - 3.4e5 bytes in FP64.  Sampled outputs, the top planes included, against
    the oracle's rows."""
    nx, ny, nz = 126, 112, 6233
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=17)
    if prec == "fp64":
        y = t.apply_K(dev(rho), dev(v)).cpu().numpy()
        tol = 1e-12
    else:
        y = t.apply_K(dev(rho, torch.float32), dev(v, torch.float32), prec="fp32").double().cpu().numpy()
        tol = 2e-5
    t.close()
    rng = np.random.default_rng(3)
    NX1, NY1 = nx + 1, ny + 1
    top = [3 * (int(i) + NX1 * (int(j) + NY1 * k)) + int(c)
           for k in (nz - 1, nz) for i, j, c in zip(rng.integers(0, NX1, 200),
                                                     rng.integers(0, NY1, 200),
                                                     rng.integers(0, 3, 200))]
    dofs = np.concatenate([_samples(nx, ny, nz, rng, n=600), np.array(top, dtype=np.int64)])
    y_ref = fem.apply_K_rows(nx, ny, nz, rho, v, fixed, dofs, KE)
    assert np.max(np.abs(y[dofs] - y_ref)) <= tol * np.max(np.abs(y_ref))
    assert np.all(np.isfinite(y[dofs]))


def test_apply_K_every_dof_fixed_is_identity():
    """With every DOF fixed K_c = I: y = v exactly in every precision, and a solve of a
    zero load converges at once to u = 0."""
    from paper_2604_18020_amd import Tosimp
    nx, ny, nz = 9, 5, 4
    t = Tosimp(0).set_mesh(nx, ny, nz)
    n_dof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    t.set_bcs(np.arange(n_dof))
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=8)
    assert np.array_equal(t.apply_K(dev(rho), dev(v)).cpu().numpy(), v)
    v32 = v.astype(np.float32)
    for prec in ("fp32", "bf16_mfma", "fp16_mfma"):
        y = t.apply_K(dev(rho, torch.float32), dev(v32), prec=prec).cpu().numpy()
        assert np.array_equal(y, v32), prec
    t.set_loads(torch.zeros(n_dof, dtype=torch.float64, device="cuda:0"))
    u = torch.ones(n_dof, dtype=torch.float64, device="cuda:0")
    st = t.pcg_solve(dev(rho), torch.zeros(n_dof, dtype=torch.float64, device="cuda:0"), u,
                     tol=1e-8)
    t.close()
    assert st["iterations"] == 0 and st["rc"] == 0
    assert torch.count_nonzero(u).item() == 0


@pytest.mark.parametrize("penal", [3.0, 2.5])
@pytest.mark.parametrize("level", [0.0, 1.0])
def test_apply_K_density_extremes(level, penal):
    """x = 0 everywhere (E = Emin: K scaled by 1e-9; the general-penalty path takes
    x^p = 0 without evaluating pow at 0) and x = 1 (E = E0), FP64 and FP32."""
    nx, ny, nz = 17, 9, 11
    t, fixed, _ = gpu_problem(nx, ny, nz, penal=penal)
    rho = np.full(nx * ny * nz, level)
    _, v = si.random_density_and_vector(nx, ny, nz, seed=9)
    y_ref = _oracle_y(nx, ny, nz, rho, v, fixed, penal=penal)
    free = ~fem.fixed_mask(v.size, fixed)
    y = t.apply_K(dev(rho), dev(v)).cpu().numpy()
    # free rows against their own scale (1e-9 of the fixed rows' when x = 0)
    assert maxrel(y[free], y_ref[free]) <= 1e-12
    assert np.array_equal(y[~free], v[~free])
    v32 = v.astype(np.float32)
    y32 = t.apply_K(dev(rho, torch.float32), dev(v32), prec="fp32").double().cpu().numpy()
    y32_ref = _oracle_y(nx, ny, nz, rho, v32.astype(np.float64), fixed, penal=penal)
    assert rel(y32[free], y32_ref[free]) <= 1e-5
    assert np.array_equal(y32[~free], v32[~free].astype(np.float64))
    t.close()


SCATTERS = ["atomic_element", "atomic_brick"]


@pytest.mark.parametrize("scatter", SCATTERS)
@pytest.mark.parametrize("dims", [(16, 8, 8), (37, 19, 23), (1, 1, 1), (2, 1, 3), (15, 14, 40),
                                  (9, 17, 5), (8, 8, 4)])
def test_apply_K_atomic_scatter_matches_oracle(dims, scatter):
    """The atomic-scatter forms (Alg. "Fused Gather-GEMM-Scatter": one thread per element,
    and 8x8x4 bricks reduced in LDS) against the oracle at the default kernel's bounds, on
    meshes that cut the bricks raggedly or fit one exactly; fixed rows give y = v."""
    nx, ny, nz = dims
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=11)
    y_ref = _oracle_y(nx, ny, nz, rho, v, fixed)
    y = t.apply_K(dev(rho), dev(v), scatter=scatter).cpu().numpy()
    assert rel(y, y_ref) <= 1e-12 and maxrel(y, y_ref) <= 1e-12
    assert np.array_equal(y[fixed], v[fixed])
    v32 = v.astype(np.float32).astype(np.float64)
    for xdt in (torch.float32, torch.float64):
        y = t.apply_K(dev(rho, xdt), dev(v, torch.float32), prec="fp32",
                      scatter=scatter).double().cpu().numpy()
        assert rel(y, y_ref) <= 1e-5 and maxrel(y, y_ref) <= 2e-5
        assert np.array_equal(y[fixed], v32[fixed])
    t.close()


@pytest.mark.parametrize("scatter", SCATTERS)
def test_apply_K_atomic_scatter_general_penal_nu_h(scatter):
    nx, ny, nz = 12, 12, 20
    t, fixed, _ = gpu_problem(nx, ny, nz, kind="torsion", penal=2.5, nu=0.25, h=0.5)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=3)
    y = t.apply_K(dev(rho), dev(v), scatter=scatter).cpu().numpy()
    y_ref = _oracle_y(nx, ny, nz, rho, v, fixed, penal=2.5, nu=0.25, h=0.5)
    assert maxrel(y, y_ref) <= 1e-12
    t.close()


@pytest.mark.parametrize("scatter,prec", [("atomic_element", "fp32"), ("atomic_brick", "fp32"),
                                          ("atomic_brick", "fp64")])
def test_apply_K_atomic_scatter_full_size_sampled(scatter, prec):
    """340x170x85, the launch the scatter study times, on sampled outputs computed one by
    one by the oracle (brick seams every 8 / 8 / 4 elements among the samples)."""
    nx, ny, nz = 340, 170, 85
    t, fixed, _ = gpu_problem(nx, ny, nz)
    rho, v = si.random_density_and_vector(nx, ny, nz, seed=42)
    dt = torch.float64 if prec == "fp64" else torch.float32
    y = t.apply_K(dev(rho, dt), dev(v, dt), prec=prec, scatter=scatter).double().cpu().numpy()
    t.close()
    rng = np.random.default_rng(1)
    dofs = _samples(nx, ny, nz, rng)
    NX1, NY1 = nx + 1, ny + 1
    seams = [3 * (int(rng.choice([0, 8, 16, 64, 336, 340])) + NX1 * (int(rng.choice([0, 8, 16, 168, 170]))
             + NY1 * int(rng.choice([0, 4, 8, 84, 85])))) + int(rng.integers(0, 3)) for _ in range(300)]
    dofs = np.concatenate([dofs, np.array(seams, dtype=np.int64)])
    y_ref = fem.apply_K_rows(nx, ny, nz, rho, v, fixed, dofs, KE)
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert np.max(np.abs(y[dofs] - y_ref)) <= tol * np.max(np.abs(y_ref))
    assert np.all(np.isfinite(y))


def test_apply_K_atomic_scatter_refuses_mfma():
    from paper_2604_18020_amd import TosimpError
    t, _, _ = gpu_problem(4, 3, 2)
    x = torch.full((24,), 0.5, dtype=torch.float32, device="cuda:0")
    v = torch.zeros(t.n_dof, dtype=torch.float32, device="cuda:0")
    for s in SCATTERS:
        with pytest.raises(TosimpError):
            t.apply_K(x, v, prec="bf16_mfma", scatter=s)
    t.close()
