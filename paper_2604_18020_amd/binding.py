"""ctypes binding of libtosimp.so (argument marshalling only).

Every numerical step runs in the library's HIP kernels; torch tensors are used only as
device memory and torch's current stream as the stream.  If the shared object is not
built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtosimp.so")

OK, NOT_CONVERGED, FALLBACK_USED = 0, 1, 2
F64, F32 = 0, 1
V_ZERO_ON_FIXED = 0x100
SCATTER = {"owner": 0, "atomic_element": 0x200, "atomic_brick": 0x400}
PREC = {"fp64": 0, "fp32": 1, "bf16_mfma": 2, "fp16_mfma": 3}
FILTER = {"forward": 0, "adjoint": 1}
SOLVE = {"plain_fp64": 0, "ir": 1}
PRECOND = {"jacobi": 0, "nn": 1, "mg": 2}
_DT = {torch.float64: F64, torch.float32: F32}


class TosimpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tosimp error {code}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("mode", C.c_int),
                ("inner_prec", C.c_int), ("inner_tol", C.c_double), ("max_outer", C.c_int),
                ("precond", C.c_int), ("check_every", C.c_int), ("enforce_rule", C.c_int),
                ("kappa", C.c_double), ("harvest_r", C.c_void_p), ("harvest_u", C.c_void_p),
                ("harvest_cap", C.c_int), ("harvest_every", C.c_int), ("fcg_window", C.c_int),
                ("eager", C.c_int), ("nn_stall", C.c_int), ("mg_degree", C.c_int),
                ("mg_alpha", C.c_double), ("harvest_ustar", C.c_void_p)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer_iterations", C.c_int),
                ("fallbacks", C.c_int), ("status", C.c_int),
                ("rel_residual", C.c_double), ("true_rel_residual", C.c_double),
                ("harvested", C.c_int), ("restarts", C.c_int), ("b_dot_u", C.c_double),
                ("b_dot_u_corrected", C.c_double), ("escalations", C.c_int),
                ("kappa", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepOpts(C.Structure):
    _fields_ = [("volfrac", C.c_double), ("move", C.c_double), ("solve", SolveOpts),
                ("beta", C.c_double), ("eta", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("compliance", C.c_double), ("change", C.c_double), ("volume", C.c_double),
                ("bisection_steps", C.c_int), ("solve", SolveStats), ("grayness", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "solve"}
        d["solve"] = self.solve.as_dict()
        return d


class ProtocolOpts(C.Structure):
    _fields_ = [("iters", C.c_int), ("volfrac", C.c_double), ("eta", C.c_double),
                ("restart_factor", C.c_double), ("eligible_penal", C.c_double),
                ("eligible_gray", C.c_double), ("nphases", C.c_int),
                ("phases", C.POINTER(C.c_double)), ("solve", SolveOpts)]


class ProtocolRecord(C.Structure):
    _fields_ = [("it", C.c_int), ("cg_iterations", C.c_int), ("bisection_steps", C.c_int),
                ("restart", C.c_int), ("eligible", C.c_int), ("selected", C.c_int),
                ("penal", C.c_double), ("beta", C.c_double), ("move", C.c_double),
                ("rmin", C.c_double), ("compliance", C.c_double), ("grayness", C.c_double),
                ("change", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2604_18020_amd/build.py` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P, I, D, L = C.c_void_p, C.c_int, C.c_double, C.c_int64
    sig = {
        "tosimp_create": (I, [I, P, C.POINTER(P)]),
        "tosimp_destroy": (I, [P]),
        "tosimp_set_stream": (I, [P, P]),
        "tosimp_last_error": (C.c_char_p, [P]),
        "tosimp_version": (C.c_char_p, []),
        "tosimp_set_mesh": (I, [P, I, I, I, D, D, D, D, D, D]),
        "tosimp_set_bcs": (I, [P, P, L]),
        "tosimp_set_loads": (I, [P, P]),
        "tosimp_counts": (I, [P, P, P, P]),
        "tosimp_apply_K": (I, [P, P, I, P, P, I]),
        "tosimp_diag_K": (I, [P, P, I, P, I]),
        "tosimp_pcg_solve": (I, [P, P, P, P, C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
        "tosimp_sensitivity": (I, [P, P, P, P, C.POINTER(D)]),
        "tosimp_filter": (I, [P, P, P, I]),
        "tosimp_project": (I, [P, P, P, P, D, D]),
        "tosimp_oc_update": (I, [P, P, P, D, D, P, P, C.POINTER(D), C.POINTER(I)]),
        "tosimp_simp_step": (I, [P, P, P, P, C.POINTER(StepOpts), C.POINTER(StepStats)]),
        "tosimp_set_params": (I, [P, D, D]),
        "tosimp_grayness": (I, [P, P, C.POINTER(D)]),
        "tosimp_simp_protocol": (I, [P, P, P, P, P, C.POINTER(ProtocolOpts),
                                     C.POINTER(ProtocolRecord), C.POINTER(I), C.POINTER(D)]),
        "tosimp_lanczos": (I, [P, P, P, I, I, P, P, C.POINTER(I)]),
        "tosimp_lanczos_noalloc": (I, [P, P, P, I, I, P, P, C.POINTER(I)]),
        "tosimp_tridiag_extremes": (I, [P, P, I, C.POINTER(D), C.POINTER(D)]),
        "tosimp_kappa": (I, [P, P, P, I, I, D, I, C.POINTER(D), C.POINTER(D), C.POINTER(I),
                             C.POINTER(I)]),
        "tosimp_mg_apply": (I, [P, P, P, P, I, I, D]),
        "tosimp_mg_levels": (I, [P, P, I]),
        "tosimp_nn_create": (I, [P, I, I]),
        "tosimp_nn_num_params": (I, [P, C.POINTER(L)]),
        "tosimp_nn_set_weights": (I, [P, P, L]),
        "tosimp_nn_get_weights": (I, [P, P, L]),
        "tosimp_nn_set_density": (I, [P, P, I]),
        "tosimp_nn_apply": (I, [P, P, P]),
        "tosimp_nn_precondition": (I, [P, P, P, P]),
        "tosimp_nn_forward": (I, [P, P, P]),
        "tosimp_nn_loss_grad": (I, [P, P, P, C.POINTER(D), P]),
        "tosimp_nn_train_step": (I, [P, P, P, I, D, C.POINTER(D)]),
        "tosimp_nn_make_targets": (I, [P, P, P, I]),
        "tosimp_nn_set_loss": (I, [P, I]),
        "tosimp_nn_sample_grad": (I, [P, P, P, C.POINTER(D), P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = res, args
    return lib


LIB = _load()


def _ptr(t: torch.Tensor, dtype=None, numel=None, device=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, context on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Tosimp:
    """One library context bound to a device; follows torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            s = torch.cuda.current_stream(self.device).cuda_stream
        rc = LIB.tosimp_create(self.device, C.c_void_p(s), C.byref(h))
        if rc != 0:
            raise TosimpError(rc, "tosimp_create failed")
        self._h = h
        self.n_elem = self.n_node = self.n_dof = 0

    def close(self):
        if getattr(self, "_h", None):
            LIB.tosimp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ plumbing
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        LIB.tosimp_set_stream(self._h, C.c_void_p(s))

    def _check(self, rc):
        if rc < 0:
            raise TosimpError(rc, LIB.tosimp_last_error(self._h).decode())
        return rc

    def _dev(self, t, dtype=None, numel=None, name="tensor"):
        return _ptr(t, dtype, numel, self.device, name)

    # ------------------------------------------------------------------ set-up
    def set_mesh(self, nx, ny, nz, h=1.0, E0=1.0, Emin=1e-9, nu=0.3, penal=3.0, rmin=1.5):
        self._sync_stream()
        self._check(LIB.tosimp_set_mesh(self._h, nx, ny, nz, h, E0, Emin, nu, penal, rmin))
        ne, nn, nd = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(LIB.tosimp_counts(self._h, C.byref(ne), C.byref(nn), C.byref(nd)))
        self.n_elem, self.n_node, self.n_dof = ne.value, nn.value, nd.value
        self.dims = (nx, ny, nz)
        return self

    def set_bcs(self, fixed_dofs):
        a = np.ascontiguousarray(np.asarray(fixed_dofs, dtype=np.int64))
        self._check(LIB.tosimp_set_bcs(self._h, a.ctypes.data_as(C.c_void_p), a.size))

    def set_loads(self, f: torch.Tensor):
        self._sync_stream()
        self._check(LIB.tosimp_set_loads(self._h, self._dev(f, torch.float64, self.n_dof, "f")))

    # ------------------------------------------------------------------ operator
    def apply_K(self, x, v, y=None, prec="fp64", v_zero_on_fixed=False, scatter="owner"):
        """v_zero_on_fixed: the caller guarantees v = 0 on fixed DOFs (skips the BC bytes).
        scatter: "owner" (deterministic default), "atomic_element" or "atomic_brick"."""
        p = PREC[prec] | SCATTER[scatter]
        vt = torch.float64 if PREC[prec] == 0 else torch.float32
        if y is None:
            y = torch.empty_like(v)
        self._sync_stream()
        self._check(LIB.tosimp_apply_K(
            self._h, self._dev(x, None, self.n_elem, "x"), _DT[x.dtype],
            self._dev(v, vt, self.n_dof, "v"), self._dev(y, vt, self.n_dof, "y"), p | (V_ZERO_ON_FIXED if v_zero_on_fixed else 0)))
        return y

    def diag_K(self, x, dtype=torch.float64):
        d = torch.empty(self.n_dof, dtype=dtype, device=x.device)
        self._sync_stream()
        self._check(LIB.tosimp_diag_K(self._h, self._dev(x, None, self.n_elem, "x"),
                                      _DT[x.dtype], self._dev(d, dtype, self.n_dof, "d"),
                                      _DT[dtype]))
        return d

    # ------------------------------------------------------------------ solve
    @staticmethod
    def solve_opts(tol=1e-8, maxit=20000, mode="plain_fp64", inner_prec="fp32",
                   inner_tol=1e-5, max_outer=30, precond="jacobi", check_every=16,
                   enforce_rule=False, kappa=0.0, fcg_window=1, eager=False, nn_stall=0,
                   mg_degree=0, mg_alpha=0.0):
        return SolveOpts(tol, maxit, SOLVE[mode], PREC[inner_prec], inner_tol, max_outer,
                         PRECOND[precond], check_every, int(enforce_rule), kappa, None, None,
                         0, 0, int(fcg_window), int(bool(eager)), int(nn_stall),
                         int(mg_degree), float(mg_alpha))

    def _opts_with_harvest(self, harvest, harvest_every, harvest_ustar=None, **kw):
        o = self.solve_opts(**kw)
        if harvest_ustar is not None:
            o.harvest_ustar = self._dev(harvest_ustar, torch.float64, self.n_dof, "harvest_ustar").value
        if harvest is not None:
            hr, hu = harvest
            cap = hr.shape[0]
            o.harvest_r = self._dev(hr, torch.float32, cap * self.n_dof, "harvest_r").value
            o.harvest_u = self._dev(hu, torch.float32, cap * self.n_dof, "harvest_u").value
            o.harvest_cap, o.harvest_every = cap, int(harvest_every)
        return o

    def pcg_solve(self, x, b, u, harvest=None, harvest_every=1, harvest_ustar=None, **kw):
        """harvest: optional (r, u) pair of FP32 device tensors [cap, n_dof] (plain FP64);
        with harvest_ustar (FP64 reference solution) u receives ustar - u_k."""
        o = self._opts_with_harvest(harvest, harvest_every, harvest_ustar, **kw)
        s = SolveStats()
        self._sync_stream()
        rc = self._check(LIB.tosimp_pcg_solve(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(b, torch.float64, self.n_dof, "b"),
            self._dev(u, torch.float64, self.n_dof, "u"), C.byref(o), C.byref(s)))
        d = s.as_dict()
        d["rc"] = rc
        return d

    # ------------------------------------------------------------------ SIMP
    def sensitivity(self, x, u, dc=None):
        if dc is None:
            dc = torch.empty(self.n_elem, dtype=torch.float64, device=x.device)
        c = C.c_double()
        self._sync_stream()
        self._check(LIB.tosimp_sensitivity(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(u, torch.float64, self.n_dof, "u"),
            self._dev(dc, torch.float64, self.n_elem, "dc"), C.byref(c)))
        return dc, c.value

    def filter(self, inp, mode="forward", out=None):
        if out is None:
            out = torch.empty_like(inp)
        self._sync_stream()
        self._check(LIB.tosimp_filter(self._h, self._dev(inp, torch.float64, self.n_elem, "in"),
                                      self._dev(out, torch.float64, self.n_elem, "out"),
                                      FILTER[mode]))
        return out

    def project(self, xbar, beta, eta=0.5, g=None, out=None):
        """Heaviside projection of xbar, or (with g) g times its derivative at xbar."""
        if out is None:
            out = torch.empty_like(xbar)
        self._sync_stream()
        self._check(LIB.tosimp_project(
            self._h, self._dev(xbar, torch.float64, self.n_elem, "xbar"),
            None if g is None else self._dev(g, torch.float64, self.n_elem, "g"),
            self._dev(out, torch.float64, self.n_elem, "out"), float(beta), float(eta)))
        return out

    def oc_update(self, x, dc, volfrac, move=0.2, x_new=None, xphys_new=None):
        xn = torch.empty_like(x) if x_new is None else x_new
        xpn = torch.empty_like(x) if xphys_new is None else xphys_new
        ch, st = C.c_double(), C.c_int()
        self._sync_stream()
        self._check(LIB.tosimp_oc_update(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(dc, torch.float64, self.n_elem, "dc"), volfrac, move,
            self._dev(xn, torch.float64, self.n_elem, "x_new"),
            self._dev(xpn, torch.float64, self.n_elem, "xphys_new"), C.byref(ch), C.byref(st)))
        return xn, xpn, ch.value, st.value

    def set_params(self, penal, rmin):
        self._sync_stream()
        self._check(LIB.tosimp_set_params(self._h, float(penal), float(rmin)))

    def grayness(self, rho):
        g = C.c_double()
        self._sync_stream()
        self._check(LIB.tosimp_grayness(self._h, self._dev(rho, torch.float64, self.n_elem, "rho"),
                                        C.byref(g)))
        return g.value

    def simp_protocol(self, x, u, iters=120, volfrac=0.3, eta=0.5, restart_factor=1.12,
                      eligible_penal=3.0, eligible_gray=0.25, phases=None, x_sel=None,
                      xphys=None, **solve_kw):
        """Three-field SIMP with continuation, restart and selection.  phases: None (the
        paper's four) or a sequence of (last_it, penal, beta, move, rmin_end or None).
        Returns (records, it_selected, c_selected, x_sel, xphys)."""
        x_sel = torch.empty_like(x) if x_sel is None else x_sel
        xphys = torch.empty_like(x) if xphys is None else xphys
        if phases is None:
            nph, arr = 0, None
        else:
            flat = [float(v if v is not None else 0.0) for ph in phases for v in ph]
            nph, arr = len(phases), (C.c_double * len(flat))(*flat)
        o = ProtocolOpts(int(iters), volfrac, eta, restart_factor, eligible_penal, eligible_gray,
                         nph, arr, self.solve_opts(**solve_kw))
        rec = (ProtocolRecord * int(iters))()
        its, cs = C.c_int(), C.c_double()
        self._sync_stream()
        self._check(LIB.tosimp_simp_protocol(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(x_sel, torch.float64, self.n_elem, "x_sel"),
            self._dev(xphys, torch.float64, self.n_elem, "xphys"),
            self._dev(u, torch.float64, self.n_dof, "u"), C.byref(o), rec, C.byref(its),
            C.byref(cs)))
        return [r.as_dict() for r in rec], its.value, cs.value, x_sel, xphys

    def simp_step(self, x, xphys, u, volfrac=0.3, move=0.2, harvest=None, harvest_every=1,
                  beta=0.0, eta=0.5, **solve_kw):
        o = StepOpts(volfrac, move, self._opts_with_harvest(harvest, harvest_every, **solve_kw),
                     float(beta), float(eta))
        s = StepStats()
        self._sync_stream()
        rc = self._check(LIB.tosimp_simp_step(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(xphys, torch.float64, self.n_elem, "xphys"),
            self._dev(u, torch.float64, self.n_dof, "u"), C.byref(o), C.byref(s)))
        d = s.as_dict()
        d["rc"] = rc
        return d

    # ------------------------------------------------------------------ Lanczos
    def lanczos(self, x, v0, k, jacobi_scaled=False):
        a = np.zeros(k)
        b = np.zeros(max(k, 1))
        m = C.c_int()
        self._sync_stream()
        self._check(LIB.tosimp_lanczos(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(v0, torch.float64, self.n_dof, "v0"), k, int(jacobi_scaled),
            a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), C.byref(m)))
        return a[:m.value].copy(), b[:max(m.value - 1, 0)].copy()


    def lanczos_noalloc(self, x, v0, k, jacobi_scaled=False):
        """tosimp_lanczos_noalloc: the same coefficients, kept in the library's fixed
        device array (no allocation inside the call)."""
        a = np.zeros(k)
        b = np.zeros(max(k, 1))
        m = C.c_int()
        self._sync_stream()
        self._check(LIB.tosimp_lanczos_noalloc(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(v0, torch.float64, self.n_dof, "v0"), int(k), int(jacobi_scaled),
            a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), C.byref(m)))
        return a[:m.value].copy(), b[:max(m.value - 1, 0)].copy()

    def kappa(self, x, v0, kmax=5000, jacobi_scaled=True, rtol=1e-3, window=50):
        """Lanczos extremes with the stopping rule: (lmin, lmax, steps, converged)."""
        lo, hi, st, cv = C.c_double(), C.c_double(), C.c_int(), C.c_int()
        self._sync_stream()
        self._check(LIB.tosimp_kappa(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(v0, torch.float64, self.n_dof, "v0"), int(kmax), int(jacobi_scaled),
            float(rtol), int(window), C.byref(lo), C.byref(hi), C.byref(st), C.byref(cv)))
        return lo.value, hi.value, st.value, bool(cv.value)

    # ------------------------------------------------------------------ multigrid
    def mg_apply(self, x, r, z=None, degree=0, alpha=0.0):
        """One V-cycle z = V(r) for K_c(x) (FP64 or FP32 by r's dtype)."""
        if z is None:
            z = torch.empty_like(r)
        prec = PREC["fp64"] if r.dtype == torch.float64 else PREC["fp32"]
        self._sync_stream()
        self._check(LIB.tosimp_mg_apply(
            self._h, self._dev(x, torch.float64, self.n_elem, "x"),
            self._dev(r, r.dtype, self.n_dof, "r"), self._dev(z, r.dtype, self.n_dof, "z"),
            prec, int(degree), float(alpha)))
        return z

    def mg_levels(self, cap=16):
        dims = (C.c_int * (3 * cap))()
        self._sync_stream()
        n = LIB.tosimp_mg_levels(self._h, dims, cap)
        if n < 0:
            self._check(n)
        return [tuple(dims[3 * l:3 * l + 3]) for l in range(n)]

    # ------------------------------------------------------------------ learned preconditioner
    def nn_create(self, base=16, bf16=True):
        self._sync_stream()
        self._check(LIB.tosimp_nn_create(self._h, int(base), int(bool(bf16))))
        self.nn_base = int(base)
        n = C.c_int64()
        self._check(LIB.tosimp_nn_num_params(self._h, C.byref(n)))
        self.nn_params = n.value
        return self

    def nn_set_weights(self, w):
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
        self._sync_stream()
        self._check(LIB.tosimp_nn_set_weights(self._h, a.ctypes.data_as(C.c_void_p), a.size))

    def nn_get_weights(self):
        a = np.zeros(self.nn_params, dtype=np.float32)
        self._sync_stream()
        self._check(LIB.tosimp_nn_get_weights(self._h, a.ctypes.data_as(C.c_void_p), a.size))
        return a

    def nn_set_density(self, x):
        self._sync_stream()
        self._check(LIB.tosimp_nn_set_density(self._h, self._dev(x, None, self.n_elem, "x"),
                                              _DT[x.dtype]))

    def nn_apply(self, r, z=None):
        if z is None:
            z = torch.empty_like(r)
        self._sync_stream()
        self._check(LIB.tosimp_nn_apply(self._h, self._dev(r, torch.float32, self.n_dof, "r"),
                                        self._dev(z, torch.float32, self.n_dof, "z")))
        return z

    def nn_precondition(self, x32, r, z=None):
        if z is None:
            z = torch.empty_like(r)
        self._sync_stream()
        self._check(LIB.tosimp_nn_precondition(
            self._h, self._dev(x32, torch.float32, self.n_elem, "x32"),
            self._dev(r, torch.float32, self.n_dof, "r"),
            self._dev(z, torch.float32, self.n_dof, "z")))
        return z

    def nn_forward(self, x4):
        out = torch.empty(self.n_node, 3, dtype=torch.float32, device=x4.device)
        self._sync_stream()
        self._check(LIB.tosimp_nn_forward(self._h, self._dev(x4, torch.float32, 4 * self.n_node,
                                                             "x4"),
                                          self._dev(out, torch.float32, 3 * self.n_node, "out")))
        return out

    def nn_loss_grad(self, x4, target3, want_grad=True):
        loss = C.c_double()
        g = np.zeros(self.nn_params, dtype=np.float32) if want_grad else None
        self._sync_stream()
        self._check(LIB.tosimp_nn_loss_grad(
            self._h, self._dev(x4, torch.float32, 4 * self.n_node, "x4"),
            self._dev(target3, torch.float32, 3 * self.n_node, "target"), C.byref(loss),
            g.ctypes.data_as(C.c_void_p) if want_grad else None))
        return loss.value, g

    def nn_train_step(self, r_batch, e_batch, lr=1e-3):
        nb = r_batch.shape[0]
        loss = C.c_double()
        self._sync_stream()
        self._check(LIB.tosimp_nn_train_step(
            self._h, self._dev(r_batch, torch.float32, nb * self.n_dof, "r_batch"),
            self._dev(e_batch, torch.float32, nb * self.n_dof, "e_batch"), nb, lr,
            C.byref(loss)))
        return loss.value

    def nn_set_loss(self, kind="mse"):
        self._check(LIB.tosimp_nn_set_loss(self._h, {"mse": 0, "energy": 1}[kind]))

    def nn_sample_grad(self, r, e, want_grad=True):
        loss = C.c_double()
        g = np.zeros(self.nn_params, dtype=np.float32) if want_grad else None
        self._sync_stream()
        self._check(LIB.tosimp_nn_sample_grad(
            self._h, self._dev(r, torch.float32, self.n_dof, "r"),
            self._dev(e, torch.float32, self.n_dof, "e"), C.byref(loss),
            g.ctypes.data_as(C.c_void_p) if want_grad else None))
        return loss.value, g

    def nn_make_targets(self, u_star, harvest_u, count):
        if harvest_u.numel() < int(count) * self.n_dof:
            raise ValueError("harvest_u holds fewer than count x n_dof values")
        self._sync_stream()
        self._check(LIB.tosimp_nn_make_targets(
            self._h, self._dev(u_star, torch.float64, self.n_dof, "u_star"),
            self._dev(harvest_u, torch.float32, None, "harvest_u"), int(count)))


def tridiag_extremes(alpha, beta):
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    lo, hi = C.c_double(), C.c_double()
    rc = LIB.tosimp_tridiag_extremes(a.ctypes.data_as(C.c_void_p),
                                     b.ctypes.data_as(C.c_void_p) if b.size else None,
                                     a.size, C.byref(lo), C.byref(hi))
    if rc != 0:
        raise TosimpError(rc, "tridiag_extremes")
    return lo.value, hi.value


def version() -> str:
    return LIB.tosimp_version().decode()
