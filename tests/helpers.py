"""Shared test helpers: build a GPU context and the matching oracle objects."""
import numpy as np

import synth_inputs as si


def gpu_problem(nx, ny, nz, kind="cantilever", penal=3.0, nu=0.3, rmin=1.5, h=1.0):
    import torch
    from paper_2604_18020_amd import Tosimp

    if kind in ("cantilever", "torsion", "mbb", "bridge"):
        fixed, f = si.bcs_and_load(kind, nx, ny, nz)
    elif kind == "midpoint":
        fixed, f = si.cantilever_fixed_dofs(nx, ny, nz), si.cantilever_midpoint_load(nx, ny, nz)
    elif kind == "free":
        fixed, f = np.zeros(0, dtype=np.int64), np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    else:
        raise KeyError(kind)
    t = Tosimp(0).set_mesh(nx, ny, nz, h=h, nu=nu, penal=penal, rmin=rmin)
    t.set_bcs(fixed)
    t.set_loads(torch.tensor(f, dtype=torch.float64, device="cuda:0"))
    return t, fixed, f


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))
