"""CPU checks of the C ABI: the shared library loads and exports every declared entry
point; host-only entry points (tridiagonal extremes) and argument validation work
without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:int|const char\*|void)\s+(tosimp_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for must in ["tosimp_create", "tosimp_set_mesh", "tosimp_set_bcs", "tosimp_set_loads",
                 "tosimp_apply_K", "tosimp_pcg_solve", "tosimp_sensitivity", "tosimp_filter",
                 "tosimp_oc_update", "tosimp_simp_step", "tosimp_lanczos", "tosimp_kappa",
                 "tosimp_set_params", "tosimp_grayness", "tosimp_simp_protocol",
                 "tosimp_project"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2604_18020_amd import LIB_PATH
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_tridiag_extremes_host():
    from paper_2604_18020_amd import tridiag_extremes
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(50), rng.uniform(0.1, 1.0, 49)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ev = np.linalg.eigvalsh(T)
    lo, hi = tridiag_extremes(a, b)
    assert abs(lo - ev[0]) < 1e-12 and abs(hi - ev[-1]) < 1e-12
    lo1, hi1 = tridiag_extremes(np.array([2.5]), np.array([]))
    assert lo1 == pytest.approx(2.5) and hi1 == pytest.approx(2.5)


def test_null_context_is_rejected():
    from paper_2604_18020_amd.binding import LIB
    assert LIB.tosimp_set_mesh(None, 1, 1, 1, 1.0, 1.0, 1e-9, 0.3, 3.0, 1.5) < 0
    assert LIB.tosimp_apply_K(None, None, 0, None, None, 0) < 0
    assert LIB.tosimp_destroy(None) == 0


def test_binding_structures_match_the_header(tmp_path):
    """The ctypes mirrors of the option and statistics structures have the C layout:
    sizes and field offsets from a C program compiled against include/tosimp.h."""
    import shutil
    import subprocess
    from paper_2604_18020_amd import binding as b
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tosimp_solve_opts": b.SolveOpts, "tosimp_solve_stats": b.SolveStats,
               "tosimp_step_opts": b.StepOpts, "tosimp_step_stats": b.StepStats,
               "tosimp_protocol_opts": b.ProtocolOpts,
               "tosimp_protocol_record": b.ProtocolRecord}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tosimp.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_binding_flags_match_the_header():
    """The flag values the binding OR-s into the operator's precision are the header's."""
    from paper_2604_18020_amd import binding as b
    txt = open(os.path.join(ROOT, "include", "tosimp.h")).read()
    defs = {k: int(v, 0) for k, v in re.findall(r"#define (TOSIMP_\w+) (0x[0-9a-fA-F]+|\d+)", txt)}
    assert b.V_ZERO_ON_FIXED == defs["TOSIMP_V_ZERO_ON_FIXED"]
    assert b.SCATTER["atomic_element"] == defs["TOSIMP_SCATTER_ATOMIC_ELEMENT"]
    assert b.SCATTER["atomic_brick"] == defs["TOSIMP_SCATTER_ATOMIC_BRICK"]
    assert b.SCATTER["owner"] == 0
    flags = [defs["TOSIMP_V_ZERO_ON_FIXED"], defs["TOSIMP_SCATTER_ATOMIC_ELEMENT"],
             defs["TOSIMP_SCATTER_ATOMIC_BRICK"]]
    assert all(f & 0xff == 0 for f in flags) and len({f for f in flags}) == 3
