"""The C-ABI library loads and exports every symbol the header declares;
host-only entry points agree with the oracle (CPU only, no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import bath

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iesh.h")
LIB = os.path.join(ROOT, "paper_2212_00518_amd", "libiesh.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(iesh_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("iesh_create", "iesh_step", "iesh_run", "iesh_hop_probs"):
        assert required in names


@pytest.fixture(scope="module")
def libiesh():
    if not os.path.exists(LIB):
        pytest.fail("libiesh.so is not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(libiesh):
    missing = [n for n in declared_functions() if not hasattr(libiesh, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2212_00518_amd import _lib
    assert sorted(_lib.SYMBOLS) == declared_functions()


def test_version(libiesh):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert libiesh.iesh_version(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == 0
    assert (a.value, b.value) >= (0, 1)


@pytest.mark.parametrize("kind,M", [("trapezoid", 20), ("trapezoid", 200),
                                    ("trapezoid_midpoint", 33), ("gauss_legendre", 40),
                                    ("gauss_legendre", 200), ("gauss_legendre", 320)])
def test_library_discretisation_matches_oracle(kind, M):
    from paper_2212_00518_amd import _lib
    eps, w = _lib.discretize(kind, M, 0.1)
    e_ref, w_ref = bath.discretise(kind, M, 0.1)
    assert np.max(np.abs(eps - e_ref)) < 1e-15
    assert np.max(np.abs(w - w_ref)) < 1e-15


@pytest.mark.parametrize("kind,M,mu,placement", [("gauss_legendre", 40, 0.01, "shift"),
                                                 ("gauss_legendre", 100, -0.02, "split"),
                                                 ("trapezoid", 20, 0.03, "shift")])
def test_band_placement_for_a_chemical_potential(kind, M, mu, placement):
    """The library's grid for a chemical potential mu equals the oracle's, and
    the states below mu are half of the bath when the band or the
    Gauss-Legendre split follows mu."""
    from paper_2212_00518_amd import bath_grid, electrons_below
    from oracle import models
    from workloads import get_config
    b = dict(kind=kind, M=M, W=0.1, mu=mu, placement=placement)
    eps, w = bath_grid(b, M)
    cfg = get_config("c1")
    cfg["bath"] = b
    m = models.from_config(cfg, M=M)
    e_ref = np.diag(m.H(np.array([0.0])))[1:]
    assert np.max(np.abs(eps - e_ref)) < 1e-15
    assert abs(np.sum(w) - 0.1) < 1e-14
    assert electrons_below(eps, mu) == M // 2


def test_discretisation_rejects_bad_arguments(libiesh):
    from paper_2212_00518_amd import _lib
    e = np.zeros(3)
    w = np.zeros(3)
    dp = ctypes.POINTER(ctypes.c_double)
    L = _lib.lib()
    # odd M for the Gauss-Legendre split, empty band
    assert L.iesh_discretize(2, 3, -1.0, 1.0, 0.0, e.ctypes.data_as(dp), w.ctypes.data_as(dp)) < 0
    assert L.iesh_discretize(0, 3, 1.0, 1.0, 0.0, e.ctypes.data_as(dp), w.ctypes.data_as(dp)) < 0


def test_product_path_does_not_use_the_oracle():
    """The package and the library sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2212_00518_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_binding_structs_match_the_header_layout(tmp_path):
    """Size and field offsets of every descriptor struct, as the C compiler
    lays them out from include/iesh.h, equal the ctypes binding's."""
    import shutil
    import subprocess
    from paper_2212_00518_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"iesh_model_desc": _lib.ModelDesc, "iesh_run_desc": _lib.RunDesc,
               "iesh_event": _lib.Event, "iesh_sizes": _lib.Sizes}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "iesh.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])
