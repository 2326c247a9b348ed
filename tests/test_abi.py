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
    from paper_2212_00518_amd import bath_levels
    from oracle import models
    from workloads import get_config
    b = dict(kind=kind, M=M, W=0.1, mu=mu, placement=placement)
    eps, w, lead, n_below = bath_levels(b, M)
    cfg = get_config("c1")
    cfg["bath"] = b
    m = models.from_config(cfg, M=M)
    e_ref = np.diag(m.H(np.array([0.0])))[1:]
    assert np.max(np.abs(eps - e_ref)) < 1e-15
    assert abs(np.sum(w) - 0.1) < 1e-14
    assert lead is None
    assert n_below == M // 2 == int(np.sum(e_ref < mu))


@pytest.mark.parametrize("kind,M,mu,placement", [("trapezoid", 256, 0.0, "shift"),
                                                 ("gauss_legendre", 200, 0.01, "shift"),
                                                 ("trapezoid_midpoint", 64, -0.02, "split")])
def test_two_lead_bath_matches_the_oracle(kind, M, mu, placement):
    """Two leads on one grid from the library (iesh_bath) equal the oracle's
    construction: the one-lead grid of M/2 levels with every level listed once
    per lead at half its weight, lead 0 first; the levels below mu are
    counted over both leads."""
    from paper_2212_00518_amd import bath_levels
    from oracle import bath as obath
    b = dict(kind=kind, M=M, W=0.1, mu=mu, placement=placement, leads=2)
    eps, w, lead, n_below = bath_levels(b, M)
    centre = mu if placement == "shift" else 0.0
    e1, w1 = obath.discretise(kind, M // 2, 0.1, eps_f=mu, centre=centre)
    e_ref, w_ref, l_ref = obath.two_leads(e1, w1)
    assert np.max(np.abs(eps - e_ref)) < 1e-15 and np.max(np.abs(w - w_ref)) < 1e-16
    assert np.array_equal(lead, l_ref)
    assert n_below == int(np.sum(e_ref < mu))
    assert abs(np.sum(w) - 0.1) < 1e-14


def test_bath_rejects_bad_descriptors(libiesh):
    from paper_2212_00518_amd import _lib
    with pytest.raises(_lib.IeshError):
        _lib.bath("gauss_legendre", 6, 0.1, n_leads=2)      # 3 levels per lead: odd
    with pytest.raises(_lib.IeshError):
        _lib.bath("trapezoid", 7, 0.1, n_leads=2)           # not a multiple of the leads
    with pytest.raises(_lib.IeshError):
        _lib.bath("trapezoid", 8, 0.1, n_leads=3)
    with pytest.raises(_lib.IeshError):
        _lib.bath("gauss_legendre", 8, 0.1, mu=0.2, placement="split")  # split outside the band


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


def _valid_case():
    """A valid two-lead multi-coordinate descriptor set (plain dicts)."""
    from workloads import get_config
    cfg = get_config("c5")
    e = np.repeat(np.linspace(-0.05, 0.05, 6), 2)
    w = np.full(12, 0.1 / 12)
    lead = np.tile(np.array([0, 1], dtype=np.int32), 6)
    run = dict(n_traj=4, precision="fp64", dt=20.0, kT=1e-3, seed=0)
    return cfg["model"], e, w, lead, run


@pytest.mark.parametrize("change,message", [
    (lambda m, e, w, l, r, n: r.update(dt=0.0), "dt must be > 0"),
    (lambda m, e, w, l, r, n: r.update(kT=-1.0), "kT must be >= 0"),
    (lambda m, e, w, l, r, n: r.update(n_traj=0), "n_traj"),
    (lambda m, e, w, l, r, n: r.update(elec_substeps=65), "elec_substeps"),
    (lambda m, e, w, l, r, n: r.update(dt_levels=3), "hop_gmax"),
    (lambda m, e, w, l, r, n: r.update(dt_levels=31, hop_gmax=0.1), "dt_levels"),
    (lambda m, e, w, l, r, n: r.update(bias=0.01, kT=0.0), "kT > 0"),
    (lambda m, e, w, l, r, n: r.update(exit_dof=6), "exit_dof"),
    (lambda m, e, w, l, r, n: r.update(hop_filter_off=2), "hop_filter_off"),
    (lambda m, e, w, l, r, n: e.__setitem__(3, 0.2), "ascending"),
    (lambda m, e, w, l, r, n: w.__setitem__(0, 0.0), "weights"),
    (lambda m, e, w, l, r, n: l.__setitem__(0, 2), "lead labels"),
    (lambda m, e, w, l, r, n: n.__setitem__(0, 13), "n_elec"),
])
def test_create_rejects_bad_arguments_before_any_device_call(change, message):
    """Argument errors come back as IESH_EINVAL with their reason, on a host
    without a GPU (iesh_create checks everything before its first device
    call)."""
    from paper_2212_00518_amd import _lib
    model, e, w, lead, run = _valid_case()
    n_elec = [6]
    change(model, e, w, lead, run, n_elec)
    with pytest.raises(_lib.IeshError, match=message):
        _lib.Ensemble([_lib.model_desc(model, e, w, n_elec[0], lead)], run)


def test_bias_needs_lead_labels_in_every_model():
    from paper_2212_00518_amd import _lib
    model, e, w, lead, run = _valid_case()
    run.update(bias=0.01)
    with pytest.raises(_lib.IeshError, match="lead labels in every model"):
        _lib.Ensemble([_lib.model_desc(model, e, w, 6, lead), _lib.model_desc(model, e, w, 6)], run,
                      traj_model=np.array([0, 1, 0, 1], dtype=np.int32))


def test_models_of_a_context_need_the_same_coordinate_count():
    from paper_2212_00518_amd import _lib
    from workloads import get_config
    model, e, w, lead, run = _valid_case()
    c1 = get_config("c1")["model"]
    with pytest.raises(_lib.IeshError, match="same n_dof"):
        _lib.Ensemble([_lib.model_desc(model, e, w, 6, lead), _lib.model_desc(c1, e, w, 6)], run,
                      traj_model=np.array([0, 1, 0, 1], dtype=np.int32))


@pytest.mark.parametrize("n,batch,kind,message", [
    (0, 1, 0, "n out of range"), (337, 1, 0, "n out of range"), (4, -1, 0, "batch"),
    (4, 1, 7, "mem_kind"),
])
def test_dense_eigensolver_rejects_bad_arguments_without_a_gpu(libiesh, n, batch, kind, message):
    from paper_2212_00518_amd import _lib
    L = _lib.lib()
    H = np.eye(2)  # only read after the checks pass
    lam = np.zeros(2)
    Q = np.zeros_like(H)
    rc = L.iesh_eigh_batched(H.ctypes.data_as(ctypes.c_void_p), n, batch,
                             lam.ctypes.data_as(ctypes.c_void_p), Q.ctypes.data_as(ctypes.c_void_p),
                             None, kind, None)
    assert rc == _lib.IESH_EINVAL
    assert message in L.iesh_last_error(None).decode()
    # an empty batch is a no-op
    assert L.iesh_eigh_batched(None, 4, 0, None, None, None, 0, None) == _lib.IESH_OK


def test_iteration_cap_is_checked():
    from paper_2212_00518_amd import _lib
    model, e, w, lead, run = _valid_case()
    run.update(eig_max_iter=129)
    with pytest.raises(_lib.IeshError, match="eig_max_iter"):
        _lib.Ensemble([_lib.model_desc(model, e, w, 6, lead)], run)
