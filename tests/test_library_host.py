"""Host-side checks of the C-ABI library that need no GPU: the shared
library loads, exports every entry point declared in include/tetmf.h, and the
mesh validation errors of tetmf_mesh_create."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    import paper_2509_10226_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return pkg


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tetmf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tetmf_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares a signature for each of them
    assert set(names) <= set(L._SIGS)


def test_status_strings(L):
    lib = L.lib()
    assert lib.tetmf_status_string(0) == b"ok"
    assert lib.tetmf_status_string(-3) == b"non-conforming mesh"


def test_mesh_create_counts(L):
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15)
    m = L.Mesh(xyz, tets)
    c = synth.kuhn_counts(3)
    assert m.n_face == c["n_iface"] + c["n_bface"]
    assert m.n_interior_face == c["n_iface"]


def test_mesh_errors(L):
    xyz, tets = synth.kuhn_cube_mesh(2)
    bad = tets.copy()
    bad[3, 2] = xyz.shape[0]
    with pytest.raises(L.TetmfError) as e:
        L.Mesh(xyz, bad)
    assert e.value.status == -1
    flat = xyz.copy()
    t0 = tets[0]
    flat[t0[3]] = flat[t0[0]] + 0.5 * (flat[t0[1]] - flat[t0[0]]) + 0.5 * (flat[t0[2]] - flat[t0[0]])
    with pytest.raises(L.TetmfError) as e:
        L.Mesh(flat, tets[:1])
    assert e.value.status == -2
    rep = tets.copy()
    rep[0, 1] = rep[0, 0]
    with pytest.raises(L.TetmfError) as e:
        L.Mesh(xyz, rep)
    assert e.value.status == -2
    # a triangle shared by three cells
    three = np.vstack([tets, tets[:1, [1, 0, 2, 3]]])
    with pytest.raises(L.TetmfError) as e:
        L.Mesh(xyz, three)
    assert e.value.status == -3
