"""Seeded input generators: meshes and quadrature rules (no GPU)."""
import itertools
import math

import numpy as np
import pytest

import synth


@pytest.mark.parametrize("n,jit", [(1, 0.0), (3, 0.15), (6, 0.15)])
def test_kuhn_mesh_valid(n, jit):
    xyz, tets = synth.kuhn_cube_mesh(n, jit, seed=0)
    c = synth.kuhn_counts(n)
    assert xyz.shape == (c["n_vert"], 3) and tets.shape == (c["n_cell"], 4)
    X = xyz[tets]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(J)
    assert det.min() > 0
    assert abs(det.sum() / 6 - 1.0) < 1e-13
    # boundary vertices stay on the cube surface
    onb = np.any((np.abs(xyz) < 1e-15) | (np.abs(xyz - 1) < 1e-15), axis=1)
    assert onb.sum() == (n + 1) ** 3 - max(n - 1, 0) ** 3


def test_faces_closed_form():
    from collections import Counter
    for n in (1, 2, 4):
        _, tets = synth.kuhn_cube_mesh(n)
        cnt = Counter()
        for t in tets:
            for f in range(4):
                cnt[tuple(sorted(int(t[i]) for i in range(4) if i != f))] += 1
        c = synth.kuhn_counts(n)
        assert sum(v == 1 for v in cnt.values()) == c["n_bface"]
        assert sum(v == 2 for v in cnt.values()) == c["n_iface"]
        assert max(cnt.values()) == 2


def test_jitter_bound_and_seed():
    xyz0, _ = synth.kuhn_cube_mesh(4)
    xyz1, _ = synth.kuhn_cube_mesh(4, 0.15, seed=0)
    xyz2, _ = synth.kuhn_cube_mesh(4, 0.15, seed=0)
    assert np.array_equal(xyz1, xyz2)
    assert np.abs(xyz1 - xyz0).max() <= 0.15 / 4 + 1e-15


def test_shuffle_is_relabelling():
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15)
    xs, ts = synth.shuffle_mesh(xyz, tets, seed=0)
    a = np.sort(np.sort(xyz[tets].reshape(-1, 12), axis=1), axis=0)
    b = np.sort(np.sort(xs[ts].reshape(-1, 12), axis=1), axis=0)
    assert np.array_equal(a, b)


def test_five_tet_mesh_valid():
    xyz, tets = synth.five_tet_cube_mesh(3)
    X = xyz[tets]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(J)
    assert det.min() > 0 and abs(det.sum() / 6 - 1) < 1e-13


@pytest.mark.parametrize("shape,deg", [("tet", 2), ("tet", 4), ("tet", 6), ("tri", 2), ("tri", 4), ("tri", 6)])
def test_rule_moments(shape, deg):
    """Exactness on all monomials of degree <= deg, positive weights, interior points."""
    P, W = synth.tet_rule(deg) if shape == "tet" else synth.tri_rule(deg)
    dim = P.shape[1]
    assert W.min() > 0
    assert P.min() > 0 and (1 - P.sum(axis=1)).min() > 0
    for e in itertools.product(range(deg + 1), repeat=dim):
        if sum(e) > deg:
            continue
        exact = np.prod([math.factorial(k) for k in e]) / math.factorial(sum(e) + dim)
        q = W @ np.prod(P ** np.array(e), axis=1)
        assert abs(q - exact) <= 1e-14 * exact


def test_rule_sizes():
    assert [synth.tet_rule(d)[1].size for d in (2, 4, 6)] == [4, 14, 24]
    assert [synth.tri_rule(d)[1].size for d in (2, 4, 6)] == [3, 6, 12]
