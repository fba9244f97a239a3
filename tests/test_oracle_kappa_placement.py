"""Where the per-point coefficient acts: pins against closed forms.

The coefficient of the forms (eq. (2), eq. (3)) is a field sampled at the
quadrature points.  The operator takes it as an array, cell point q of cell
e at the physical point X0 + J x_q (J built from the cell's vertices in the
given order) and face point q of face F at a + s_q (b - a) + t_q (c - a) for
the face's vertices sorted by global id, a < b < c.  A mistake in that
pairing (another vertex order, a transposed table, points of an unsorted
face triple) leaves A 1 = 0, symmetry, linearity and the indicator
derivatives intact, so it needs its own pin: a linear field kappa(x) is
sampled at the points by that convention, and for global polynomial data the
forms are then integrals with closed forms on the unit cube.

Cell term (any jittered mesh; kappa linear and q1, q2 of degree <= p, so the
integrand has degree <= 2p - 1, within the degree-2p rule):
    I_h(q1)^T K(kappa) I_h(q2) = int_Omega kappa grad q1 . grad q2.

Face terms (SIPG, unjittered Kuhn mesh with N even so that x = 1/2 is a mesh
plane; u = q1 on the cells with x < 1/2 and 0 elsewhere, v = q2 everywhere):
jumps of v vanish, the only jump of u is across x = 1/2, so
    u^T A v = int_{x<1/2} kappa_c grad q1 . grad q2
              - int_{x=1/2} kappa_f q1 d_x q2
              + sum over the boundary of the half box of
                int kappa_f (-q1 d_n q2 - q2 d_n q1 + 2 tau q1 q2)
with tau = (p+1)^2 |F| / |K| = 3 (p+1)^2 / h on every boundary face of the
unjittered mesh (|F| = h^2/2, |K| = h^3/6).  Pairs with deg q1 + deg q2 <=
2p - 1 keep kappa q1 q2 within the degree-2p face rule.

The closed forms use int_0^L t^m dt = L^(m+1)/(m+1) only.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

# kappa(x) = K0 + KX . x: positive on the unit cube, all components distinct
K0 = 2.0
KX = (0.7, -0.4, 0.3)


def kappa_at(x):
    x = np.asarray(x, dtype=np.float64)
    return K0 + x[..., 0] * KX[0] + x[..., 1] * KX[1] + x[..., 2] * KX[2]


def cell_points(xyz, tets, qpts):
    """Physical rule points [n_cell, n_q, 3]: X0 + J x_q, vertices as given."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(tets)]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    return X[:, None, 0, :] + np.einsum("eab,qb->eqa", J, qpts)


def canonical_faces(tets):
    """Sorted vertex triples of all faces, in lexicographic order."""
    t = np.asarray(tets, dtype=np.int64)
    tri = np.concatenate([np.sort(t[:, [i for i in range(4) if i != f]], axis=1) for f in range(4)])
    return np.unique(tri, axis=0)


def face_points(xyz, tri, fpts):
    """Physical face points [n_face, n_qf, 3]: a + s (b - a) + t (c - a)."""
    P = np.asarray(xyz, dtype=np.float64)[tri]
    a, b, c = P[:, 0], P[:, 1], P[:, 2]
    return (a[:, None, :] + fpts[None, :, 0:1] * (b - a)[:, None, :]
            + fpts[None, :, 1:2] * (c - a)[:, None, :])


# ---------------------------------------------------------------- polynomials
# A polynomial is a dict {(i, j, k): coefficient} for x^i y^j z^k.

def mono(e):
    return {tuple(e): 1.0}


def pmul(a, b):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = (ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2])
            out[e] = out.get(e, 0.0) + ca * cb
    return out


def padd(*ps):
    out = {}
    for p in ps:
        for e, c in p.items():
            out[e] = out.get(e, 0.0) + c
    return out


def pscale(a, s):
    return {e: c * s for e, c in a.items()}


def pdiff(a, k):
    out = {}
    for e, c in a.items():
        if e[k] > 0:
            f = list(e)
            f[k] -= 1
            out[tuple(f)] = out.get(tuple(f), 0.0) + c * e[k]
    return out


def kappa_poly():
    return {(0, 0, 0): K0, (1, 0, 0): KX[0], (0, 1, 0): KX[1], (0, 0, 1): KX[2]}


def peval(a, x):
    x = np.asarray(x, dtype=np.float64)
    return sum(c * x[..., 0] ** e[0] * x[..., 1] ** e[1] * x[..., 2] ** e[2] for e, c in a.items())


def box_int(a, lo, hi):
    """int over the box prod [lo_k, hi_k] (lo_k == hi_k: that coordinate is
    fixed and not integrated)."""
    s = 0.0
    for e, c in a.items():
        t = c
        for k in range(3):
            if lo[k] == hi[k]:
                t *= lo[k] ** e[k]
            else:
                t *= (hi[k] ** (e[k] + 1) - lo[k] ** (e[k] + 1)) / (e[k] + 1)
        s += t
    return s


def grad_dot(q1, q2):
    return padd(*[pmul(pdiff(q1, k), pdiff(q2, k)) for k in range(3)])


def monomials(p):
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]


# ---------------------------------------------------------------- closed forms

def cell_closed_form(q1, q2, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    return box_int(pmul(kappa_poly(), grad_dot(q1, q2)), lo, hi)


def half_box_face_closed_form(q1, q2, p, h):
    """Face part of u^T A v for u = q1 on x < 1/2 (see the module docstring)."""
    kap = kappa_poly()
    tau = 3.0 * (p + 1) ** 2 / h
    # interface x = 1/2: -int kappa q1 d_x q2
    s = -box_int(pmul(kap, pmul(q1, pdiff(q2, 0))), (0.5, 0.0, 0.0), (0.5, 1.0, 1.0))
    # boundary of the half box: (fixed coordinate k, value, outward normal sign)
    for k, val, sgn in ((0, 0.0, -1.0), (1, 0.0, -1.0), (1, 1.0, 1.0), (2, 0.0, -1.0), (2, 1.0, 1.0)):
        lo = [0.0, 0.0, 0.0]
        hi = [0.5, 1.0, 1.0]
        lo[k] = hi[k] = val
        integrand = padd(pscale(pmul(q1, pdiff(q2, k)), -sgn), pscale(pmul(q2, pdiff(q1, k)), -sgn),
                         pscale(pmul(q1, q2), 2.0 * tau))
        s += box_int(pmul(kap, integrand), lo, hi)
    return s


# ---------------------------------------------------------------- self-checks of the closed forms

def test_closed_form_helpers():
    """The polynomial integrator against direct values: int_0^1 x^2 = 1/3,
    int over [0,1/2]x[0,1]^2 of x y = 1/16, a face at y = 1 of z^2 = 1/6."""
    assert box_int(mono((2, 0, 0)), (0, 0, 0), (1, 1, 1)) == pytest.approx(1 / 3, rel=1e-15)
    assert box_int(mono((1, 1, 0)), (0, 0, 0), (0.5, 1, 1)) == pytest.approx(1 / 16, rel=1e-15)
    assert box_int(mono((0, 3, 2)), (0, 1, 0), (0.5, 1, 1)) == pytest.approx(0.5 / 3, rel=1e-15)
    assert grad_dot(mono((1, 1, 0)), mono((2, 0, 0))) == {(1, 1, 0): 2.0}
    x = np.array([[0.3, 0.2, 0.9]])
    assert peval(kappa_poly(), x)[0] == pytest.approx(kappa_at(x)[0], rel=1e-15)


# ---------------------------------------------------------------- cell pins

@pytest.mark.parametrize("p", [1, 2, 3])
def test_cell_kappa_placement_cg(p):
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 0)
    qp, qw = synth.tet_rule(2 * p)
    kap = kappa_at(cell_points(xyz, tets, qp))
    K, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap)
    X = d["xyz"]
    for e1 in monomials(p):
        for e2 in monomials(p):
            ex = cell_closed_form(mono(e1), mono(e2))
            got = peval(mono(e1), X) @ (K @ peval(mono(e2), X))
            assert abs(got - ex) <= 1e-12 * max(1.0, abs(ex)), (e1, e2, got, ex)


@pytest.mark.parametrize("p", [2, 3])
def test_cell_kappa_placement_detects_other_vertex_order(p):
    """Sampling the field with the cell's vertices rotated (another X0 and J
    for the same cell) misses the closed form: the pin sees the pairing."""
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 0)
    qp, qw = synth.tet_rule(2 * p)
    wrong = kappa_at(cell_points(xyz, np.roll(tets, 1, axis=1), qp))
    K, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=wrong)
    X = d["xyz"]
    worst = 0.0
    for e1 in monomials(p):
        for e2 in monomials(p):
            ex = cell_closed_form(mono(e1), mono(e2))
            got = peval(mono(e1), X) @ (K @ peval(mono(e2), X))
            worst = max(worst, abs(got - ex) / max(1.0, abs(ex)))
    assert worst > 1e-6


# ---------------------------------------------------------------- face pins

def _dg_half_box(p, n, kc, kf):
    xyz, tets = synth.kuhn_cube_mesh(n, 0.0, 0)
    qp, qw = synth.tet_rule(2 * p)
    fp, fw = synth.tri_rule(2 * p)
    A, faces = oracle.assemble_dg(xyz, tets, p, qp, qw, fp, fw, kc, kf, bc="dirichlet")
    return xyz, tets, A, faces


def dg_node_xyz(xyz, tets, p):
    """Node coordinates [n_cell * n_dof, 3] in the oracle's DG numbering."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(tets)]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    xn = oracle.basis.nodes(p)[:, 1:] / p
    return (X[:, None, 0, :] + np.einsum("eab,kb->eka", J, xn)).reshape(-1, 3)


def half_box_pairs(p):
    return [(e1, e2) for e1 in monomials(p) for e2 in monomials(p) if sum(e1) + sum(e2) <= 2 * p - 1]


def half_box_vectors(xyz, tets, p, e1, e2):
    nd = oracle.basis.nodes(p).shape[0]
    Xn = dg_node_xyz(xyz, tets, p)
    cen = np.asarray(xyz)[np.asarray(tets)].mean(axis=1)
    left = np.repeat(cen[:, 0] < 0.5, nd)
    u = np.where(left, peval(mono(e1), Xn), 0.0)
    v = peval(mono(e2), Xn)
    return u, v


def half_box_expected(p, n, e1, e2):
    return (cell_closed_form(mono(e1), mono(e2), hi=(0.5, 1.0, 1.0))
            + half_box_face_closed_form(mono(e1), mono(e2), p, 1.0 / n))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_face_kappa_placement_dg(p):
    n = 2
    xyz, tets = synth.kuhn_cube_mesh(n, 0.0, 0)
    qp, _ = synth.tet_rule(2 * p)
    fp, _ = synth.tri_rule(2 * p)
    tri = canonical_faces(tets)
    kc = kappa_at(cell_points(xyz, tets, qp))
    kf = kappa_at(face_points(xyz, tri, fp))
    xyz, tets, A, faces = _dg_half_box(p, n, kc, kf)
    # the oracle's face order is the canonical (lexicographic) one
    assert np.array_equal(faces["tri"], tri)
    for e1, e2 in half_box_pairs(p):
        u, v = half_box_vectors(xyz, tets, p, e1, e2)
        ex = half_box_expected(p, n, e1, e2)
        scale = max(1.0, abs(ex), 3.0 * (p + 1) ** 2 * n)
        assert abs(u @ (A @ v) - ex) <= 1e-12 * scale, (e1, e2, u @ (A @ v), ex)
        assert abs(v @ (A @ u) - ex) <= 1e-12 * scale


@pytest.mark.parametrize("p", [2, 3])
def test_face_kappa_placement_detects_unsorted_face_frame(p):
    """Face coefficients sampled at the points of an unsorted vertex triple
    (the same point set under the symmetric rule, another pairing of values
    with points) miss the closed form."""
    n = 2
    xyz, tets = synth.kuhn_cube_mesh(n, 0.0, 0)
    qp, _ = synth.tet_rule(2 * p)
    fp, _ = synth.tri_rule(2 * p)
    tri = canonical_faces(tets)
    kc = kappa_at(cell_points(xyz, tets, qp))
    wrong = kappa_at(face_points(xyz, tri[:, [1, 2, 0]], fp))
    xyz, tets, A, _ = _dg_half_box(p, n, kc, wrong)
    worst = 0.0
    for e1, e2 in half_box_pairs(p):
        u, v = half_box_vectors(xyz, tets, p, e1, e2)
        ex = half_box_expected(p, n, e1, e2)
        worst = max(worst, abs(u @ (A @ v) - ex) / max(1.0, abs(ex)))
    assert worst > 1e-6


def test_face_point_sets_agree_under_rotation():
    """The mutation above is a pure re-pairing: the rotated frame gives the
    same set of face points (symmetric rule), so only the pairing differs."""
    xyz, tets = synth.kuhn_cube_mesh(2, 0.0, 0)
    fp, _ = synth.tri_rule(6)
    tri = canonical_faces(tets)
    a = face_points(xyz, tri, fp)
    b = face_points(xyz, tri[:, [1, 2, 0]], fp)
    for f in range(0, tri.shape[0], 17):
        d = np.linalg.norm(a[f][:, None, :] - b[f][None, :, :], axis=2)
        assert d.min(axis=1).max() < 1e-14
        assert not np.allclose(a[f], b[f])
