"""Pins that tie the oracle to facts fixed by the paper's problem and by
mathematics (none of them re-types the oracle's own formula):

P1  A 1 = 0 for the Neumann stiffness (any positive coefficient), CG and DG
P2  symmetry of the bilinear forms (eq. (2), eq. (3))
P3  exact integration of polynomial data: I_h(q1)^T K I_h(q2) = int grad q1 . grad q2
    and the same for the mass matrix, on the jittered unit cube
P4  mass: 1^T M_e 1 = |K_e|, 1^T M 1 = |Omega|
P5  positive semi-definiteness; constants are the only Neumann kernel
P6  linearity in the coefficient
P7  textbook P1 element matrices
P8  exact rational brute force on 6- and 48-tet meshes (oracle/exact.py)
P11 closed-form sizes; the paper's unique-DoFs-per-cell counts (golden file)
plus the DG penalty identity for piecewise constants and derivative pins for
the coefficient gradients (A is linear in kappa, so the derivative is the
matrix assembled with an indicator coefficient).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle.exact import assemble_exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mesh(n=3, jit=0.15, seed=0):
    return synth.kuhn_cube_mesh(n, jit, seed)


# ---------------------------------------------------------------- P1, P2, P5, P6

@pytest.mark.parametrize("p", [1, 2, 3])
def test_cg_neumann_kernel_and_symmetry(p):
    xyz, tets = _mesh()
    qp, qw = synth.tet_rule(2 * p)
    kap = synth.lognormal(0, 1, (tets.shape[0], qw.size), sigma=1.0)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap)
    rowabs = abs(A).sum(axis=1).max()
    assert np.abs(A @ np.ones(A.shape[0])).max() <= 1e-13 * rowabs
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = rng.standard_normal(A.shape[0])
        u -= u.mean()
        assert u @ (A @ u) > 0


def test_cg_linear_in_kappa():
    xyz, tets = _mesh(2)
    qp, qw = synth.tet_rule(6)
    k1 = synth.lognormal(0, 1, (tets.shape[0], qw.size))
    k2 = synth.lognormal(1, 1, (tets.shape[0], qw.size))
    A1, _ = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=k1)
    A2, _ = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=k2)
    A3, _ = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=2.0 * k1 - 0.5 * k2)
    assert abs(A3 - (2.0 * A1 - 0.5 * A2)).max() <= 1e-14 * abs(A3).max()


# ---------------------------------------------------------------- P3, P4

def _monomials(p):
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]


def _cube_int(e):
    return np.prod([1.0 / (k + 1) for k in e])


def _grad_dot_int(e1, e2):
    s = 0.0
    for k in range(3):
        if e1[k] == 0 or e2[k] == 0:
            continue
        f1 = list(e1)
        f2 = list(e2)
        f1[k] -= 1
        f2[k] -= 1
        s += e1[k] * e2[k] * _cube_int([a + b for a, b in zip(f1, f2)])
    return s


@pytest.mark.parametrize("p", [1, 2, 3])
def test_cg_polynomial_exactness(p):
    xyz, tets = _mesh(3, 0.15)
    qp, qw = synth.tet_rule(2 * p)
    K, d = oracle.assemble_cg(xyz, tets, p, qp, qw)
    M, _ = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=np.zeros((tets.shape[0], qw.size)), sigma=1.0, dofs=d)
    X = d["xyz"]
    mons = _monomials(p)
    I = {e: X[:, 0] ** e[0] * X[:, 1] ** e[1] * X[:, 2] ** e[2] for e in mons}
    for e1 in mons:
        for e2 in mons:
            k_ex = _grad_dot_int(e1, e2)
            m_ex = _cube_int([a + b for a, b in zip(e1, e2)])
            assert abs(I[e1] @ (K @ I[e2]) - k_ex) <= 1e-12 * max(1.0, abs(k_ex))
            assert abs(I[e1] @ (M @ I[e2]) - m_ex) <= 1e-12


@pytest.mark.parametrize("p", [2, 3])
def test_reduced_rule_stiffness(p):
    """Modified (reduced) cell integration, Sec. 3.3: on affine cells the
    stiffness integrand grad phi_i . grad phi_j has degree 2p - 2, so with a
    unit coefficient a rule exact to degree 2p - 2 gives the same matrix as the
    degree-2p rule, and the polynomial-exactness pin holds for it."""
    xyz, tets = _mesh(3, 0.15)
    qr, wr = synth.tet_rule(2 * p - 2)
    qf, wf = synth.tet_rule(2 * p)
    assert wr.size < wf.size
    Kr, d = oracle.assemble_cg(xyz, tets, p, qr, wr)
    Kf, _ = oracle.assemble_cg(xyz, tets, p, qf, wf, dofs=d)
    assert abs(Kr - Kf).max() <= 1e-13 * abs(Kf).max()
    X = d["xyz"]
    mons = _monomials(p)
    I = {e: X[:, 0] ** e[0] * X[:, 1] ** e[1] * X[:, 2] ** e[2] for e in mons}
    for e1 in mons:
        for e2 in mons:
            k_ex = _grad_dot_int(e1, e2)
            assert abs(I[e1] @ (Kr @ I[e2]) - k_ex) <= 1e-12 * max(1.0, abs(k_ex))


def test_mass_sums_and_volume():
    xyz, tets = _mesh(3, 0.15)
    qp, qw = synth.tet_rule(4)
    M, d = oracle.assemble_cg(xyz, tets, 2, qp, qw, kappa=np.zeros((tets.shape[0], qw.size)), sigma=1.0)
    assert abs(M.sum() - 1.0) < 1e-13
    # per cell: a one-cell "mesh" assembles exactly M_e
    geo = oracle.Geometry(xyz, tets)
    for e in (0, 17, 101):
        Me, _ = oracle.assemble_cg(xyz, tets[e:e + 1], 2, qp, qw, kappa=np.zeros((1, qw.size)), sigma=1.0)
        assert abs(Me.sum() - geo.vol[e]) < 1e-16


# ---------------------------------------------------------------- P7

def test_p1_textbook():
    xyz, tets = _mesh(2, 0.15)
    qp, qw = synth.tet_rule(2)
    geo = oracle.Geometry(xyz, tets)
    for e in (0, 5, 33):
        kap = np.full((1, qw.size), 2.5)
        A, d = oracle.assemble_cg(xyz, tets[e:e + 1], 1, qp, qw, kappa=kap, sigma=3.0)
        # node order of this one-cell mesh: keys sort by vertex id
        verts = np.sort(tets[e])
        X = xyz[verts]
        Jm = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
        Ji = np.linalg.inv(Jm)
        gl = np.vstack([-Ji.sum(axis=0), Ji])  # rows: grad lambda_i
        vol = abs(np.linalg.det(Jm)) / 6
        K = 2.5 * vol * gl @ gl.T
        M = vol * (np.ones((4, 4)) + np.eye(4)) / 20
        assert np.allclose(A.toarray(), K + 3.0 * M, rtol=1e-13, atol=1e-16)
        assert abs(vol - geo.vol[e]) < 1e-15 * vol


# ---------------------------------------------------------------- P8

def _rational_mesh(n, seed):
    xyz, tets = synth.kuhn_cube_mesh(n)
    m = n + 1
    rng = np.random.default_rng(seed)
    xq = []
    for vid in range(m ** 3):
        i, j, k = vid % m, (vid // m) % m, vid // (m * m)
        c = [Fraction(i, n), Fraction(j, n), Fraction(k, n)]
        if 0 < i < n and 0 < j < n and 0 < k < n and seed is not None:
            c = [ci + Fraction(int(rng.integers(-9, 10)), 64 * n) for ci in c]
        xq.append(c)
    xf = np.array([[float(v) for v in c] for c in xq])
    return xq, xf, tets


@pytest.mark.parametrize("n,p,seed,sigma", [(1, 1, None, 0), (1, 2, None, 1), (1, 3, None, 0),
                                            (2, 2, 5, 0), (2, 3, 5, 1), (3, 1, 6, 1), (3, 2, 6, 0)])
def test_exact_rational(n, p, seed, sigma):
    xq, xf, tets = _rational_mesh(n, seed)
    qp, qw = synth.tet_rule(2 * p)
    A, d = oracle.assemble_cg(xf, tets, p, qp, qw, sigma=float(sigma))
    E = assemble_exact(xq, tets, p, sigma=Fraction(sigma))
    lookup = {tuple(np.round(x * 2 ** 20).astype(np.int64)): i for i, x in enumerate(d["xyz"])}

    def idx(c):
        return lookup[tuple(int(round(float(v) * 2 ** 20)) for v in c)]
    dense = A.toarray()
    seen = np.zeros_like(dense, dtype=bool)
    scale = max(abs(float(v)) for v in E.values())
    for (ci, cj), v in E.items():
        i, j = idx(ci), idx(cj)
        assert abs(dense[i, j] - float(v)) <= 1e-15 * scale * 8
        seen[i, j] = True
    assert np.abs(dense[~seen]).max(initial=0.0) <= 1e-15 * scale


# ---------------------------------------------------------------- P11 + golden

def test_unique_dofs_per_cell_golden():
    """Paper's unique DoFs per cell on the 5-tet cube split: the N^3 coefficient
    of the DoF count (third finite difference of the cubic count) / 5."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "unique_dofs_per_cell.txt")) if not l.startswith("#")]
    for p_s, u_s, nd_s in rows:
        p = int(p_s)
        counts = []
        for n in (1, 2, 3, 4):
            xyz, tets = synth.five_tet_cube_mesh(n)
            d = oracle.cg_dofs(xyz, tets, p)
            counts.append(d["xyz"].shape[0])
            assert d["dofmap"].shape[1] == int(nd_s)
        lead = (counts[3] - 3 * counts[2] + 3 * counts[1] - counts[0]) / 6.0
        assert abs(lead / 5.0 - float(u_s)) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_kuhn_closed_form_counts(p):
    for n in (2, 3):
        xyz, tets = synth.kuhn_cube_mesh(n, 0.1)
        d = oracle.cg_dofs(xyz, tets, p)
        assert d["xyz"].shape[0] == (p * n + 1) ** 3
        assert d["constrained"].sum() == (p * n + 1) ** 3 - (p * n - 1) ** 3


# ---------------------------------------------------------------- gradients, load vector

def test_cg_kappa_grad_matches_indicator_assembly():
    xyz, tets = _mesh(2)
    qp, qw = synth.tet_rule(4)
    rng = np.random.default_rng(4)
    A0, d = oracle.assemble_cg(xyz, tets, 2, qp, qw)
    u = rng.uniform(-1, 1, A0.shape[0])
    g = rng.uniform(-1, 1, A0.shape[0])
    dk = oracle.cg_kappa_grad(xyz, tets, 2, qp, qw, u, g, dofs=d)
    for e, q in [(0, 0), (7, 3), (40, 13)]:
        ind = np.zeros((tets.shape[0], qw.size))
        ind[e, q] = 1.0
        Ai, _ = oracle.assemble_cg(xyz, tets, 2, qp, qw, kappa=ind, dofs=d)
        ref = g @ (Ai @ u)
        assert abs(dk[e, q] - ref) <= 1e-13 * max(1e-3, abs(ref))


def test_load_vector():
    xyz, tets = _mesh(3, 0.15)
    qp, qw = synth.tet_rule(6)
    b = oracle.load_vector(xyz, tets, 3, qp, qw)
    assert abs(b.sum() - 1.0) < 1e-13
    M, d = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=np.zeros((tets.shape[0], qw.size)), sigma=1.0)
    assert np.allclose(b, M @ np.ones(M.shape[0]), atol=1e-16)
    geo = oracle.Geometry(xyz, tets)
    xq = geo.X0[:, None, :] + np.einsum("eij,qj->eqi", geo.J, qp)
    bx = oracle.load_vector(xyz, tets, 3, qp, qw, f=xq[:, :, 0])
    assert abs(bx.sum() - 0.5) < 1e-13
    bd = oracle.load_vector(xyz, tets, 3, qp, qw, dirichlet=True)
    assert np.all(bd[d["constrained"]] == 0)


def test_dirichlet_rows_identity():
    xyz, tets = _mesh(2)
    qp, qw = synth.tet_rule(6)
    A, d = oracle.assemble_cg(xyz, tets, 3, qp, qw, dirichlet=True)
    c = d["constrained"]
    u = np.random.default_rng(5).standard_normal(A.shape[0])
    y = A @ u
    assert np.array_equal(y[c], u[c])
    u2 = u.copy()
    u2[c] = 0
    assert np.allclose(y[~c], (A @ u2)[~c], rtol=0, atol=1e-14)


def test_cg_rows_match_assembly():
    xyz, tets = _mesh(3)
    qp, qw = synth.tet_rule(6)
    kap = synth.lognormal(0, 1, (tets.shape[0], qw.size))
    A, d = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=kap)
    cells = np.array([0, 5, 77, 161])
    locs = np.array([0, 3, 11, 19])
    keys, rows = oracle.cg_rows(xyz, tets, 3, qp, qw, cells, locs, kappa=kap)
    for e, j, row in zip(cells, locs, rows):
        i = d["dofmap"][e, j]
        assert len(row) == A[i].nnz
        for ck, v in row.items():
            coord = sum(m * xyz[vv] for vv, m in ck) / 3
            jj = np.argmin(np.abs(d["xyz"] - coord).sum(axis=1))
            assert abs(A[i, jj] - v) <= 1e-15 * abs(A).max()


# ---------------------------------------------------------------- DG

def _dg(p=2, n=2, bc="neumann", kap=True):
    xyz, tets = _mesh(n)
    qp, qw = synth.tet_rule(2 * p)
    fp, fw = synth.tri_rule(2 * p)
    nf = oracle.find_faces(tets)["tri"].shape[0]
    kc = synth.lognormal(0, 1, (tets.shape[0], qw.size)) if kap else None
    kf = synth.lognormal(0, 3, (nf, fw.size)) if kap else None
    A, faces = oracle.assemble_dg(xyz, tets, p, qp, qw, fp, fw, kc, kf, bc=bc)
    return xyz, tets, A, faces, (qp, qw, fp, fw), kc, kf


@pytest.mark.parametrize("p", [1, 2, 3])
def test_dg_neumann_kernel_symmetric(p):
    _, _, A, _, _, _, _ = _dg(p)
    assert np.abs(A @ np.ones(A.shape[0])).max() <= 1e-12 * abs(A).sum(axis=1).max()
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_dg_polynomial_exactness(p):
    xyz, tets = _mesh(2, 0.15)
    qp, qw = synth.tet_rule(2 * p)
    fp, fw = synth.tri_rule(2 * p)
    A, _ = oracle.assemble_dg(xyz, tets, p, qp, qw, fp, fw, bc="neumann")
    geo = oracle.Geometry(xyz, tets)
    xn = oracle.basis.node_coords(p)
    X = (geo.X0[:, None, :] + np.einsum("eij,kj->eki", geo.J, xn)).reshape(-1, 3)
    mons = _monomials(p)
    for e1 in mons:
        for e2 in mons:
            q1 = X[:, 0] ** e1[0] * X[:, 1] ** e1[1] * X[:, 2] ** e1[2]
            q2 = X[:, 0] ** e2[0] * X[:, 1] ** e2[1] * X[:, 2] ** e2[2]
            assert abs(q1 @ (A @ q2) - _grad_dot_int(e1, e2)) <= 1e-12


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_dg_penalty_identity(bc):
    p = 2
    xyz, tets, A, faces, _, _, _ = _dg(p, bc=bc, kap=False)
    geo = oracle.Geometry(xyz, tets)
    c = np.random.default_rng(6).standard_normal(tets.shape[0])
    u = np.repeat(c, 10)
    ref = 0.0
    for f in range(faces["tri"].shape[0]):
        a, b, cc = xyz[faces["tri"][f]]
        area = 0.5 * np.linalg.norm(np.cross(b - a, cc - a))
        k0, k1 = faces["cells"][f]
        if k1 >= 0:
            tau = (p + 1) ** 2 * area / min(geo.vol[k0], geo.vol[k1])
            ref += tau * area * (c[k0] - c[k1]) ** 2
        elif bc == "dirichlet":
            tau = (p + 1) ** 2 * area / geo.vol[k0]
            ref += 2 * tau * area * c[k0] ** 2
    assert abs(u @ (A @ u) - ref) <= 1e-12 * ref


def test_dg_dirichlet_spd():
    _, _, A, _, _, _, _ = _dg(2, bc="dirichlet")
    w = np.linalg.eigvalsh(A.toarray())
    assert w.min() > 0


def test_dg_kappa_grad_matches_indicator_assembly():
    p = 2
    xyz, tets, A, faces, (qp, qw, fp, fw), kc, kf = _dg(p, bc="dirichlet")
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, A.shape[0])
    g = rng.uniform(-1, 1, A.shape[0])
    dkc, dkf = oracle.dg_kappa_grad(xyz, tets, p, qp, qw, fp, fw, u, g, bc="dirichlet")
    nf = faces["tri"].shape[0]
    for e, q in [(0, 1), (30, 5)]:
        ic = np.zeros_like(kc)
        ic[e, q] = 1
        Ai, _ = oracle.assemble_dg(xyz, tets, p, qp, qw, fp, fw, ic, np.zeros_like(kf), bc="dirichlet")
        assert abs(dkc[e, q] - g @ (Ai @ u)) <= 1e-13
    bnd = np.flatnonzero(faces["cells"][:, 1] < 0)[3]
    for f, q in [(0, 0), (11, 4), (int(bnd), 2)]:
        iff = np.zeros_like(kf)
        iff[f, q] = 1
        Ai, _ = oracle.assemble_dg(xyz, tets, p, qp, qw, fp, fw, np.zeros_like(kc), iff, bc="dirichlet")
        assert abs(dkf[f, q] - g @ (Ai @ u)) <= 1e-12


def test_dg_rows_match_assembly():
    p = 3
    xyz, tets, A, faces, (qp, qw, fp, fw), kc, kf = _dg(p, bc="dirichlet")
    sel = np.array([0, 9, 20, 47])
    R = oracle.dg_rows(xyz, tets, p, qp, qw, fp, fw, sel, kc, kf, bc="dirichlet")
    rows = (sel[:, None] * 20 + np.arange(20)).ravel()
    assert abs(R - A[rows]).max() <= 1e-15 * abs(A).max()


@pytest.mark.parametrize("p,bc", [(2, "neumann"), (3, "neumann"), (2, "dirichlet"), (3, "dirichlet")])
def test_dg_consistency_by_parts(p, bc):
    """Consistency of SIPG: for a polynomial u of degree p (no jumps) and any
    broken v, integration by parts gives
      neumann:   a(u, v) = (-lap u, v) + int_dOmega d_n u v
      dirichlet: a(u, v) = (-lap u, v) + int_dOmega (-u d_n v + 2 tau u v).
    This pins the sign and the 1/2 of the face consistency terms, which the
    polynomial and penalty pins cannot see."""
    from oracle.basis import eval_basis
    xyz, tets = _mesh(2, 0.15)
    qp, qw = synth.tet_rule(2 * p)
    fp, fw = synth.tri_rule(2 * p)
    A, faces = oracle.assemble_dg(xyz, tets, p, qp, qw, fp, fw, bc=bc)
    geo = oracle.Geometry(xyz, tets)
    nd = {2: 10, 3: 20}[p]

    def u_fn(x):
        return x[..., 0] ** 2 * x[..., 1] + 3 * x[..., 2] - 0.5 * x[..., 0] * x[..., 1] * x[..., 2] if p == 3 else \
            x[..., 0] ** 2 - x[..., 1] * x[..., 2] + 2 * x[..., 0]

    def grad_u(x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        if p == 3:
            return np.stack([2 * X * Y - 0.5 * Y * Z, X ** 2 - 0.5 * X * Z, 3 - 0.5 * X * Y], axis=-1)
        return np.stack([2 * X + 2, -Z, -Y], axis=-1)

    def mlap_u(x):
        return -2 * x[..., 1] if p == 3 else -2.0 * np.ones(x.shape[:-1])
    xn = oracle.basis.node_coords(p)
    Xn = geo.X0[:, None, :] + np.einsum("eij,kj->eki", geo.J, xn)
    uvec = u_fn(Xn).ravel()
    v = np.random.default_rng(8).uniform(-1, 1, tets.shape[0] * nd)
    V = v.reshape(-1, nd)
    phi, gref = eval_basis(p, qp)
    xq = geo.X0[:, None, :] + np.einsum("eij,qj->eqi", geo.J, qp)
    rhs = np.einsum("q,e,eq,qk,ek->", qw, np.abs(geo.detJ), mlap_u(xq), phi, V)
    bnd = np.flatnonzero(faces["cells"][:, 1] < 0)
    for f in bnd:
        a, b, c = xyz[faces["tri"][f]]
        nvec = np.cross(b - a, c - a)
        area = 0.5 * np.linalg.norm(nvec)
        nvec /= np.linalg.norm(nvec)
        k = faces["cells"][f, 0]
        if np.dot(xyz[tets[k]].mean(axis=0) - a, nvec) > 0:
            nvec = -nvec
        x = a + fp[:, 0:1] * (b - a) + fp[:, 1:2] * (c - a)
        om = fw * 2 * area
        xh = (geo.Jinv[k] @ (x - geo.X0[k]).T).T
        pv, pg = eval_basis(p, xh)
        vv = pv @ V[k]
        dnv = np.einsum("i,qik,k->q", geo.Jinv[k] @ nvec, pg, V[k])  # n . J^{-T} grad_ref
        if bc == "neumann":
            rhs += om @ (grad_u(x) @ nvec * vv)
        else:
            tau = (p + 1) ** 2 * area / geo.vol[k]
            rhs += om @ (-u_fn(x) * dnv + 2 * tau * u_fn(x) * vv)
    lhs = v @ (A @ uvec)
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(rhs))
