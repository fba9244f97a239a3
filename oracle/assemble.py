"""Assembly of the global FP64 sparse matrices, coefficient gradients and
load vectors, straight from the weak forms.

Continuous Galerkin (eq. (2), with a coefficient kappa per quadrature point
and an optional mass term sigma (u, v) as in the Helmholtz-type eq. (19),
the velocity step of the dual splitting in Sec. 4.2):

    A_e[i, j] = sum_q w_q |det J| ( kappa_{e,q} grad phi_i . grad phi_j
                                    + sigma phi_i phi_j )  at x_q,

with grad phi = J^{-T} grad_ref phi (Sec. 2.2).  A = sum_e G_e^T A_e G_e
(eq. (5)).  Curved cells (Sec. 3.2) use the Jacobian J_q of the
reference-to-physical map at each point instead of the affine J.  Homogeneous Dirichlet: constrained rows and columns are replaced
by the identity, the reading that a masked gather skips constrained DoFs
(Sec. 2.4, instruction scheduling) and the operator returns them unchanged.

SIPG discontinuous Galerkin (eq. (3), eq. (7)): the same cell matrices on
cell-local DoFs plus, for every interior face F = K- n K+ (K- has the smaller
cell id, n points out of K-), with [[v]] = v- - v+ and {{w}} = (w- + w+)/2:

    a_F(u, v) = sum_q omega_q kappa_{F,q} ( -{{d_n v}} [[u]] - [[v]] {{d_n u}}
                                            + tau_F [[u]] [[v]] ),
    tau_F = eta (p+1)^2 |F| / min(|K-|, |K+|).

The face points are x_q = a + s_q (b - a) + t_q (c - a) for the face's
vertices sorted by global id a < b < c, omega_q = w_q 2|F|.  Boundary faces
(the paper leaves them to "suitable modifications"): 'neumann' adds nothing;
'dirichlet' applies the mirror principle u+ = -u-, grad u+ = grad u-, i.e.
    sum_q omega_q kappa ( -u d_n v - v d_n u + 2 tau_F u v ),
    tau_F = eta (p+1)^2 |F| / |K|.
Each side evaluates its basis at the physical face points through its own
inverse affine map, so no orientation tables are involved.
"""
import numpy as np
import scipy.sparse as sp

from .basis import eval_basis, nodes
from .mesh import Geometry, cg_dofs, find_faces


def _point_geometry(geo, cells, nq, jac):
    """J^{-1} and |det J| at every rule point: [e, q, 3, 3] and [e, q].

    Straight-sided cells repeat the affine values; curved cells (Sec. 3.2)
    take the Jacobian of the reference-to-physical map at each point, given
    as jac [n_cell, n_q, 3, 3] with jac[e, q, a, b] = d x_a / d xi_b."""
    if jac is None:
        Jinv = np.repeat(geo.Jinv[cells][:, None], nq, axis=1)
        adet = np.repeat(np.abs(geo.detJ[cells])[:, None], nq, axis=1)
        return Jinv, adet
    Jq = np.asarray(jac, dtype=np.float64)[cells]
    return np.linalg.inv(Jq), np.abs(np.linalg.det(Jq))


def _cell_matrices(geo, cells, p, qpts, qw, kappa, sigma, jac=None):
    """Element matrices [len(cells), n_dof, n_dof] (stiffness with kappa + sigma*mass)."""
    phi, gref = eval_basis(p, qpts)  # [nq, nd], [nq, 3, nd]
    Jinv, adet = _point_geometry(geo, cells, qw.size, jac)
    B = np.einsum("eqji,qjk->eqik", Jinv, gref)  # J^{-T} grad_ref: [e, q, 3, nd]
    kap = np.ones((cells.size, qw.size)) if kappa is None else kappa[cells]
    s = qw[None, :] * adet * kap
    A = np.einsum("eq,eqik,eqil->ekl", s, B, B)
    if sigma:
        A = A + sigma * np.einsum("eq,qk,ql->ekl", qw[None, :] * adet, phi, phi)
    return A


def _chunks(n, size=20000):
    for s in range(0, n, size):
        yield np.arange(s, min(n, s + size))


def assemble_cg(xyz, tets, p, qpts, qw, kappa=None, sigma=0.0, dirichlet=False, dofs=None, jac=None):
    """Global CG matrix (CSR, FP64) and the DoF description from ``cg_dofs``.
    jac: per-point Jacobians of curved cells (see ``_point_geometry``); the
    DoF identities still come from the straight-sided vertex mesh."""
    geo = Geometry(xyz, tets)
    if np.any(geo.detJ <= 0):
        raise ValueError("oracle expects positively oriented cells")
    d = cg_dofs(xyz, tets, p) if dofs is None else dofs
    dm = d["dofmap"]
    n = d["xyz"].shape[0]
    rows, cols, vals = [], [], []
    for c in _chunks(geo.n_cell):
        Ae = _cell_matrices(geo, c, p, qpts, qw, kappa, sigma, jac)
        nd = dm.shape[1]
        rows.append(np.repeat(dm[c], nd, axis=1).ravel())
        cols.append(np.tile(dm[c], (1, nd)).ravel())
        vals.append(Ae.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sum_duplicates()
    if dirichlet:
        A = _apply_dirichlet(A, d["constrained"])
    return A, d


def _apply_dirichlet(A, constrained):
    keep = sp.diags((~constrained).astype(np.float64))
    A = keep @ A @ keep + sp.diags(constrained.astype(np.float64))
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    return A


def cg_kappa_grad(xyz, tets, p, qpts, qw, u, g, dofs=None, jac=None):
    """d(g^T A(kappa) u) / d kappa_{e,q} = w_q |det J| (grad u . grad g)(x_q)."""
    geo = Geometry(xyz, tets)
    d = cg_dofs(xyz, tets, p) if dofs is None else dofs
    dm = d["dofmap"]
    _, gref = eval_basis(p, qpts)
    out = np.empty((geo.n_cell, qw.size))
    for c in _chunks(geo.n_cell):
        Jinv, adet = _point_geometry(geo, c, qw.size, jac)
        B = np.einsum("eqji,qjk->eqik", Jinv, gref)
        gu = np.einsum("eqik,ek->eqi", B, u[dm[c]])
        gg = np.einsum("eqik,ek->eqi", B, g[dm[c]])
        out[c] = qw[None, :] * adet * np.sum(gu * gg, axis=2)
    return out


def load_vector(xyz, tets, p, qpts, qw, f=None, dirichlet=False, dofs=None, jac=None):
    """b_i = sum_e sum_q w_q |det J| f_{e,q} phi_i(x_q); zero on constrained rows."""
    geo = Geometry(xyz, tets)
    d = cg_dofs(xyz, tets, p) if dofs is None else dofs
    dm = d["dofmap"]
    phi, _ = eval_basis(p, qpts)
    fv = np.ones((geo.n_cell, qw.size)) if f is None else f
    _, adet = _point_geometry(geo, np.arange(geo.n_cell), qw.size, jac)
    loc = np.einsum("eq,qk->ek", qw[None, :] * adet * fv, phi)
    b = np.zeros(d["xyz"].shape[0])
    np.add.at(b, dm.ravel(), loc.ravel())
    if dirichlet:
        b[d["constrained"]] = 0.0
    return b


# ---------------------------------------------------------------------------
# discontinuous Galerkin

def _face_geometry(geo, faces, fidx):
    tri = faces["tri"][fidx]
    a, b, c = (geo.xyz[tri[:, k]] for k in range(3))
    area_vec = 0.5 * np.cross(b - a, c - a)
    area = np.linalg.norm(area_vec, axis=1)
    n = area_vec / area[:, None]
    c0 = faces["cells"][fidx, 0]
    opp = geo.xyz[geo.tets[c0, faces["local"][fidx, 0]]]
    flip = np.sum((opp - a) * n, axis=1) > 0
    n[flip] *= -1.0
    return a, b, c, area, n


def _side_eval(geo, cells, x, p):
    """Basis values [f, q, nd] and physical gradients [f, q, 3, nd] of ``cells`` at points x [f, q, 3]."""
    xh = np.einsum("fij,fqj->fqi", geo.Jinv[cells], x - geo.X0[cells][:, None, :])
    nf, nq = x.shape[:2]
    val, gref = eval_basis(p, xh.reshape(-1, 3))
    nd = val.shape[1]
    val = val.reshape(nf, nq, nd)
    gref = gref.reshape(nf, nq, 3, nd)
    grad = np.einsum("fji,fqjk->fqik", geo.Jinv[cells], gref)
    return val, grad


def dg_face_data(geo, faces, fidx, p, fpts, fw):
    a, b, c, area, n = _face_geometry(geo, faces, fidx)
    x = a[:, None, :] + fpts[None, :, 0:1] * (b - a)[:, None, :] + fpts[None, :, 1:2] * (c - a)[:, None, :]
    omega = fw[None, :] * 2.0 * area[:, None]
    return x, omega, area, n


def _dg_face_blocks(geo, faces, fidx, p, fpts, fw, kappa_face, eta):
    """Interior-face blocks [f, 2, 2, nd, nd] indexed (test side, trial side)."""
    x, omega, area, n = dg_face_data(geo, faces, fidx, p, fpts, fw)
    cm, cp = faces["cells"][fidx, 0], faces["cells"][fidx, 1]
    vm, gm = _side_eval(geo, cm, x, p)
    vp, gpl = _side_eval(geo, cp, x, p)
    dnm = np.einsum("fi,fqik->fqk", n, gm)
    dnp = np.einsum("fi,fqik->fqk", n, gpl)
    kap = np.ones_like(omega) if kappa_face is None else kappa_face[fidx]
    s = omega * kap
    tau = eta * (p + 1) ** 2 * area / np.minimum(geo.vol[cm], geo.vol[cp])
    jump = [vm, -vp]            # contribution of each side to [[.]]
    avg = [0.5 * dnm, 0.5 * dnp]  # contribution of each side to {{d_n .}}
    nd = vm.shape[2]
    out = np.empty((fidx.size, 2, 2, nd, nd))
    for si in range(2):
        for sj in range(2):
            out[:, si, sj] = (
                -np.einsum("fq,fqi,fqj->fij", s, avg[si], jump[sj])
                - np.einsum("fq,fqi,fqj->fij", s, jump[si], avg[sj])
                + np.einsum("fq,f,fqi,fqj->fij", s, tau, jump[si], jump[sj])
            )
    return out


def _dg_boundary_blocks(geo, faces, fidx, p, fpts, fw, kappa_face, eta):
    x, omega, area, n = dg_face_data(geo, faces, fidx, p, fpts, fw)
    cm = faces["cells"][fidx, 0]
    v, g = _side_eval(geo, cm, x, p)
    dn = np.einsum("fi,fqik->fqk", n, g)
    kap = np.ones_like(omega) if kappa_face is None else kappa_face[fidx]
    s = omega * kap
    tau = eta * (p + 1) ** 2 * area / geo.vol[cm]
    return (-np.einsum("fq,fqi,fqj->fij", s, v, dn) - np.einsum("fq,fqi,fqj->fij", s, dn, v)
            + 2.0 * np.einsum("fq,f,fqi,fqj->fij", s, tau, v, v))


def assemble_dg(xyz, tets, p, qpts, qw, fpts, fw, kappa_cell=None, kappa_face=None,
                eta=1.0, bc="dirichlet", sigma=0.0):
    """Global SIPG matrix (CSR, FP64); DoF (e, j) has index e*n_dof + j (j lexicographic)."""
    geo = Geometry(xyz, tets)
    if np.any(geo.detJ <= 0):
        raise ValueError("oracle expects positively oriented cells")
    faces = find_faces(tets)
    nd = nodes(p).shape[0]
    nc = geo.n_cell
    n = nc * nd
    loc = np.arange(nd)
    rows, cols, vals = [], [], []
    for c in _chunks(nc):
        Ae = _cell_matrices(geo, c, p, qpts, qw, kappa_cell, sigma)
        base = c[:, None] * nd + loc[None, :]
        rows.append(np.repeat(base, nd, axis=1).ravel())
        cols.append(np.tile(base, (1, nd)).ravel())
        vals.append(Ae.ravel())
    interior = np.flatnonzero(faces["cells"][:, 1] >= 0)
    for c in _chunks(interior.size, 10000):
        fidx = interior[c]
        blk = _dg_face_blocks(geo, faces, fidx, p, fpts, fw, kappa_face, eta)
        side = faces["cells"][fidx]
        for si in range(2):
            for sj in range(2):
                bi = side[:, si][:, None] * nd + loc[None, :]
                bj = side[:, sj][:, None] * nd + loc[None, :]
                rows.append(np.repeat(bi, nd, axis=1).ravel())
                cols.append(np.tile(bj, (1, nd)).ravel())
                vals.append(blk[:, si, sj].ravel())
    if bc == "dirichlet":
        boundary = np.flatnonzero(faces["cells"][:, 1] < 0)
        for c in _chunks(boundary.size, 10000):
            fidx = boundary[c]
            blk = _dg_boundary_blocks(geo, faces, fidx, p, fpts, fw, kappa_face, eta)
            bi = faces["cells"][fidx, 0][:, None] * nd + loc[None, :]
            rows.append(np.repeat(bi, nd, axis=1).ravel())
            cols.append(np.tile(bi, (1, nd)).ravel())
            vals.append(blk.ravel())
    elif bc != "neumann":
        raise ValueError(bc)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sum_duplicates()
    return A, faces


def dg_kappa_grad(xyz, tets, p, qpts, qw, fpts, fw, u, g, eta=1.0, bc="dirichlet"):
    """Gradients of g^T A u with respect to the cell and face coefficients."""
    geo = Geometry(xyz, tets)
    faces = find_faces(tets)
    nd = nodes(p).shape[0]
    U = u.reshape(-1, nd)
    Gv = g.reshape(-1, nd)
    _, gref = eval_basis(p, qpts)
    B = np.einsum("eji,qjk->eqik", geo.Jinv, gref)
    gu = np.einsum("eqik,ek->eqi", B, U)
    gg = np.einsum("eqik,ek->eqi", B, Gv)
    dkc = qw[None, :] * np.abs(geo.detJ)[:, None] * np.sum(gu * gg, axis=2)
    dkf = np.zeros((faces["tri"].shape[0], fw.size))
    interior = np.flatnonzero(faces["cells"][:, 1] >= 0)
    x, omega, area, n = dg_face_data(geo, faces, interior, p, fpts, fw)
    cm, cp = faces["cells"][interior, 0], faces["cells"][interior, 1]
    vm, gm = _side_eval(geo, cm, x, p)
    vp, gpl = _side_eval(geo, cp, x, p)
    tau = eta * (p + 1) ** 2 * area / np.minimum(geo.vol[cm], geo.vol[cp])

    def traces(V):
        val = np.einsum("fqk,fk->fq", vm, V[cm]) - np.einsum("fqk,fk->fq", vp, V[cp])
        avg = 0.5 * (np.einsum("fi,fqik,fk->fq", n, gm, V[cm]) + np.einsum("fi,fqik,fk->fq", n, gpl, V[cp]))
        return val, avg
    ju, au = traces(U)
    jg, ag = traces(Gv)
    dkf[interior] = omega * (-ag * ju - jg * au + tau[:, None] * ju * jg)
    if bc == "dirichlet":
        bnd = np.flatnonzero(faces["cells"][:, 1] < 0)
        x, omega, area, n = dg_face_data(geo, faces, bnd, p, fpts, fw)
        c0 = faces["cells"][bnd, 0]
        v, gr = _side_eval(geo, c0, x, p)
        tau = eta * (p + 1) ** 2 * area / geo.vol[c0]
        uu = np.einsum("fqk,fk->fq", v, U[c0])
        gv = np.einsum("fqk,fk->fq", v, Gv[c0])
        du = np.einsum("fi,fqik,fk->fq", n, gr, U[c0])
        dg = np.einsum("fi,fqik,fk->fq", n, gr, Gv[c0])
        dkf[bnd] = omega * (-gv * du - uu * dg + 2.0 * tau[:, None] * uu * gv)
    return dkc, dkf


# ---------------------------------------------------------------------------
# selected rows for large meshes

def cg_rows(xyz, tets, p, qpts, qw, cell_of_row, local_of_row, kappa=None, sigma=0.0, jac=None):
    """Rows of the CG matrix for DoFs given as (cell, local node) pairs.

    Returns a list of dicts {column key: value}, where a key is the sorted
    tuple of (global vertex id, multiplicity) identifying a continuous node
    (the DoF identity of ``mesh.cg_dofs``), plus the list of row keys.  Only
    the cells that contain the row's node are assembled.
    """
    tets = np.asarray(tets, dtype=np.int64)
    al = nodes(p)
    geo = Geometry(xyz, tets)

    def key(e, j):
        a = al[j]
        return tuple(sorted((int(tets[e, i]), int(a[i])) for i in range(4) if a[i] > 0))

    # vertex -> cells
    order = np.argsort(tets.ravel(), kind="stable")
    vsorted = tets.ravel()[order]
    starts = np.searchsorted(vsorted, np.arange(xyz.shape[0] + 1))
    out, rkeys = [], []
    for e0, j0 in zip(cell_of_row, local_of_row):
        rk = key(e0, j0)
        support = [v for v, _ in rk]
        cand = order[starts[support[0]]:starts[support[0] + 1]] // 4
        cells = np.array(sorted(c for c in set(cand.tolist()) if all(v in tets[c] for v in support)))
        Ae = _cell_matrices(geo, cells, p, qpts, qw, kappa, sigma, jac)
        row = {}
        for ci, c in enumerate(cells):
            jj = [j for j in range(al.shape[0]) if key(c, j) == rk]
            assert len(jj) == 1
            for k in range(al.shape[0]):
                ck = key(c, k)
                row[ck] = row.get(ck, 0.0) + Ae[ci, jj[0], k]
        out.append(row)
        rkeys.append(rk)
    return rkeys, out


def dg_rows(xyz, tets, p, qpts, qw, fpts, fw, cells_sel, kappa_cell=None, kappa_face=None,
            eta=1.0, bc="dirichlet"):
    """Rows of the SIPG matrix belonging to the cells ``cells_sel``.

    Returns (rows [len(cells_sel)*nd, n_cell*nd] as CSR) with the global DoF
    numbering of ``assemble_dg``.  Only the selected cells and their faces are
    assembled.
    """
    geo = Geometry(xyz, tets)
    faces = find_faces(tets)
    nd = nodes(p).shape[0]
    nc = geo.n_cell
    sel = np.asarray(cells_sel, dtype=np.int64)
    pos = -np.ones(nc, dtype=np.int64)
    pos[sel] = np.arange(sel.size)
    loc = np.arange(nd)
    rows, cols, vals = [], [], []
    Ae = _cell_matrices(geo, sel, p, qpts, qw, kappa_cell, 0.0)
    rows.append(np.repeat(pos[sel][:, None] * nd + loc, nd, axis=1).ravel())
    cols.append(np.tile(sel[:, None] * nd + loc, (1, nd)).ravel())
    vals.append(Ae.ravel())
    touch = np.flatnonzero(np.isin(faces["cells"][:, 0], sel) | np.isin(faces["cells"][:, 1], sel))
    interior = touch[faces["cells"][touch, 1] >= 0]
    if interior.size:
        blk = _dg_face_blocks(geo, faces, interior, p, fpts, fw, kappa_face, eta)
        side = faces["cells"][interior]
        for si in range(2):
            keep = pos[side[:, si]] >= 0
            for sj in range(2):
                bi = pos[side[keep, si]][:, None] * nd + loc
                bj = side[keep, sj][:, None] * nd + loc
                rows.append(np.repeat(bi, nd, axis=1).ravel())
                cols.append(np.tile(bj, (1, nd)).ravel())
                vals.append(blk[keep, si, sj].ravel())
    if bc == "dirichlet":
        bnd = touch[faces["cells"][touch, 1] < 0]
        if bnd.size:
            blk = _dg_boundary_blocks(geo, faces, bnd, p, fpts, fw, kappa_face, eta)
            c0 = faces["cells"][bnd, 0]
            bi = pos[c0][:, None] * nd + loc
            bj = c0[:, None] * nd + loc
            rows.append(np.repeat(bi, nd, axis=1).ravel())
            cols.append(np.tile(bj, (1, nd)).ravel())
            vals.append(blk.ravel())
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(sel.size * nd, nc * nd))
    R.sum_duplicates()
    return R


def vector_operator(A, n_components):
    """The operator of a vector-valued problem without coupling between the
    components (the vector Poisson/Helmholtz problem of Sec. 3.2 and the
    remark after it): one copy of the scalar operator per component, for
    vectors stored component by component, u = [u_1; u_2; ...; u_d].  With a
    Dirichlet scalar operator every component is constrained the same way."""
    return sp.block_diag([A] * n_components, format="csr")


def vector_kappa_grad(grad_fn, u, g, n_components, n_dofs):
    """d(g^T A(kappa) u)/d kappa for the vector operator: the sum over the
    components of the scalar gradient (grad_fn(u_c, g_c))."""
    return sum(grad_fn(u[c * n_dofs:(c + 1) * n_dofs], g[c * n_dofs:(c + 1) * n_dofs])
               for c in range(n_components))
