"""Mesh quantities for the oracle: affine geometry, faces, DoF identities.

Geometry (Sec. 2.2, the paragraph after eq. (5)): each cell is the affine
image x = X0 + J x_hat of the reference tetrahedron with
J = [X1 - X0 | X2 - X0 | X3 - X0]; physical gradients are J^{-T} times
reference gradients and |det J| is the volume scale.

Continuous Galerkin DoF identity: node alpha of a cell is identified by the
sorted tuple of (global vertex id, alpha_i) over the vertices with
alpha_i > 0.  Two cells share a node exactly when these tuples agree, for any
vertex order inside the cells.  Global DoF order is the sorted order of the
keys.  A node is constrained (homogeneous Dirichlet) when all its support
vertices lie on one boundary face.

Faces: the triple of sorted global vertex ids.  Faces are ordered
lexicographically by that triple; a face with one cell is a boundary face.
"""
import numpy as np

from .basis import nodes


class Geometry:
    def __init__(self, xyz, tets):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        X = self.xyz[self.tets]  # [nc, 4, 3]
        self.X0 = X[:, 0, :]
        self.J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        self.detJ = np.linalg.det(self.J)
        self.Jinv = np.linalg.inv(self.J)
        self.vol = np.abs(self.detJ) / 6.0

    @property
    def n_cell(self):
        return self.tets.shape[0]


def find_faces(tets):
    """Faces as sorted vertex triples in lexicographic order.

    Returns dict with
      tri   [nf, 3] sorted vertex ids
      cells [nf, 2] adjacent cells (second = -1 on the boundary), first < second
      local [nf, 2] local face index (= index of the opposite vertex) in each cell
    """
    tets = np.asarray(tets, dtype=np.int64)
    nc = tets.shape[0]
    tri = np.empty((nc, 4, 3), dtype=np.int64)
    for f in range(4):
        others = [i for i in range(4) if i != f]
        tri[:, f, :] = tets[:, others]
    tri = np.sort(tri, axis=2).reshape(-1, 3)
    cell = np.repeat(np.arange(nc), 4)
    loc = np.tile(np.arange(4), nc)
    order = np.lexsort((cell, tri[:, 2], tri[:, 1], tri[:, 0]))
    tri, cell, loc = tri[order], cell[order], loc[order]
    new = np.ones(tri.shape[0], dtype=bool)
    new[1:] = np.any(tri[1:] != tri[:-1], axis=1)
    start = np.flatnonzero(new)
    counts = np.diff(np.append(start, tri.shape[0]))
    if np.any(counts > 2):
        raise ValueError("non-manifold mesh: a triangle is shared by more than two cells")
    nf = start.size
    cells = -np.ones((nf, 2), dtype=np.int64)
    local = -np.ones((nf, 2), dtype=np.int64)
    cells[:, 0] = cell[start]
    local[:, 0] = loc[start]
    two = counts == 2
    cells[two, 1] = cell[start[two] + 1]
    local[two, 1] = loc[start[two] + 1]
    return {"tri": tri[start], "cells": cells, "local": local}


def cg_dofs(xyz, tets, p):
    """Continuous DoF map.

    Returns dict with
      dofmap [nc, n_dof] global DoF of each local node (local order = lexicographic alpha)
      xyz    [n_dofs, 3] node coordinates
      constrained [n_dofs] bool (all support vertices on one boundary face)
    """
    tets = np.asarray(tets, dtype=np.int64)
    xyz = np.asarray(xyz, dtype=np.float64)
    al = nodes(p)
    nc, nd = tets.shape[0], al.shape[0]
    big = np.iinfo(np.int64).max
    # key of (cell, node): up to three (vertex id, multiplicity) pairs sorted by
    # vertex id, padded with (big, 0)
    vid = np.full((nc, nd, 4), big, dtype=np.int64)
    mul = np.zeros((nc, nd, 4), dtype=np.int64)
    for j, a in enumerate(al):
        for i in range(4):
            if a[i] > 0:
                vid[:, j, i] = tets[:, i]
                mul[:, j, i] = a[i]
    order = np.argsort(vid, axis=2, kind="stable")
    vid = np.take_along_axis(vid, order, axis=2)
    mul = np.take_along_axis(mul, order, axis=2)
    key = np.concatenate([vid[..., :3], mul[..., :3]], axis=2).reshape(-1, 6)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    dofmap = inv.reshape(nc, nd)
    coords = np.zeros((uniq.shape[0], 3))
    for s in range(3):
        ok = uniq[:, s] != big
        coords[ok] += uniq[ok, 3 + s][:, None] * xyz[uniq[ok, s]]
    coords /= p
    faces = find_faces(tets)
    bnd = faces["tri"][faces["cells"][:, 1] < 0]
    nv = np.int64(xyz.shape[0] + 1)
    bv = np.unique(bnd.ravel())
    be = np.unique(np.concatenate([bnd[:, 0] * nv + bnd[:, 1], bnd[:, 0] * nv + bnd[:, 2],
                                   bnd[:, 1] * nv + bnd[:, 2]]))
    bf = np.unique((bnd[:, 0] * nv + bnd[:, 1]) * nv + bnd[:, 2])
    nsup = np.sum(uniq[:, :3] != big, axis=1)
    constrained = np.zeros(uniq.shape[0], dtype=bool)
    one = nsup == 1
    constrained[one] = np.isin(uniq[one, 0], bv)
    two = nsup == 2
    constrained[two] = np.isin(uniq[two, 0] * nv + uniq[two, 1], be)
    three = nsup == 3
    constrained[three] = np.isin((uniq[three, 0] * nv + uniq[three, 1]) * nv + uniq[three, 2], bf)
    return {"dofmap": dofmap, "xyz": coords, "constrained": constrained}
