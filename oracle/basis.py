"""Nodal Lagrange basis of degree p on the reference tetrahedron.

Reference cell: vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1); barycentric
coordinates l0 = 1 - x - y - z, l1 = x, l2 = y, l3 = z.  Nodes are the
equispaced points sum_i alpha_i X_i / p for multi-indices alpha in N^4 with
|alpha| = p, enumerated lexicographically.  The shape function of node alpha
is Silvester's product  prod_i prod_{k < alpha_i} (p l_i - k) / (k + 1),
which is 1 at its own node and 0 at every other node.  The paper's E matrix
(eq. (6)) is the table of reference gradients of these functions at the
quadrature points.
"""
import itertools

import numpy as np

# gradients of the barycentric coordinates with respect to (x, y, z)
GRAD_LAMBDA = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def nodes(p):
    """Multi-indices alpha (n_dof x 4), lexicographic, |alpha| = p."""
    return np.array([a for a in itertools.product(range(p + 1), repeat=4) if sum(a) == p], dtype=np.int64)


def node_coords(p):
    """Reference coordinates of the nodes (n_dof x 3)."""
    return nodes(p)[:, 1:].astype(np.float64) / p


def _factor(a, lam, p):
    """prod_{k<a} (p lam - k)/(k+1) and its derivative in lam (arrays)."""
    val = np.ones_like(lam)
    der = np.zeros_like(lam)
    for k in range(a):
        f = (p * lam - k) / (k + 1)
        der = der * f + val * (p / (k + 1))
        val = val * f
    return val, der


def eval_basis(p, pts):
    """Values [n_pts, n_dof] and reference gradients [n_pts, 3, n_dof]."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    lam = np.stack([1.0 - pts.sum(axis=1), pts[:, 0], pts[:, 1], pts[:, 2]], axis=1)
    al = nodes(p)
    n = pts.shape[0]
    nd = al.shape[0]
    val = np.ones((n, nd))
    dlam = np.zeros((n, 4, nd))  # d phi / d lambda_i, lambdas treated as independent
    for j, a in enumerate(al):
        fs = [_factor(int(a[i]), lam[:, i], p) for i in range(4)]
        v = np.ones(n)
        for i in range(4):
            v = v * fs[i][0]
        val[:, j] = v
        for i in range(4):
            d = fs[i][1]
            for k in range(4):
                if k != i:
                    d = d * fs[k][0]
            dlam[:, i, j] = d
    grad = np.einsum("nij,ik->nkj", dlam, GRAD_LAMBDA)
    return val, grad
