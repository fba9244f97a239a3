"""Shared set-up for the GPU parity tests: builds a mesh, the library
operator and the oracle matrix on the same seeded inputs, and maps library
DoFs to oracle DoFs through their coordinates (the two sides number DoFs
independently)."""
import numpy as np
from scipy.spatial import cKDTree

import oracle
import synth


def cg_map(op_xyz, oracle_xyz, h):
    tree = cKDTree(oracle_xyz)
    dist, idx = tree.query(op_xyz)
    assert dist.max() < 1e-9 * h, "library DoF without an oracle match"
    assert np.unique(idx).size == idx.size
    return idx


def dg_map(op_xyz, op_cell, xyz, tets, p):
    """Oracle index (cell * nd + j, j lexicographic) of every library DG DoF."""
    geo = oracle.Geometry(xyz, tets)
    xn = oracle.basis.node_coords(p)
    Xn = geo.X0[:, None, :] + np.einsum("eij,kj->eki", geo.J, xn)  # [nc, nd, 3]
    nd = xn.shape[0]
    cand = Xn[op_cell]                                         # [n_dofs, nd, 3]
    d = np.linalg.norm(cand - op_xyz[:, None, :], axis=2)
    j = np.argmin(d, axis=1)
    assert d[np.arange(j.size), j].max() < 1e-12
    idx = op_cell.astype(np.int64) * nd + j
    assert np.unique(idx).size == idx.size
    return idx


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def row_err(v, A, u, idx=None):
    """Largest entry-wise error of v against y = A u, each entry measured
    against its row scale sum_j |a_ij| |u_j| (so a wrong entry in a
    small-magnitude row is not hidden by the norm of the whole vector).
    idx maps the entries of v to rows of A (library -> oracle numbering).
    Rows with a zero scale must match exactly."""
    y = A @ u
    s = abs(A) @ np.abs(u)
    if idx is not None:
        y, s = y[idx], s[idx]
    d = np.abs(np.asarray(v, dtype=np.float64) - y)
    zero = s == 0
    if np.any(d[zero] != 0):
        return float("inf")
    return float(np.max(d[~zero] / s[~zero])) if np.any(~zero) else 0.0
