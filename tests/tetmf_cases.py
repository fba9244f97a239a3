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
