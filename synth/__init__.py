"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds no arithmetic of the operator itself: it only produces
meshes, coefficients and vectors.  Both sides receive the same raw arrays
(vertex coordinates, tetrahedron vertex lists, quadrature rules, coefficient
samples, vectors) and do everything else on their own.

Mesh recipe (the paper measures on a refined tetrahedral cube, Sec. 2.3 and
Sec. 4.1; the patient-specific lung mesh of Sec. 4.2 is not available, so a
seeded shuffle of cell and vertex order stands in for its "unordered" state):

* vertices on the lattice (i, j, k) in [0, N]^3, id = i + (N+1)(j + (N+1)k),
  coordinates h (i, j, k) with h = 1/N;
* every lattice cube c = i + N(j + N k) is split into 6 Kuhn tetrahedra,
  cell id 6c + m, where m indexes the axis permutation pi in
  ``itertools.permutations((0, 1, 2))`` order; the tet walks from the cube's
  lower corner along e_pi(0), e_pi(1), e_pi(2); odd permutations swap their
  last two vertices so that every cell is positively oriented;
* interior vertices are jittered: ``default_rng(seed).uniform(-a h, a h,
  (n_vert, 3))`` is drawn for all vertices in id order and the rows of
  boundary vertices are zeroed, so the domain stays the unit cube.

Curved cells (a stand-in for curvilinear meshes, Sec. 3.2): the straight
mesh is pushed through the smooth global map
    Phi(x, y, z) = (x + e y^2, y + e z^2, z + e x^2),
so the reference-to-physical map of cell K is Phi(X0 + J_K xi) and its
Jacobian at a reference point xi is grad Phi(X) J_K, X = X0 + J_K xi.
``curved_jacobians`` tabulates these per cell and rule point (the input a
curvilinear operator receives); ``curved_map`` applies Phi to points.

Random streams: ``default_rng([seed, s])`` with s = 1 cell coefficients,
2 input vector, 3 face coefficients, 4 right-hand side f, 5 finite-difference
picks, 9 shuffle permutations.
"""
import itertools

import numpy as np

STREAM_KAPPA_CELL = 1
STREAM_U = 2
STREAM_KAPPA_FACE = 3
STREAM_F = 4
STREAM_FD = 5
STREAM_SHUFFLE = 9


def _perm_parity(p):
    inv = 0
    for a in range(len(p)):
        for b in range(a + 1, len(p)):
            inv += p[a] > p[b]
    return inv % 2


def kuhn_cube_mesh(n, jitter=0.0, seed=0):
    """Unit cube split into n^3 cubes x 6 Kuhn tets.

    Returns (xyz float64 [n_vert, 3], tets int32 [n_cell, 4]).
    ``jitter`` is the maximum displacement in units of h.
    """
    n = int(n)
    m = n + 1
    h = 1.0 / n
    ii, jj, kk = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    # vertex id = i + m (j + m k): flatten with i fastest
    lat = np.stack([ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")], axis=1)
    xyz = lat.astype(np.float64) * h
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=(m ** 3, 3))
        on_bnd = np.any((lat == 0) | (lat == n), axis=1)
        d[on_bnd] = 0.0
        xyz = xyz + d
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    corner = np.stack([ci.ravel(order="F"), cj.ravel(order="F"), ck.ravel(order="F")], axis=1)
    eye = np.eye(3, dtype=np.int64)
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for mi, pi in enumerate(itertools.permutations((0, 1, 2))):
        v = [corner.copy()]
        for a in pi:
            v.append(v[-1] + eye[a])
        if _perm_parity(pi):
            v[2], v[3] = v[3], v[2]
        for s in range(4):
            tets[:, mi, s] = v[s][:, 0] + m * (v[s][:, 1] + m * v[s][:, 2])
    return xyz, tets.reshape(-1, 4).astype(np.int32)


def shuffle_mesh(xyz, tets, seed=0):
    """Seeded random relabelling of cells and vertices (stream 9)."""
    rng = np.random.default_rng([seed, STREAM_SHUFFLE])
    cperm = rng.permutation(tets.shape[0])
    vperm = rng.permutation(xyz.shape[0])
    new_id = np.empty_like(vperm)
    new_id[vperm] = np.arange(vperm.size)
    xyz2 = xyz[vperm]
    tets2 = new_id[tets[cperm]].astype(np.int32)
    return xyz2, tets2


def kuhn_counts(n):
    """Closed-form sizes of the Kuhn cube mesh."""
    return {
        "n_vert": (n + 1) ** 3,
        "n_cell": 6 * n ** 3,
        "n_bface": 12 * n ** 2,
        "n_iface": (24 * n ** 3 - 12 * n ** 2) // 2,
    }


def lognormal(seed, stream, shape, mu=0.0, sigma=0.5):
    rng = np.random.default_rng([seed, stream])
    return np.exp(mu + sigma * rng.standard_normal(shape))


def uniform(seed, stream, n, lo=-1.0, hi=1.0):
    rng = np.random.default_rng([seed, stream])
    return rng.uniform(lo, hi, size=n)


def fd_picks(seed, n_total, count):
    rng = np.random.default_rng([seed, STREAM_FD])
    return rng.choice(n_total, size=count, replace=False)


from .quadrature import tet_rule, tri_rule  # noqa: E402,F401


def five_tet_cube_mesh(n):
    """Unit cube split into n^3 cubes x 5 tetrahedra (the subdivision the paper
    uses for its unique-DoF counts, Sec. 2.3).  Neighbouring cubes alternate
    between the two mirror-image splits so that face diagonals match."""
    n = int(n)
    m = n + 1
    h = 1.0 / n
    ii, jj, kk = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    lat = np.stack([ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")], axis=1)
    xyz = lat.astype(np.float64) * h
    even = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    odd = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]

    def split(center, corners):
        tets = [list(center)]
        for c in corners:
            nb = [v for v in center if sum(abs(a - b) for a, b in zip(v, c)) == 1]
            tets.append([c] + nb)
        return tets

    out = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                local = split(even, odd) if (i + j + k) % 2 == 0 else split(odd, even)
                for t in local:
                    ids = [(i + a) + m * ((j + b) + m * (k + c)) for (a, b, c) in t]
                    P = xyz[ids]
                    if np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)) < 0:
                        ids[2], ids[3] = ids[3], ids[2]
                    out.append(ids)
    return xyz, np.array(out, dtype=np.int32)


def curved_map(x, eps):
    """Phi applied to points x [..., 3] (see the module docstring)."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([x[..., 0] + eps * x[..., 1] ** 2, x[..., 1] + eps * x[..., 2] ** 2,
                     x[..., 2] + eps * x[..., 0] ** 2], axis=-1)


def curved_jacobians(xyz, tets, qpts, eps):
    """[n_cell, n_q, 3, 3] Jacobians d x / d xi of Phi(X0 + J_K xi) at the
    rule points, row a = physical coordinate, column b = reference one."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(tets)]
    JK = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    P = X[:, None, 0, :] + np.einsum("eab,qb->eqa", JK, np.asarray(qpts, dtype=np.float64))
    x, y, z = P[..., 0], P[..., 1], P[..., 2]
    # D Phi = [[1, 2 eps y, 0], [0, 1, 2 eps z], [2 eps x, 0, 1]] times J_K,
    # row by row (the zero and unit entries written out)
    out = np.empty(P.shape[:2] + (3, 3))
    J0, J1, J2 = JK[:, None, 0, :], JK[:, None, 1, :], JK[:, None, 2, :]
    out[:, :, 0, :] = J0 + (2 * eps * y)[..., None] * J1
    out[:, :, 1, :] = J1 + (2 * eps * z)[..., None] * J2
    out[:, :, 2, :] = (2 * eps * x)[..., None] * J0 + J2
    return out
