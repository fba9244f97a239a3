"""Exact rational brute force for the continuous Galerkin matrices.

Used only to pin ``assemble.assemble_cg``.  Everything here is computed with
``fractions.Fraction``: the nodal basis is expanded as a polynomial in the
barycentric coordinates, products of basis functions (and of their
barycentric derivatives) are expanded monomial by monomial, and every
monomial is integrated in closed form,

    int_K l0^b0 l1^b1 l2^b2 l3^b3 dx = |det J| b0! b1! b2! b3! / (|b| + 3)!.

Physical gradients follow from grad l_i, the rows of J^{-1} (i = 1, 2, 3)
and grad l0 = -(grad l1 + grad l2 + grad l3), all rational for rational
vertex coordinates.  No quadrature is involved, so agreement with the
quadrature-based oracle pins its basis, geometry, quadrature use and
assembly at once.

DoFs are identified by their exact rational coordinates (a mechanism
independent of the oracle's vertex-multiset keys).
"""
import itertools
from fractions import Fraction
from math import factorial


def _poly_mul(a, b):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return out


def _basis_polys(p):
    """Lagrange basis of degree p as polynomials in (l0, l1, l2, l3)."""
    al = [a for a in itertools.product(range(p + 1), repeat=4) if sum(a) == p]
    polys = []
    for a in al:
        poly = {(0, 0, 0, 0): Fraction(1)}
        for i in range(4):
            for k in range(a[i]):
                # (p l_i - k) / (k + 1)
                lin = {}
                e = [0, 0, 0, 0]
                e[i] = 1
                lin[tuple(e)] = Fraction(p, k + 1)
                if k:
                    lin[(0, 0, 0, 0)] = Fraction(-k, k + 1)
                poly = _poly_mul(poly, lin)
        polys.append(poly)
    return al, polys


def _dpoly(poly, i):
    out = {}
    for e, c in poly.items():
        if e[i] > 0:
            e2 = list(e)
            e2[i] -= 1
            out[tuple(e2)] = out.get(tuple(e2), 0) + c * e[i]
    return out


def _integral_ref(poly):
    """sum_b c_b b!/(|b|+3)!  (the integral divided by |det J|)."""
    s = Fraction(0)
    for e, c in poly.items():
        num = 1
        for k in e:
            num *= factorial(k)
        s += c * Fraction(num, factorial(sum(e) + 3))
    return s


def _reference_tables(p):
    al, polys = _basis_polys(p)
    nd = len(al)
    dpolys = [[_dpoly(ph, i) for i in range(4)] for ph in polys]
    S = [[[[None] * nd for _ in range(nd)] for _ in range(4)] for _ in range(4)]
    for a in range(4):
        for b in range(4):
            for i in range(nd):
                for j in range(nd):
                    S[a][b][i][j] = _integral_ref(_poly_mul(dpolys[i][a], dpolys[j][b]))
    Mref = [[_integral_ref(_poly_mul(polys[i], polys[j])) for j in range(nd)] for i in range(nd)]
    return al, S, Mref


def _inv3(J):
    a, b, c = J[0]
    d, e, f = J[1]
    g, h, i = J[2]
    det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g)
    inv = [[(e * i - f * h) / det, (c * h - b * i) / det, (b * f - c * e) / det],
           [(f * g - d * i) / det, (a * i - c * g) / det, (c * d - a * f) / det],
           [(d * h - e * g) / det, (b * g - a * h) / det, (a * e - b * d) / det]]
    return det, inv


def assemble_exact(xyz, tets, p, sigma=Fraction(0)):
    """Exact CG matrix as {(coord_i, coord_j): Fraction} with coords = rational node coordinates.

    ``xyz`` must hold Fractions.  kappa = 1.
    """
    al, S, Mref = _reference_tables(p)
    nd = len(al)
    A = {}
    for t in tets:
        X = [xyz[int(v)] for v in t]
        J = [[X[k + 1][r] - X[0][r] for k in range(3)] for r in range(3)]
        det, Jinv = _inv3(J)
        adet = abs(det)
        gl = [None] * 4
        for i in range(1, 4):
            gl[i] = Jinv[i - 1]
        gl[0] = [-(gl[1][r] + gl[2][r] + gl[3][r]) for r in range(3)]
        G = [[sum(gl[a][r] * gl[b][r] for r in range(3)) for b in range(4)] for a in range(4)]
        coords = [tuple(sum(Fraction(int(a[i])) * X[i][r] for i in range(4)) / p for r in range(3)) for a in al]
        for i in range(nd):
            for j in range(nd):
                v = Fraction(0)
                for a in range(4):
                    for b in range(4):
                        if G[a][b]:
                            v += G[a][b] * S[a][b][i][j]
                v = adet * (v + sigma * Mref[i][j])
                key = (coords[i], coords[j])
                A[key] = A.get(key, 0) + v
    return A
