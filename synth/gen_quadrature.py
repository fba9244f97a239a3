"""Generate the symmetric simplex quadrature rules used as problem data.

With a coefficient sampled per quadrature point the rule is part of the
problem statement, so it is generated once, committed as ``rules.json`` and
read by both sides.  The paper takes its rules from published symmetric
families (Sec. 2.3, the paragraph after eq. (9)); here each rule is found from
its orbit structure by solving the moment equations (least squares in double
precision, then Gauss-Newton refinement in 40-digit arithmetic) and accepted
only with positive weights and interior points.

Run:  python -m synth.gen_quadrature   (rewrites synth/rules.json)
"""
import itertools
import json
import math
import os

import mpmath as mp
import numpy as np
from scipy.optimize import least_squares

HERE = os.path.dirname(os.path.abspath(__file__))

# orbit kinds: (name, number of free parameters); each orbit also has a weight
TET_ORBITS = {"S4": 0, "S31": 1, "S22": 1, "S211": 2}
TRI_ORBITS = {"S3": 0, "S21": 1, "S111": 2}

STRUCTURES = {
    ("tet", 2): ["S31"],
    ("tet", 4): ["S31", "S31", "S22"],
    ("tet", 6): ["S31", "S31", "S31", "S211"],
    ("tri", 2): ["S21"],
    ("tri", 4): ["S21", "S21"],
    ("tri", 6): ["S21", "S21", "S111"],
}


def _unique_perms(vals):
    seen = []
    for p in itertools.permutations(range(len(vals))):
        t = tuple(vals[i] for i in p)
        key = tuple(t)
        if key not in [s[0] for s in seen]:
            seen.append((key, t))
    return [s[1] for s in seen]


def orbit_points(kind, params, mod=np):
    """Barycentric points of one orbit, in a fixed order."""
    one = mod.mpf(1) if mod is mp else 1.0
    if kind == "S4":
        return [(one / 4,) * 4]
    if kind == "S31":
        a = params[0]
        b = one - 3 * a
        return [tuple(b if i == k else a for i in range(4)) for k in range(4)]
    if kind == "S22":
        a = params[0]
        b = one / 2 - a
        out = []
        for pair in itertools.combinations(range(4), 2):
            out.append(tuple(a if i in pair else b for i in range(4)))
        return out
    if kind == "S211":
        a, b = params
        c = one - 2 * a - b
        out = []
        for pair in itertools.combinations(range(4), 2):
            rest = [i for i in range(4) if i not in pair]
            for bi in (0, 1):
                v = [None] * 4
                for i in pair:
                    v[i] = a
                v[rest[bi]] = b
                v[rest[1 - bi]] = c
                out.append(tuple(v))
        return out
    if kind == "S3":
        return [(one / 3,) * 3]
    if kind == "S21":
        a = params[0]
        b = one - 2 * a
        return [tuple(b if i == k else a for i in range(3)) for k in range(3)]
    if kind == "S111":
        a, b = params
        c = one - a - b
        out = []
        for p in itertools.permutations(range(3)):
            v = [None] * 3
            v[p[0]], v[p[1]], v[p[2]] = a, b, c
            out.append(tuple(v))
        return out
    raise ValueError(kind)


def monomials(dim, degree):
    return [e for e in itertools.product(range(degree + 1), repeat=dim) if sum(e) <= degree]


def exact_moment(e, mod=np):
    """Integral of x^e over the reference simplex (unit vertices)."""
    dim = len(e)
    num = 1
    for k in e:
        num *= math.factorial(k)
    den = math.factorial(sum(e) + dim)
    if mod is mp:
        return mp.mpf(num) / den
    return num / den


def unpack(shape, structure, x, mod=np):
    orbits = TET_ORBITS if shape == "tet" else TRI_ORBITS
    pts, wts = [], []
    i = 0
    for kind in structure:
        npar = orbits[kind]
        params = x[i:i + npar]
        w = x[i + npar]
        i += npar + 1
        op = orbit_points(kind, params, mod)
        pts.extend(op)
        wts.extend([w] * len(op))
    return pts, wts


def residual(shape, degree, structure, x, mod=np):
    pts, wts = unpack(shape, structure, x, mod)
    dim = 3 if shape == "tet" else 2
    res = []
    for e in monomials(dim, degree):
        s = 0
        for p, w in zip(pts, wts):
            term = w
            for d in range(dim):
                term = term * p[d + 1] ** e[d]
            s = s + term
        res.append(s - exact_moment(e, mod))
    return res


def residual_np(shape, degree, structure, x):
    pts, wts = unpack(shape, structure, x)
    P = np.array(pts, dtype=np.float64)[:, 1:]
    W = np.array(wts, dtype=np.float64)
    dim = P.shape[1]
    mons = monomials(dim, degree)
    E = np.array(mons)
    vals = np.prod(P[:, None, :] ** E[None, :, :], axis=2)
    exact = np.array([exact_moment(e) for e in mons])
    return W @ vals - exact


def solve(shape, degree, seed=0, tries=400, want=8):
    structure = STRUCTURES[(shape, degree)]
    orbits = TET_ORBITS if shape == "tet" else TRI_ORBITS
    nvar = sum(orbits[k] + 1 for k in structure)
    rng = np.random.default_rng(seed)
    vol = 1.0 / 6.0 if shape == "tet" else 0.5
    npts = len(unpack(shape, structure, np.ones(nvar) * 0.1)[0])
    best = None
    found = 0
    for _ in range(tries):
        x0 = []
        for kind in structure:
            x0.extend(rng.uniform(0.01, 0.45, orbits[kind]).tolist())
            x0.append(vol / npts * rng.uniform(0.3, 1.7))
        sol = least_squares(lambda x: residual_np(shape, degree, structure, x), np.array(x0),
                            xtol=1e-15, ftol=1e-15, gtol=1e-15)
        if sol.cost > 1e-26:
            continue
        pts, wts = unpack(shape, structure, sol.x)
        if min(wts) <= 0:
            continue
        if min(min(p) for p in pts) <= 1e-6:
            continue
        score = min(min(p) for p in pts)
        if best is None or score > best[0]:
            best = (score, sol.x)
        found += 1
        if found >= want:
            break
    if best is None:
        raise RuntimeError(f"no rule found for {shape} degree {degree}")
    return structure, refine(shape, degree, structure, best[1])


def refine(shape, degree, structure, x):
    """Gauss-Newton in 40-digit arithmetic on the (consistent) moment system."""
    mp.mp.dps = 40
    xv = mp.matrix([mp.mpf(float(v)) for v in x])
    n = len(x)
    for _ in range(8):
        r = mp.matrix(residual(shape, degree, structure, list(xv), mp))
        J = mp.matrix(len(r), n)
        for j in range(n):
            h = mp.mpf(10) ** -20
            xp = xv.copy()
            xp[j] += h
            rp = mp.matrix(residual(shape, degree, structure, list(xp), mp))
            for i in range(len(r)):
                J[i, j] = (rp[i] - r[i]) / h
        JT = J.T
        dx = mp.lu_solve(JT * J, JT * r)
        xv = xv - dx
    r = residual(shape, degree, structure, list(xv), mp)
    assert max(abs(v) for v in r) < mp.mpf(10) ** -30, "refinement did not converge"
    return list(xv)


def main():
    out = {"tet": {}, "tri": {}}
    for (shape, degree) in sorted(STRUCTURES):
        structure, x = solve(shape, degree)
        pts, wts = unpack(shape, structure, x, mp)
        dim = 3 if shape == "tet" else 2
        out[shape][str(degree)] = {
            "orbits": structure,
            "points": [[mp.nstr(p[d + 1], 20) for d in range(dim)] for p in pts],
            "weights": [mp.nstr(w, 20) for w in wts],
        }
        print(shape, degree, len(wts), "points")
    with open(os.path.join(HERE, "rules.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
