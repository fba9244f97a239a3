"""Loader for the committed simplex quadrature rules (reference tetrahedron
with vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1), weights summing to 1/6;
reference triangle (0,0), (1,0), (0,1), weights summing to 1/2)."""
import json
import os

import numpy as np

_RULES = None


def _load():
    global _RULES
    if _RULES is None:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "rules.json")) as f:
            _RULES = json.load(f)
    return _RULES


def _get(shape, degree):
    r = _load()[shape][str(int(degree))]
    pts = np.array([[float(v) for v in p] for p in r["points"]], dtype=np.float64)
    wts = np.array([float(v) for v in r["weights"]], dtype=np.float64)
    return pts, wts


def tet_rule(degree):
    """Symmetric rule exact for polynomials of total degree <= ``degree``."""
    return _get("tet", degree)


def tri_rule(degree):
    return _get("tri", degree)


def available():
    r = _load()
    return {k: sorted(int(d) for d in v) for k, v in r.items()}
