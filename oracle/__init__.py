"""Plain FP64 CPU oracle for the matrix-free tetrahedral Galerkin operators.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports it, and this package
never imports the product path: the two share nothing but the seeded raw
inputs produced by ``synth``.

What it computes is the definition the matrix-free method reaches up to
rounding order: the assembled global sparse matrix of the weak forms of
eq. (2) (continuous Galerkin Poisson), eq. (3) (SIPG discontinuous Galerkin)
and the Helmholtz-type form of eq. (19) (stiffness plus a mass term), built
cell by cell from element matrices evaluated with the shared quadrature rule,
and then applied with a sparse matrix-vector product (the matrix-based
comparison of Sec. 3.2).

Modules
  basis     nodal Lagrange basis in Silvester's product form
  mesh      geometry, faces, DoF identities, Dirichlet constraints
  assemble  CG/DG assembly, coefficient gradients, load vector, row samples
  exact     exact rational brute force used to pin ``assemble``
  smoother  Jacobi-preconditioned Chebyshev smoother (Sec. 4.1)

Parity unpinned: nothing — every function here has at least one pin in
``tests/test_oracle_*.py`` (closed forms, exact rational arithmetic,
invariants); see the test docstrings for which pin covers which function.
"""
from .basis import nodes, eval_basis  # noqa: F401
from .mesh import Geometry, cg_dofs, find_faces  # noqa: F401
from .smoother import chebyshev  # noqa: F401
from .assemble import (  # noqa: F401
    assemble_cg, assemble_dg, cg_kappa_grad, dg_kappa_grad, load_vector, cg_rows, dg_rows, vector_operator,
    vector_kappa_grad,
)
