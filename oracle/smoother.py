"""Jacobi-preconditioned Chebyshev smoother on an assembled matrix (test
infrastructure, like the rest of this package).

Sec. 4.1 smooths every multigrid level with a Chebyshev iteration
preconditioned by the point Jacobi diagonal (five pre- and five
post-smoothing steps).  This is the classical three-term Chebyshev
acceleration for an operator whose preconditioned spectrum lies in
[lambda_min, lambda_max], written out step by step with dense/sparse
numpy products in FP64:

    theta = (lambda_max + lambda_min) / 2,  delta = (lambda_max - lambda_min) / 2
    r_0 = b - A x_0,  d_0 = D^-1 r_0 / theta,  x_1 = x_0 + d_0,  rho_0 = delta / theta
    for k = 1, ..., degree - 1:
        r_k = b - A x_k
        rho_k = 1 / (2 theta / delta - rho_{k-1})
        d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D^-1 r_k
        x_{k+1} = x_k + d_k

After degree steps the error x* - x is multiplied by
p(D^-1 A), p(t) = T_degree((theta - t) / delta) / T_degree(theta / delta),
the pin used by the tests.
"""
import numpy as np


def chebyshev(A, inv_diag, b, x0, degree, lambda_min, lambda_max):
    """x after `degree` Chebyshev-Jacobi steps from x0 (x0 None: zero)."""
    theta = 0.5 * (lambda_max + lambda_min)
    delta = 0.5 * (lambda_max - lambda_min)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    d = inv_diag * r / theta
    x = x + d
    rho_prev = delta / theta
    for _ in range(1, degree):
        r = b - A @ x
        rho = 1.0 / (2.0 * theta / delta - rho_prev)
        d = rho * rho_prev * d + (2.0 * rho / delta) * (inv_diag * r)
        x = x + d
        rho_prev = rho
    return x
