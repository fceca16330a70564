"""B-spline basis and Gauss quadrature (oracle; test infrastructure only).

Every cell space is spanned by the same reference functions N_i pushed forward
by the cell map (paper Sec. 2.2.1, eq. (6)).  The reference functions here are
tensor products of univariate B-splines of degree p on an open uniform knot
vector, evaluated with the Cox-de Boor recursion.

Pins: partition of unity, linear precision with Greville abscissae, derivative
against central differences (tests/test_oracle_assembly.py).
"""
from __future__ import annotations

import numpy as np


def bspline_basis(knots: np.ndarray, p: int, x: np.ndarray):
    """All univariate B-splines of degree p and their first derivatives at x.

    Cox-de Boor: N_{i,0} = 1 on [t_i, t_{i+1}) (the last non-empty span is
    closed on the right), N_{i,q} = (x-t_i)/(t_{i+q}-t_i) N_{i,q-1}
    + (t_{i+q+1}-x)/(t_{i+q+1}-t_{i+1}) N_{i+1,q-1}; the derivative is
    N'_{i,p} = p/(t_{i+p}-t_i) N_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}.
    Returns (values, derivatives), each of shape (len(x), n) with
    n = len(knots) - p - 1.
    """
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = t.size - 1
    # degree 0
    N = np.zeros((x.size, m))
    for i in range(m):
        if t[i] < t[i + 1]:
            inside = (x >= t[i]) & (x < t[i + 1])
            N[:, i] = inside
    # right end: x == last knot belongs to the last non-empty span
    last = max(i for i in range(m) if t[i] < t[i + 1])
    N[x == t[-1], :] = 0.0
    N[x == t[-1], last] = 1.0
    prev = N
    for q in range(1, p + 1):
        cur = np.zeros((x.size, m - q))
        for i in range(m - q):
            d1 = t[i + q] - t[i]
            d2 = t[i + q + 1] - t[i + 1]
            a = (x - t[i]) / d1 * prev[:, i] if d1 > 0 else 0.0
            b = (t[i + q + 1] - x) / d2 * prev[:, i + 1] if d2 > 0 else 0.0
            cur[:, i] = a + b
        if q == p:
            lower = prev  # degree p-1
        prev = cur
    vals = prev
    n = t.size - p - 1
    der = np.zeros((x.size, n))
    if p > 0:
        for i in range(n):
            d1 = t[i + p] - t[i]
            d2 = t[i + p + 1] - t[i + 1]
            a = p / d1 * lower[:, i] if d1 > 0 else 0.0
            b = p / d2 * lower[:, i + 1] if d2 > 0 else 0.0
            der[:, i] = a - b
    return vals, der


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre rule mapped to [0,1] (library primitive)."""
    xg, wg = np.polynomial.legendre.leggauss(n)
    return 0.5 * (xg + 1.0), 0.5 * wg
