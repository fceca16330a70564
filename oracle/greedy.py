"""Greedy selection of the principal cells (oracle; test infrastructure only).

Paper Sec. 4.2.2, Algorithm 4 (a truncated Gram-Schmidt process on the
normalised snapshots) and eqs. (55)-(56):

  Delta_0^(s) = A^(s) / ||A^(s)||_2
  for i = 1, 2, ...:
      sigma_i  = argmax_s ||Delta_{i-1}^(s)||_inf
      zeta_i   = Delta_{i-1}^(sigma_i) / ||Delta_{i-1}^(sigma_i)||_2
      beta_i^(s) = Delta_{i-1}^(s) . zeta_i
      Delta_i^(s) = Delta_{i-1}^(s) - beta_i^(s) zeta_i
      stop when max_s ||Delta_i^(s)||_inf <= tol or i = n_principal
  Å^(s) = ||A^(s)|| Z beta^(s) = [A^(sigma_1) ... A^(sigma_K)] alpha^(s)    (56)

The snapshot A^(s) is the pulled-back material tensor at all quadrature
points, so the cell stiffness is exactly linear in it and the same alpha
gives K̃^(s) = sum_k alpha_k K^(sigma_k) (eq. (38)).  Since ||A|| Z^T A^(sigma_j)
is upper triangular in (i, j), alpha^(s) solves that triangular system with
right-hand side ||A^(s)|| beta^(s).

Ties in the argmax: the smallest cell index among those within a relative
1e-12 of the maximum.

Pins (tests/test_oracle_dd_rom.py): Z^T Z = I, non-increasing residual,
interpolation alpha^(sigma_i) = e_i (eq. (55)), exact recovery (zero residual)
after m picks on lattices with exactly m distinct cells.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

TIE_RTOL = 1e-12


def greedy(A: np.ndarray, n_principal: int, tol: float = 1e-12, principal_in=None):
    """Run Algorithm 4 on snapshots A (N, n).  Returns dict with sigma, alpha, ..."""
    N = A.shape[0]
    if principal_in is not None:
        n_principal = len(principal_in)
    norms = np.linalg.norm(A, axis=1)
    Delta = A / norms[:, None]
    sigma, Z, beta, resid = [], [], [], []
    for i in range(n_principal):
        inf = np.abs(Delta).max(axis=1)
        if principal_in is not None:
            s = int(principal_in[i])
        else:
            m = inf.max()
            if m <= tol:
                break
            s = int(np.nonzero(inf >= m * (1.0 - TIE_RTOL))[0].min())
        z = Delta[s] / np.linalg.norm(Delta[s])
        b = Delta @ z
        Delta = Delta - b[:, None] * z[None, :]
        sigma.append(s)
        Z.append(z)
        beta.append(b)
        resid.append(np.abs(Delta).max(axis=1).max())
    K = len(sigma)
    Z = np.array(Z).T                         # (n, K)
    beta = np.array(beta).T                   # (N, K)
    sigma = np.array(sigma, dtype=np.int64)
    # upper-triangular U[i, j] = ||A^(sigma_j)|| beta_i^(sigma_j), i <= j
    U = np.triu((norms[sigma][None, :] * beta[sigma].T))
    rhs = (norms[:, None] * beta).T           # (K, N)
    alpha = sl.solve_triangular(U, rhs, lower=False).T   # (N, K)
    return dict(sigma=sigma, alpha=alpha, Z=Z, beta=beta, norms=norms, residuals=np.array(resid),
                U=U)
