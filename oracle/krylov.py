"""Krylov solvers (oracle; test infrastructure only).

* PCG for the interface problem with F̊ preconditioned by M̊_D^-1 (paper
  Sec. 3.2.3; tolerance tol_CG on the unpreconditioned relative residual
  ||r_k|| / ||r_0||, lambda_0 = 0).
* Right-preconditioned flexible GMRES (Saad 1993) for the saddle system (16)
  with the iFETI-DP block preconditioner (44) (Sec. 2.3: "GMRES for
  example"); flexible because the preconditioner contains an inner PCG
  stopped by tolerance and the nonlinear reduced solve (46).  x_0 = 0,
  relres = ||b - A x|| / ||b||.

Pins (tests/test_oracle_dd_rom.py): PCG equals a dense solve on SPD systems
and reports breakdown when p^T A p <= 0; FGMRES equals a dense solve and
converges in one iteration with the exact inverse as preconditioner.
"""
from __future__ import annotations

import numpy as np


class Breakdown(RuntimeError):
    pass


def pcg(apply_A, apply_M, b, tol=1e-11, maxit=1000):
    """Returns (x, iterations, relres history)."""
    x = np.zeros_like(b)
    r = b.copy()
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return x, 0, hist
    z = apply_M(r)
    p = z.copy()
    rho = r @ z
    it = 0
    while it < maxit:
        q = apply_A(p)
        pq = p @ q
        if not np.isfinite(pq) or pq <= 0.0:
            raise Breakdown(f"p^T A p = {pq} at iteration {it}")
        a = rho / pq
        x += a * p
        r -= a * q
        it += 1
        rel = np.linalg.norm(r) / r0
        hist.append(rel)
        if rel <= tol:
            break
        z = apply_M(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, it, hist


def fgmres(apply_A, apply_P, b, tol=1e-8, maxit=200):
    """Right-preconditioned flexible GMRES without restart.  Returns (x, its, history)."""
    n = b.size
    beta = np.linalg.norm(b)
    hist = [1.0]
    if beta == 0.0:
        return np.zeros_like(b), 0, hist
    V = [b / beta]
    Zs = []
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    it = 0
    for j in range(maxit):
        z = apply_P(V[j])
        Zs.append(z)
        w = apply_A(z)
        for i in range(j + 1):                  # modified Gram-Schmidt
            H[i, j] = w @ V[i]
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] != 0.0 else w)
        for i in range(j):                      # apply previous Givens rotations
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        it = j + 1
        hist.append(abs(g[j + 1]) / beta)
        if abs(g[j + 1]) / beta <= tol or H[j, j] == 0.0:
            break
    y = np.linalg.solve(np.triu(H[:it, :it]), g[:it])
    x = np.zeros(n)
    for i in range(it):
        x += y[i] * Zs[i]
    return x, it, hist
