"""Krylov solvers (oracle; test infrastructure only).

* PCG for the interface problem with F̊ preconditioned by M̊_D^-1 (paper
  Sec. 3.2.3; tolerance tol_CG on the unpreconditioned relative residual
  ||r_k|| / ||r_0||, lambda_0 = 0).
* Right-preconditioned flexible GMRES (Saad 1993) for the saddle system (16)
  with the iFETI-DP block preconditioner (44) (Sec. 2.3: "GMRES for
  example"); flexible because the preconditioner contains an inner PCG
  stopped by tolerance and the nonlinear reduced solve (46).  x_0 = 0,
  relres = ||b - A x|| / ||b||.

* Block PCG for several right-hand sides at once (O'Leary's block conjugate
  gradient, the N4 variant for many load cases), in the breakdown-free form:
  the search block is orthonormalised at every step from the eigendecomposition
  of its Gram matrix and directions of relative eigenvalue <= drop are dropped,
  so right-hand sides that are (nearly) linearly dependent do not break the
  recurrence; the step and conjugation coefficients are small dense solves.

Pins (tests/test_oracle_dd_rom.py, tests/test_oracle_solve.py): PCG equals a
dense solve on SPD systems and reports breakdown when p^T A p <= 0; FGMRES
equals a dense solve and converges in one iteration with the exact inverse as
preconditioner; block PCG with one column follows PCG, reaches the dense
solution for rank-deficient blocks, and needs no more iterations than the
single-column solves.
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


def _orth(W, drop):
    """Orthonormal basis of the column space of W from the eigendecomposition of D W^T W D, D the
    inverse column norms (zero for zero columns), directions of relative eigenvalue <= drop removed.
    The scaling makes the drop test one of linear dependence: a load case whose residual is much smaller
    than the others' keeps its direction."""
    G = W.T @ W
    d = np.diag(G).copy()
    D = np.where(d > 0.0, 1.0 / np.sqrt(np.where(d > 0.0, d, 1.0)), 0.0)
    Gs = D[:, None] * G * D[None, :]
    lam, V = np.linalg.eigh(0.5 * (Gs + Gs.T))
    keep = lam > drop * max(lam.max(), 0.0)
    if not np.any(keep):
        return W[:, :0]
    return W @ (D[:, None] * V[:, keep] / np.sqrt(lam[keep]))


def block_pcg(apply_A, apply_M, B, tol=1e-11, maxit=1000, drop=1e-12):
    """Block PCG on A X = B (B: n x s), X_0 = 0, until ||r_j|| <= tol ||b_j|| for every column j.
    apply_A / apply_M act on one vector.  Returns (X, iterations, history of the largest relative
    residual)."""
    n, s = B.shape
    X = np.zeros_like(B)
    R = B.copy()
    nb = np.linalg.norm(B, axis=0)
    live = nb > 0.0
    hist = [1.0 if live.any() else 0.0]
    if not live.any():
        return X, 0, hist

    def block(fn, Y):
        return np.stack([fn(Y[:, j]) for j in range(Y.shape[1])], axis=1) if Y.shape[1] else Y.copy()

    P = _orth(block(apply_M, R), drop)
    it = 0
    while it < maxit and P.shape[1] > 0:
        Q = block(apply_A, P)
        PQ = P.T @ Q
        PQ = 0.5 * (PQ + PQ.T)
        if not np.all(np.isfinite(PQ)) or np.linalg.eigvalsh(PQ).min() <= 0.0:
            raise Breakdown(f"P^T A P not positive definite at iteration {it}")
        alpha = np.linalg.solve(PQ, P.T @ R)
        X += P @ alpha
        R -= Q @ alpha
        it += 1
        rel = np.where(live, np.linalg.norm(R, axis=0) / np.where(live, nb, 1.0), 0.0)
        hist.append(float(rel.max()))
        if rel.max() <= tol:
            break
        Z = block(apply_M, R)
        beta = -np.linalg.solve(PQ, Q.T @ Z)
        P = _orth(Z + P @ beta, drop)
    return X, it, hist


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
