"""Principal bank, coefficient systems and ROM local operators (oracle; test infrastructure only).

Principal cell k (cell sigma_k chosen by the greedy), with K = K^(sigma_k)
partitioned as in eq. (12) and r = (i, d):
  U_rp = K_rr^-1 K_rp                          eq. (29)
  U_rd = K_rr^-1 T_rd                          eq. (28)
  F_dd = T_dr K_rr^-1 T_rd                     eq. (27)
  S_pp = K_pp - K_pr K_rr^-1 K_rp              eq. (22)
  S_dd = K_dd - K_di K_ii^-1 K_id              eq. (30)  (= F_dd^-1, Sec. 3.1.1)
  K_rr^-1 (explicit, for the reduced solves of eq. (46a))

Per-cell coefficients (eqs. (40)-(42)), energy products taken with the cell's
own operator K^(s), as the paper writes them:
  A[i,j] = tr(U_rp^(i)T K_rr^(s) U_rp^(j)),  b[i] = tr(U_rp^(i)T K_rp^(s))
  M[i,j] = tr(U_rd^(i)T K_rr^(s) U_rd^(j)),  d[i] = tr(U_rd^(i)T T_rd) = tr(F_dd^(i))
  A pi = b,  M delta = d  (Cholesky; symmetric pseudo-inverse with relative
  eigenvalue cut 1e-13 if the Cholesky fails)
ROM local operators, eq. (43): Ů_rp = sum pi_k U_rp^(k),
  S̊_pp = sym(K̊_pp - K̊_rp^T Ů_rp), Ů_rd = sum delta_k U_rd^(k),
  F̊_dd = sum delta_k F_dd^(k), S̊_dd = sum alpha_k S_dd^(k),  sym(X) = (X+X^T)/2.
Coarse problem (Sec. 3.2.1): S̊_PP = sum_s A_p S̊_pp^(s) A_p^T, factored once
by a banded Cholesky; optionally (the approximative coarse solvers Sec. 3.2.1
allows) replaced by block Jacobi over consecutive blocks of B primal dofs.

Pins (tests/test_oracle_dd_rom.py): S_dd F_dd = I, K_rr U_rp = K_rp, S_pp of a
floating cell annihilates the corner values of rigid modes, pi = delta = e_i at
principal cells, ROM operators equal the exact ones on identical-cell lattices;
block-Jacobi coarse solve: exact for B >= nP, diagonal scaling for B = 1,
symmetric positive definite (tests/test_oracle_solve.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp

from .assembly import dense

EIG_CUT = 1e-13


def spd_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve SPD A x = b by Cholesky; pseudo-inverse fallback (relative cut 1e-13)."""
    try:
        c = sl.cho_factor(A, lower=True)
        if np.all(np.isfinite(c[0])):
            return sl.cho_solve(c, b)
    except (np.linalg.LinAlgError, ValueError):
        pass
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    keep = w > EIG_CUT * max(w.max(), 0.0)
    inv = np.where(keep, 1.0 / np.where(keep, w, 1.0), 0.0)
    return V @ (inv[:, None] * (V.T @ b)) if b.ndim == 2 else V @ (inv * (V.T @ b))


class PrincipalBank:
    def __init__(self, ref, dd, Kvals_principal: np.ndarray):
        self.K = Kvals_principal.shape[0]
        ir, ii, idd, ip = dd.idx_r, dd.idx_i, dd.idx_d, dd.idx_p
        ni = dd.n_i
        self.Krr, self.Krp, self.Kpp, self.Kinv = [], [], [], []
        self.Urp, self.Urd, self.Fdd, self.Spp, self.Sdd = [], [], [], [], []
        self.Krr_sparse = []
        for k in range(self.K):
            Kd = dense(ref, Kvals_principal[k])
            Krr = Kd[np.ix_(ir, ir)]
            Krp = Kd[np.ix_(ir, ip)]
            Kpp = Kd[np.ix_(ip, ip)]
            c = sl.cho_factor(Krr, lower=True)
            Kinv = sl.cho_solve(c, np.eye(dd.n_r))
            Urp = sl.cho_solve(c, Krp)
            Urd = Kinv[:, ni:]
            Fdd = Kinv[ni:, ni:]
            Spp = Kpp - Krp.T @ Urp
            Kii = Kd[np.ix_(ii, ii)]
            Kid = Kd[np.ix_(ii, idd)]
            Kdd = Kd[np.ix_(idd, idd)]
            Sdd = Kdd - Kid.T @ sl.cho_solve(sl.cho_factor(Kii, lower=True), Kid)
            self.Krr.append(Krr); self.Krp.append(Krp); self.Kpp.append(Kpp); self.Kinv.append(Kinv)
            self.Urp.append(Urp); self.Urd.append(Urd); self.Fdd.append(Fdd)
            self.Spp.append(Spp); self.Sdd.append(Sdd)
            self.Krr_sparse.append(sp.csr_matrix(Krr))
        stack = lambda xs: np.array(xs)
        self.Krr, self.Krp, self.Kpp, self.Kinv = map(stack, (self.Krr, self.Krp, self.Kpp, self.Kinv))
        self.Urp, self.Urd, self.Fdd, self.Spp, self.Sdd = map(stack, (self.Urp, self.Urd, self.Fdd,
                                                                      self.Spp, self.Sdd))
        self.W = self.Urp[:, ni:, :]          # T_dr U_rp^(k), (K, n_d, n_p)


def cell_blocks(ref, dd, vals: np.ndarray):
    """Sparse K_rr^(s) and K_rp^(s) of one cell from its pattern values."""
    K = sp.csr_matrix((vals, (ref.pat_rows, ref.pat_cols)), shape=(ref.n_dof, ref.n_dof))
    Kr = K[dd.idx_r]
    return Kr[:, dd.idx_r].tocsr(), Kr[:, dd.idx_p].tocsr()


def cell_coefficients(ref, dd, bank: PrincipalBank, Kvals: np.ndarray, cells=None):
    """pi^(s), delta^(s) of eq. (41) with the traces of eq. (42), shape (len(cells), K) each."""
    N = Kvals.shape[0]
    cells = np.arange(N) if cells is None else np.atleast_1d(cells)
    K = bank.K
    Urp = bank.Urp.transpose(1, 0, 2).reshape(dd.n_r, K * dd.n_p)        # [U_rp^(1) ... U_rp^(K)]
    Urd = bank.Urd.transpose(1, 0, 2).reshape(dd.n_r, K * dd.n_d)        # [U_rd^(1) ... U_rd^(K)]
    dvec = np.einsum("kdd->k", bank.Fdd)
    pi = np.zeros((cells.size, K))
    delta = np.zeros((cells.size, K))
    for t, s in enumerate(cells):
        Krr, Krp = cell_blocks(ref, dd, Kvals[s])
        KUp = (Krr @ Urp).reshape(dd.n_r, K, dd.n_p)
        KUd = (Krr @ Urd).reshape(dd.n_r, K, dd.n_d)
        A = np.einsum("rip,rjp->ij", bank.Urp.transpose(1, 0, 2), KUp)
        M = np.einsum("rid,rjd->ij", bank.Urd.transpose(1, 0, 2), KUd)
        b = np.einsum("irp,rp->i", bank.Urp, Krp.toarray())
        pi[t] = spd_solve(A, b)
        delta[t] = spd_solve(M, dvec)
    return pi, delta


def rom_Spp(bank: PrincipalBank, alpha: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """S̊_pp^(s) = sym(K̊_pp - K̊_rp^T Ů_rp) for every cell, (N, n_p, n_p) (eq. (43))."""
    Kpp = np.einsum("sm,mab->sab", alpha, bank.Kpp)
    Krp = np.einsum("sm,mrp->srp", alpha, bank.Krp)
    Urp = np.einsum("sk,krp->srp", pi, bank.Urp)
    X = Kpp - np.einsum("sra,srb->sab", Krp, Urp)
    return 0.5 * (X + X.transpose(0, 2, 1))


class BandedCholesky:
    """Cholesky factor of a symmetric banded matrix (LAPACK pbtrf), for S̊_PP^-1."""

    def __init__(self, S: sp.spmatrix):
        S = sp.csr_matrix(S)
        n = S.shape[0]
        coo = S.tocoo()
        bw = int(np.max(np.abs(coo.row - coo.col))) if coo.nnz else 0
        ab = np.zeros((bw + 1, n))
        low = coo.row >= coo.col
        ab[(coo.row - coo.col)[low], coo.col[low]] = coo.data[low]
        self.n, self.bw = n, bw
        self.cb = sl.cholesky_banded(ab, lower=True)

    def solve(self, b: np.ndarray) -> np.ndarray:
        if self.n == 0:
            return np.zeros_like(b)
        return sl.cho_solve_banded((self.cb, True), b)


class BlockJacobiCoarse:
    """Approximate coarse solve (Sec. 3.2.1 allows approximative coarse solvers in the inexact method):
    S̊_PP^-1 replaced by the inverse of its block-diagonal part over consecutive blocks of B primal dofs
    (dense Cholesky of each block).  Linear, symmetric positive definite and fixed, so the interface PCG
    stays valid; B >= nP is the exact solve, B = 1 is diagonal scaling."""

    def __init__(self, S: sp.spmatrix, B: int):
        S = sp.csr_matrix(S)
        self.n, self.B = S.shape[0], int(B)
        self.blocks = []
        for lo in range(0, self.n, self.B):
            hi = min(self.n, lo + self.B)
            self.blocks.append((lo, hi, sl.cho_factor(S[lo:hi, lo:hi].toarray(), lower=True)))

    def solve(self, b: np.ndarray) -> np.ndarray:
        x = np.zeros_like(b)
        for lo, hi, f in self.blocks:
            x[lo:hi] = sl.cho_solve(f, b[lo:hi])
        return x


def assemble_coarse(dd, Spp_cells: np.ndarray) -> sp.csr_matrix:
    """S̊_PP = sum_s A_p^(s) S̊_pp^(s) A_p^(s)T with Dirichlet corners removed."""
    N, n_p = dd.Ap.shape
    rows = np.repeat(dd.Ap[:, :, None], n_p, axis=2)
    cols = np.repeat(dd.Ap[:, None, :], n_p, axis=1)
    m = (rows >= 0) & (cols >= 0)
    return sp.csr_matrix((Spp_cells[m], (rows[m], cols[m])), shape=(dd.nP, dd.nP))
