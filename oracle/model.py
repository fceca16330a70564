"""ROM-based inexact FETI-DP, step by step (oracle; test infrastructure only).

Vector layouts (identical to the GPU library's, so results compare entry by entry):
  u   = (u_r^(1), ..., u_r^(N), u_P)   eq. (13); u_r^(s) in (i, d) order
  lam in R^L, rows in the order documented in oracle/dd.py

Operators (paper Sec. 3.2):
  apply_F        F̊ of eq. (48)
  apply_MD       M̊_D^-1 of eq. (49)
  apply_U/Ut     Ů and Ůᵀ, Algorithm 3 with the first term read as
                 sum_s B_d^(s) Ů_rd^(s)T v_r^(s) (eq. (28)); Ůᵀ by transposition
  apply_Kinv_rom K̊^-ROM of eq. (45) / Algorithm 2 with the reduced local
                 solves of eq. (46), the Gram matrix taken with the cell's own
                 K_rr^(s)
  apply_A        the true saddle operator of eq. (16)
  rom_local_solve the reduced local solve of eq. (46), or with local_iters > 1
                 the multi-preconditioned CG of Remark 6 (K̊^-MPCG)
  apply_MD_rom   M̊_D^-ROM of eq. (47): the Dirichlet preconditioner (30) with
                 each cell's interior solve replaced by the reduced solve of
                 eq. (46) on the interior block (principal K_ii^(σk)-1)
  apply_prec     the block preconditioner (44), Algorithm 1 (signs as printed:
                 y = -F̊^-pcg w̄ and x = K̊^-ROM v - Ůᵀ y); the interface block
                 -F̊^-pcg may instead be one application of M̊_D^-1 (49) or of
                 M̊_D^-ROM (47), the alternative of Sec. 3.2.3
  solve          right-preconditioned FGMRES on (16)

Parity: pinned by tests/test_oracle_*.py (brute-force dense operators, exact
FETI-DP on identical-cell lattices, direct Cholesky of the conforming
system, patch test).
"""
from __future__ import annotations

import time

import numpy as np
import scipy.linalg as sl

from .assembly import RefCell, cell_matrix_values, cell_loads, snapshots, dense
from .dd import DD
from .greedy import greedy
from .krylov import pcg, fgmres
from . import rom as romlib


def comb(coef: np.ndarray, mats: np.ndarray, X: np.ndarray) -> np.ndarray:
    """out_s = sum_k coef[s, k] mats[k] @ X_s  (coef (N,K), mats (K,m,n), X (N,n))."""
    out = np.zeros((X.shape[0], mats.shape[1]))
    for k in range(mats.shape[0]):
        out += coef[:, k, None] * (X @ mats[k].T)
    return out


def combT(coef: np.ndarray, mats: np.ndarray, X: np.ndarray) -> np.ndarray:
    """out_s = sum_k coef[s, k] mats[k]^T @ X_s  (mats (K,m,n), X (N,m))."""
    out = np.zeros((X.shape[0], mats.shape[2]))
    for k in range(mats.shape[0]):
        out += coef[:, k, None] * (X @ mats[k])
    return out


class Model:
    def __init__(self, problem, build_all_cells: bool = True):
        self.problem = problem
        self.ref = RefCell(problem.dim, problem.n_el, problem.degree)
        self.dd = DD(problem, self.ref)
        dd = self.dd
        self.N = problem.N
        self.nR = self.N * dd.n_r
        self.nU = self.nR + dd.nP
        self.L = dd.L
        self.Kvals = cell_matrix_values(self.ref, problem, np.arange(self.N)) if build_all_cells else None
        self.f_cells = cell_loads(self.ref, problem)            # (N, n_dof, nrhs)
        self.rhs_f = None
        self._Kii_inv = None
        self.local_iters = 1                 # > 1: multi-preconditioned local solves (Remark 6)
        if build_all_cells:
            self._build_rhs()

    # ----------------------------------------------------------- rhs (16)
    def _local_full(self, uR: np.ndarray, uP: np.ndarray, dirichlet_values: bool = False) -> np.ndarray:
        dd = self.dd
        u = np.zeros((self.N, self.ref.n_dof))
        u[:, dd.idx_r] = uR.reshape(self.N, dd.n_r)
        up = dd.restrict_primal(uP)
        if dirichlet_values:
            up = np.where(dd.p_is_dir, dd.up_dir, up)
        u[:, dd.idx_p] = up
        return u

    def cell_matvec(self, u_loc: np.ndarray, vals=None) -> np.ndarray:
        """y_s = K^(s) u_s on the shared pattern, (N, n_dof)."""
        vals = self.Kvals if vals is None else vals
        prod = vals * u_loc[:, self.ref.pat_cols]
        return np.add.reduceat(prod, self.ref.indptr[:-1], axis=1)

    def _build_rhs(self):
        dd = self.dd
        f = []
        # lifting of prescribed primal (corner) values on the Dirichlet boundary
        uD = np.zeros((self.N, self.ref.n_dof))
        uD[:, dd.idx_p] = np.where(dd.p_is_dir, dd.up_dir, 0.0)
        KuD = self.cell_matvec(uD)
        for r in range(self.problem.nrhs):
            fc = self.f_cells[:, :, r] - KuD
            fR = fc[:, dd.idx_r].reshape(-1)
            fP = dd.assemble_primal(fc[:, dd.idx_p])
            f.append(np.concatenate([fR, fP]))
        self.rhs_f = np.array(f)            # (nrhs, nU)
        self.rhs_d = dd.d.copy()            # same for every load case

    # ----------------------------------------------------------- setup
    def build_reduced_basis(self, n_principal=None, principal_in=None, tol_rb=1e-12):
        p = self.problem
        K = p.n_principal if n_principal is None else n_principal
        A = snapshots(self.ref, p, np.arange(self.N))
        g = greedy(A, K, tol=tol_rb, principal_in=principal_in)
        del A
        self.greedy_out = g
        self.sigma = g["sigma"]
        self.alpha = g["alpha"]
        self.bank = romlib.PrincipalBank(self.ref, self.dd, self.Kvals[self.sigma])
        self.pi, self.delta = romlib.cell_coefficients(self.ref, self.dd, self.bank, self.Kvals)
        self.Spp_cells = romlib.rom_Spp(self.bank, self.alpha, self.pi)
        self.SPP = romlib.assemble_coarse(self.dd, self.Spp_cells)
        self.coarse = romlib.BandedCholesky(self.SPP)
        self.coarse_approx = None
        return self.sigma

    def set_coarse_block(self, B: int):
        """B > 0: approximate coarse solve by block Jacobi over blocks of B primal dofs (Sec. 3.2.1);
        0: the exact banded Cholesky solve."""
        self.coarse_approx = romlib.BlockJacobiCoarse(self.SPP, B) if B > 0 else None

    def coarse_solve(self, z: np.ndarray) -> np.ndarray:
        if self.coarse_approx is not None:
            return self.coarse_approx.solve(z)
        return self.coarse.solve(z)

    # ----------------------------------------------------------- F̊ (48)
    def apply_F(self, lam: np.ndarray) -> np.ndarray:
        dd, b = self.dd, self.bank
        Lam = dd.gather(lam)                                          # B_d^T lam
        Y = comb(self.delta, b.Fdd, Lam)       # F̊_dd^(s) Lam_s
        c = combT(self.pi, b.W, Lam)            # (T_dr Ů_rp)^T Lam_s
        yP = self.coarse_solve(dd.assemble_primal(c))
        yp = dd.restrict_primal(yP)
        Y += comb(self.pi, b.W, yp)
        return dd.scatter(Y)

    # ----------------------------------------------------------- M̊_D^-1 (49)
    def apply_MD(self, r: np.ndarray) -> np.ndarray:
        dd, b = self.dd, self.bank
        Lam = dd.gather(r, weights=True)
        Y = comb(self.alpha, b.Sdd, Lam)
        return dd.scatter(Y, weights=True)

    # ----------------------------------------------------------- M̊_D^-ROM (47)
    def apply_MD_rom(self, r: np.ndarray) -> np.ndarray:
        """Eq. (47): sum_s D B_d^(s) S_dd^(s) B_d^(s)T D r as in (30), S_dd^(s) = K_dd - K_di K_ii^-1 K_id,
        with K_ii^(s)-1 w replaced by the reduced solve of eq. (46) on the interior block:
        R = [K_ii^(σk)-1 w]_k, x = R (Rᵀ K_ii^(s) R)^-1 Rᵀ w."""
        dd = self.dd
        ni = dd.n_i
        if self._Kii_inv is None:
            self._Kii_inv = []
            for s in self.sigma:
                Krr, _ = romlib.cell_blocks(self.ref, dd, self.Kvals[s])
                self._Kii_inv.append(np.linalg.inv(Krr[:ni, :ni].toarray()))
        Lam = dd.gather(r, weights=True)
        Y = np.zeros_like(Lam)
        for s in range(self.N):
            Krr, _ = romlib.cell_blocks(self.ref, dd, self.Kvals[s])
            Kii, Kid = Krr[:ni, :ni], Krr[:ni, ni:]
            w = Kid @ Lam[s]
            x = np.zeros(ni)
            if np.any(w):
                R = np.stack([Ki @ w for Ki in self._Kii_inv], axis=1)
                x = R @ romlib.spd_solve(R.T @ (Kii @ R), R.T @ w)
            Y[s] = Krr[ni:, ni:] @ Lam[s] - Krr[ni:, :ni] @ x
        return dd.scatter(Y, weights=True)

    # ----------------------------------------------------------- Ů, Ůᵀ (Alg. 3)
    def _split(self, v):
        return v[:self.nR].reshape(self.N, self.dd.n_r), v[self.nR:]

    def apply_U(self, v: np.ndarray) -> np.ndarray:
        dd, b = self.dd, self.bank
        vR, vP = self._split(v)
        t = combT(self.pi, b.Urp, vR)           # Ů_rp^T v_r
        zP = self.coarse_solve(vP - dd.assemble_primal(t))
        zp = dd.restrict_primal(zP)
        Y = combT(self.delta, b.Urd, vR) - comb(self.pi, b.W, zp)
        return dd.scatter(Y)

    def apply_Ut(self, y: np.ndarray) -> np.ndarray:
        dd, b = self.dd, self.bank
        Lam = dd.gather(y)
        c = combT(self.pi, b.W, Lam)
        xP = -self.coarse_solve(dd.assemble_primal(c))
        xp = dd.restrict_primal(xP)
        xR = comb(self.delta, b.Urd, Lam) - comb(self.pi, b.Urp, xp)
        return np.concatenate([xR.reshape(-1), xP])

    # ----------------------------------------------------------- K̊^-ROM (45)-(46)
    def rom_local_solve(self, vR: np.ndarray, iters=None) -> np.ndarray:
        """Eq. (46): x_r = R (R^T K_rr^(s) R)^-1 R^T v_r, R = [K_rr^(sigma_k)-1 v_r]_k, per cell.

        iters > 1 (default: self.local_iters): the multi-preconditioned CG of Remark 6 with the
        principal inverses as the preconditioners.  Iteration t takes Z = [K_rr^(σk)-1 r]_k, makes it
        K_rr^(s)-conjugate to every earlier block (Z -= P_j G_j^-1 (K_rr^(s) P_j)^T Z), and minimises the
        energy error over its span: x += Z a, r -= K_rr^(s) Z a, a = (Z^T K_rr^(s) Z)^-1 Z^T r.  The
        first iteration is eq. (46)."""
        iters = self.local_iters if iters is None else iters
        if iters > 1:
            return self._mpcg_local_solve(vR, iters)
        b = self.bank
        N, nr = vR.shape
        K = b.K
        R = np.stack([vR @ b.Kinv[k].T for k in range(K)], axis=2)   # (N, n_r, K)
        x = np.zeros_like(vR)
        for s in range(N):
            if not np.any(vR[s]):
                continue
            Krr, _ = romlib.cell_blocks(self.ref, self.dd, self.Kvals[s])
            G = R[s].T @ (Krr @ R[s])
            c = romlib.spd_solve(G, R[s].T @ vR[s])
            x[s] = R[s] @ c
        return x

    def _mpcg_local_solve(self, vR: np.ndarray, iters: int) -> np.ndarray:
        b = self.bank
        x = np.zeros_like(vR)
        for s in range(vR.shape[0]):
            if not np.any(vR[s]):
                continue
            Krr, _ = romlib.cell_blocks(self.ref, self.dd, self.Kvals[s])
            r = vR[s].copy()
            blocks = []
            for _ in range(iters):
                Z = np.stack([Ki @ r for Ki in b.Kinv], axis=1)
                for P, KP, G in blocks:
                    Z = Z - P @ romlib.spd_solve(G, KP.T @ Z)
                KZ = Krr @ Z
                G = Z.T @ KZ
                a = romlib.spd_solve(G, Z.T @ r)
                x[s] += Z @ a
                r -= KZ @ a
                blocks.append((Z, KZ, G))
        return x

    def apply_Kinv_rom(self, v: np.ndarray) -> np.ndarray:
        dd, b = self.dd, self.bank
        vR, vP = self._split(v)
        t = combT(self.pi, b.Urp, vR)
        xP = self.coarse_solve(vP - dd.assemble_primal(t))
        xR = self.rom_local_solve(vR)
        xp = dd.restrict_primal(xP)
        xR = xR - comb(self.pi, b.Urp, xp)
        return np.concatenate([xR.reshape(-1), xP])

    # ----------------------------------------------------------- true operator (16)
    def apply_K(self, u: np.ndarray) -> np.ndarray:
        dd = self.dd
        uR, uP = self._split(u)
        y = self.cell_matvec(self._local_full(uR, uP))
        return np.concatenate([y[:, dd.idx_r].reshape(-1), dd.assemble_primal(y[:, dd.idx_p])])

    def apply_Bt(self, lam: np.ndarray) -> np.ndarray:
        dd = self.dd
        out = np.zeros((self.N, dd.n_r))
        out[:, dd.n_i:] = dd.gather(lam)
        return np.concatenate([out.reshape(-1), np.zeros(dd.nP)])

    def apply_B(self, u: np.ndarray) -> np.ndarray:
        uR, _ = self._split(u)
        return self.dd.scatter(uR[:, self.dd.n_i:])

    def apply_A(self, x: np.ndarray) -> np.ndarray:
        u, lam = x[:self.nU], x[self.nU:]
        return np.concatenate([self.apply_K(u) + self.apply_Bt(lam), self.apply_B(u)])

    # ----------------------------------------------------------- interface PCG
    def solve_interface(self, rhs: np.ndarray, tol=1e-11, maxit=1000):
        return pcg(self.apply_F, self.apply_MD, rhs, tol=tol, maxit=maxit)

    # ----------------------------------------------------------- Alg. 1 / (44)
    def apply_prec(self, x: np.ndarray, inner_tol=1e-11, inner_maxit=1000, interface="pcg") -> np.ndarray:
        """interface: "pcg" F̊^-pcg (PCG on (48) with (49)), "md" one application of M̊_D^-1 (49),
        "mdrom" one application of M̊_D^-ROM (47)."""
        v, w = x[:self.nU], x[self.nU:]
        wbar = w - self.apply_U(v)
        if interface == "pcg":
            lam, its, _ = self.solve_interface(wbar, tol=inner_tol, maxit=inner_maxit)
        elif interface == "md":
            lam, its = self.apply_MD(wbar), 0
        elif interface == "mdrom":
            lam, its = self.apply_MD_rom(wbar), 0
        else:
            raise ValueError(f"unknown interface block {interface!r}")
        y = -lam
        self.inner_its.append(its)
        xo = self.apply_Kinv_rom(v) - self.apply_Ut(y)
        return np.concatenate([xo, y])

    def solve(self, rhs_index=0, tol=1e-8, maxit=100, inner_tol=1e-11, inner_maxit=1000, interface="pcg"):
        """FGMRES on (16).  Returns dict(u, lam, outer_its, inner_its, relres, time)."""
        self.inner_its = []
        b = np.concatenate([self.rhs_f[rhs_index], self.rhs_d])
        t0 = time.perf_counter()
        x, its, hist = fgmres(self.apply_A, lambda r: self.apply_prec(r, inner_tol, inner_maxit, interface), b,
                              tol=tol, maxit=maxit)
        t1 = time.perf_counter()
        res = np.linalg.norm(b - self.apply_A(x)) / np.linalg.norm(b)
        return dict(u=x[:self.nU], lam=x[self.nU:], outer_its=its, inner_its=list(self.inner_its),
                    relres=res, history=hist, time=t1 - t0)

    # ----------------------------------------------------------- helpers
    def full_cell_displacements(self, u: np.ndarray) -> np.ndarray:
        """Per-cell (N, n_dof) field with Dirichlet corner values filled in."""
        uR, uP = self._split(u)
        return self._local_full(uR, uP, dirichlet_values=True)
