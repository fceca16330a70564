"""Plain definition of the solution: conforming FE system by direct Cholesky (oracle; tests only).

At convergence the ROM-based inexact FETI-DP solution (u, lam) of the saddle
system (16) satisfies B u = d, i.e. the torn field is continuous, and is the
Galerkin solution of (5a)-(5b) on the C0-glued lattice of cell spaces (6)
with the Dirichlet data (3c) and the tractions (3d).  This module assembles
that conforming system directly (cells glued at their shared control points),
eliminates the Dirichlet dofs, orders the unknowns by reverse Cuthill-McKee
and solves with a banded LAPACK Cholesky.  The multipliers follow from the
first block row of (16): B^T lam = f - K u, solved in the least-squares sense
(unique since B has full row rank).

Used as the reference for full solves on small lattices.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla

from .rom import BandedCholesky


def conforming_solve(model, rhs_index: int = 0):
    p, ref, dd = model.problem, model.ref, model.dd
    dim, N = p.dim, p.N
    cdof = (dd.gid[:, :, None] * dim + np.arange(dim)[None, None, :]).reshape(N, ref.n_dof)
    n_glob = int(np.prod(dd.Gshape)) * dim
    rows = cdof[:, ref.pat_rows].ravel()
    cols = cdof[:, ref.pat_cols].ravel()
    K = sp.csr_matrix((model.Kvals.ravel(), (rows, cols)), shape=(n_glob, n_glob))
    f = np.bincount(cdof.ravel(), weights=model.f_cells[:, :, rhs_index].ravel(), minlength=n_glob)
    # Dirichlet dofs and prescribed values u0(x) at their control points
    is_dir = np.zeros(n_glob, dtype=bool)
    uD = np.zeros(n_glob)
    dmask = np.repeat(dd.on_dir[:, :, None], dim, axis=2).reshape(N, ref.n_dof)
    is_dir[cdof[dmask]] = True
    X = p.ctrl.reshape(N * ref.n_ctrl, dim)
    u0 = (X @ p.u0_grad.T).reshape(N, ref.n_ctrl * dim)
    uD[cdof[dmask]] = u0[dmask]
    used = np.zeros(n_glob, dtype=bool)
    used[cdof.ravel()] = True
    free = np.nonzero(used & ~is_dir)[0]
    rhs = f - K @ uD
    Kff = K[free][:, free].tocsr()
    perm = csgraph.reverse_cuthill_mckee(Kff, symmetric_mode=True)
    Kp = Kff[perm][:, perm]
    chol = BandedCholesky(Kp)
    uf = np.empty(free.size)
    uf[perm] = chol.solve(rhs[free][perm])
    u = uD.copy()
    u[free] = uf
    # torn layout (13)
    u_loc = u[cdof]                                              # (N, n_dof)
    uR = u_loc[:, dd.idx_r].reshape(-1)
    uP = np.zeros(dd.nP)
    m = dd.Ap >= 0
    uP[dd.Ap[m]] = u_loc[:, dd.idx_p][m]
    ut = np.concatenate([uR, uP])
    # multipliers from the first block row of (16)
    res = model.rhs_f[rhs_index] - model.apply_K(ut)
    resR = res[:model.nR]
    BR = sp.csr_matrix((dd.ent_sign, (dd.ent_row, dd.ent_cell * dd.n_r + dd.n_i + dd.ent_slot)),
                       shape=(dd.L, model.nR))
    lam = spla.spsolve((BR @ BR.T).tocsc(), BR @ resR)
    return dict(u=ut, lam=np.asarray(lam), u_global=u, cdof=cdof)
