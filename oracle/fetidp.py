"""Exact (standard) FETI-DP on small lattices (oracle; test infrastructure only).

Paper Sec. 2.2.4: every local K_rr^(s) is factored; the interface operator is
F = B_R K_RR^-1 B_R^T + B_R K_RR^-1 K_RP S_PP^-1 K_PR K_RR^-1 B_R^T (eq. (24))
with S_PP assembled from the exact local primal Schur complements (22), the
right-hand side d̄ of eq. (25), the Dirichlet preconditioner (30), and the
displacements recovered by eqs. (21) then (20).  This is the comparator the
paper reports beside its ROM solver ("Loc. It." equality) and the limit the
ROM operators must reach when the reduced basis is exact.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from .assembly import dense
from .krylov import pcg
from .rom import BandedCholesky, assemble_coarse


class ExactFETIDP:
    def __init__(self, model):
        self.m = model
        dd, ref = model.dd, model.ref
        N = model.N
        ir, ii, idd, ip = dd.idx_r, dd.idx_i, dd.idx_d, dd.idx_p
        ni = dd.n_i
        self.fac, self.Urp, self.Fdd, self.Sdd, Spp = [], [], [], [], []
        self.Krp = []
        for s in range(N):
            Kd = dense(ref, model.Kvals[s])
            Krr = Kd[np.ix_(ir, ir)]
            Krp = Kd[np.ix_(ir, ip)]
            c = sl.cho_factor(Krr, lower=True)
            Urp = sl.cho_solve(c, Krp)
            T = np.zeros((dd.n_r, dd.n_d))
            T[ni:, :] = np.eye(dd.n_d)
            self.fac.append(c)
            self.Krp.append(Krp)
            self.Urp.append(Urp)
            self.Fdd.append(sl.cho_solve(c, T)[ni:, :])
            Kii = Kd[np.ix_(ii, ii)]
            Kid = Kd[np.ix_(ii, idd)]
            self.Sdd.append(Kd[np.ix_(idd, idd)] - Kid.T @ sl.cho_solve(sl.cho_factor(Kii, lower=True), Kid))
            Spp.append(Kd[np.ix_(ip, ip)] - Krp.T @ Urp)
        self.Spp = np.array(Spp)
        self.SPP = assemble_coarse(dd, self.Spp)
        self.coarse = BandedCholesky(self.SPP)

    def KRR_solve(self, vR):
        return np.array([sl.cho_solve(self.fac[s], vR[s]) for s in range(self.m.N)])

    def apply_F(self, lam):
        dd = self.m.dd
        Lam = dd.gather(lam)
        Y = np.array([self.Fdd[s] @ Lam[s] for s in range(self.m.N)])
        c = np.array([self.Urp[s][dd.n_i:].T @ Lam[s] for s in range(self.m.N)])
        yp = dd.restrict_primal(self.coarse.solve(dd.assemble_primal(c)))
        Y += np.array([self.Urp[s][dd.n_i:] @ yp[s] for s in range(self.m.N)])
        return dd.scatter(Y)

    def apply_MD(self, r):
        dd = self.m.dd
        Lam = dd.gather(r, weights=True)
        Y = np.array([self.Sdd[s] @ Lam[s] for s in range(self.m.N)])
        return dd.scatter(Y, weights=True)

    def solve(self, rhs_index=0, tol=1e-11, maxit=1000):
        m, dd = self.m, self.m.dd
        N = m.N
        f = m.rhs_f[rhs_index]
        fR = f[:m.nR].reshape(N, dd.n_r)
        fP = f[m.nR:]
        KfR = self.KRR_solve(fR)                                         # K_RR^-1 f_R
        g = fP - dd.assemble_primal(np.array([self.Krp[s].T @ KfR[s] for s in range(N)]))
        Sg = self.coarse.solve(g)
        sgp = dd.restrict_primal(Sg)
        corr = np.array([self.Urp[s] @ sgp[s] for s in range(N)])      # K_RR^-1 K_RP S^-1 g
        dbar = -m.rhs_d + dd.scatter((KfR - corr)[:, dd.n_i:])         # eq. (25)
        lam, its, hist = pcg(self.apply_F, self.apply_MD, dbar, tol=tol, maxit=maxit)
        # recovery, eqs. (21) and (20)
        Lam = dd.gather(lam)
        BtL = np.zeros((N, dd.n_r))
        BtL[:, dd.n_i:] = Lam
        KBtL = self.KRR_solve(BtL)
        uP = self.coarse.solve(g + dd.assemble_primal(np.array([self.Krp[s].T @ KBtL[s] for s in range(N)])))
        up = dd.restrict_primal(uP)
        uR = self.KRR_solve(fR - np.array([self.Krp[s] @ up[s] for s in range(N)]) - BtL)
        return dict(u=np.concatenate([uR.reshape(-1), uP]), lam=lam, its=its, history=hist)
