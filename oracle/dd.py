"""Domain-decomposition bookkeeping (oracle; test infrastructure only).

* dof partition u^(s) = (u_i, u_d, u_p), u_r = (u_i, u_d)      paper eq. (12)
  - p: the cell corners (primal variables, Sec. 2.2.2 and [18, 46]);
  - d: the other control points on the cell boundary (dual);
  - i: interior control points.
  Local dofs are node-major with interleaved components (dof = dim*a + comp)
  and every class keeps ascending local dof order; the partition is the same
  for every cell because all cells share one reference discretisation.
* jump operator B = [B_R 0], B_r^(s) = B_d^(s) T_dr, entries 0/+1/-1      eq. (14)-(15)
  - one multiplier per matching dof pair; where m>2 cells share a dof (3D
    cell edges) the copies, sorted by cell index, are chained pairwise
    (+1 on the lower cell, -1 on the higher) so that B keeps full rank;
  - Dirichlet data on dual dofs enter through one +1 row per cell copy with
    d = u0 (Sec. 2.2.2); no interface row joins two copies on the Dirichlet
    boundary;
  - row order: interface rows sorted by (global control point, component,
    chain position), then Dirichlet rows in the same key order.
* weights D^(s): multiplicity scaling, 1/2 on interface rows and 1 on
  Dirichlet rows; in 2D this gives sum_s B_d B_d^T D = I_L             eq. (30)
* primal assembly A_p^(s): cell corner dof -> global primal dof, lattice
  vertices on the Dirichlet boundary eliminated (value lifted into f)  eq. (18)

Pins (tests/test_oracle_dd_rom.py): B annihilates any conforming field scattered
to the cells, rank B = L, sum_s B_d B_d^T D = I in 2D, row counts.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from latticegen import cell_coords


class DD:
    def __init__(self, problem, ref):
        dim, nc = problem.dim, ref.nc
        self.dim = dim
        N = problem.N
        self.N = N
        # local multi-index of each control point (x fastest)
        loc = np.stack(np.unravel_index(np.arange(ref.n_ctrl), (nc,) * dim, order="F"), axis=1)
        onb = (loc == 0) | (loc == nc - 1)
        corner = onb.all(axis=1)
        bnd = onb.any(axis=1) & ~corner
        inner = ~onb.any(axis=1)
        comps = np.arange(dim)
        dofs_of = lambda mask: (np.nonzero(mask)[0][:, None] * dim + comps[None, :]).ravel()
        self.idx_i = dofs_of(inner)
        self.idx_d = dofs_of(bnd)
        self.idx_p = dofs_of(corner)
        self.idx_r = np.concatenate([self.idx_i, self.idx_d])
        self.n_i, self.n_d, self.n_p = self.idx_i.size, self.idx_d.size, self.idx_p.size
        self.n_r = self.n_i + self.n_d
        self.dual_ctrl = np.nonzero(bnd)[0]
        self.corner_ctrl = np.nonzero(corner)[0]

        coords = cell_coords(problem.shape)
        G = np.array([n * (nc - 1) + 1 for n in problem.shape])
        self.Gshape = G
        gpos = coords[:, None, :] * (nc - 1) + loc[None, :, :]            # (N, n_ctrl, dim)
        self.gid = np.ravel_multi_index(tuple(gpos[..., j] for j in range(dim)), tuple(G), order="F")
        # Dirichlet global control points
        on_dir = np.zeros(gpos.shape[:2], dtype=bool)
        for face in problem.dirichlet_faces:
            axis, side = face // 2, face % 2
            tgt = 0 if side == 0 else G[axis] - 1
            on_dir |= gpos[..., axis] == tgt
        self.on_dir = on_dir

        # ---------------- multipliers over dual control points
        nd_ctrl = self.dual_ctrl.size
        cs = np.repeat(np.arange(N), nd_ctrl)
        cc = np.tile(np.arange(nd_ctrl), N)                                # dual ctrl slot
        g = self.gid[cs, self.dual_ctrl[cc]]
        dirflag = on_dir[cs, self.dual_ctrl[cc]]
        order = np.lexsort((cs, g))
        cs, cc, g, dirflag = cs[order], cc[order], g[order], dirflag[order]
        same_next = np.zeros(g.size, dtype=bool)
        same_next[:-1] = g[:-1] == g[1:]
        # chain position inside each group
        start = np.ones(g.size, dtype=bool)
        start[1:] = g[1:] != g[:-1]
        grp = np.cumsum(start) - 1
        first = np.nonzero(start)[0]
        pos = np.arange(g.size) - first[grp]
        # interface rows: consecutive pairs in non-Dirichlet groups
        a_idx = np.nonzero(same_next & ~dirflag)[0]
        b_idx = a_idx + 1
        # Dirichlet rows: every copy in Dirichlet groups
        d_idx = np.nonzero(dirflag)[0]
        rows = []
        for comp in range(dim):
            rows.append(("i", comp, a_idx))
        for comp in range(dim):
            rows.append(("d", comp, d_idx))
        # order: interface rows by (g, comp, pos); then Dirichlet rows by (g, comp, pos)
        key_i = np.concatenate([np.stack([g[a_idx], np.full(a_idx.size, c), pos[a_idx], a_idx], 1)
                                for c in range(dim)])
        key_i = key_i[np.lexsort((key_i[:, 2], key_i[:, 1], key_i[:, 0]))]
        key_d = np.concatenate([np.stack([g[d_idx], np.full(d_idx.size, c), pos[d_idx], d_idx], 1)
                                for c in range(dim)])
        key_d = key_d[np.lexsort((key_d[:, 2], key_d[:, 1], key_d[:, 0]))]
        Li, Ld = key_i.shape[0], key_d.shape[0]
        self.L = Li + Ld
        self.L_interface = Li
        # entries (row, cell, dual slot j, sign)
        ent_r, ent_s, ent_j, ent_v = [], [], [], []
        r = np.arange(Li)
        e1 = key_i[:, 3]
        e2 = e1 + 1
        comp = key_i[:, 1]
        ent_r += [r, r]
        ent_s += [cs[e1], cs[e2]]
        ent_j += [cc[e1] * dim + comp, cc[e2] * dim + comp]
        ent_v += [np.ones(Li), -np.ones(Li)]
        r = Li + np.arange(Ld)
        e = key_d[:, 3]
        comp = key_d[:, 1]
        ent_r += [r]
        ent_s += [cs[e]]
        ent_j += [cc[e] * dim + comp]
        ent_v += [np.ones(Ld)]
        self.ent_row = np.concatenate(ent_r)
        self.ent_cell = np.concatenate(ent_s)
        self.ent_slot = np.concatenate(ent_j)
        self.ent_sign = np.concatenate(ent_v)
        # B_D: (L, N*n_d) stacked local dual jump operators [B_d^(1) ... B_d^(N)]
        self.BD = sp.csr_matrix((self.ent_sign, (self.ent_row, self.ent_cell * self.n_d + self.ent_slot)),
                                shape=(self.L, N * self.n_d))
        # Dirichlet data d (eq. (14)): u0 at the control point of the row
        dvec = np.zeros(self.L)
        a_ctrl = self.dual_ctrl[cc[e]]
        X = problem.ctrl[cs[e], a_ctrl]                                    # (Ld, dim)
        u0 = X @ problem.u0_grad.T
        dvec[Li:] = u0[np.arange(Ld), comp]
        self.d = dvec
        # multiplicity weights
        self.Dw = np.concatenate([np.full(Li, 0.5), np.ones(Ld)])

        # ---------------- primal assembly
        V = np.array(problem.shape) + 1
        corner_off = loc[self.corner_ctrl] // (nc - 1)                     # (2^d, dim) in {0,1}
        vpos = coords[:, None, :] + corner_off[None, :, :]                  # (N, 2^d, dim)
        vdir = np.zeros(vpos.shape[:2], dtype=bool)
        for face in problem.dirichlet_faces:
            axis, side = face // 2, face % 2
            tgt = 0 if side == 0 else V[axis] - 1
            vdir |= vpos[..., axis] == tgt
        vid_all = np.ravel_multi_index(tuple(vpos[..., j] for j in range(dim)), tuple(V), order="F")
        # free vertices numbered in lexicographic (x fastest) order
        all_v = np.stack(np.unravel_index(np.arange(np.prod(V)), tuple(V), order="F"), axis=1)
        vfree = np.ones(all_v.shape[0], dtype=bool)
        for face in problem.dirichlet_faces:
            axis, side = face // 2, face % 2
            tgt = 0 if side == 0 else V[axis] - 1
            vfree &= all_v[:, axis] != tgt
        num = -np.ones(all_v.shape[0], dtype=np.int64)
        num[vfree] = np.arange(vfree.sum())
        self.n_vert_free = int(vfree.sum())
        self.nP = self.n_vert_free * dim
        vnum = num[vid_all]                                                 # (N, 2^d)
        Ap = np.where(vnum[:, :, None] >= 0, vnum[:, :, None] * dim + comps[None, None, :], -1)
        self.Ap = Ap.reshape(N, self.n_p)                                   # (N, n_p), -1: Dirichlet
        # prescribed values on Dirichlet primal dofs (for lifting)
        Xc = problem.ctrl[:, self.corner_ctrl, :]                           # (N, 2^d, dim)
        u0c = Xc @ problem.u0_grad.T
        self.up_dir = np.where(vdir[:, :, None], u0c, 0.0).reshape(N, self.n_p)
        self.p_is_dir = np.repeat(vdir, dim, axis=1)
        # sparse A_p: (nP, N*n_p)
        m = self.Ap >= 0
        s_idx, p_idx = np.nonzero(m)
        self.AP = sp.csr_matrix((np.ones(s_idx.size), (self.Ap[m], s_idx * self.n_p + p_idx)),
                                shape=(self.nP, N * self.n_p))

    # ------------------------------------------------------------ helpers
    def gather(self, lam: np.ndarray, weights: bool = False) -> np.ndarray:
        """Lambda_s = B_d^(s)T lam (optionally of D lam), shape (N, n_d)."""
        x = lam * self.Dw if weights else lam
        return (self.BD.T @ x).reshape(self.N, self.n_d)

    def scatter(self, Y: np.ndarray, weights: bool = False) -> np.ndarray:
        """sum_s B_d^(s) Y_s (optionally followed by D), shape (L,)."""
        out = self.BD @ Y.reshape(-1)
        return out * self.Dw if weights else out

    def assemble_primal(self, c: np.ndarray) -> np.ndarray:
        """sum_s A_p^(s) c_s, c of shape (N, n_p)."""
        return self.AP @ c.reshape(-1)

    def restrict_primal(self, xP: np.ndarray) -> np.ndarray:
        """A_p^(s)T x_P for every cell, shape (N, n_p) (zero on Dirichlet corners)."""
        return (self.AP.T @ xP).reshape(self.N, self.n_p)
