"""Cell stiffness assembly (oracle; test infrastructure only).

Follows the paper's pulled-back bilinear form (Sec. 4.2.1, eq. (52)): on the
reference cell, a^(s)(u,v) = integral of grad_xi(u) : Ĉ^(s) : grad_xi(v),
where the fourth-order field Ĉ^(s) carries the material tensor and the cell
map.  In the gradient form used here

    Ĉ_ijkl = det(J) * sum_{m,n} C_imkn (J^-1)_jm (J^-1)_ln ,   J_mj = dx_m/dxi_j,

which gives the same energy as eps(u):C:eps(v) by the minor symmetries of the
isotropic Hooke tensor C (eq. (3b); plane strain in 2D).  The stiffness is
K_(a,i),(b,k) = sum_q w_q dN_a/dxi_j Ĉ_ijkl dN_b/dxi_l, i.e. the stiffness is
linear in the values of Ĉ at the quadrature points, which is the property the
lookup-table assembly of eqs. (53)-(54) exploits and the greedy (Alg. 4)
relies on.  Material: ersatz strut field, E_in inside struts and E_out
elsewhere (sharp indicator or tanh-smoothed).

Loads: consistent nodal forces of a constant traction, eq. (5b), integrated
with the physical length/area element of the loaded face.

Pins (tests/test_oracle_assembly.py): symmetry, rigid-body null space of a
floating cell (nullity exactly 3 in 2D, 6 in 3D), total load = traction x face
measure, sum of cell volumes = lattice volume, patch test through the full
solvers.
"""
from __future__ import annotations

import itertools

import numpy as np

from latticegen import open_uniform_knots, cell_coords
from .bspline import bspline_basis, gauss_legendre_01


class RefCell:
    """Reference-cell tables shared by all cells (eq. (6))."""

    def __init__(self, dim: int, n_el: int, p: int = 2):
        self.dim, self.n_el, self.p = dim, n_el, p
        self.nc = n_el + p
        self.n_ctrl = self.nc ** dim
        self.n_dof = self.n_ctrl * dim
        self.knots = open_uniform_knots(n_el, p)
        xg, wg = gauss_legendre_01(p + 1)
        self.nq1 = xg.size
        # 1D tables: element e, local point g, local function l (global e+l)
        x1 = (np.arange(n_el)[:, None] + xg[None, :]) / n_el      # (n_el, nq1)
        v1, d1 = bspline_basis(self.knots, p, x1.ravel())
        v1 = v1.reshape(n_el, self.nq1, self.nc)
        d1 = d1.reshape(n_el, self.nq1, self.nc)
        w1 = wg / n_el
        ne = n_el ** dim
        nq = self.nq1 ** dim
        nl = (p + 1) ** dim
        self.n_elem, self.nq, self.nloc = ne, nq, nl
        self.xi = np.zeros((ne, nq, dim))
        self.w = np.zeros((ne, nq))
        self.N = np.zeros((ne, nq, nl))
        self.dN = np.zeros((ne, nq, nl, dim))
        self.elem_ctrl = np.zeros((ne, nl), dtype=np.int64)
        for E, e in enumerate(_lex(n_el, dim)):
            for l, lo in enumerate(_lex(p + 1, dim)):
                self.elem_ctrl[E, l] = _flat([e[j] + lo[j] for j in range(dim)], self.nc)
            for q, g in enumerate(_lex(self.nq1, dim)):
                self.xi[E, q] = [x1[e[j], g[j]] for j in range(dim)]
                self.w[E, q] = np.prod([w1[g[j]] for j in range(dim)])
                for l, lo in enumerate(_lex(p + 1, dim)):
                    vals = [v1[e[j], g[j], e[j] + lo[j]] for j in range(dim)]
                    ders = [d1[e[j], g[j], e[j] + lo[j]] for j in range(dim)]
                    self.N[E, q, l] = np.prod(vals)
                    for j in range(dim):
                        self.dN[E, q, l, j] = ders[j] * np.prod([vals[i] for i in range(dim) if i != j])
        # shared sparsity pattern of the cell stiffness (dense lookup of positions)
        look = -np.ones((self.n_dof, self.n_dof), dtype=np.int64)
        rows, cols = [], []
        for E in range(ne):
            dofs = (self.elem_ctrl[E][:, None] * dim + np.arange(dim)[None, :]).ravel()
            rr, cc = np.meshgrid(dofs, dofs, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        look[rows, cols] = 1
        r_idx, c_idx = np.nonzero(look >= 0)          # row-major order = CSR order
        self.nnz = r_idx.size
        look[r_idx, c_idx] = np.arange(self.nnz)
        self.pat_rows, self.pat_cols = r_idx, c_idx
        self.indptr = np.concatenate([[0], np.cumsum(np.bincount(r_idx, minlength=self.n_dof))])
        self.indices = c_idx
        self.pos = np.zeros((ne, (nl * dim) ** 2), dtype=np.int64)
        for E in range(ne):
            dofs = (self.elem_ctrl[E][:, None] * dim + np.arange(dim)[None, :]).ravel()
            self.pos[E] = look[dofs[:, None], dofs[None, :]].ravel()
        self.lookup = look


def _lex(n, dim):
    """Multi-indices of an n^dim grid, x fastest."""
    for t in itertools.product(range(n), repeat=dim):
        yield t[::-1]


def _flat(idx, n):
    s = 0
    for j in reversed(range(len(idx))):
        s = s * n + idx[j]
    return s


# ------------------------------------------------------------ material field
def strut_distance(xi: np.ndarray, dim: int) -> np.ndarray:
    """Distance (reference units) from xi in [0,1]^d to the nearest strut axis.

    2D: the cell frame (4 edges) and both diagonals, Euclidean distance to the
    segments ("hollow square with a cross", paper Fig. 7(a)).
    3D: the 12 cube edges, Chebyshev distance in the two transverse
    coordinates (square cross-section struts).
    """
    if dim == 2:
        segs = [((0, 0), (1, 0)), ((1, 0), (1, 1)), ((1, 1), (0, 1)), ((0, 1), (0, 0)),
                ((0, 0), (1, 1)), ((1, 0), (0, 1))]
        best = np.full(xi.shape[:-1], np.inf)
        for a, b in segs:
            a = np.asarray(a, float)
            b = np.asarray(b, float)
            ab = b - a
            t = np.clip(((xi - a) @ ab) / (ab @ ab), 0.0, 1.0)
            proj = a + t[..., None] * ab
            best = np.minimum(best, np.linalg.norm(xi - proj, axis=-1))
        return best
    best = np.full(xi.shape[:-1], np.inf)
    for axis in range(3):
        others = [j for j in range(3) if j != axis]
        for c1 in (0.0, 1.0):
            for c2 in (0.0, 1.0):
                d = np.maximum(np.abs(xi[..., others[0]] - c1), np.abs(xi[..., others[1]] - c2))
                best = np.minimum(best, d)
    return best


def young_modulus(xi: np.ndarray, width, problem):
    """E at reference points for a cell of strut width `width` (and dE/dw)."""
    dist = strut_distance(xi, problem.dim) * problem.h
    half = 0.5 * float(width)
    if problem.smooth_eps > 0.0:
        eps = problem.smooth_eps
        t = np.tanh((half - dist) / eps)
        E = problem.E_out + (problem.E_in - problem.E_out) * 0.5 * (1.0 + t)
        dE = (problem.E_in - problem.E_out) * 0.5 * (1.0 - t * t) * (0.5 / eps)
        return E, dE
    E = np.where(dist < half, problem.E_in, problem.E_out)
    return E, np.zeros_like(E)


def hooke(dim: int, nu: float) -> np.ndarray:
    """Isotropic Hooke tensor for E = 1: C_imkn = lam d_im d_kn + mu (d_ik d_mn + d_in d_mk).

    In 2D this is plane strain (the same Lame constants, restricted to the plane).
    """
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    I = np.eye(dim)
    return (lam * np.einsum("im,kn->imkn", I, I)
            + mu * (np.einsum("ik,mn->imkn", I, I) + np.einsum("in,mk->imkn", I, I)))


def geometry(ref: RefCell, ctrl: np.ndarray):
    """J (cells, E, q, m, j), det J and J^-1 for control points ctrl (cells, n_ctrl, dim)."""
    P = ctrl[:, ref.elem_ctrl, :]                       # (S, E, nl, dim)
    J = np.einsum("selm,eqlj->seqmj", P, ref.dN)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                              # Jinv[..., j, m]
    return J, det, Jinv


def pulled_back_tensor(ref: RefCell, problem, cells, with_derivative=False):
    """Ĉ^(s) at every quadrature point, shape (S, E, q, d, d, d, d) (eq. (52))."""
    cells = np.atleast_1d(cells)
    _, det, Jinv = geometry(ref, problem.ctrl[cells])
    E, dE = _E_cells(ref, problem, cells)
    C = hooke(problem.dim, problem.nu)
    base = np.einsum("seq,imkn,seqjm,seqln->seqijkl", det, C, Jinv, Jinv, optimize=True)
    Chat = E[..., None, None, None, None] * base
    if with_derivative:
        return Chat, dE[..., None, None, None, None] * base
    return Chat


def _E_cells(ref, problem, cells):
    E = np.empty((cells.size, ref.n_elem, ref.nq))
    dE = np.empty_like(E)
    for i, s in enumerate(cells):
        E[i], dE[i] = young_modulus(ref.xi, problem.widths[s], problem)
    return E, dE


def element_matrices(ref: RefCell, Chat: np.ndarray) -> np.ndarray:
    """K_e = sum_q w_q dN_a,j Ĉ_ijkl dN_b,l, shape (S, E, nl*d, nl*d)."""
    d = ref.dim
    Ke = np.einsum("eq,eqaj,seqijkl,eqbl->seaibk", ref.w, ref.dN, Chat, ref.dN, optimize=True)
    S = Chat.shape[0]
    n = ref.nloc * d
    return Ke.reshape(S, ref.n_elem, n, n)


def cell_matrix_values(ref: RefCell, problem, cells, chunk: int = 64) -> np.ndarray:
    """Stiffness values of the given cells on the shared pattern, (S, nnz)."""
    cells = np.atleast_1d(cells)
    out = np.zeros((cells.size, ref.nnz))
    for c0 in range(0, cells.size, chunk):
        cs = cells[c0:c0 + chunk]
        Ke = element_matrices(ref, pulled_back_tensor(ref, problem, cs))
        blk = out[c0:c0 + cs.size]
        for E in range(ref.n_elem):
            blk[:, ref.pos[E]] += Ke[:, E].reshape(cs.size, -1)
    return out


def cell_derivative_values(ref: RefCell, problem, cells) -> np.ndarray:
    """dK^(s)/dw_s on the shared pattern (width derivative of eq. (52))."""
    cells = np.atleast_1d(cells)
    _, dC = pulled_back_tensor(ref, problem, cells, with_derivative=True)
    Ke = element_matrices(ref, dC)
    out = np.zeros((cells.size, ref.nnz))
    for E in range(ref.n_elem):
        out[:, ref.pos[E]] += Ke[:, E].reshape(cells.size, -1)
    return out


def dense(ref: RefCell, vals: np.ndarray) -> np.ndarray:
    K = np.zeros((ref.n_dof, ref.n_dof))
    K[ref.pat_rows, ref.pat_cols] = vals
    return K


def snapshots(ref: RefCell, problem, cells, chunk: int = 256) -> np.ndarray:
    """Greedy snapshot of each cell: Ĉ^(s) at all quadrature points, all d^4 entries."""
    cells = np.atleast_1d(cells)
    n = ref.n_elem * ref.nq * problem.dim ** 4
    out = np.zeros((cells.size, n))
    for c0 in range(0, cells.size, chunk):
        cs = cells[c0:c0 + chunk]
        out[c0:c0 + cs.size] = pulled_back_tensor(ref, problem, cs).reshape(cs.size, n)
    return out


# ------------------------------------------------------------------- loads
def face_cells(problem, face: int) -> np.ndarray:
    axis, side = face // 2, face % 2
    coords = cell_coords(problem.shape)
    target = 0 if side == 0 else problem.shape[axis] - 1
    return np.nonzero(coords[:, axis] == target)[0]


def cell_loads(ref: RefCell, problem) -> np.ndarray:
    """Consistent nodal forces of the constant tractions, (N, n_dof, nrhs) (eq. (5b))."""
    d = problem.dim
    f = np.zeros((problem.N, ref.n_dof, problem.nrhs))
    if problem.load_face < 0:
        return f
    axis, side = problem.load_face // 2, problem.load_face % 2
    tang = [j for j in range(d) if j != axis]
    xg, wg = gauss_legendre_01(ref.p + 1)
    n_el = ref.n_el
    pts1 = ((np.arange(n_el)[:, None] + xg[None, :]) / n_el).ravel()
    w1 = np.tile(wg / n_el, n_el)
    grids = np.meshgrid(*([pts1] * (d - 1)), indexing="ij")
    wgrid = np.meshgrid(*([w1] * (d - 1)), indexing="ij")
    nf = pts1.size ** (d - 1)
    xi = np.zeros((nf, d))
    for t, g in zip(tang, grids):
        xi[:, t] = g.ravel()
    xi[:, axis] = float(side)
    wf = np.prod([g.ravel() for g in wgrid], axis=0)
    # full tensor basis at face points
    v, dv = bspline_basis(ref.knots, ref.p, xi.ravel())
    v = v.reshape(nf, d, ref.nc)
    dv = dv.reshape(nf, d, ref.nc)
    Nf = np.ones((nf, ref.n_ctrl))
    dNf = np.ones((nf, ref.n_ctrl, d))
    for a, idx in enumerate(_lex(ref.nc, d)):
        Nf[:, a] = np.prod([v[:, j, idx[j]] for j in range(d)], axis=0)
        for jj in range(d):
            dNf[:, a, jj] = np.prod([dv[:, j, idx[j]] if j == jj else v[:, j, idx[j]] for j in range(d)], axis=0)
    for s in face_cells(problem, problem.load_face):
        P = problem.ctrl[s]                                    # (n_ctrl, d)
        T = np.einsum("am,qaj->qmj", P, dNf)                   # dx_m/dxi_j
        if d == 2:
            meas = np.linalg.norm(T[:, :, tang[0]], axis=1)
        else:
            meas = np.linalg.norm(np.cross(T[:, :, tang[0]], T[:, :, tang[1]]), axis=1)
        wq = wf * meas
        base = np.einsum("q,qa->a", wq, Nf)                    # integral of N_a
        for r in range(problem.nrhs):
            f[s, :, r] = (base[:, None] * problem.tractions[r][None, :]).ravel()
    return f
