"""Seeded synthetic lattice problems (problem data only, no solver arithmetic).

This module is the single source of inputs shared by the CPU oracle and the
GPU library.  It defines *what* is solved: the lattice of cells, the per-cell
spline geometry (control points), the strut widths of the ersatz material, the
Dirichlet faces and the tractions.  It contains none of the method's
computations (no basis functions, quadrature, stiffness, decomposition or
Krylov steps); both solver sides compute those independently from these data.

Geometry (paper Sec. 2.2.1, eq. (6) and Sec. 4.1, eqs. (50)-(51)): every cell is
the image of the same reference cell [0,1]^d under its own spline map whose
control points are the macro map evaluated at the Greville abscissae of the
open uniform quadratic knot vector.  Neighbouring cells therefore share the
control points of their common boundary (a matching, conforming decomposition
as required for pointwise multipliers, Sec. 2.2.2).

Workloads: the paper's own lattices (its multipatch cells and NURBS macro
shapes) are not reproducible here, so these synthetic lattices stand in for
them; sizes follow the five configurations the build is measured on:

  c1  2D  4x4 cells,  8x8 quadratic elements/cell, sin-sin map a=0.05h, w=0.2h, 4 principal cells
  c2  2D 64x64 cells, 16x16 elements/cell, sin-sin map a=0.15h, w linear 0.15h..0.30h in x, 12 principal cells
  c3  3D 16x16x8 cells, 6x6x6 elements/cell, 3-mode seeded map <=0.1h, cubic frame w=0.2h, 16 principal cells
  c4  c2 with 32 load cases (seeded traction directions/magnitudes)
  c5  3D 12x12x12 cells as c3 with per-cell widths U[0.15,0.30]h, smoothed indicator
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

__all__ = ["Problem", "make", "tiny", "CONFIG_NAMES", "greville_abscissae", "c4_tractions",
           "open_uniform_knots", "cell_index", "cell_coords"]

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")

# Face ids: 0: X=0, 1: X=L_x, 2: Y=0, 3: Y=L_y, 4: Z=0, 5: Z=L_z.
FACE_XMIN, FACE_XMAX, FACE_YMIN, FACE_YMAX, FACE_ZMIN, FACE_ZMAX = range(6)


@dataclasses.dataclass
class Problem:
    """One synthetic lattice problem.

    Arrays are float64 / int64 numpy arrays.  Cell s sits at lattice position
    (ix, iy[, iz]) with s = ix + nx*(iy + ny*iz).  Within a cell the control
    point a = ax + nc*(ay + nc*az) (x fastest), nc = n_el + degree.
    """
    name: str
    dim: int
    shape: tuple                 # (nx, ny) or (nx, ny, nz)
    n_el: int                    # elements per direction per cell
    degree: int                  # spline degree (2: quadratic)
    h: float                     # cell size in the lattice (reference) frame
    E_in: float
    E_out: float
    nu: float
    smooth_eps: float            # 0: sharp strut indicator; >0: tanh smoothing width
    ctrl: np.ndarray             # (N, n_ctrl, dim) control points of each cell map
    widths: np.ndarray           # (N,) strut width of each cell (physical units of h)
    dirichlet_faces: tuple       # faces clamped (u = u0 there)
    u0_grad: np.ndarray          # (dim, dim): prescribed u0(x) = u0_grad @ x on Dirichlet faces
    load_face: int               # face carrying the traction (-1: none)
    tractions: np.ndarray        # (nrhs, dim) constant traction per load case
    n_principal: int             # number of principal cells requested from the greedy

    @property
    def N(self) -> int:
        return int(np.prod(self.shape))

    @property
    def nc(self) -> int:
        return self.n_el + self.degree

    @property
    def n_ctrl(self) -> int:
        return self.nc ** self.dim

    @property
    def n_dof(self) -> int:
        return self.n_ctrl * self.dim

    @property
    def nrhs(self) -> int:
        return int(self.tractions.shape[0])

    @property
    def plane_strain(self) -> bool:
        return self.dim == 2

    def lengths(self):
        return tuple(n * self.h for n in self.shape)


def open_uniform_knots(n_el: int, degree: int) -> np.ndarray:
    """Open uniform knot vector on [0,1] with n_el elements (geometry input)."""
    inner = np.arange(1, n_el) / n_el
    return np.concatenate([np.zeros(degree + 1), inner, np.ones(degree + 1)])


def greville_abscissae(n_el: int, degree: int) -> np.ndarray:
    """Greville points: averages of `degree` consecutive interior knots."""
    kn = open_uniform_knots(n_el, degree)
    nc = n_el + degree
    return np.array([kn[a + 1:a + 1 + degree].mean() for a in range(nc)])


def cell_coords(shape: Sequence[int]) -> np.ndarray:
    """(N, dim) integer lattice coordinates of every cell, x fastest."""
    dim = len(shape)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    coords = np.stack([g.transpose(tuple(range(dim))[::-1]).ravel() for g in grids], axis=1)
    return coords.astype(np.int64)


def cell_index(c, shape) -> int:
    s = 0
    for j in reversed(range(len(shape))):
        s = s * shape[j] + int(c[j])
    return s


# ----------------------------------------------------------------- macro maps
def _map_sinsin(X: np.ndarray, L, amp: float) -> np.ndarray:
    """x = X + amp sin(2 pi X/Lx) sin(2 pi Y/Ly), y = Y (2D)."""
    out = X.copy()
    out[..., 0] = X[..., 0] + amp * np.sin(2 * np.pi * X[..., 0] / L[0]) * np.sin(2 * np.pi * X[..., 1] / L[1])
    return out


def _fourier3_params(seed: int, h: float):
    rng = np.random.default_rng(seed)
    comp = rng.integers(0, 3, size=3)
    k = rng.integers(1, 3, size=(3, 3))
    a = rng.uniform(0.0, 0.1 * h / 3.0, size=3)
    return comp, k, a


def _map_fourier3(X: np.ndarray, L, params) -> np.ndarray:
    """x = X + sum_m a_m e_{c_m} prod_j sin(pi k_mj X_j / L_j) (3D); vanishes on all outer faces."""
    comp, k, a = params
    out = X.copy()
    for m in range(3):
        prod = np.ones(X.shape[:-1])
        for j in range(3):
            prod = prod * np.sin(np.pi * k[m, j] * X[..., j] / L[j])
        out[..., comp[m]] += a[m] * prod
    return out


def _control_points(shape, n_el, degree, h, macro) -> np.ndarray:
    dim = len(shape)
    gv = greville_abscissae(n_el, degree)
    nc = gv.size
    # local reference points of control points, a = ax + nc*(ay + nc*az)
    loc = np.stack(np.meshgrid(*([gv] * dim), indexing="ij"), axis=-1)  # [ax,ay,(az),dim]
    loc = loc.transpose(tuple(range(dim))[::-1] + (dim,)).reshape(-1, dim)  # x fastest
    coords = cell_coords(shape).astype(np.float64)
    X = (coords[:, None, :] + loc[None, :, :]) * h                     # (N, n_ctrl, dim)
    return macro(X)


def _build(name, dim, shape, n_el, *, amp=0.0, map_kind="sinsin", map_seed=3, width=("const", 0.2),
           n_principal=4, tractions=None, smooth=False, E_in=1.0, E_out=1e-3, nu=0.3, degree=2, h=1.0,
           dirichlet_faces=(FACE_XMIN,), load_face=FACE_XMAX, u0_grad=None) -> Problem:
    L = tuple(n * h for n in shape)
    if map_kind == "sinsin":
        macro = (lambda X: _map_sinsin(X, L, amp * h)) if amp != 0.0 else (lambda X: X.copy())
    elif map_kind == "fourier3":
        params = _fourier3_params(map_seed, h)
        macro = lambda X: _map_fourier3(X, L, params)
    elif map_kind == "identity":
        macro = lambda X: X.copy()
    else:
        raise ValueError(map_kind)
    ctrl = _control_points(shape, n_el, degree, h, macro)
    N = ctrl.shape[0]
    coords = cell_coords(shape)
    kind = width[0]
    if kind == "const":
        widths = np.full(N, width[1] * h)
    elif kind == "linx":
        nx = shape[0]
        widths = (width[1] + (width[2] - width[1]) * coords[:, 0] / max(nx - 1, 1)) * h
    elif kind == "uniform":
        rng = np.random.default_rng(width[3])
        widths = rng.uniform(width[1], width[2], size=N) * h
    elif kind == "levels":          # m distinct widths cycling over x (exact-ROM lattices)
        lv = np.asarray(width[1], dtype=np.float64)
        widths = lv[coords[:, 0] % lv.size] * h
    else:
        raise ValueError(kind)
    if tractions is None:
        tractions = np.zeros((1, dim))
        tractions[0, 0] = 1.0
    tractions = np.atleast_2d(np.asarray(tractions, dtype=np.float64))
    eps = (h / n_el) / 4.0 if smooth else 0.0
    if u0_grad is None:
        u0_grad = np.zeros((dim, dim))
    return Problem(name=name, dim=dim, shape=tuple(shape), n_el=n_el, degree=degree, h=h,
                   E_in=E_in, E_out=E_out, nu=nu, smooth_eps=eps, ctrl=ctrl, widths=widths,
                   dirichlet_faces=tuple(dirichlet_faces), u0_grad=np.asarray(u0_grad, dtype=np.float64),
                   load_face=load_face, tractions=tractions, n_principal=n_principal)


def c4_tractions(n: int = 32, seed: int = 4) -> np.ndarray:
    """The seeded load cases of c4: constant tractions m (cos phi, sin phi), m ~ U[0.5, 1], phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    mag = rng.uniform(0.5, 1.0, size=n)
    phi = rng.uniform(0.0, 2 * np.pi, size=n)
    return np.stack([mag * np.cos(phi), mag * np.sin(phi)], axis=1)


def make(name: str, n_principal: Optional[int] = None) -> Problem:
    """The five measured configurations (see module docstring)."""
    if name == "c1":
        p = _build("c1", 2, (4, 4), 8, amp=0.05, width=("const", 0.2), n_principal=4)
    elif name == "c2":
        p = _build("c2", 2, (64, 64), 16, amp=0.15, width=("linx", 0.15, 0.30), n_principal=12)
    elif name == "c3":
        p = _build("c3", 3, (16, 16, 8), 6, map_kind="fourier3", map_seed=3, width=("const", 0.2),
                   n_principal=16)
    elif name == "c4":
        p = _build("c4", 2, (64, 64), 16, amp=0.15, width=("linx", 0.15, 0.30), n_principal=12,
                   tractions=c4_tractions())
    elif name == "c5":
        p = _build("c5", 3, (12, 12, 12), 6, map_kind="fourier3", map_seed=3,
                   width=("uniform", 0.15, 0.30, 5), n_principal=16, smooth=True)
    else:
        raise KeyError(name)
    if n_principal is not None:
        p.n_principal = n_principal
    return p


def tiny(dim: int = 2, shape=(2, 2), n_el: int = 3, **kw) -> Problem:
    """Small lattices for tests: same recipe, any size.

    Keyword arguments are those of the configuration builder: amp, map_kind,
    map_seed, width, n_principal, tractions, smooth, E_in, E_out, nu,
    dirichlet_faces, load_face, u0_grad.
    """
    kw.setdefault("amp", 0.05)
    if dim == 3 and "map_kind" not in kw:
        kw["map_kind"] = "fourier3"
    return _build(kw.pop("name", "tiny"), dim, shape, n_el, **kw)


def fd_cells(N: int, count: int = 20, seed: int = 55) -> np.ndarray:
    """Cells whose width derivative is checked by finite differences."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=min(count, N), replace=False))
