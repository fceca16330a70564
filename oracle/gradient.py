"""Compliance and its width gradient (oracle; test infrastructure only).

Compliance c = f^T u with u the solution of the saddle system (16).  The loads
do not depend on the strut widths and the system is self-adjoint, so
dc/dw_s = -u_s^T (dK^(s)/dw_s) u_s, where u_s is the cell's full local
displacement and dK^(s)/dw_s is the width derivative of the cell stiffness of
eq. (52): the pulled-back tensor is linear in the Young modulus, so
dĈ/dw = (dE/dw) Ĉ/E with the smoothed strut indicator
E = E_out + (E_in - E_out)(1 + tanh((w/2 - dist)/eps))/2.

Pins (tests/test_oracle_gradient.py): central finite differences of the
compliance computed by the direct conforming solver, and a brute-force dense
derivative of the assembled cell matrix.
"""
from __future__ import annotations

import copy

import numpy as np

from .assembly import cell_derivative_values
from .direct import conforming_solve


def compliance(model, u: np.ndarray, rhs_index: int = 0) -> float:
    return float(model.rhs_f[rhs_index] @ u)


def compliance_gradient(model, u: np.ndarray, cells=None) -> np.ndarray:
    """dc/dw_s for the given cells (all by default), from the torn solution u (eq. (13) layout)."""
    cells = np.arange(model.N) if cells is None else np.atleast_1d(cells)
    U = model.full_cell_displacements(u)                         # (N, n_dof)
    dK = cell_derivative_values(model.ref, model.problem, cells)  # (S, nnz)
    g = np.zeros(cells.size)
    for t, s in enumerate(cells):
        us = U[s]
        g[t] = -np.sum(dK[t] * us[model.ref.pat_rows] * us[model.ref.pat_cols])
    return g


def compliance_direct(problem, widths=None) -> float:
    """Compliance from the direct conforming solve, optionally with other widths."""
    from .model import Model
    p = copy.copy(problem)
    if widths is not None:
        p.widths = np.asarray(widths, dtype=np.float64).copy()
    m = Model(p)
    r = conforming_solve(m)
    return compliance(m, r["u"])
