"""Pins of the oracle's compliance gradient (CPU only)."""
import numpy as np
import pytest

import latticegen
from oracle import Model
from oracle.assembly import RefCell, cell_matrix_values, cell_derivative_values, dense
from oracle.direct import conforming_solve
from oracle.gradient import compliance_gradient, compliance_direct


def _smooth(dim):
    if dim == 2:
        return latticegen.tiny(2, (3, 2), 3, smooth=True, width=("uniform", 0.15, 0.30, 5), n_principal=3)
    return latticegen.tiny(3, (2, 2, 1), 2, smooth=True, width=("uniform", 0.15, 0.30, 5), n_principal=2)


@pytest.mark.parametrize("dim", [2, 3])
def test_cell_derivative_matches_finite_difference(dim):
    p = _smooth(dim)
    ref = RefCell(dim, p.n_el)
    s = 1
    h = 1e-6
    dK = cell_derivative_values(ref, p, [s])[0]
    w0 = p.widths[s]
    p.widths[s] = w0 + h
    Kp = cell_matrix_values(ref, p, [s])[0]
    p.widths[s] = w0 - h
    Km = cell_matrix_values(ref, p, [s])[0]
    p.widths[s] = w0
    fd = (Kp - Km) / (2 * h)
    assert np.abs(fd - dK).max() <= 1e-6 * np.abs(dK).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_adjoint_gradient_matches_central_difference_of_compliance(dim):
    p = _smooth(dim)
    m = Model(p)
    u = conforming_solve(m)["u"]
    g = compliance_gradient(m, u)
    h = 1e-6
    for s in range(p.N):
        wp = p.widths.copy(); wp[s] += h
        wm = p.widths.copy(); wm[s] -= h
        fd = (compliance_direct(p, wp) - compliance_direct(p, wm)) / (2 * h)
        assert abs(fd - g[s]) <= 1e-5 * np.abs(g).max(), (s, fd, g[s])
    assert np.all(g < 0)          # thicker struts -> stiffer lattice -> smaller compliance


def test_sharp_indicator_has_zero_width_derivative():
    p = latticegen.tiny(2, (2, 2), 3, n_principal=2)
    ref = RefCell(2, p.n_el)
    assert np.abs(cell_derivative_values(ref, p, [0])).max() == 0.0
