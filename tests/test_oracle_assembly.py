"""Pins of the oracle's discretisation: basis, geometry, stiffness, loads (CPU only)."""
import numpy as np
import pytest

import latticegen
from oracle.bspline import bspline_basis, gauss_legendre_01
from oracle.assembly import (RefCell, cell_matrix_values, dense, cell_loads, geometry, hooke,
                             strut_distance)


@pytest.mark.parametrize("n_el", [1, 3, 8])
def test_partition_of_unity_and_linear_precision(n_el):
    kn = latticegen.open_uniform_knots(n_el, 2)
    x = np.linspace(0, 1, 101)
    v, d = bspline_basis(kn, 2, x)
    assert np.allclose(v.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(d.sum(axis=1), 0.0, atol=1e-12)
    g = latticegen.greville_abscissae(n_el, 2)
    assert np.allclose(v @ g, x, atol=1e-14)          # linear precision with Greville points
    assert np.allclose(d @ g, 1.0, atol=1e-12)
    assert np.all(v >= -1e-15)


def test_basis_derivative_matches_central_difference():
    kn = latticegen.open_uniform_knots(4, 2)
    x = np.array([0.03, 0.2, 0.41, 0.66, 0.9])
    h = 1e-6
    _, d = bspline_basis(kn, 2, x)
    vp, _ = bspline_basis(kn, 2, x + h)
    vm, _ = bspline_basis(kn, 2, x - h)
    assert np.allclose(d, (vp - vm) / (2 * h), atol=1e-7)


def test_quadratic_bspline_known_values():
    # single element: Bernstein polynomials of degree 2
    kn = latticegen.open_uniform_knots(1, 2)
    x = np.array([0.0, 0.25, 0.5, 1.0])
    v, _ = bspline_basis(kn, 2, x)
    expect = np.stack([(1 - x) ** 2, 2 * x * (1 - x), x ** 2], axis=1)
    assert np.allclose(v, expect, atol=1e-15)


def test_gauss_rule_exact_for_degree_5():
    x, w = gauss_legendre_01(3)
    for k in range(6):
        assert np.isclose(np.sum(w * x ** k), 1.0 / (k + 1), atol=1e-15)


def _floating_cell(dim, n_el):
    shape = (3, 3) if dim == 2 else (3, 3, 3)
    p = latticegen.tiny(dim, shape, n_el)
    s = latticegen.cell_index((1,) * dim, shape)
    return p, RefCell(dim, n_el), s


@pytest.mark.parametrize("dim,n_el,nullity", [(2, 3, 3), (2, 8, 3), (3, 2, 6)])
def test_cell_stiffness_symmetric_with_rigid_nullspace(dim, n_el, nullity):
    p, ref, s = _floating_cell(dim, n_el)
    K = dense(ref, cell_matrix_values(ref, p, [s])[0])
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    # rigid modes built from the control points (isoparametric => exact)
    P = p.ctrl[s]
    modes = []
    for c in range(dim):
        t = np.zeros_like(P)
        t[:, c] = 1.0
        modes.append(t.ravel())
    rot_pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for a, b in rot_pairs:
        r = np.zeros_like(P)
        r[:, a] = -P[:, b]
        r[:, b] = P[:, a]
        modes.append(r.ravel())
    Rm = np.array(modes).T
    assert np.abs(K @ Rm).max() <= 1e-11 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.all(ev[:nullity] < 1e-11 * ev[-1])
    assert ev[nullity] > 1e-9 * ev[-1]


def test_total_area_and_load():
    p = latticegen.make("c1")
    ref = RefCell(2, p.n_el)
    _, det, _ = geometry(ref, p.ctrl)
    area = np.einsum("eq,seq->", ref.w, det)
    assert np.isclose(area, 16.0, rtol=1e-13)      # the macro map fixes the lattice boundary
    f = cell_loads(ref, p)
    tot = f[:, :, 0].reshape(p.N, -1, 2).sum(axis=(0, 1))
    assert np.allclose(tot, [4.0 * 1.0, 0.0], atol=1e-13)   # traction (1,0) on an edge of length 4


def test_total_volume_and_load_3d():
    p = latticegen.tiny(3, (2, 2, 2), 2, tractions=[[0.3, -0.2, 0.5]])
    ref = RefCell(3, 2)
    _, det, _ = geometry(ref, p.ctrl)
    assert np.isclose(np.einsum("eq,seq->", ref.w, det), 8.0, rtol=1e-13)
    f = cell_loads(ref, p)
    tot = f[:, :, 0].reshape(p.N, -1, 3).sum(axis=(0, 1))
    assert np.allclose(tot, 4.0 * np.array([0.3, -0.2, 0.5]), atol=1e-13)


def test_hooke_plane_strain_values():
    C = hooke(2, 0.3)
    lam = 0.3 / (1.3 * 0.4)
    mu = 1 / 2.6
    assert np.isclose(C[0, 0, 0, 0], lam + 2 * mu)
    assert np.isclose(C[0, 0, 1, 1], lam)
    assert np.isclose(C[0, 1, 0, 1], mu)
    assert np.isclose(C[0, 1, 1, 0], mu)


def test_strut_distance_2d_and_3d():
    xi = np.array([[0.5, 0.5], [0.5, 0.0], [0.25, 0.5], [0.3, 0.1]])
    d = strut_distance(xi, 2)
    assert np.allclose(d[:3], [0.0, 0.0, 0.25 / np.sqrt(2)])
    xi3 = np.array([[0.5, 0.5, 0.5], [0.5, 0.05, 0.02], [0.0, 0.4, 0.3]])
    d3 = strut_distance(xi3, 3)
    assert np.allclose(d3, [0.5, 0.05, 0.3])


def _bspline_integrals(n_el, p=2):
    """Integral over [0, 1] of each B-spline of the open uniform knot vector: the textbook identity
    int N_a = (Xi_{a+p+1} - Xi_a) / (p + 1)."""
    kn = latticegen.open_uniform_knots(n_el, p)
    return np.array([(kn[a + p + 1] - kn[a]) / (p + 1) for a in range(n_el + p)])


@pytest.mark.parametrize("dim", [2, 3])
def test_cell_loads_closed_form_on_straight_face(dim):
    """Consistent loads (5b) entry by entry.  The macro maps fix the lattice boundary and Greville
    control points reproduce affine maps, so the loaded face X = L_x is flat and each cell's face map is
    affine with measure h^(dim-1) dxi: the load on face control point a is t h^(dim-1) prod_j int N_{a_j}
    over the tangential directions, and every other entry (other control points, cells off the face)
    is zero.  A load on the wrong face, wrong per-node weights or a wrong measure fails here."""
    if dim == 2:
        t = np.array([0.7, -0.4])
        p = latticegen.tiny(2, (3, 2), 4, tractions=[t])
    else:
        t = np.array([0.3, -0.2, 0.5])
        p = latticegen.tiny(3, (2, 2, 2), 3, tractions=[t])
    assert p.load_face == 1  # X = L_x
    ref = RefCell(dim, p.n_el)
    f = cell_loads(ref, p)[:, :, 0].reshape(p.N, -1, dim)
    I1 = _bspline_integrals(p.n_el)
    nc = p.nc
    expect = np.zeros_like(f)
    coords = latticegen.cell_coords(p.shape)
    for s in range(p.N):
        if coords[s, 0] != p.shape[0] - 1:
            continue
        for a in range(p.n_ctrl):
            mi = [(a // nc ** j) % nc for j in range(dim)]
            if mi[0] != nc - 1:
                continue
            w = p.h ** (dim - 1) * np.prod([I1[mi[j]] for j in range(1, dim)])
            expect[s, a] = w * t
    assert np.abs(f - expect).max() <= 1e-14 * np.abs(expect).max()
