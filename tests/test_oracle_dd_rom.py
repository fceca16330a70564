"""Pins of the oracle's decomposition, greedy and ROM operators (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import latticegen
from oracle import Model
import oracle.rom as romlib
from oracle.assembly import dense
from oracle.greedy import greedy
from oracle.fetidp import ExactFETIDP
from oracle.krylov import pcg, fgmres, Breakdown


@pytest.fixture(scope="module")
def m2():
    m = Model(latticegen.tiny(2, (3, 3), 3, n_principal=3))
    m.build_reduced_basis()
    return m


@pytest.fixture(scope="module")
def m3():
    m = Model(latticegen.tiny(3, (2, 2, 2), 2, n_principal=3))
    m.build_reduced_basis()
    return m


@pytest.fixture(scope="module")
def m_ident():
    """Identical cells: the reduced basis has one element and is exact (Remark 11)."""
    m = Model(latticegen.tiny(2, (3, 3), 3, amp=0.0, map_kind="identity", n_principal=3))
    m.build_reduced_basis()
    return m


# ------------------------------------------------------------------ DD
def _conforming_field(m, rng):
    """A random conforming field scattered to the torn layout (13)."""
    dd, N = m.dd, m.N
    g = rng.standard_normal((int(np.prod(dd.Gshape)), m.problem.dim))
    g[dd.gid[dd.on_dir]] = 0.0                                  # satisfies u0 = 0 on Gamma_D
    loc = g[dd.gid].reshape(N, -1)
    uR = loc[:, dd.idx_r].reshape(-1)
    uP = np.zeros(dd.nP)
    mask = dd.Ap >= 0
    uP[dd.Ap[mask]] = loc[:, dd.idx_p][mask]
    return np.concatenate([uR, uP])


@pytest.mark.parametrize("which", ["m2", "m3"])
def test_jump_of_conforming_field_is_zero(which, request):
    m = request.getfixturevalue(which)
    u = _conforming_field(m, np.random.default_rng(0))
    assert np.abs(m.apply_B(u) - m.rhs_d).max() < 1e-14


@pytest.mark.parametrize("which", ["m2", "m3"])
def test_B_full_rank_and_entries(which, request):
    m = request.getfixturevalue(which)
    B = m.dd.BD.toarray()
    assert np.linalg.matrix_rank(B) == m.L
    assert set(np.unique(B)) <= {-1.0, 0.0, 1.0}
    # interface rows: one +1 and one -1; Dirichlet rows: a single +1
    Li = m.dd.L_interface
    assert np.all((B[:Li] == 1).sum(1) == 1) and np.all((B[:Li] == -1).sum(1) == 1)
    assert np.all((B[Li:] == 1).sum(1) == 1) and np.all((B[Li:] != 0).sum(1) == 1)


def test_weights_partition_identity_2d(m2):
    dd = m2.dd
    B = dd.BD.toarray()
    S = np.zeros((m2.L, m2.L))
    for s in range(m2.N):
        Bs = B[:, s * dd.n_d:(s + 1) * dd.n_d]
        S += Bs @ Bs.T @ np.diag(dd.Dw)
    assert np.allclose(S, np.eye(m2.L), atol=1e-15)


def test_sizes_match_formulas():
    p = latticegen.make("c1")
    m = Model(p, build_all_cells=False)
    dd = m.dd
    assert (dd.n_i, dd.n_d, dd.n_p, dd.n_r) == (128, 64, 8, 192)
    # 24 interior edges x 8 dual ctrl pts x 2 comps, plus 4 clamped cells x 8 x 2 Dirichlet rows
    assert dd.L == 24 * 8 * 2 + 4 * 8 * 2 == 448
    assert dd.nP == 4 * 5 * 2 == 40
    m3 = Model(latticegen.tiny(3, (2, 2, 2), 6), build_all_cells=False)
    assert (m3.dd.n_i, m3.dd.n_d, m3.dd.n_p) == (648, 864, 24)


# ------------------------------------------------------------------ greedy
def test_greedy_orthonormal_monotone_interpolatory(m2):
    g = m2.greedy_out
    Z = g["Z"]
    assert np.allclose(Z.T @ Z, np.eye(Z.shape[1]), atol=1e-12)
    r = g["residuals"]
    assert np.all(np.diff(r) <= 1e-15)
    assert np.allclose(g["alpha"][g["sigma"]], np.eye(len(g["sigma"])), atol=1e-12)   # eq. (55)
    assert len(set(g["sigma"].tolist())) == len(g["sigma"])


def test_greedy_exact_after_m_distinct_cells():
    # identity map and 3 distinct widths: exactly 3 distinct cells
    p = latticegen.tiny(2, (6, 2), 3, map_kind="identity", amp=0.0, width=("levels", [0.1, 0.3, 0.6]),
                        n_principal=6)
    m = Model(p)
    m.build_reduced_basis()
    assert len(np.unique(np.round(m.Kvals, 10), axis=0)) == 3
    assert len(m.sigma) == 3
    assert m.greedy_out["residuals"][-1] < 1e-14
    # affine decomposition reproduces every cell stiffness (eq. (38))
    Kt = m.alpha @ m.Kvals[m.sigma]
    assert np.abs(Kt - m.Kvals).max() < 1e-12 * np.abs(m.Kvals).max()


def test_greedy_tie_break_smallest_index():
    A = np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.0, 1.0]])
    g = greedy(A, 2)
    assert list(g["sigma"]) == [0, 2]


# ------------------------------------------------------------------ principal bank
def test_principal_identities(m2):
    b = m2.bank
    for k in range(b.K):
        assert np.allclose(b.Sdd[k] @ b.Fdd[k], np.eye(m2.dd.n_d), atol=1e-9)       # S_dd = F_dd^-1
        assert np.allclose(b.Krr[k] @ b.Urp[k], b.Krp[k], atol=1e-12)
        assert np.allclose(b.Kinv[k] @ b.Krr[k], np.eye(m2.dd.n_r), atol=1e-9)


def test_floating_Spp_annihilates_rigid_corner_values():
    p = latticegen.tiny(2, (3, 3), 3, n_principal=9, dirichlet_faces=(0,))
    m = Model(p)
    s = latticegen.cell_index((1, 1), p.shape)
    m.build_reduced_basis(principal_in=[s])
    P = p.ctrl[s][m.dd.corner_ctrl]
    t = np.zeros_like(P); t[:, 0] = 1
    rot = np.stack([-P[:, 1], P[:, 0]], 1)
    for v in (t, rot):
        assert np.abs(m.bank.Spp[0] @ v.ravel()).max() < 1e-10


def test_pi_delta_unit_at_principal_cells(m2):
    sig = m2.sigma
    assert np.allclose(m2.pi[sig], np.eye(len(sig)), atol=1e-8)
    assert np.allclose(m2.delta[sig], np.eye(len(sig)), atol=1e-8)


# ------------------------------------------------------------------ operators
def _dense_rom_F(m):
    """F̊ of eq. (48) formed explicitly as an L x L matrix from dense blocks."""
    dd, b = m.dd, m.bank
    B = dd.BD.toarray()
    L = m.L
    F = np.zeros((L, L))
    BUrp = np.zeros((L, dd.nP))
    for s in range(m.N):
        Bs = B[:, s * dd.n_d:(s + 1) * dd.n_d]
        Fs = sum(m.delta[s, k] * b.Fdd[k] for k in range(b.K))
        F += Bs @ Fs @ Bs.T
        Ap = np.zeros((dd.nP, dd.n_p))
        for j in range(dd.n_p):
            if dd.Ap[s, j] >= 0:
                Ap[dd.Ap[s, j], j] = 1.0
        Us = sum(m.pi[s, k] * b.Urp[k] for k in range(b.K))            # n_r x n_p
        BUrp += Bs @ Us[dd.n_i:] @ Ap.T
    S = m.SPP.toarray()
    return F + BUrp @ np.linalg.solve(S, BUrp.T)


def test_apply_F_equals_dense_definition(m2):
    F = _dense_rom_F(m2)
    rng = np.random.default_rng(1)
    lam = rng.standard_normal(m2.L)
    assert np.allclose(m2.apply_F(lam), F @ lam, rtol=1e-11, atol=1e-12 * np.abs(F).max())
    assert np.allclose(F, F.T, atol=1e-10 * np.abs(F).max())


def _dense_K_B(m):
    I = np.eye(m.nU)
    K = np.array([m.apply_K(I[:, j]) for j in range(m.nU)]).T
    B = np.array([m.apply_B(I[:, j]) for j in range(m.nU)]).T
    return K, B


def test_exact_F_is_BKinvBt(m2):
    """Eq. (26): the exact FETI-DP operator equals B K^-1 B^T."""
    K, B = _dense_K_B(m2)
    ex = ExactFETIDP(m2)
    I = np.eye(m2.L)
    Fex = np.array([ex.apply_F(I[:, j]) for j in range(m2.L)]).T
    assert np.allclose(Fex, B @ np.linalg.solve(K, B.T), atol=1e-10 * np.abs(Fex).max())
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())
    assert np.all(np.linalg.eigvalsh(K) > 0)


def test_rom_operators_exact_for_identical_cells(m_ident):
    m = m_ident
    assert len(m.sigma) == 1
    ex = ExactFETIDP(m)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(m.L)
    assert np.allclose(m.apply_F(lam), ex.apply_F(lam), rtol=1e-10, atol=1e-12)
    assert np.allclose(m.apply_MD(lam), ex.apply_MD(lam), rtol=1e-10, atol=1e-12)
    K, B = _dense_K_B(m)
    v = rng.standard_normal(m.nU)
    assert np.allclose(m.apply_U(v), B @ np.linalg.solve(K, v), rtol=1e-9, atol=1e-11)
    assert np.allclose(m.apply_Ut(lam), np.linalg.solve(K, B.T @ lam), rtol=1e-9, atol=1e-11)
    assert np.allclose(m.apply_Kinv_rom(v), np.linalg.solve(K, v), rtol=1e-9, atol=1e-11)


def test_Kinv_rom_exact_when_every_cell_is_principal():
    p = latticegen.tiny(2, (2, 2), 3, n_principal=4)
    m = Model(p)
    m.build_reduced_basis(principal_in=[0, 1, 2, 3])
    assert len(m.sigma) == 4
    K, _ = _dense_K_B(m)
    v = np.random.default_rng(3).standard_normal(m.nU)
    assert np.allclose(m.apply_Kinv_rom(v), np.linalg.solve(K, v), rtol=1e-8, atol=1e-10)


def test_rom_local_solve_exact_on_principal_cell(m2):
    rng = np.random.default_rng(4)
    vR = rng.standard_normal((m2.N, m2.dd.n_r))
    x = m2.rom_local_solve(vR)
    for k, s in enumerate(m2.sigma):
        assert np.allclose(x[s], m2.bank.Kinv[k] @ vR[s], rtol=1e-8, atol=1e-10)


def test_Ut_is_transpose_of_U(m2):
    rng = np.random.default_rng(5)
    v = rng.standard_normal(m2.nU)
    y = rng.standard_normal(m2.L)
    assert np.isclose(y @ m2.apply_U(v), v @ m2.apply_Ut(y), rtol=1e-11)


# ------------------------------------------------------------------ Krylov
def test_pcg_matches_dense_and_detects_breakdown():
    rng = np.random.default_rng(6)
    Q = rng.standard_normal((30, 30))
    A = Q @ Q.T + 30 * np.eye(30)
    b = rng.standard_normal(30)
    x, its, _ = pcg(lambda v: A @ v, lambda v: v / np.diag(A), b, tol=1e-13)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-11)
    with pytest.raises(Breakdown):
        pcg(lambda v: -v, lambda v: v, b)


def test_fgmres_matches_dense_and_one_step_with_exact_inverse():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((25, 25)) + 10 * np.eye(25)
    b = rng.standard_normal(25)
    x, its, _ = fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-13, maxit=25)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10)
    Ainv = np.linalg.inv(A)
    x1, its1, _ = fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-10)
    assert its1 == 1 and np.allclose(x1, np.linalg.solve(A, b), rtol=1e-10)


def test_MD_rom_is_exact_dirichlet_when_every_cell_is_principal():
    """Eq. (47) with every cell principal: the reduced interior solve contains K_ii^(s)-1 w itself, so
    M̊_D^-ROM is the exact Dirichlet preconditioner (30) (interior Cholesky in the exact FETI-DP)."""
    p = latticegen.tiny(2, (2, 2), 3, n_principal=4)
    m = Model(p)
    m.build_reduced_basis(principal_in=[0, 1, 2, 3])
    ex = ExactFETIDP(m)
    lam = np.random.default_rng(6).standard_normal(m.L)
    assert np.allclose(m.apply_MD_rom(lam), ex.apply_MD(lam), rtol=1e-9, atol=1e-11)


def test_MD_rom_is_exact_dirichlet_for_identical_cells(m_ident):
    ex = ExactFETIDP(m_ident)
    lam = np.random.default_rng(7).standard_normal(m_ident.L)
    assert np.allclose(m_ident.apply_MD_rom(lam), ex.apply_MD(lam), rtol=1e-9, atol=1e-11)


def test_MD_rom_positively_homogeneous_and_energy_positive(m2):
    """The reduced solve is a Galerkin projection onto a space spanned by the input's own principal
    solves: scaling the input scales the output, and rᵀ M̊_D^-ROM r ≥ rᵀ M_D^-1 r > 0 (a Galerkin
    approximation of K_ii^-1 w under-estimates wᵀ K_ii^-1 w, so S̃_dd over-estimates S_dd)."""
    ex = ExactFETIDP(m2)
    r = np.random.default_rng(8).standard_normal(m2.L)
    y = m2.apply_MD_rom(r)
    assert np.allclose(m2.apply_MD_rom(-2.5 * r), -2.5 * y, rtol=1e-12, atol=1e-13)
    assert r @ y >= r @ ex.apply_MD(r) * (1 - 1e-12) > 0


def test_mpcg_local_solve_improves_and_converges(m2):
    """Remark 6: the multi-preconditioned CG local solve minimises the K_rr^(s)-energy error over a
    growing conjugate space, so the error never grows with the iteration count, the first iteration
    is eq. (46), and enough iterations give K_rr^(s)-1 v (checked against a dense solve per cell)."""
    rng = np.random.default_rng(9)
    vR = rng.standard_normal((m2.N, m2.dd.n_r))
    exact = np.array([np.linalg.solve(romlib.cell_blocks(m2.ref, m2.dd, m2.Kvals[s])[0].toarray(), vR[s])
                      for s in range(m2.N)])
    x1 = m2.rom_local_solve(vR, iters=1)
    assert np.allclose(m2._mpcg_local_solve(vR, 1), x1, rtol=1e-10, atol=1e-12)
    prev = None
    for it in (1, 2, 3, 5):
        x = m2.rom_local_solve(vR, iters=it)
        err = []
        for s in range(m2.N):
            Krr = romlib.cell_blocks(m2.ref, m2.dd, m2.Kvals[s])[0]
            e = x[s] - exact[s]
            err.append(e @ (Krr @ e))
        err = np.array(err)
        if prev is not None:
            assert np.all(err <= prev * (1 + 1e-8) + 1e-20)
        prev = err
    n_r, K = m2.dd.n_r, m2.bank.K
    xf = m2.rom_local_solve(vR, iters=n_r // K + 4)
    assert np.allclose(xf, exact, rtol=1e-8, atol=1e-10)
