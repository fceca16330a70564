"""Full-solve pins of the oracle: the ROM-FETI-DP reaches the conforming FE solution (CPU only)."""
import numpy as np
import pytest

import latticegen
from oracle import Model
from oracle.direct import conforming_solve
from oracle.fetidp import ExactFETIDP


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dim,shape,n_el,K", [
    (2, (1, 1), 3, 1), (2, (2, 2), 3, 2), (2, (3, 3), 3, 3), (2, (4, 2), 4, 3), (3, (2, 2, 2), 2, 3)])
def test_rom_fetidp_equals_direct_cholesky(dim, shape, n_el, K):
    m = Model(latticegen.tiny(dim, shape, n_el, n_principal=K))
    m.build_reduced_basis()
    r = m.solve(tol=1e-12, inner_tol=1e-13, maxit=60)
    ref = conforming_solve(m)
    assert r["relres"] < 1e-11
    assert _rel(r["u"], ref["u"]) < 1e-10
    assert _rel(r["lam"], ref["lam"]) < 1e-9
    # energy identity f^T u = u^T K u (no Dirichlet lifting: u0 = 0)
    f = m.rhs_f[0]
    assert np.isclose(f @ r["u"], r["u"] @ m.apply_K(r["u"]), rtol=1e-9)


def test_c1_solve_matches_direct():
    m = Model(latticegen.make("c1"))
    m.build_reduced_basis()
    r = m.solve(tol=1e-12, inner_tol=1e-13)
    ref = conforming_solve(m)
    assert _rel(r["u"], ref["u"]) < 1e-10
    assert r["outer_its"] < 20


@pytest.mark.parametrize("dim,shape", [(2, (3, 2)), (3, (2, 2, 1))])
def test_patch_test_uniform_strain_reproduced(dim, shape):
    """Homogeneous material, u0 = eps x on the whole boundary => u = eps P at every control point."""
    eps = np.array([[1e-3, 2e-4], [-5e-4, 3e-4]]) if dim == 2 else \
        np.array([[1e-3, 2e-4, 0.0], [-5e-4, 3e-4, 1e-4], [2e-4, 0.0, -4e-4]])
    faces = tuple(range(2 * dim))
    p = latticegen.tiny(dim, shape, 3 if dim == 2 else 2, E_out=1.0, dirichlet_faces=faces, load_face=-1,
                        u0_grad=eps, tractions=np.zeros((1, dim)), n_principal=2)
    m = Model(p)
    m.build_reduced_basis()
    r = m.solve(tol=1e-13, inner_tol=1e-14, maxit=80)
    u = m.full_cell_displacements(r["u"]).reshape(p.N, -1, dim)
    expect = p.ctrl @ eps.T
    assert np.abs(u - expect).max() < 1e-12 * np.abs(expect).max() * 1e3
    ref = conforming_solve(m)
    ud = ref["u_global"][ref["cdof"]].reshape(p.N, -1, dim)
    assert np.abs(ud - expect).max() < 1e-10 * np.abs(expect).max()


def test_identical_cells_one_global_iteration():
    """Remark 11: with identical cells the ROM is exact and one global iteration suffices."""
    p = latticegen.tiny(2, (4, 3), 3, amp=0.0, map_kind="identity", n_principal=4)
    m = Model(p)
    m.build_reduced_basis()
    assert len(m.sigma) == 1
    r = m.solve(tol=1e-8, inner_tol=1e-12)
    assert r["outer_its"] == 1


def test_local_iterations_match_standard_fetidp():
    """Tables 1-2: the interface PCG needs (about) as many iterations as standard FETI-DP."""
    m = Model(latticegen.tiny(2, (4, 4), 4, n_principal=4))
    m.build_reduced_basis()
    r = m.solve(tol=1e-8, inner_tol=1e-11)
    ex = ExactFETIDP(m).solve(tol=1e-11)
    assert abs(np.median(r["inner_its"]) - ex["its"]) <= 2


def test_more_principals_fewer_outer_iterations():
    m = Model(latticegen.make("c1"))
    its = []
    for K in (1, 4):
        m.build_reduced_basis(n_principal=K)
        its.append(m.solve(tol=1e-8)["outer_its"])
    assert its[1] <= its[0]


@pytest.mark.parametrize("interface", ["md", "mdrom"])
def test_interface_block_variants_reach_direct_solution(interface):
    """Alg. 1 with the interface block -F̊^-pcg replaced by one application of M̊_D^-1 (49) or of
    M̊_D^-ROM (47): FGMRES still reaches the conforming solution of (16), with more outer iterations."""
    m = Model(latticegen.tiny(2, (3, 3), 3, n_principal=3))
    m.build_reduced_basis()
    r = m.solve(tol=1e-12, maxit=200, interface=interface)
    ref = conforming_solve(m)
    assert r["relres"] < 1e-11
    assert _rel(r["u"], ref["u"]) < 1e-9
    assert r["outer_its"] >= m.solve(tol=1e-12, inner_tol=1e-13)["outer_its"]
    assert sum(r["inner_its"]) == 0


def test_mpcg_local_solves_reach_direct_solution():
    """K̊^-MPCG (Remark 6, two multi-preconditioned CG iterations per local solve) inside Alg. 1: the
    outer FGMRES reaches the conforming solution, in no more outer iterations than with eq. (46)."""
    m = Model(latticegen.tiny(2, (3, 3), 3, n_principal=3))
    m.build_reduced_basis()
    r1 = m.solve(tol=1e-12, inner_tol=1e-13, maxit=80)
    m.local_iters = 2
    r2 = m.solve(tol=1e-12, inner_tol=1e-13, maxit=80)
    ref = conforming_solve(m)
    assert r2["relres"] < 1e-11
    assert _rel(r2["u"], ref["u"]) < 1e-10
    assert r2["outer_its"] <= r1["outer_its"]


@pytest.mark.parametrize("dim,shape,n_el", [(2, (3, 2), 3), (3, (2, 2, 2), 2)])
def test_exact_fetidp_solve_equals_direct_cholesky(dim, shape, n_el):
    """Standard FETI-DP (Sec. 2.2.4): the right-hand side d̄ of eq. (25), PCG on F (24) with M_D (30) and
    the recovery of eqs. (21) then (20) reach the conforming solution of (16) and its multipliers."""
    p = latticegen.tiny(dim, shape, n_el, n_principal=2)
    m = Model(p)
    ref = conforming_solve(m)
    r = ExactFETIDP(m).solve(tol=1e-13, maxit=500)
    eu = np.linalg.norm(r["u"] - ref["u"]) / np.linalg.norm(ref["u"])
    el = np.linalg.norm(r["lam"] - ref["lam"]) / np.linalg.norm(ref["lam"])
    assert eu < 1e-10, eu
    assert el < 1e-9, el


def test_block_jacobi_coarse_solve_limits_and_spd():
    """Approximate coarse solve (Sec. 3.2.1): block Jacobi over blocks of B primal dofs is the exact
    banded Cholesky solve for B >= nP, diagonal scaling for B = 1, and symmetric positive definite for
    any B (so F̊ stays symmetric and the interface PCG valid)."""
    from oracle.rom import BlockJacobiCoarse
    m = Model(latticegen.tiny(2, (5, 4), 3, n_principal=3))
    m.build_reduced_basis()
    n = m.dd.nP
    rng = np.random.default_rng(3)
    z, w = rng.standard_normal(n), rng.standard_normal(n)
    exact = m.coarse.solve(z)
    assert _rel(BlockJacobiCoarse(m.SPP, n).solve(z), exact) < 1e-12
    assert _rel(BlockJacobiCoarse(m.SPP, n + 7).solve(z), exact) < 1e-12
    assert np.allclose(BlockJacobiCoarse(m.SPP, 1).solve(z), z / m.SPP.diagonal(), rtol=1e-13)
    for B in (2, 5, 16):
        bj = BlockJacobiCoarse(m.SPP, B)
        a, b = w @ bj.solve(z), z @ bj.solve(w)
        assert abs(a - b) <= 1e-12 * abs(a)
        assert z @ bj.solve(z) > 0
    m.set_coarse_block(8)
    l1, l2 = rng.standard_normal(m.L), rng.standard_normal(m.L)
    a, b = l1 @ m.apply_F(l2), l2 @ m.apply_F(l1)
    assert abs(a - b) <= 1e-11 * abs(a)


@pytest.mark.parametrize("B", [1, 8])
def test_block_jacobi_coarse_solve_reaches_direct_solution(B):
    """With the approximate coarse solve in every coarse correction, the outer FGMRES on the true
    operator (16) still reaches the conforming solution."""
    m = Model(latticegen.tiny(2, (4, 3), 3, n_principal=3))
    m.build_reduced_basis()
    m.set_coarse_block(B)
    r = m.solve(tol=1e-12, inner_tol=1e-13, maxit=150)
    assert _rel(r["u"], conforming_solve(m)["u"]) < 1e-9


def test_block_pcg_one_column_follows_pcg_and_rank_deficient_blocks_converge():
    """O'Leary's block CG (breakdown-free form): with one column it is PCG; on a block whose columns are
    linearly dependent (b1, b2, b1 + b2, 2 b1) every column reaches the dense solution without
    breakdown, in no more iterations than the single-column solves; on F̊ with M̊_D^-1 likewise."""
    from oracle.krylov import pcg, block_pcg
    rng = np.random.default_rng(4)
    n = 60
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Qm @ np.diag(np.logspace(0, 3, n)) @ Qm.T
    Dm = 1.0 / np.diag(A)
    fA, fM = (lambda v: A @ v), (lambda v: Dm * v)
    b1, b2 = rng.standard_normal(n), rng.standard_normal(n)
    x1, it1, h1 = pcg(fA, fM, b1, tol=1e-12)
    X, itb, hb = block_pcg(fA, fM, b1[:, None], tol=1e-12)
    # the same iterates in exact arithmetic: equal residual histories until finite-precision loss of
    # orthogonality separates the two recurrences, and the same converged solution
    assert np.allclose(hb[:15], h1[:15], rtol=1e-8, atol=0.0)
    assert abs(itb - it1) <= 3 and _rel(X[:, 0], x1) < 1e-10
    B = np.stack([b1, b2, b1 + b2, 2 * b1], axis=1)
    X, itb, _ = block_pcg(fA, fM, B, tol=1e-12)
    ref = np.linalg.solve(A, B)
    assert max(_rel(X[:, j], ref[:, j]) for j in range(4)) < 1e-10
    assert itb <= max(pcg(fA, fM, B[:, j], tol=1e-12)[1] for j in range(4))
    m = Model(latticegen.tiny(2, (3, 3), 3, n_principal=3))
    m.build_reduced_basis()
    R = rng.standard_normal((m.L, 3))
    R[:, 2] = R[:, 0] - 0.5 * R[:, 1]
    X, itb, _ = block_pcg(m.apply_F, m.apply_MD, R, tol=1e-12)
    Fd = np.stack([m.apply_F(e) for e in np.eye(m.L)], axis=1)
    ref = np.linalg.solve(Fd, R)
    assert max(_rel(X[:, j], ref[:, j]) for j in range(3)) < 1e-9
    # a load case 1e-9 times smaller than the others keeps its own direction (the drop test compares
    # unit columns), and a zero load case stays zero
    B = np.stack([b1, 1e-9 * b2, np.zeros(n), 2 * b1], axis=1)
    X, itb, _ = block_pcg(fA, fM, B, tol=1e-12)
    ref = np.linalg.solve(A, B)
    assert max(_rel(X[:, j], ref[:, j]) for j in (0, 1, 3)) < 1e-10
    assert not X[:, 2].any()
