"""Boundary of the library through the C ABI (needs an MI355X).

* Dirichlet data u0(x) = G x (eq. (3c)): d of eq. (14) on the Dirichlet rows and the lifting of the
  eliminated primal corners, against the oracle's right-hand side; the patch test (homogeneous
  material, u0 = eps x on the whole boundary, no load) reproduces u = eps P at every control point;
  a clamped-plus-displaced lattice under load reaches the oracle's solution.
* Failure statuses: EMAXIT (iteration limits), EBREAKDOWN (a non-finite right-hand side), ENOTSPD (a
  principal K_rr made singular by void regions with E_out = 0), EINVAL (width gradient with the sharp
  strut indicator) — each returned with a message, the context usable afterwards.
* Options are merged (ifeti_get_options), and two stale-state regressions: a cached PCG graph after
  the coarse partition changes, and the fragment copy of a rebuilt exact coarse inverse.
"""
import dataclasses

import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


EPS = {2: np.array([[1e-3, 2e-4], [-5e-4, 3e-4]]),
       3: np.array([[1e-3, 2e-4, 0.0], [-5e-4, 3e-4, 1e-4], [2e-4, 0.0, -4e-4]])}


@pytest.mark.parametrize("dim,shape,n_el", [(2, (3, 2), 3), (3, (2, 2, 2), 2), (3, (2, 2, 1), 2)])
def test_patch_test_through_gpu(dim, shape, n_el):
    """Homogeneous material and u0 = eps x on every face, no load: the GPU solve gives u = eps P at every
    control point (Greville geometry is isoparametric), and f, d equal the oracle's."""
    _cuda()
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print(f"[gpu boundary] patch test dim={dim} shape={shape}", flush=True)
    eps = EPS[dim]
    p = latticegen.tiny(dim, shape, n_el, E_out=1.0, dirichlet_faces=tuple(range(2 * dim)), load_face=-1,
                        u0_grad=eps, tractions=np.zeros((1, dim)), n_principal=2)
    m = Model(p)
    m.build_reduced_basis()
    ctx = ifeti.setup(p, principal_in=m.sigma)
    f, d = ctx.get_rhs()
    assert rel(host(d), m.rhs_d) < 1e-14
    assert np.linalg.norm(host(f) - m.rhs_f[0]) <= 1e-13 * max(np.linalg.norm(m.rhs_f[0]), 1e-30)
    u, lam, info = ctx.solve(f, d, tol=1e-13, inner_tol=1e-14, maxit=80)
    s = ctx.sizes
    cu = host(ctx.cell_displacements(u)).reshape(p.N, s.n_ctrl, dim)
    expect = p.ctrl @ eps.T
    err = np.abs(cu - expect).max() / np.abs(expect).max()
    print(f"patch test dim={dim} shape={shape}: outer {info['outer_its'][0]}, max |u - eps P| / max |eps P| "
          f"= {err:.2e}")
    assert err < 1e-12
    ctx.close()


def test_displaced_face_under_load_matches_oracle():
    """Left face displaced by u0 = G x, traction on the right face: right-hand side and solution of
    (16) against the oracle (same principal cells)."""
    _cuda()
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    G = np.array([[2e-3, -1e-3], [5e-4, 1e-3]])
    p = latticegen.tiny(2, (4, 3), 4, u0_grad=G, tractions=[[0.4, -0.2]], n_principal=3)
    m = Model(p)
    m.build_reduced_basis()
    ctx = ifeti.setup(p, principal_in=m.sigma)
    f, d = ctx.get_rhs()
    assert rel(host(d), m.rhs_d) < 1e-14
    assert rel(host(f), m.rhs_f[0]) < 1e-13
    ro = m.solve(tol=1e-12, inner_tol=1e-13)
    u, lam, info = ctx.solve(f, d, tol=1e-12, inner_tol=1e-13)
    eu, el = rel(host(u), ro["u"]), rel(host(lam), ro["lam"])
    print(f"displaced face: u err {eu:.2e}, lam err {el:.2e}")
    assert eu < 1e-9 and el < 1e-9
    ctx.close()


@pytest.fixture(scope="module")
def small():
    _cuda()
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print("[gpu boundary] small lattice", flush=True)
    p = latticegen.tiny(2, (4, 3), 3, n_principal=3)
    m = Model(p)
    m.build_reduced_basis()
    ctx = ifeti.setup(p, principal_in=m.sigma)
    yield p, m, ctx
    ctx.close()


def _reference_solve(ctx):
    f, d = ctx.get_rhs()
    u, lam, info = ctx.solve(f, d, tol=1e-10, inner_tol=1e-11)
    return host(u), host(lam)


def test_emaxit_keeps_partial_result_and_context(small):
    from paper_2308_11371_amd import ifeti
    p, m, ctx = small
    u_ref, lam_ref = _reference_solve(ctx)
    rhs = dev(np.random.default_rng(5).standard_normal(m.L))
    lam, its, rel_, st = ctx.solve_interface(rhs, tol=1e-12, maxit=1, check=False)
    assert st == ifeti.IFETI_EMAXIT
    assert "iteration limit" in ifeti.load().ifeti_last_error().decode()
    assert its[0] == 1 and 0 < rel_[0] < 1 and np.all(np.isfinite(host(lam)))
    f, d = ctx.get_rhs()
    u, lam, info = ctx.solve(f, d, tol=1e-10, inner_tol=1e-11, maxit=1, check=False)
    assert info["status"] == ifeti.IFETI_EMAXIT and info["outer_its"][0] == 1
    assert np.all(np.isfinite(host(u)))
    u2, lam2 = _reference_solve(ctx)
    assert np.array_equal(u2, u_ref) and np.array_equal(lam2, lam_ref)


def test_ebreakdown_on_non_finite_input(small):
    from paper_2308_11371_amd import ifeti
    p, m, ctx = small
    u_ref, lam_ref = _reference_solve(ctx)
    rhs = np.random.default_rng(6).standard_normal(m.L)
    rhs[7] = np.nan
    lam, its, rel_, st = ctx.solve_interface(dev(rhs), tol=1e-11, check=False)
    assert st == ifeti.IFETI_EBREAKDOWN
    assert "breakdown" in ifeti.load().ifeti_last_error().decode()
    assert its[0] == 0
    f, d = ctx.get_rhs()
    fn = f.clone()
    fn[3] = float("inf")
    u, lam, info = ctx.solve(fn, d, tol=1e-10, inner_tol=1e-11, check=False)
    assert info["status"] == ifeti.IFETI_EBREAKDOWN
    u2, lam2 = _reference_solve(ctx)
    assert np.array_equal(u2, u_ref) and np.array_equal(lam2, lam_ref)


def test_enotspd_singular_principal_then_recovery():
    """E_out = 0 with thin struts leaves control points whose whole support is void: the principal
    K_rr is singular and the offline phase returns ENOTSPD; the context then rebuilds with full
    struts and solves."""
    _cuda()
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print("[gpu boundary] ENOTSPD", flush=True)
    p = latticegen.tiny(2, (2, 2), 16, amp=0.0, map_kind="identity", E_out=0.0, width=("const", 0.02),
                        n_principal=1)
    ctx = ifeti.Context.from_problem(p)
    ctrl = dev(p.ctrl)
    ctx.build_cells(ctrl, dev(p.widths), p.tractions)
    with pytest.raises(ifeti.IfetiError) as e:
        ctx.build_reduced_basis(1)
    assert e.value.status == ifeti.IFETI_ENOTSPD
    assert "positive definite" in str(e.value)
    with pytest.raises(ifeti.IfetiError) as e2:  # no reduced basis: the operators refuse
        ctx.apply_F(dev(np.zeros(ctx.sizes.L)))
    assert e2.value.status == ifeti.IFETI_EINVAL
    q = dataclasses.replace(p, widths=np.full(p.N, 1.0))  # struts cover the cells: E = E_in everywhere
    ctx.build_cells(ctrl, dev(q.widths), q.tractions)
    ctx.build_reduced_basis(1)
    m = Model(q)
    m.build_reduced_basis(principal_in=list(ctx.sigma))
    f, d = ctx.get_rhs()
    u, lam, info = ctx.solve(f, d, tol=1e-12, inner_tol=1e-13)
    ro = m.solve(tol=1e-12, inner_tol=1e-13)
    assert rel(host(u), ro["u"]) < 1e-9
    ctx.close()


def test_sharp_indicator_gradient_rejected(small):
    from paper_2308_11371_amd import ifeti
    p, m, ctx = small
    assert p.smooth_eps == 0.0
    f, d = ctx.get_rhs()
    with pytest.raises(ifeti.IfetiError) as e:
        ctx.compliance_grad(f, f)
    assert e.value.status == ifeti.IFETI_EINVAL and "smooth" in str(e.value)


def test_set_options_merges(small):
    from paper_2308_11371_amd import ifeti
    p, m, ctx = small
    ctx.set_options(use_graph=1, autotune=1, pcg_maxit=321)
    ctx.set_options(precision=ifeti.IFETI_FP32_LOCAL)
    o = ctx.get_options()
    assert (o["use_graph"], o["autotune"], o["pcg_maxit"], o["precision"]) == (1, 1, 321, ifeti.IFETI_FP32_LOCAL)
    ctx.reset_options()
    assert ctx.get_options() == ifeti.DEFAULT_OPTIONS


def test_graph_after_coarse_partition_change_equals_eager():
    """A cached PCG graph holds the partitioned coarse solve's buffers and row counts: after the
    partition changes, the graph solve must equal the eager solve with the new partition bitwise."""
    _cuda()
    from paper_2308_11371_amd import ifeti
    p = latticegen.tiny(2, (10, 7), 3, n_principal=4)
    ctx = ifeti.setup(p)
    rhs = dev(np.random.default_rng(8).standard_normal(ctx.sizes.L))
    ctx.set_options(coarse_parts=2, use_graph=1)
    ctx.solve_interface(rhs, tol=1e-11)               # captures a graph with the 2-block partition
    for parts in (3, 5):
        ctx.set_options(coarse_parts=parts, use_graph=0)
        lam0, its0, _, _ = ctx.solve_interface(rhs, tol=1e-11)
        ctx.set_options(use_graph=1)
        lam1, its1, _, _ = ctx.solve_interface(rhs, tol=1e-11)
        assert list(its1) == list(its0)
        assert np.array_equal(host(lam1), host(lam0)), f"coarse_parts={parts}"
    ctx.close()


def test_exact_block_solve_after_width_update_and_rebuild():
    """The exact coarse inverse is rebuilt in place by ifeti_build_exact after a width update; its
    fragment copy (used by the coarse contraction of >= 4 load cases) must follow."""
    _cuda()
    from oracle import Model
    from oracle.fetidp import ExactFETIDP
    from paper_2308_11371_amd import ifeti
    tr = np.array([[1.0, 0.0], [0.2, 0.9], [-0.6, 0.4], [0.5, -0.5]])
    p = latticegen.tiny(2, (5, 3), 3, smooth=True, width=("uniform", 0.15, 0.30, 9), tractions=tr,
                        n_principal=3)
    ctx = ifeti.setup(p)
    ctx.build_exact()
    f, d = ctx.get_rhs()
    ctx.exact_solve(f, d, nrhs=4, tol=1e-12)          # builds the fragment copy of the coarse inverse
    w2 = p.widths * 1.15
    ctx.update_widths(dev(w2))
    ctx.build_exact()
    f, d = ctx.get_rhs()
    u, lam, info = ctx.exact_solve(f, d, nrhs=4, tol=1e-12)
    q = dataclasses.replace(p, widths=w2)
    m = Model(q)
    ex = ExactFETIDP(m)
    U = host(u).reshape(4, -1)
    for r in range(4):
        ro = ex.solve(rhs_index=r, tol=1e-12)
        assert rel(U[r], ro["u"]) < 1e-9, f"load case {r}: {rel(U[r], ro['u']):.2e}"
    ctx.close()
