"""GPU library vs CPU oracle, call by call through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = {
    "tiny2d": lambda: latticegen.tiny(2, (3, 3), 3, n_principal=3),
    "ragged2d": lambda: latticegen.tiny(2, (5, 3), 4, n_principal=4, tractions=[[0.3, -0.7]]),
    "c1": lambda: latticegen.make("c1"),
    "tiny3d": lambda: latticegen.tiny(3, (2, 2, 2), 2, n_principal=3),
}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    _cuda()
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print(f"[gpu parity] case {request.param}", flush=True)
    prob = CASES[request.param]()
    m = Model(prob)
    m.build_reduced_basis()
    ctx = ifeti.setup(prob, principal_in=m.sigma)
    yield request.param, prob, m, ctx
    ctx.close()


def test_sizes_and_rhs(pair):
    name, prob, m, ctx = pair
    s = ctx.sizes
    dd = m.dd
    assert (s.n_i, s.n_d, s.n_p, s.n_r, s.L, s.nP, s.nU) == (dd.n_i, dd.n_d, dd.n_p, dd.n_r, m.L, dd.nP, m.nU)
    f, d = ctx.get_rhs()
    assert rel(host(f)[:m.nU], m.rhs_f[0]) < 1e-13
    assert np.array_equal(host(d)[:m.L], m.rhs_d)


def test_greedy_and_coefficients(pair):
    name, prob, m, ctx = pair
    from paper_2308_11371_amd import ifeti
    ctx2 = ifeti.setup(prob)                     # the library's own greedy
    s2 = ctx2.build_reduced_basis(prob.n_principal)
    assert list(s2) == list(m.sigma)             # index work: bit-exact
    a, p, d = ctx2.get_coefficients()
    assert np.abs(a - m.alpha).max() < 1e-10 * max(1.0, np.abs(m.alpha).max())
    assert rel(p, m.pi) < 1e-8
    assert rel(d, m.delta) < 1e-8
    ctx2.close()


def _rand(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


@pytest.mark.parametrize("op", ["F", "MD", "U", "Ut", "Kinv_rom", "A"])
def test_operator_parity(pair, op):
    name, prob, m, ctx = pair
    nU, L = m.nU, m.L
    if op in ("F", "MD"):
        x = _rand(L, 11)
    elif op == "Ut":
        x = _rand(L, 12)
    elif op == "A":
        x = _rand(nU + L, 13)
    else:
        x = _rand(nU, 14)
    expect = {"F": m.apply_F, "MD": m.apply_MD, "U": m.apply_U, "Ut": m.apply_Ut,
              "Kinv_rom": m.apply_Kinv_rom, "A": m.apply_A}[op](x)
    got = host(getattr(ctx, "apply_" + op)(dev(x)))
    assert rel(got, expect) < 1e-11, f"{name} {op}: rel err {rel(got, expect):.3e}"


def test_matrix_free_true_operator(pair):
    """The matrix-free cell operator (Remark 9: from the pulled-back tensor at the quadrature points and
    the shared 1D tables) gives the oracle's assembled K^(s) products in the true operator (16), agrees
    with the stencil form to rounding, is bitwise the same for a block of load cases as for single
    ones, and the outer solve reaches the same solution with it."""
    name, prob, m, ctx = pair
    x = _rand(m.nU + m.L, 13)
    X = np.stack([_rand(m.nU + m.L, 90 + r) for r in range(3)])
    stencil = host(ctx.apply_A(dev(x)))
    ctx.set_options(true_operator=1)
    try:
        got = host(ctx.apply_A(dev(x)))
        assert rel(got, m.apply_A(x)) < 1e-11, f"{name}: rel err {rel(got, m.apply_A(x)):.3e}"
        assert rel(got, stencil) < 1e-12
        Y = host(ctx.apply_A(dev(X.ravel()), nrhs=3)).reshape(3, -1)
        for r in range(3):
            assert np.array_equal(Y[r], host(ctx.apply_A(dev(X[r]))))
        ro = m.solve(tol=1e-12, inner_tol=1e-13, maxit=80)
        f, d = ctx.get_rhs()
        u, lam, info = ctx.solve(f[:m.nU].contiguous(), d[:m.L].contiguous(), tol=1e-12, inner_tol=1e-13,
                                 maxit=80)
        assert info["relres"][0] < 1e-11
        assert rel(host(u), ro["u"]) < 1e-9
    finally:
        ctx.reset_options()


def test_MD_rom_parity(pair):
    """M̊_D^-ROM of eq. (47) (Dirichlet preconditioner with reduced interior solves) against the
    oracle, for a single vector and a block of three."""
    name, prob, m, ctx = pair
    x = _rand(m.L, 15)
    got = host(ctx.apply_MD_rom(dev(x)))
    expect = m.apply_MD_rom(x)
    assert rel(got, expect) < 1e-10, f"{name}: rel err {rel(got, expect):.3e}"
    X = np.stack([_rand(m.L, 40 + r) for r in range(3)])
    Y = host(ctx.apply_MD_rom(dev(X.ravel()), nrhs=3)).reshape(3, m.L)
    for r in range(3):
        assert rel(Y[r], m.apply_MD_rom(X[r])) < 1e-10


@pytest.mark.parametrize("block,label", [(1, "md"), (2, "mdrom")])
def test_interface_block_variants(pair, block, label):
    """Alg. 1 with the interface block replaced by one application of (49) or (47): the outer FGMRES
    reaches the oracle's solution with the oracle's outer iteration count (±1)."""
    name, prob, m, ctx = pair
    ro = m.solve(tol=1e-10, maxit=400, interface=label)
    f, d = ctx.get_rhs()
    ctx.set_options(interface_block=block, fgmres_restart=400)  # 3D corner-only coarse spaces: >200 outer
    try:
        u, lam, info = ctx.solve(f[:m.nU].contiguous(), d[:m.L].contiguous(), tol=1e-10, maxit=400)
    finally:
        ctx.reset_options()
    assert info["relres"][0] < 1e-10
    assert rel(host(u), ro["u"]) < 1e-8
    # rounding differences may move the stop by a step or two over a few hundred iterations
    assert abs(int(info["outer_its"][0]) - ro["outer_its"]) <= max(1, ro["outer_its"] // 50)
    assert int(info["inner_its"][0]) == 0


@pytest.mark.parametrize("iters", [2, 3])
def test_mpcg_local_parity(pair, iters):
    """K̊^-MPCG (Remark 6): K̊^-ROM with multi-preconditioned CG local solves against the oracle's, and
    the outer solve with two iterations per local solve reaches the oracle's solution."""
    name, prob, m, ctx = pair
    v = _rand(m.nU, 14)
    ctx.set_options(local_iters=iters)
    m.local_iters = iters
    try:
        got = host(ctx.apply_Kinv_rom(dev(v)))
        expect = m.apply_Kinv_rom(v)
        assert rel(got, expect) < 1e-10, f"{name} MPCG {iters}: rel err {rel(got, expect):.3e}"
        if iters == 2:
            ro = m.solve(tol=1e-10, inner_tol=1e-12, maxit=80)
            f, d = ctx.get_rhs()
            u, lam, info = ctx.solve(f[:m.nU].contiguous(), d[:m.L].contiguous(), tol=1e-10, inner_tol=1e-12,
                                     maxit=80)
            assert info["relres"][0] < 1e-10
            assert rel(host(u), ro["u"]) < 1e-8
            assert abs(int(info["outer_its"][0]) - ro["outer_its"]) <= 1
    finally:
        ctx.reset_options()
        m.local_iters = 1


def test_fgmres_restart_growth(pair):
    """A solve with a larger Krylov limit than earlier solves of the same context grows the device
    tables of Krylov-block pointers; every entry must be valid again (regression: the grown table
    lost its entries while the host mirror still held them)."""
    name, prob, m, ctx = pair
    f, d = ctx.get_rhs()
    f = f[:m.nU].contiguous()
    d = d[:m.L].contiguous()
    try:
        ctx.set_options(fgmres_restart=30)
        u0, lam0, i0 = ctx.solve(f, d, tol=1e-10, maxit=30)
        ctx.set_options(fgmres_restart=300)
        u1, lam1, i1 = ctx.solve(f, d, tol=1e-10, maxit=300)
    finally:
        ctx.reset_options()
    assert np.array_equal(host(u0), host(u1)) and np.array_equal(host(lam0), host(lam1))


def test_overlap_local_bitwise(pair):
    """Reduced local solves on a third stream beside Ů v and the interface PCG: the same kernels on the
    same inputs, so the solve is bitwise that of the single-stream order."""
    name, prob, m, ctx = pair
    f, d = ctx.get_rhs()
    f = f[:m.nU].contiguous()
    d = d[:m.L].contiguous()
    ctx.set_options(overlap_local=0)
    try:
        u0, lam0, i0 = ctx.solve(f, d, tol=1e-10, maxit=80)
        ctx.set_options(overlap_local=1)
        u1, lam1, i1 = ctx.solve(f, d, tol=1e-10, maxit=80)
    finally:
        ctx.reset_options()
    assert np.array_equal(host(u0), host(u1)) and np.array_equal(host(lam0), host(lam1))
    assert int(i0["outer_its"][0]) == int(i1["outer_its"][0])


def test_cell_displacements(pair):
    """Per-cell view of u (eq. (13) layout -> each cell's own dofs, clamped corners zero): bitwise the
    oracle's, for one and two load cases."""
    name, prob, m, ctx = pair
    U = np.stack([_rand(m.nU, 80 + r) for r in range(2)])
    n_dof = m.ref.n_dof
    got = host(ctx.cell_displacements(dev(U.ravel()), nrhs=2)).reshape(2, m.N, n_dof)
    for r in range(2):
        assert np.array_equal(got[r], m.full_cell_displacements(U[r]))


def test_multi_rhs_equals_single(pair):
    name, prob, m, ctx = pair
    L = m.L
    X = np.stack([_rand(L, 20 + r) for r in range(3)])
    Y = host(ctx.apply_F(dev(X.ravel()), nrhs=3)).reshape(3, L)
    for r in range(3):
        y1 = host(ctx.apply_F(dev(X[r])))
        assert np.array_equal(Y[r], y1)
    U = np.stack([_rand(m.nU, 30 + r) for r in range(2)])
    K2 = host(ctx.apply_Kinv_rom(dev(U.ravel()), nrhs=2)).reshape(2, m.nU)
    for r in range(2):
        assert np.array_equal(K2[r], host(ctx.apply_Kinv_rom(dev(U[r]))))


def test_bitwise_repeatable(pair):
    name, prob, m, ctx = pair
    x = dev(_rand(m.L, 40))
    a = host(ctx.apply_F(x))
    b = host(ctx.apply_F(x))
    assert np.array_equal(a, b)


def test_interface_pcg(pair):
    name, prob, m, ctx = pair
    rhs = _rand(m.L, 50)
    lam_o, its_o, _ = m.solve_interface(rhs, tol=1e-12)
    lam, its, relres, st = ctx.solve_interface(dev(rhs), tol=1e-12)
    assert rel(host(lam), lam_o) < 1e-9
    assert abs(int(its[0]) - its_o) <= 2
    assert relres[0] <= 1e-12


def test_full_solve(pair):
    name, prob, m, ctx = pair
    ro = m.solve(tol=1e-12, inner_tol=1e-13, maxit=80)
    f, d = ctx.get_rhs()
    u, lam, info = ctx.solve(f[:m.nU].contiguous(), d[:m.L].contiguous(), tol=1e-12, inner_tol=1e-13, maxit=80)
    assert info["relres"][0] < 1e-11
    assert rel(host(u), ro["u"]) < 1e-9
    assert rel(host(lam), ro["lam"]) < 1e-9
    assert abs(int(info["outer_its"][0]) - ro["outer_its"]) <= 1


def test_recover_displacement(pair):
    name, prob, m, ctx = pair
    v = _rand(m.nU, 60)
    y = _rand(m.L, 61)
    expect = m.apply_Kinv_rom(v) - m.apply_Ut(y)
    got = host(ctx.recover_displacement(dev(v), dev(y)))
    assert rel(got, expect) < 1e-11


def test_block_rhs_equals_single_solves():
    """Block form: nrhs independent recurrences sharing every operator application equal nrhs
    single-load-case solves (interface PCG bitwise per iteration count, full solve to rounding)."""
    _cuda()
    from paper_2308_11371_amd import ifeti
    tr = np.array([[1.0, 0.0], [0.3, -0.8], [-0.5, 0.5]])
    prob = latticegen.tiny(2, (4, 3), 3, n_principal=3, tractions=tr)
    ctx = ifeti.setup(prob)
    s = ctx.sizes
    rng = np.random.default_rng(70)
    R = rng.standard_normal((3, s.L))
    R[2] *= 1e-3                                   # a load case that converges at a different pace
    lam3, its3, rel3, st = ctx.solve_interface(dev(R.ravel()), nrhs=3, tol=1e-11)
    for r in range(3):
        lam1, its1, rel1, _ = ctx.solve_interface(dev(R[r]), nrhs=1, tol=1e-11)
        assert its1[0] == its3[r]
        assert rel(host(lam3)[r * s.L:(r + 1) * s.L], host(lam1)) < 1e-12
    f, d = ctx.get_rhs()
    u3, l3, info3 = ctx.solve(f, d, nrhs=3, tol=1e-11, inner_tol=1e-12)
    for r in range(3):
        u1, l1, info1 = ctx.solve(f[r * s.nU:(r + 1) * s.nU].contiguous(), d[r * s.L:(r + 1) * s.L].contiguous(),
                                  tol=1e-11, inner_tol=1e-12)
        assert info1["outer_its"][0] == info3["outer_its"][r]
        assert rel(host(u3)[r * s.nU:(r + 1) * s.nU], host(u1)) < 1e-10
    ctx.close()


def test_five_rhs_match_single(pair):
    """Five load cases at once take the block forms (coarse tiles, per-cell combined small-side
    products, the restriction/prolongation and the true operator over load-case groups); each load case
    matches its single apply."""
    name, prob, m, ctx = pair
    L, nU = m.L, m.nU
    X = np.stack([_rand(L, 80 + r) for r in range(5)])
    V = np.stack([_rand(nU, 90 + r) for r in range(5)])
    S = np.stack([_rand(nU + L, 100 + r) for r in range(5)])
    for op, Z, n in (("F", X, L), ("Ut", X, nU), ("U", V, L), ("Kinv_rom", V, nU), ("A", S, nU + L)):
        Y = host(getattr(ctx, "apply_" + op)(dev(Z.ravel()), nrhs=5)).reshape(5, n)
        for r in range(5):
            y1 = host(getattr(ctx, "apply_" + op)(dev(Z[r])))
            assert rel(Y[r], y1) < 1e-12, f"{name} {op} rhs {r}: {rel(Y[r], y1):.2e}"


def test_graph_replay_equals_eager():
    """HIP-graph form of the interface PCG (first iteration eager, second captured, the rest replayed
    with host convergence polls in between): multipliers and iteration counts bitwise those of the
    eager loop, for one and for three load cases, twice in a row."""
    _cuda()
    from paper_2308_11371_amd import ifeti
    tr = np.array([[1.0, 0.0], [0.3, -0.8], [-0.5, 0.5]])
    prob = latticegen.tiny(2, (4, 3), 3, n_principal=3, tractions=tr)
    ctx = ifeti.setup(prob)
    s = ctx.sizes
    R = np.random.default_rng(71).standard_normal((3, s.L))
    for nrhs in (1, 3):
        rhs = dev(R[:nrhs].ravel())
        ctx.set_options(use_graph=0)
        lam0, its0, rel0, _ = ctx.solve_interface(rhs, nrhs=nrhs, tol=1e-11)
        ref = host(lam0)
        ctx.set_options(use_graph=1)
        for rep in range(2):
            lam1, its1, rel1, _ = ctx.solve_interface(rhs, nrhs=nrhs, tol=1e-11)
            assert list(its1) == list(its0)
            assert np.array_equal(host(lam1), ref), f"nrhs={nrhs} rep={rep}"
    f, d = ctx.get_rhs()
    ctx.set_options(use_graph=0)
    u0, l0, i0 = ctx.solve(f, d, nrhs=3, tol=1e-10, inner_tol=1e-12)
    ctx.set_options(use_graph=1)
    u1, l1, i1 = ctx.solve(f, d, nrhs=3, tol=1e-10, inner_tol=1e-12)
    assert np.array_equal(host(u0), host(u1)) and np.array_equal(host(l0), host(l1))
    assert list(i0["inner_its"]) == list(i1["inner_its"])
    ctx.close()


def test_autotuned_tiles_match_defaults():
    """With the tile autotuner on, each contraction shape is timed over its candidate tiles on first use
    and the fastest kept; every operator still matches the oracle-checked default path to rounding."""
    _cuda()
    from paper_2308_11371_amd import ifeti
    prob = latticegen.tiny(2, (5, 3), 4, n_principal=4, tractions=[[0.3, -0.7]])
    ctx = ifeti.setup(prob)
    s = ctx.sizes
    xs = {"F": _rand(s.L, 11), "MD": _rand(s.L, 12), "Ut": _rand(s.L, 13), "U": _rand(s.nU, 14),
          "Kinv_rom": _rand(s.nU, 15)}
    ref = {op: host(getattr(ctx, "apply_" + op)(dev(x))) for op, x in xs.items()}
    ctx.set_options(autotune=1)
    for rep in range(2):  # first call tunes, second uses the kept choice
        for op, x in xs.items():
            got = host(getattr(ctx, "apply_" + op)(dev(x)))
            assert rel(got, ref[op]) < 1e-13, f"{op} rep {rep}: {rel(got, ref[op]):.2e}"
    ctx.close()
