"""Edge cases of the GPU path through the C ABI (needs an MI355X): empty batches are rejected, zero
inputs give exact zeros, a zero load gives the zero solution without iterating, and the largest
supported reduced basis (40 principal cells, the limit of the contraction kernels' coefficient
staging) matches the oracle while 41 is rejected."""
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


@pytest.fixture(scope="module")
def small():
    _cuda()
    from paper_2308_11371_amd import ifeti
    print("[gpu edge] tiny2d", flush=True)
    prob = latticegen.tiny(2, (3, 3), 3, n_principal=3)
    ctx = ifeti.setup(prob)
    yield ctx
    ctx.close()


def test_empty_batch_rejected(small):
    from paper_2308_11371_amd import ifeti
    ctx = small
    s = ctx.sizes
    x = torch.zeros(s.L, dtype=torch.float64, device="cuda")
    y = torch.zeros(s.L, dtype=torch.float64, device="cuda")
    for fn in (ctx.lib.ifeti_apply_F, ctx.lib.ifeti_apply_MD, ctx.lib.ifeti_apply_MD_rom):
        assert fn(ctx.h, x.data_ptr(), y.data_ptr(), 0) == ifeti.IFETI_EINVAL
    u = torch.zeros(s.nU + s.L, dtype=torch.float64, device="cuda")
    assert ctx.lib.ifeti_apply_A(ctx.h, u.data_ptr(), u.clone().data_ptr(), 0) == ifeti.IFETI_EINVAL


@pytest.mark.parametrize("op", ["F", "MD", "MD_rom", "U", "Ut", "Kinv_rom", "A"])
def test_zero_input_gives_zero(small, op):
    ctx = small
    s = ctx.sizes
    n = {"F": s.L, "MD": s.L, "MD_rom": s.L, "Ut": s.L, "U": s.nU, "Kinv_rom": s.nU, "A": s.nU + s.L}[op]
    got = host(getattr(ctx, "apply_" + op)(torch.zeros(n, dtype=torch.float64, device="cuda")))
    assert np.all(got == 0.0), f"{op}: max |y| = {np.abs(got).max():.3e}"


def test_zero_load_zero_solution(small):
    ctx = small
    s = ctx.sizes
    f = torch.zeros(s.nU, dtype=torch.float64, device="cuda")
    d = torch.zeros(s.L, dtype=torch.float64, device="cuda")
    u, lam, info = ctx.solve(f, d, tol=1e-10, maxit=50)
    assert np.all(host(u) == 0.0) and np.all(host(lam) == 0.0)
    assert int(info["outer_its"][0]) == 0


def test_largest_reduced_basis_matches_oracle():
    """40 principal cells of an 8 x 6 lattice with per-cell widths: every contraction stages 40
    coefficients per column.  Tolerance: at K = 40 the coefficient systems of eq. (41) reach condition
    numbers of about 2e10 (computed below), and the GPU forms their traces (42) by another arithmetic
    route (trace tables and a snapshot contraction), so π and δ agree only to rounding amplified in
    their ill-determined directions; the products then agree to about 3e-10 (1e-13 at K = 4).  A lost
    or misplaced coefficient changes them by 1e-3 or more."""
    _cuda()
    from oracle import Model
    import oracle.rom as romlib
    from paper_2308_11371_amd import ifeti
    prob = latticegen.tiny(2, (8, 6), 4, amp=0.15, width=("uniform", 0.15, 0.30, 9), smooth=True, n_principal=40)
    m = Model(prob)
    m.build_reduced_basis(n_principal=40)
    assert len(m.sigma) == 40
    b, dd = m.bank, m.dd
    Urp = b.Urp.transpose(1, 0, 2).reshape(dd.n_r, -1)
    Krr, _ = romlib.cell_blocks(m.ref, dd, m.Kvals[0])
    A = np.einsum("rip,rjp->ij", b.Urp.transpose(1, 0, 2), (Krr @ Urp).reshape(dd.n_r, 40, dd.n_p))
    assert np.linalg.cond(A) > 1e8      # the regime the tolerance is set for
    ctx = ifeti.setup(prob, principal_in=m.sigma)
    try:
        rng = np.random.default_rng(17)
        lam = rng.standard_normal(m.L)
        v = rng.standard_normal(m.nU)
        for op, x, ref in (("F", lam, m.apply_F), ("MD", lam, m.apply_MD), ("U", v, m.apply_U),
                           ("Ut", lam, m.apply_Ut), ("Kinv_rom", v, m.apply_Kinv_rom)):
            got = host(getattr(ctx, "apply_" + op)(dev(x)))
            assert rel(got, ref(x)) < 2e-9, f"{op}: rel err {rel(got, ref(x)):.3e}"
    finally:
        ctx.close()
    with pytest.raises(ifeti.IfetiError):
        ifeti.setup(latticegen.tiny(2, (8, 6), 4, amp=0.15, width=("uniform", 0.15, 0.30, 9), smooth=True,
                                    n_principal=41))


@pytest.mark.parametrize("shape,K", [((1, 1), 1), ((4, 1), 2), ((1, 3), 1)])
def test_degenerate_lattices_match_direct(shape, K):
    """A single cell (no interface multipliers, only Dirichlet rows), one-cell-wide strips, and a
    single principal cell: the solve reaches the direct solution of the conforming problem."""
    _cuda()
    from oracle import Model
    from oracle.direct import conforming_solve
    from paper_2308_11371_amd import ifeti
    prob = latticegen.tiny(2, shape, 3, n_principal=K)
    m = Model(prob)
    m.build_reduced_basis()
    ctx = ifeti.setup(prob, principal_in=m.sigma)
    try:
        f, d = ctx.get_rhs()
        u, lam, info = ctx.solve(f[:m.nU].contiguous(), d[:m.L].contiguous(), tol=1e-12, inner_tol=1e-13, maxit=80)
        ref = conforming_solve(m)
        assert info["relres"][0] < 1e-11
        assert rel(host(u), ref["u"]) < 1e-9
    finally:
        ctx.close()
