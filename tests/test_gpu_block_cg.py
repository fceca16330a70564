"""Block PCG across load cases (option block_cg) against the oracle's block PCG and dense solves
(needs an MI355X).

O'Leary's block conjugate gradients in the breakdown-free form: all load cases' interface problems
(48) in one block Krylov space, the search block re-orthonormalised every iteration with linearly
dependent directions dropped.  Checked: the multipliers of every load case against the dense solution
of F̊, the block iteration count against the oracle's, dependent, tiny and zero load cases, and the
full solve (16) with the block form inside the preconditioner against the single-load-case solves.
"""
import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=["tiny2d", "ragged3d"])
def pair(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print(f"[gpu block cg] case {request.param}", flush=True)
    if request.param == "tiny2d":
        prob = latticegen.tiny(2, (4, 3), 3, n_principal=3)
    else:
        prob = latticegen.tiny(3, (3, 2, 2), 2, n_principal=4)
    m = Model(prob)
    m.build_reduced_basis()
    ctx = ifeti.setup(prob, principal_in=m.sigma)
    Fd = np.stack([m.apply_F(e) for e in np.eye(m.L)], axis=1)
    yield request.param, m, ctx, Fd
    ctx.close()


def _block_rhs(L, seed):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((L, 6))
    R[:, 2] = R[:, 0] - 0.5 * R[:, 1]     # dependent on two others
    R[:, 3] *= 1e-9                       # far below the others: keeps its own direction
    R[:, 4] = 0.0                         # zero load case
    R[:, 5] = 2.0 * R[:, 0]               # parallel to the first
    return R


def test_block_pcg_matches_dense_and_oracle(pair):
    from oracle.krylov import block_pcg
    name, m, ctx, Fd = pair
    R = _block_rhs(m.L, 11)
    ref = np.linalg.solve(Fd, R)
    Xo, ito, _ = block_pcg(m.apply_F, m.apply_MD, R, tol=1e-12)
    ctx.set_options(block_cg=1)
    try:
        lam, its, relres, st = ctx.solve_interface(dev(R.T.ravel()), nrhs=6, tol=1e-12)
    finally:
        ctx.reset_options()
    X = host(lam).reshape(6, m.L)
    errs = [rel(X[j], ref[:, j]) for j in range(6)]
    print(f"[gpu block cg] {name}: {int(its[0])} block its (oracle {ito}), errors {np.max(errs):.1e}, "
          f"relres {np.max(relres):.1e}", flush=True)
    assert st == 0
    assert max(errs) < 1e-9
    assert not X[4].any() and relres[4] == 0.0 and its[4] == 0
    assert max(relres) <= 1e-12
    assert abs(int(its[0]) - ito) <= max(2, ito // 10)
    assert max(rel(X[j], Xo[:, j]) for j in range(6)) < 1e-9


def test_block_pcg_needs_fewer_iterations_than_separate(pair):
    """Independent load cases: the block space holds every column's Krylov space, so the block count
    is at most the largest single count."""
    name, m, ctx, Fd = pair
    R = np.random.default_rng(12).standard_normal((4, m.L))
    _, its1, _, _ = ctx.solve_interface(dev(R.ravel()), nrhs=4, tol=1e-11)
    ctx.set_options(block_cg=1)
    try:
        lam, itsb, relres, st = ctx.solve_interface(dev(R.ravel()), nrhs=4, tol=1e-11)
    finally:
        ctx.reset_options()
    assert st == 0 and max(relres) <= 1e-11
    assert int(itsb[0]) <= int(max(its1))
    X = host(lam).reshape(4, m.L)
    assert max(rel(X[j], np.linalg.solve(Fd, R[j])) for j in range(4)) < 1e-8


def test_full_solve_with_block_interface(pair):
    """FGMRES on (16) with the block form inside the preconditioner: every load case's displacements
    and multipliers equal its single-load-case solve to the stop tolerance."""
    name, m, ctx, Fd = pair
    s = ctx.sizes
    f, d = ctx.get_rhs()
    # the problem's load, an independent random load, and the problem's load scaled by 1e-4
    F3 = torch.cat([f[:s.nU], dev(np.random.default_rng(13).standard_normal(s.nU)), 1e-4 * f[:s.nU]])
    D3 = torch.cat([d[:s.L], torch.zeros_like(d[:s.L]), 1e-4 * d[:s.L]])
    ctx.set_options(block_cg=1)
    try:
        u3, l3, info3 = ctx.solve(F3, D3, nrhs=3, tol=1e-11, inner_tol=1e-12)
    finally:
        ctx.reset_options()
    U3 = host(u3).reshape(3, s.nU)
    for r in range(3):
        u1, l1, info1 = ctx.solve(F3[r * s.nU:(r + 1) * s.nU].contiguous(), D3[r * s.L:(r + 1) * s.L].contiguous(),
                                  tol=1e-11, inner_tol=1e-12)
        assert rel(U3[r], host(u1)) < 1e-9
    assert info3["relres"].max() <= 1e-10
