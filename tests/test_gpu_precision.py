"""Precision form: fp32 / bf16 principal contractions with FP64 PCG, coarse solve and outer FGMRES
(needs an MI355X).  The outer FP64 iteration on the true operator (16) refines the result back to the
FP64 solution; the error of every result against the FP64 oracle is checked."""
import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


CASES = {
    "c1": lambda: latticegen.make("c1"),
    # ragged tile counts (rows and columns), a traction load, and a 3D lattice
    "ragged2d": lambda: latticegen.tiny(2, (5, 3), 4, n_principal=4, tractions=[[0.3, -0.7]]),
    "tiny3d": lambda: latticegen.tiny(3, (2, 2, 2), 2, n_principal=3),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print(f"[gpu precision] case {request.param}", flush=True)
    prob = CASES[request.param]()
    m = Model(prob)
    m.build_reduced_basis()
    ctx = ifeti.setup(prob, principal_in=m.sigma)
    yield prob, m, ctx
    ctx.close()


@pytest.mark.parametrize("prec,tol_op", [("fp32", 2e-6), ("bf16", 3e-2)])
def test_operators_low_precision(pair, prec, tol_op):
    from paper_2308_11371_amd import ifeti
    prob, m, ctx = pair
    p = {"fp32": ifeti.IFETI_FP32_LOCAL, "bf16": ifeti.IFETI_BF16_LOCAL}[prec]
    ctx.set_options(precision=p)
    try:
        lam = np.random.default_rng(3).standard_normal(m.L)
        v = np.random.default_rng(4).standard_normal(m.nU)
        for name, x, ref in (("F", lam, m.apply_F(lam)), ("MD", lam, m.apply_MD(lam)),
                             ("Ut", lam, m.apply_Ut(lam)), ("U", v, m.apply_U(v)),
                             ("Kinv_rom", v, m.apply_Kinv_rom(v))):
            got = getattr(ctx, "apply_" + name)(torch.tensor(x, device="cuda")).cpu().numpy()
            err = rel(got, ref)
            print(f"{prec} {name}: rel err {err:.2e}")
            assert err < tol_op
        # a block of load cases takes the same contraction per column
        X = np.random.default_rng(5).standard_normal((3, m.L))
        Y = ctx.apply_F(torch.tensor(X.ravel(), device="cuda"), nrhs=3).cpu().numpy().reshape(3, m.L)
        for r in range(3):
            assert rel(Y[r], m.apply_F(X[r])) < tol_op
        # a block of load cases in the reduced local solve: each column equals its single apply bitwise
        V = np.random.default_rng(6).standard_normal((3, m.nU))
        Z = ctx.apply_Kinv_rom(torch.tensor(V.ravel(), device="cuda"), nrhs=3).cpu().numpy().reshape(3, m.nU)
        for r in range(3):
            assert rel(Z[r], m.apply_Kinv_rom(V[r])) < tol_op
            one = ctx.apply_Kinv_rom(torch.tensor(V[r], device="cuda")).cpu().numpy()
            assert np.array_equal(Z[r], one)
    finally:
        ctx.reset_options()


@pytest.mark.parametrize("prec,inner", [("fp32", 1e-6), ("bf16", 1e-3)])
def test_refined_solve_matches_fp64_oracle(pair, prec, inner):
    from paper_2308_11371_amd import ifeti
    prob, m, ctx = pair
    ro = m.solve(tol=1e-12, inner_tol=1e-13)
    p = {"fp32": ifeti.IFETI_FP32_LOCAL, "bf16": ifeti.IFETI_BF16_LOCAL}[prec]
    ctx.set_options(precision=p)
    try:
        f, d = ctx.get_rhs()
        u, lam, info = ctx.solve(f, d, tol=1e-10, inner_tol=inner, maxit=100)
        err = rel(u.cpu().numpy(), ro["u"])
        print(f"{prec}: outer {info['outer_its'][0]} relres {info['relres'][0]:.1e} u err {err:.2e}")
        assert info["relres"][0] <= 1e-10
        assert err < 1e-6
    finally:
        ctx.reset_options()


@pytest.mark.parametrize("prec,inner", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_bf16_preconditioner_refined_solve(pair, prec, inner):
    """BF16 Dirichlet preconditioner (49) under FP64 or FP32 operators: PCG needs only a symmetric
    positive definite preconditioner, and the outer FP64 FGMRES reaches the FP64 oracle's solution."""
    from paper_2308_11371_amd import ifeti
    prob, m, ctx = pair
    ro = m.solve(tol=1e-12, inner_tol=1e-13)
    p = {"fp64": ifeti.IFETI_FP64, "fp32": ifeti.IFETI_FP32_LOCAL}[prec]
    ctx.set_options(precision=p, md_precision=ifeti.IFETI_BF16_LOCAL)
    try:
        f, d = ctx.get_rhs()
        u, lam, info = ctx.solve(f, d, tol=1e-10, inner_tol=inner, maxit=100)
        err = rel(u.cpu().numpy(), ro["u"])
        print(f"{prec} + bf16 M_D: outer {info['outer_its'][0]} relres {info['relres'][0]:.1e} u err {err:.2e}")
        assert info["relres"][0] <= 1e-10
        assert err < 1e-6
    finally:
        ctx.reset_options()

