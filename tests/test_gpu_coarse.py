"""Coarse solve S̊_PP^-1 (Sec. 3.2.1): the partitioned direct solve (interior blocks, separator Schur
complement) against the oracle's banded Cholesky, through the operators that contain it, for several
block counts, 1-3 load cases and a 3D band (needs an MI355X)."""
import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = {
    # 10x7 cells: 11x8 vertices, left column clamped -> nP = 160; blocks of unequal size for p = 3
    "2d": (lambda: latticegen.tiny(2, (10, 7), 3, n_principal=4), (1, 2, 3, 5)),
    "3d": (lambda: latticegen.tiny(3, (4, 3, 3), 2, n_principal=3), (1, 2)),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    _cuda()
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print(f"[gpu coarse] case {request.param}", flush=True)
    make, parts = CASES[request.param]
    prob = make()
    m = Model(prob)
    m.build_reduced_basis()
    ctx = ifeti.setup(prob, principal_in=m.sigma)
    yield request.param, parts, m, ctx
    ctx.close()


def test_partitioned_matches_oracle(pair):
    name, parts, m, ctx = pair
    rng = np.random.default_rng(7)
    lam = rng.standard_normal((3, m.L))
    v = rng.standard_normal(m.nU)
    F_ref = [m.apply_F(lam[r]) for r in range(3)]
    U_ref = m.apply_U(v)
    Ut_ref = m.apply_Ut(lam[0])
    ref_sym = None
    for p in parts:
        print(f"[gpu coarse] {name} coarse_parts={p}", flush=True)
        ctx.set_options(coarse_parts=p)
        F3 = host(ctx.apply_F(dev(lam.ravel()), nrhs=3)).reshape(3, m.L)
        for r in range(3):
            assert rel(F3[r], F_ref[r]) < 1e-11, f"{name} p={p} rhs {r}: {rel(F3[r], F_ref[r]):.2e}"
            # 1-3 load cases per launch: each load case bitwise as alone
            assert np.array_equal(F3[r], host(ctx.apply_F(dev(lam[r]))))
        F2 = host(ctx.apply_F(dev(lam[:2].ravel()), nrhs=2)).reshape(2, m.L)
        assert np.array_equal(F2, F3[:2])
        U = host(ctx.apply_U(dev(v)))
        Ut = host(ctx.apply_Ut(dev(lam[0])))
        assert rel(U, U_ref) < 1e-11 and rel(Ut, Ut_ref) < 1e-11
        if p == 1:
            ref_sym = F3
        else:
            assert rel(F3, ref_sym) < 1e-12      # partitioned vs explicit inverse: rounding only
    ctx.reset_options()


def test_block_count_beyond_the_band_is_rejected(pair):
    name, parts, m, ctx = pair
    from paper_2308_11371_amd import ifeti
    with pytest.raises(ifeti.IfetiError):
        ctx.set_options(coarse_parts=10_000)
    # the context falls back to the explicit inverse and stays usable
    x = np.random.default_rng(3).standard_normal(m.L)
    assert rel(host(ctx.apply_F(dev(x))), m.apply_F(x)) < 1e-11
    ctx.reset_options()


@pytest.mark.parametrize("B", [1, 7, 64])
def test_block_jacobi_coarse_matches_oracle(pair, B):
    """Approximate coarse solve (option coarse_approx = B, Sec. 3.2.1): every operator that contains the
    coarse solve against the oracle with the same block-Jacobi approximation, for one and three load
    cases, and the outer solve still reaching the conforming solution."""
    from oracle.direct import conforming_solve
    name, parts, m, ctx = pair
    m.set_coarse_block(B)
    try:
        rng = np.random.default_rng(11)
        lam = rng.standard_normal((3, m.L))
        v = rng.standard_normal(m.nU)
        ctx.set_options(coarse_approx=B)
        F3 = host(ctx.apply_F(dev(lam.ravel()), nrhs=3)).reshape(3, m.L)
        for r in range(3):
            assert rel(F3[r], m.apply_F(lam[r])) < 1e-11, f"{name} B={B} F rhs {r}"
        assert rel(host(ctx.apply_U(dev(v))), m.apply_U(v)) < 1e-11
        assert rel(host(ctx.apply_Ut(dev(lam[0]))), m.apply_Ut(lam[0])) < 1e-11
        assert rel(host(ctx.apply_Kinv_rom(dev(v))), m.apply_Kinv_rom(v)) < 1e-11
        ctx.set_options(fgmres_restart=300, pcg_maxit=3000)
        f, d = ctx.get_rhs()
        u, lam_s, info = ctx.solve(f, d, tol=1e-12, inner_tol=1e-13, maxit=300)
        e = rel(host(u), conforming_solve(m)["u"])
        print(f"[gpu coarse] {name} block Jacobi B={B}: outer {info['outer_its'][0]}, PCG {info['inner_its'][0]}, "
              f"u vs direct {e:.1e}", flush=True)
        assert e < 1e-9
    finally:
        m.set_coarse_block(0)
        ctx.reset_options()


@pytest.mark.parametrize("nrhs", [4, 17, 35])
def test_partitioned_tiles_for_blocks_of_load_cases(pair, nrhs):
    """Four or more load cases take the partitioned phases as FP64 MFMA tiles (16 or 32 load cases a
    pass, more in passes of 32): F̊, Ů and K̊^-ROM of every load case against the oracle, for every block
    count."""
    name, parts, m, ctx = pair
    rng = np.random.default_rng(11 + nrhs)
    lam = rng.standard_normal((nrhs, m.L))
    v = rng.standard_normal((nrhs, m.nU))
    pick = [0, nrhs // 2, nrhs - 1]
    F_ref = {r: m.apply_F(lam[r]) for r in pick}
    U_ref = {r: m.apply_U(v[r]) for r in pick}
    K_ref = {r: m.apply_Kinv_rom(v[r]) for r in pick}
    for p in parts:
        if p == 1:
            continue  # one block: the explicit inverse, not the partitioned phases
        ctx.set_options(coarse_parts=p)
        F = host(ctx.apply_F(dev(lam.ravel()), nrhs=nrhs)).reshape(nrhs, m.L)
        U = host(ctx.apply_U(dev(v.ravel()), nrhs=nrhs)).reshape(nrhs, m.L)
        K = host(ctx.apply_Kinv_rom(dev(v.ravel()), nrhs=nrhs)).reshape(nrhs, m.nU)
        for r in pick:
            e = max(rel(F[r], F_ref[r]), rel(U[r], U_ref[r]), rel(K[r], K_ref[r]))
            print(f"[gpu coarse] {name} p={p} nrhs={nrhs} load case {r}: {e:.1e}", flush=True)
            assert e < 1e-11
        # every load case equals its single apply (the row form) to rounding
        for r in range(nrhs):
            assert rel(F[r], host(ctx.apply_F(dev(lam[r])))) < 1e-12
    ctx.reset_options()
