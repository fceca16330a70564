"""Allocation-free F̊ apply (ifeti_apply_F_noalloc) through the C ABI (needs an MI355X): two calls in a
row, the second with fewer load cases, each equal to ifeti_apply_F bitwise (and to the oracle in 2D);
sizes beyond the scratch array's maximum and more than three load cases are rejected with EINVAL."""
import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _two_calls(ctx, L, counts, seed):
    rng = np.random.default_rng(seed)
    for nrhs in counts:
        lam = dev(rng.standard_normal(nrhs * L))
        out = torch.full((nrhs * L,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.apply_F_noalloc(lam, nrhs=nrhs, out=out)
        got = host(out)
        ref = host(ctx.apply_F(lam, nrhs=nrhs))
        assert np.array_equal(got, ref), f"nrhs={nrhs}: max diff {np.abs(got - ref).max():.3e}"
        yield nrhs, host(lam).reshape(nrhs, L), got.reshape(nrhs, L)


def test_noalloc_equals_apply_F_2d():
    _cuda()
    from oracle import Model
    from paper_2308_11371_amd import ifeti
    print("[gpu noalloc] 2D", flush=True)
    p = latticegen.tiny(2, (5, 3), 4, n_principal=4, tractions=[[0.3, -0.7]])
    m = Model(p)
    m.build_reduced_basis()
    ctx = ifeti.setup(p, principal_in=m.sigma)
    L = ctx.sizes.L
    for nrhs, lam, got in _two_calls(ctx, L, (3, 1), 21):
        for r in range(nrhs):
            want = m.apply_F(lam[r])
            assert np.linalg.norm(got[r] - want) <= 1e-11 * np.linalg.norm(want)
    with pytest.raises(ifeti.IfetiError) as e:
        ctx.apply_F_noalloc(dev(np.zeros(4 * L)), nrhs=4)
    assert e.value.status == ifeti.IFETI_EINVAL
    ctx.close()


def test_noalloc_equals_apply_F_3d_and_size_limit():
    """1024 cells of the c3 cell: two load cases fit the 32 MiB array (then one), three do not."""
    _cuda()
    from paper_2308_11371_amd import ifeti
    print("[gpu noalloc] 3D 16x8x8", flush=True)
    p = latticegen.tiny(3, (16, 8, 8), 6, width=("const", 0.2), n_principal=16)
    ctx = ifeti.setup(p)
    s = ctx.sizes
    need3 = 8 * (2 * s.N * 3 * s.n_d + s.N * 3 * s.n_p + 2 * 3 * s.nP)
    assert need3 > 32 << 20
    for _ in _two_calls(ctx, s.L, (2, 1), 22):
        pass
    with pytest.raises(ifeti.IfetiError) as e:
        ctx.apply_F_noalloc(dev(np.zeros(3 * s.L)), nrhs=3)
    assert e.value.status == ifeti.IFETI_EINVAL and "maximum" in str(e.value)
    ctx.close()
