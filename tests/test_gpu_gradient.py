"""Differentiation form: compliance gradient w.r.t. strut widths (needs an MI355X)."""
import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _smooth(dim):
    if dim == 2:
        return latticegen.tiny(2, (4, 3), 3, smooth=True, width=("uniform", 0.15, 0.30, 5), n_principal=4)
    return latticegen.tiny(3, (2, 2, 2), 2, smooth=True, width=("uniform", 0.15, 0.30, 5), n_principal=3)


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_oracle(dim):
    _cuda()
    from oracle import Model
    from oracle.direct import conforming_solve
    from oracle.gradient import compliance_gradient, compliance
    from paper_2308_11371_amd import ifeti
    prob = _smooth(dim)
    m = Model(prob)
    uo = conforming_solve(m)["u"]
    go = compliance_gradient(m, uo)
    co = compliance(m, uo)
    ctx = ifeti.setup(prob)
    ctx.set_options(pcg_maxit=400, fgmres_restart=120)
    f, d = ctx.get_rhs()
    u, lam, info = ctx.solve(f, d, tol=1e-12, inner_tol=1e-12, maxit=120)
    c, g = ctx.compliance_grad(f, u)
    g = g.cpu().numpy()
    print(f"dim {dim}: compliance {c[0]:.12e} vs {co:.12e}; grad rel err "
          f"{np.linalg.norm(g - go) / np.linalg.norm(go):.2e}")
    assert abs(c[0] - co) <= 1e-10 * abs(co)
    assert np.linalg.norm(g - go) <= 1e-8 * np.linalg.norm(go)
    ctx.close()


def test_gradient_matches_central_differences_and_autograd():
    _cuda()
    from paper_2308_11371_amd import ifeti
    prob = _smooth(3)
    ctx = ifeti.setup(prob)
    ctx.set_options(pcg_maxit=400, fgmres_restart=120)
    f, d = ctx.get_rhs()
    w = torch.tensor(prob.widths, dtype=torch.float64, device="cuda", requires_grad=True)
    c = ifeti.compliance(w, ctx, f, d, tol=1e-12, inner_tol=1e-12)
    (gw,) = torch.autograd.grad(c, w)
    gw = gw.cpu().numpy()
    h = 1e-6
    for s in (0, 3, 6):
        vals = []
        for sgn in (1, -1):
            ww = prob.widths.copy()
            ww[s] += sgn * h
            vals.append(float(ifeti.compliance(torch.tensor(ww, device="cuda"), ctx, f, d, tol=1e-12,
                                               inner_tol=1e-12)))
        fd = (vals[0] - vals[1]) / (2 * h)
        print(f"cell {s}: fd {fd:.8e} adjoint {gw[s]:.8e}")
        assert abs(fd - gw[s]) <= 1e-5 * np.abs(gw).max()
    ctx.close()


def test_c5_gradient_finite_differences_on_sampled_cells():
    """Full-size c5 (1728 cells, smoothed indicator): the adjoint gradient on all 20 seeded cells
    against (a) the oracle's FP64 gradient -u_s^T dK^(s)/dw_s u_s evaluated with the GPU's converged u,
    which checks the gradient kernel at full size, and (b) central differences (step 1e-6) of the
    compliance of two GPU solves per cell, which checks the whole chain."""
    _cuda()
    from oracle import Model
    from oracle.gradient import compliance_gradient
    from paper_2308_11371_amd import ifeti
    print("[gpu gradient] c5 setup", flush=True)
    prob = latticegen.make("c5")
    ctx = ifeti.setup(prob)
    ctx.set_options(pcg_maxit=200, fgmres_restart=100)
    f, d = ctx.get_rhs()
    w0 = torch.tensor(prob.widths, dtype=torch.float64, device="cuda")
    u, lam, info = ctx.solve(f, d, tol=1e-12, inner_tol=1e-11, maxit=100)
    c0, g = ctx.compliance_grad(f, u)
    g = g.cpu().numpy()
    assert np.all(g < 0)
    cells = latticegen.fd_cells(prob.N, count=20)
    m0 = Model(prob, build_all_cells=False)          # cell matrices only for the sampled cells
    go = compliance_gradient(m0, u.cpu().numpy(), cells=cells)
    eo = np.abs(g[cells] - go).max() / np.abs(go).max()
    print(f"[gpu gradient] c5 adjoint vs oracle on {cells.size} cells: max rel {eo:.2e}", flush=True)
    assert eo <= 1e-10
    h = 1e-6
    worst = 0.0
    for s in cells:
        vals = []
        for sgn in (1, -1):
            ww = w0.clone()
            ww[s] += sgn * h
            ctx.update_widths(ww)
            uu, _, inf = ctx.solve(f, d, tol=1e-12, inner_tol=1e-11, maxit=100)
            vals.append(ctx.compliance_grad(f, uu)[0][0])
        fd = (vals[0] - vals[1]) / (2 * h)
        worst = max(worst, abs(fd - g[s]) / abs(g[s]))
        print(f"c5 cell {s}: fd {fd:.6e} adjoint {g[s]:.6e}", flush=True)
        assert abs(fd - g[s]) <= 2e-3 * abs(g[s])
    print(f"[gpu gradient] c5 central differences on {cells.size} cells: max rel {worst:.2e}", flush=True)
    ctx.update_widths(w0)
    ctx.close()
