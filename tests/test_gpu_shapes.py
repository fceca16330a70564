"""Parity at the benchmarked kernel shapes (needs an MI355X).

Two lattices carry the measured configurations' cell discretisations and column counts (oracle samples
in tests/golden/shape_samples.json, written by tests/golden/make_shape_samples.py from oracle/ only):

  c3cell  3D 4x4x2 cells with the c3 cell (6x6x6 quadratic elements, 1536 dof, 16 principal cells):
          the large-operator contraction path, seven staging chunks per contraction, the 3D LDS
          footprints of the reduced local solve
  c4cols  2D 32x16 cells with the c2/c4 cell (648 dof, 12 principal cells) and the 32 load cases of
          c4: 16384 cell columns per contraction, the many-column precision-form path and the coarse
          solve as a contraction

Every tile candidate of every contraction family is forced in turn (option tile_candidate), so
whichever candidate the autotuner keeps for a configuration is one checked here: FP64 against the
oracle at 1e-10 of the sampled norm, FP32 / BF16 operands at the precision form's operator error.
c3cell also checks the interface PCG and the full solve; c4cols the 32-load-case block solves (FP64
and FP32 local with FP64 outer refinement) against the conforming solutions.
"""
import json
import os

import numpy as np
import pytest

import latticegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "shape_samples.json")
OPS = ("F", "MD", "U", "Ut", "Kinv_rom", "A")
INPUT_SEED = {"F": 401, "MD": 402, "U": 403, "Ut": 404, "Kinv_rom": 405, "A": 406}
N_FP64_CANDIDATES = 8   # small-operator family (the large-operator family has 5: i mod 5)
N_LP_CANDIDATES = 4
LP_TOL = {"fp32": 2e-5, "bf16": 5e-2}


def _lattice(name):
    if name == "c3cell":
        return latticegen.tiny(3, (4, 4, 2), 6, width=("const", 0.2), n_principal=16, name="c3cell")
    return latticegen.tiny(2, (32, 16), 16, amp=0.15, width=("linx", 0.15, 0.30), n_principal=12,
                           tractions=latticegen.c4_tractions(), name="c4cols")


@pytest.fixture(scope="module", params=["c3cell", "c4cols"])
def lat(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_11371_amd import ifeti
    with open(GOLDEN) as f:
        gold = json.load(f)[request.param]
    print(f"[gpu shapes] {request.param} setup", flush=True)
    prob = _lattice(request.param)
    ctx = ifeti.setup(prob)
    inputs = {}
    s = ctx.sizes
    n_in = {"F": s.L, "MD": s.L, "Ut": s.L, "U": s.nU, "Kinv_rom": s.nU, "A": s.nU + s.L}
    for op in OPS:
        X = np.random.default_rng(INPUT_SEED[op]).standard_normal((gold["nrhs"], n_in[op]))
        inputs[op] = torch.tensor(X.ravel(), dtype=torch.float64, device="cuda")
    yield request.param, prob, ctx, gold, inputs
    ctx.close()


def _errors(ctx, gold, inputs, op):
    """Largest sampled relative error and largest norm error over the load cases of one operator."""
    nrhs = gold["nrhs"]
    y = getattr(ctx, "apply_" + op)(inputs[op], nrhs=nrhs)
    torch.cuda.synchronize()
    Y = y.cpu().numpy().reshape(nrhs, -1)
    es, en = 0.0, 0.0
    for r, g in enumerate(gold["ops"][op]):
        assert Y[r].size == g["n"]
        exp = np.array(g["val"])
        es = max(es, np.linalg.norm(Y[r][np.array(g["idx"])] - exp) / np.linalg.norm(exp))
        en = max(en, abs(np.linalg.norm(Y[r]) - g["norm"]) / g["norm"])
    return es, en


def test_greedy_selection_and_sizes(lat):
    name, prob, ctx, gold, inputs = lat
    s = ctx.sizes
    assert (s.N, s.L, s.nU, s.K) == tuple(gold["sizes"][k] for k in ("N", "L", "nU", "K"))
    assert list(ctx.sigma) == gold["sigma"]


@pytest.mark.parametrize("cand", range(N_FP64_CANDIDATES))
def test_fp64_tile_candidates(lat, cand):
    name, prob, ctx, gold, inputs = lat
    ctx.set_options(tile_candidate=cand)
    try:
        for op in OPS:
            es, en = _errors(ctx, gold, inputs, op)
            print(f"[gpu shapes] {name} fp64 candidate {cand} {op}: sampled {es:.1e} norm {en:.1e}", flush=True)
            assert es <= 1e-10 and en <= 1e-10, f"{name} candidate {cand} {op}: {es:.2e} / {en:.2e}"
    finally:
        ctx.reset_options()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("cand", range(N_LP_CANDIDATES))
def test_low_precision_tile_candidates(lat, prec, cand):
    from paper_2308_11371_amd import ifeti
    name, prob, ctx, gold, inputs = lat
    p = {"fp32": ifeti.IFETI_FP32_LOCAL, "bf16": ifeti.IFETI_BF16_LOCAL}[prec]
    ctx.set_options(precision=p, tile_candidate=cand)
    try:
        for op in OPS:
            es, en = _errors(ctx, gold, inputs, op)
            print(f"[gpu shapes] {name} {prec} candidate {cand} {op}: sampled {es:.1e} norm {en:.1e}", flush=True)
            tol = 1e-10 if op == "A" else LP_TOL[prec]   # the true operator (16) stays FP64
            assert es <= tol and en <= tol, f"{name} {prec} candidate {cand} {op}: {es:.2e} / {en:.2e}"
    finally:
        ctx.reset_options()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_low_precision_library_path(lat, prec):
    """The precision form as the solves run it (no forced candidate): the narrow library product of
    (46a) gives R in FP32 for the reduced local solve (c4cols: the 32 load cases and three; c3cell: 32
    copies of its load case, 1024 cell columns)."""
    from paper_2308_11371_amd import ifeti
    name, prob, ctx, gold, inputs = lat
    ctx.set_options(precision={"fp32": ifeti.IFETI_FP32_LOCAL, "bf16": ifeti.IFETI_BF16_LOCAL}[prec])
    try:
        for op in OPS:
            es, en = _errors(ctx, gold, inputs, op)
            print(f"[gpu shapes] {name} {prec} library path {op}: sampled {es:.1e} norm {en:.1e}", flush=True)
            tol = 1e-10 if op == "A" else LP_TOL[prec]
            assert es <= tol and en <= tol, f"{name} {prec} library path {op}: {es:.2e} / {en:.2e}"
        if gold["nrhs"] < 3:
            # 32 copies of the single load case: 1024 cell columns take the narrow library product and
            # the 3D reduced local solve with R and H in FP32
            n = inputs["Kinv_rom"].numel()
            y = ctx.apply_Kinv_rom(inputs["Kinv_rom"].repeat(32), nrhs=32).cpu().numpy().reshape(32, n)
            g = gold["ops"]["Kinv_rom"][0]
            exp = np.array(g["val"])
            for r in (0, 17, 31):
                err = np.linalg.norm(y[r][np.array(g["idx"])] - exp) / np.linalg.norm(exp)
                assert err <= LP_TOL[prec], f"{name} {prec} 32 copies, column {r}: {err:.2e}"
            return
        n = inputs["Kinv_rom"].numel() // gold["nrhs"]
        y = ctx.apply_Kinv_rom(inputs["Kinv_rom"][:3 * n], nrhs=3).cpu().numpy().reshape(3, n)
        for r in range(3):
            g = gold["ops"]["Kinv_rom"][r]
            exp = np.array(g["val"])
            err = np.linalg.norm(y[r][np.array(g["idx"])] - exp) / np.linalg.norm(exp)
            assert err <= LP_TOL[prec], f"{name} {prec} three load cases, column {r}: {err:.2e}"
    finally:
        ctx.reset_options()


def test_autotuned_tiles_match_oracle(lat):
    name, prob, ctx, gold, inputs = lat
    ctx.set_options(autotune=1)
    try:
        for rep in range(2):
            for op in OPS:
                es, en = _errors(ctx, gold, inputs, op)
                assert es <= 1e-10 and en <= 1e-10, f"{name} autotuned {op}: {es:.2e}"
    finally:
        ctx.reset_options()


def _sampled(x, g):
    exp = np.array(g["val"])
    return np.linalg.norm(x[np.array(g["idx"])] - exp) / np.linalg.norm(exp)


def test_c3cell_interface_pcg_and_full_solve(lat):
    name, prob, ctx, gold, inputs = lat
    if name != "c3cell":
        pytest.skip("c3-cell lattice only")
    g = gold["pcg"]
    rhs = torch.tensor(np.random.default_rng(g["rhs_seed"]).standard_normal(ctx.sizes.L), dtype=torch.float64,
                       device="cuda")
    lam, its, rel, st = ctx.solve_interface(rhs, tol=g["tol"], maxit=3000)
    e = _sampled(lam.cpu().numpy(), g["lam"])
    print(f"[gpu shapes] c3cell PCG: {its[0]} its (oracle {g['its']}), lam samples {e:.2e}", flush=True)
    assert e <= 1e-9
    assert abs(int(its[0]) - g["its"]) <= max(2, g["its"] // 50)
    gs = gold["solve"]
    s = ctx.sizes
    f, d = ctx.get_rhs()
    ctx.set_options(fgmres_restart=200, pcg_maxit=3000)
    try:
        u, lam, info = ctx.solve(f, d, tol=gs["tol"], inner_tol=gs["inner_tol"], maxit=200, check=False)
    finally:
        ctx.reset_options()
    u = u.cpu().numpy()
    eu, el = _sampled(u, gs["u"]), _sampled(lam.cpu().numpy(), gs["lam"])
    nu = abs(np.linalg.norm(u) - gs["u"]["norm"]) / gs["u"]["norm"]
    print(f"[gpu shapes] c3cell solve: outer {info['outer_its'][0]} (oracle {gs['outer_its']}), relres "
          f"{info['relres'][0]:.1e}; u samples {eu:.2e}, lam samples {el:.2e}, u norm {nu:.1e}", flush=True)
    assert eu <= 1e-9 and el <= 1e-9 and nu <= 1e-9


@pytest.mark.parametrize("prec,block_cg", [("fp64", 0), ("fp32", 0), ("fp64", 1)])
def test_c4cols_block_solve_matches_conforming_solutions(lat, prec, block_cg):
    """32 load cases at once (shared operator applications; independent PCG recurrences, or one block
    PCG over all load cases with block_cg): each load case's displacements against the conforming
    solution, FP64 within 1e-9 and FP32 local contractions (FP64 PCG, coarse solve and outer
    refinement) within 1e-6."""
    from paper_2308_11371_amd import ifeti
    name, prob, ctx, gold, inputs = lat
    if name != "c4cols":
        pytest.skip("c4-column lattice only")
    g = gold["direct"]
    s = ctx.sizes
    nrhs = gold["nrhs"]
    f, d = ctx.get_rhs()
    p = {"fp64": ifeti.IFETI_FP64, "fp32": ifeti.IFETI_FP32_LOCAL}[prec]
    ctx.set_options(precision=p, autotune=1, block_cg=block_cg)
    try:
        u, lam, info = ctx.solve(f, d, nrhs=nrhs, tol=1e-11, inner_tol=1e-12 if prec == "fp64" else 1e-6, maxit=100)
    finally:
        ctx.reset_options()
    U = u.cpu().numpy().reshape(nrhs, s.nU)
    idx = np.array(g["u_idx"])
    worst = 0.0
    for c in range(nrhs):
        exp = np.array(g["u_val"][c])
        worst = max(worst, np.linalg.norm(U[c][idx] - exp) / np.linalg.norm(exp),
                    abs(np.linalg.norm(U[c]) - g["u_norm"][c]) / g["u_norm"][c])
    print(f"[gpu shapes] c4cols {prec} block_cg={block_cg} solve of {nrhs} load cases: outer "
          f"{int(info['outer_its'].max())}, inner {int(np.sum(info['inner_its']))}, "
          f"max relres {info['relres'].max():.1e}, worst u error {worst:.2e}", flush=True)
    assert info["relres"].max() <= 1e-9     # true residual of (16) (the outer stop test uses the estimate)
    assert worst <= (1e-9 if prec == "fp64" else 1e-6)
