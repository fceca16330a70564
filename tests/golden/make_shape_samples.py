"""Write oracle samples at the benchmarked cell shapes (calls only oracle/ and the seeded input generators).

Two lattices carry the cell discretisations and column counts the measured configurations run with,
small enough for the oracle:

  c3cell  3D 4x4x2 cells with the c3 cell: trivariate quadratic B-splines, 6x6x6 elements (1536 dof),
          cubic frame w = 0.2h, seeded 3-mode macro map, 16 principal cells
  c4cols  2D 32x16 cells with the c2/c4 cell: 16x16 elements (648 dof), w linear 0.15h..0.30h in x,
          macro amplitude 0.15h, 12 principal cells, and the 32 seeded load cases of c4, so that a
          32-load-case operator application has 16384 cell columns as at c4

Stored per lattice: the principal set; for every operator (F̊ (48), M̊_D^-1 (49), Ů, Ůᵀ (Algorithm 3),
K̊^-ROM (Algorithm 2 with eq. (46)), the saddle operator (16)) applied to seeded standard-normal
inputs (one load case for c3cell, 32 for c4cols), the norm of each load case's output and seeded
samples of its entries.  c3cell also stores the interface PCG (tol 1e-13) and the full ROM-FETI-DP
solve (FGMRES 1e-12, PCG 1e-13); c4cols the conforming solutions (the plain definition, direct
Cholesky) of its 32 load cases, each the traction-weighted combination of the two unit-traction
solutions (the finite element problem is linear in the traction).  About ten minutes of CPU.

Usage: python tests/golden/make_shape_samples.py   (writes tests/golden/shape_samples.json)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import latticegen  # noqa: E402
from oracle import Model  # noqa: E402
from oracle.direct import conforming_solve  # noqa: E402

OPS = ("F", "MD", "U", "Ut", "Kinv_rom", "A")
INPUT_SEED = {"F": 401, "MD": 402, "U": 403, "Ut": 404, "Kinv_rom": 405, "A": 406}
SAMPLE_SEED = 500


def lattice(name):
    if name == "c3cell":
        return latticegen.tiny(3, (4, 4, 2), 6, width=("const", 0.2), n_principal=16, name="c3cell")
    if name == "c4cols":
        return latticegen.tiny(2, (32, 16), 16, amp=0.15, width=("linx", 0.15, 0.30), n_principal=12,
                               tractions=latticegen.c4_tractions(), name="c4cols")
    raise KeyError(name)


def in_len(op, m):
    return {"F": m.L, "MD": m.L, "Ut": m.L, "U": m.nU, "Kinv_rom": m.nU, "A": m.nU + m.L}[op]


def samples(rng, y, k):
    idx = np.sort(rng.choice(y.size, min(k, y.size), replace=False))
    return {"n": int(y.size), "norm": float(np.linalg.norm(y)), "idx": [int(i) for i in idx],
            "val": [float(v) for v in y[idx]]}


def main():
    out = {"generator": "tests/golden/make_shape_samples.py (oracle only)"}
    for name, nrhs, per in (("c3cell", 1, 512), ("c4cols", 32, 64)):
        t0 = time.time()
        p = lattice(name)
        m = Model(p)
        m.build_reduced_basis()
        print(f"{name}: model + reduced basis {time.time() - t0:.0f} s, sigma {list(m.sigma)}", flush=True)
        rng = np.random.default_rng(SAMPLE_SEED)
        rec = {"sizes": {"N": int(m.N), "L": int(m.L), "nU": int(m.nU), "K": int(len(m.sigma))},
               "sigma": [int(s) for s in m.sigma], "nrhs": nrhs, "ops": {}}
        for op in OPS:
            t1 = time.time()
            X = np.random.default_rng(INPUT_SEED[op]).standard_normal((nrhs, in_len(op, m)))
            fn = getattr(m, "apply_" + op)
            rec["ops"][op] = [samples(rng, fn(X[r]), per) for r in range(nrhs)]
            print(f"{name} {op}: {time.time() - t1:.1f} s", flush=True)
        if name == "c3cell":
            rhs = np.random.default_rng(407).standard_normal(m.L)
            lam, its, _ = m.solve_interface(rhs, tol=1e-13, maxit=2000)
            rec["pcg"] = {"rhs_seed": 407, "tol": 1e-13, "its": int(its), "lam": samples(rng, lam, 1024)}
            t1 = time.time()
            r = m.solve(tol=1e-12, inner_tol=1e-13, maxit=200)
            print(f"{name} solve: {time.time() - t1:.0f} s, outer {r['outer_its']}, relres {r['relres']:.2e}",
                  flush=True)
            rec["solve"] = {"tol": 1e-12, "inner_tol": 1e-13, "outer_its": int(r["outer_its"]),
                            "relres": float(r["relres"]), "u": samples(rng, r["u"], 2048),
                            "lam": samples(rng, r["lam"], 1024)}
        else:
            # conforming solutions for the unit tractions, combined per load case
            t1 = time.time()
            q = lattice(name)
            q.tractions = np.eye(2)
            mq = Model(q)
            base = [conforming_solve(mq, rhs_index=i) for i in range(2)]
            print(f"{name} conforming solves: {time.time() - t1:.0f} s", flush=True)
            iu = np.sort(rng.choice(m.nU, 512, replace=False))
            U = [p.tractions[c, 0] * base[0]["u"] + p.tractions[c, 1] * base[1]["u"] for c in range(nrhs)]
            rec["direct"] = {"u_idx": [int(i) for i in iu],
                             "u_val": [[float(v) for v in U[c][iu]] for c in range(nrhs)],
                             "u_norm": [float(np.linalg.norm(U[c])) for c in range(nrhs)]}
        out[name] = rec
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shape_samples.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
