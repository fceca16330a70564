"""Write the full-size c2 golden solve (calls only oracle/ and the seeded input generators).

The oracle solves the whole 64x64-cell c2 lattice (4096 cells, 648 dof/cell, 12 principal cells,
FP64) with the ROM-based inexact FETI-DP method: right-preconditioned flexible GMRES on the saddle
system (16) with the block preconditioner of Algorithm 1, interface PCG on F̊ (48) preconditioned by
M̊_D^-1 (49), reduced local solves of eq. (46).  Tolerances are the tight parity setting (outer
relative residual 1e-12, interface PCG 1e-13), so the stored displacements are the solution of (16)
to about 1e-12 and a GPU solve at the same tolerances must agree to well within 1e-9.

Stored: the principal set, iteration counts, the norms of u and lambda, and 4096 seeded samples of
each.  Tens of minutes of CPU.

Usage: python tests/golden/make_c2_solve.py   (writes tests/golden/c2_solve.json)
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

TOL = 1e-12
INNER_TOL = 1e-13
SAMPLE_SEED = 300
N_SAMPLES = 4096


def main():
    t0 = time.time()
    prob = latticegen.make("c2")
    m = Model(prob)
    m.build_reduced_basis()
    print(f"oracle c2 model + reduced basis: {time.time() - t0:.0f} s", flush=True)
    t1 = time.time()
    r = m.solve(tol=TOL, inner_tol=INNER_TOL, maxit=200)
    print(f"oracle c2 solve: {time.time() - t1:.0f} s, outer {r['outer_its']}, relres {r['relres']:.3e}",
          flush=True)
    u, lam = r["u"], r["lam"]
    rng = np.random.default_rng(SAMPLE_SEED)
    iu = np.sort(rng.choice(u.size, N_SAMPLES, replace=False))
    il = np.sort(rng.choice(lam.size, N_SAMPLES, replace=False))
    out = {
        "config": "c2",
        "generator": "tests/golden/make_c2_solve.py (oracle only)",
        "tol": TOL,
        "inner_tol": INNER_TOL,
        "sizes": {"N": int(m.N), "L": int(m.L), "nU": int(m.nU), "K": int(len(m.sigma))},
        "sigma": [int(s) for s in m.sigma],
        "outer_its": int(r["outer_its"]),
        "inner_its_total": int(sum(r["inner_its"])),
        "relres": float(r["relres"]),
        "u_norm": float(np.linalg.norm(u)),
        "lam_norm": float(np.linalg.norm(lam)),
        "u_idx": [int(i) for i in iu],
        "u_val": [float(v) for v in u[iu]],
        "lam_idx": [int(i) for i in il],
        "lam_val": [float(v) for v in lam[il]],
        "seconds": {"setup": t1 - t0, "solve": float(r["time"])},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_solve.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
