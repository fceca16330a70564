"""Write the full-size c2 golden samples (calls only oracle/ and the seeded input generators).

The oracle builds the whole 64x64-cell c2 lattice (4096 cells, 648 dof/cell, 12 principal cells,
FP64): greedy (Algorithm 4), principal bank, coefficients of eqs. (41)-(42) and the coarse factor.
Stored: the principal set, the coefficients of 64 sampled cells, and 256 sampled entries of each
operator applied to a seeded standard-normal input: F̊ (48), M̊_D^-1 (49), Ů and Ůᵀ (Algorithm 3),
K̊^-ROM (Algorithm 2 with eq. (46)) and the saddle operator of (16).  A few minutes of CPU.

Usage: python tests/golden/make_c2_samples.py   (writes tests/golden/c2_samples.json)
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

# seeds of the inputs (standard normal) and of the sampled indices, shared with the GPU test
INPUT_SEEDS = {"F": 101, "MD": 102, "Ut": 103, "U": 104, "Kinv_rom": 105, "A": 106}
SAMPLE_SEED = 200
N_SAMPLES = 256
N_CELLS = 64


def input_length(op, m):
    return {"F": m.L, "MD": m.L, "Ut": m.L, "U": m.nU, "Kinv_rom": m.nU, "A": m.nU + m.L}[op]


def main():
    t0 = time.time()
    prob = latticegen.make("c2")
    m = Model(prob)
    m.build_reduced_basis()
    print(f"oracle c2 model + reduced basis: {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(SAMPLE_SEED)
    cells = np.sort(rng.choice(m.N, N_CELLS, replace=False))
    out = {
        "config": "c2",
        "generator": "tests/golden/make_c2_samples.py (oracle only)",
        "sizes": {"N": int(m.N), "L": int(m.L), "nU": int(m.nU), "K": int(len(m.sigma))},
        "sigma": [int(s) for s in m.sigma],
        "cells": [int(s) for s in cells],
        "alpha": m.alpha[cells].tolist(),
        "pi": m.pi[cells].tolist(),
        "delta": m.delta[cells].tolist(),
        "input_seeds": INPUT_SEEDS,
        "ops": {},
    }
    for op, seed in INPUT_SEEDS.items():
        t1 = time.time()
        x = np.random.default_rng(seed).standard_normal(input_length(op, m))
        y = getattr(m, "apply_" + op)(x)
        idx = np.sort(rng.choice(y.size, N_SAMPLES, replace=False))
        out["ops"][op] = {"n": int(y.size), "norm": float(np.linalg.norm(y)), "idx": [int(i) for i in idx],
                          "val": [float(v) for v in y[idx]]}
        print(f"{op}: {time.time() - t1:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_samples.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
