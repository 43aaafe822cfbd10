"""Write tests/golden/superop_env_chi16.json: FP64 oracle values of the ascending and
descending superoperators and of both environments of one seeded chi=16 layer, in the
LEFT and RIGHT placements (AVG is their mean, checked by the tests from these two).

Produced with the FP64 oracle only (Sec. II.B, Fig. 4a,b; Sec. II.C, Fig. 4c,d and the
appendix figure A1).  Inputs, drawn in this order from numpy's PCG64 with seed 0
(paper_1906_12030_amd/inputs.py): u, w = random_layer(16, 16); rho = random_density(16)
(G G^T / tr, G in R^{4096 x 64}); h = random_symmetric(16).

For every output X in {A_L(h), A_R(h), D_L(rho), D_R(rho), Env_u^L, Env_u^R, Env_w^L,
Env_w^R} the file stores
  * ||X||_F;
  * <X, G_1> and <X, G_2> for G_k = standard_normal(X.shape) from PCG64 seed 777: every
    entry enters these two sums;
  * X at NSAMPLE positions drawn with Generator(PCG64(12345)).choice(size, NSAMPLE,
    replace=False), sorted;
  (probes and positions are drawn once per quantity A, D, Env_u, Env_w, in that order, and
  shared by its LEFT and RIGHT outputs, so that AVG = (LEFT + RIGHT)/2 can be checked too)
and the Euler values <Env_u^P, u>, <Env_w^P, w> with e_P = tr(h D_P(rho)).

Run from the repository root:  python tests/golden/make_superop_env_chi16.py  (a few
minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mera_oracle as O  # noqa: E402
from paper_1906_12030_amd import inputs as I  # noqa: E402

CHI, SEED, PROBE_SEED, SAMPLE_SEED, NSAMPLE = 16, 0, 777, 12345, 2048
OUTPUTS = ("A_L", "A_R", "D_L", "D_R", "Env_u_L", "Env_u_R", "Env_w_L", "Env_w_R")


def inputs():
    rng = np.random.default_rng(SEED)
    u, w = I.random_layer(rng, CHI, CHI)
    rho = I.random_density(rng, CHI)
    h = I.random_symmetric(rng, CHI)
    return u, w, rho, h


def main():
    u, w, rho, h = inputs()
    probe_rng = np.random.default_rng(PROBE_SEED)
    sample_rng = np.random.default_rng(SAMPLE_SEED)
    comp = {
        "A_L": lambda: O.ascend_placement(u, w, h, "L"),
        "A_R": lambda: O.ascend_placement(u, w, h, "R"),
        "D_L": lambda: O.descend_placement(u, w, rho, "L"),
        "D_R": lambda: O.descend_placement(u, w, rho, "R"),
        "Env_u_L": lambda: O.env_u(u, w, h, rho, "L"),
        "Env_u_R": lambda: O.env_u(u, w, h, rho, "R"),
        "Env_w_L": lambda: O.env_w(u, w, h, rho, "L"),
        "Env_w_R": lambda: O.env_w(u, w, h, rho, "R"),
    }
    out = {"recipe": {"chi": CHI, "seed": SEED, "probe_seed": PROBE_SEED, "sample_seed": SAMPLE_SEED,
                      "nsample": NSAMPLE, "order": list(OUTPUTS),
                      "generator": "tests/golden/make_superop_env_chi16.py (oracle only)"}}
    vals = {}
    draws = {}
    for name in OUTPUTS:
        t0 = time.time()
        x = comp[name]()
        vals[name] = x
        q = name[:-2]  # A, D, Env_u, Env_w: LEFT and RIGHT share the probes and positions
        if q not in draws:
            g1 = probe_rng.standard_normal(x.shape)
            g2 = probe_rng.standard_normal(x.shape)
            idx = np.sort(sample_rng.choice(x.size, min(NSAMPLE, x.size), replace=False))
            draws[q] = (g1, g2, idx)
        g1, g2, idx = draws[q]
        flat = x.reshape(-1)
        out[name] = {"fro": float(np.linalg.norm(flat)), "probe": [float(np.sum(x * g1)), float(np.sum(x * g2))],
                     "index": idx.tolist(), "sample": flat[idx].tolist()}
        print(name, f"{time.time() - t0:.1f} s", out[name]["fro"], flush=True)
    for p in ("L", "R"):
        e = O.trace_product(h, vals["D_" + p])
        out["energy_" + p] = e
        out["euler_u_" + p] = float(np.sum(vals["Env_u_" + p] * u))
        out["euler_w_" + p] = float(np.sum(vals["Env_w_" + p] * w))
    with open(os.path.join(ROOT, "tests", "golden", "superop_env_chi16.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
