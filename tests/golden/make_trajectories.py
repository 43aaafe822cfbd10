"""Write tests/golden/trajectories.json: per-sweep energies of oracle optimisations.

Produced with the FP64 oracle only (Sec. II.C sweep, 30 power iterations per sweep, one
scale-invariant environment level, seeded tensors from paper_1906_12030_amd/inputs.py and an
initial fixed point of 30 power iterations):
  * chi = 4, two transitional layers (2-4-4), seeds 0, 1, 2: sweeps 1..100;
  * chi = 8, three transitional layers (2-4-8), seed 0: sweeps 1..500.
The energies are e = tr(h rho_1) + c per site after each sweep, as the oracle's sweep returns
them.

Run from the repository root:  python tests/golden/make_trajectories.py  (about 40 minutes on
8 cores, almost all of it the chi = 8 run).
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mera_oracle as O  # noqa: E402
from paper_1906_12030_amd import inputs as I  # noqa: E402

ITERS = 30
RUNS = [(4, 2, 0, 100), (4, 2, 1, 100), (4, 2, 2, 100), (8, 3, 0, 500)]


def run(chi, T, seed, sweeps):
    layers, si = I.init_mera(chi, T, seed)
    st = O.MeraState(layers, si)
    h, c = O.shifted_hamiltonian()
    O.initial_fixed_point(st, ITERS)
    es = []
    for k in range(sweeps):
        es.append(O.sweep(st, h, c, iters=ITERS))
        if k % 50 == 49:
            print(chi, seed, k + 1, es[-1], flush=True)
    return es


def main():
    out = {"recipe": {"power_iterations": ITERS, "si_levels": 1, "initial_fixed_point_iterations": ITERS,
                      "generator": "tests/golden/make_trajectories.py (oracle only)"},
           "runs": []}
    for chi, T, seed, sweeps in RUNS:
        out["runs"].append({"chi": chi, "transitional_layers": T, "seed": seed, "sweeps": sweeps,
                            "energies": run(chi, T, seed, sweeps)})
    with open(os.path.join(ROOT, "tests", "golden", "trajectories.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
