"""Write tests/golden/precision_chi16.json: FP64 oracle reference values of a seeded chi=16
scale-invariant MERA, for the precision-form comparison (FP32 and split-bf16 contractions
against FP64).

Produced with the FP64 oracle only: seeded tensors (seed 0, three transitional layers
2-4-16-16, scale-invariant layer chi=16; not optimised), rho* by 30 power iterations from
the maximally mixed density (Sec. II.B), then
  * the energy per site tr(h rho_1) + c, rho_1 descended from rho* (Sec. II.B);
  * ||rho*||_F, tr(rho*^2) and 512 entries of rho* at seeded positions.
(The scaling dimensions of this unoptimised layer have no spectral gap to speak of, so
Arnoldi does not converge in a useful time; they are compared at optimised states instead.)
Run from the repository root:  python tests/golden/make_precision_chi16.py  (about 10 min
on 8 cores).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mera_oracle as O  # noqa: E402
from paper_1906_12030_amd import inputs as I  # noqa: E402

CHI, T, SEED, ITERS, NSAMPLE = 16, 3, 0, 30, 512


def main():
    layers, si = I.init_mera(CHI, T, SEED)
    st = O.MeraState(layers, si)
    h, c = O.shifted_hamiltonian()
    O.initial_fixed_point(st, ITERS)
    e = O.energy(st, h, c)
    print("energy", e, flush=True)
    rho = st.rho_star.reshape(-1)
    idx = np.sort(np.random.default_rng(12345).choice(rho.size, NSAMPLE, replace=False))
    out = {
        "recipe": {"chi": CHI, "transitional_layers": T, "seed": SEED, "power_iterations": ITERS,
                   "rho_start": "maximally mixed", "sample_seed": 12345,
                   "generator": "tests/golden/make_precision_chi16.py (oracle only)"},
        "energy": e,
        "rho_fro": float(np.linalg.norm(rho)),
        "rho_purity": float(rho @ rho),
        "rho_sample_index": idx.tolist(),
        "rho_sample": rho[idx].tolist(),
    }
    with open(os.path.join(ROOT, "tests", "golden", "precision_chi16.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
