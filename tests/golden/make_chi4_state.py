"""Write tests/golden/chi4_state.json: an optimised chi=4 scale-invariant MERA.

Produced with the FP64 oracle only: seeded initial tensors (seed 0, two
transitional layers 2-4-4, scale-invariant layer chi=4), an initial fixed point
of 30 power iterations, then 3000 oracle sweeps with 30 power iterations each
(Sec. II.C).  The tensors (not rho*, which tests recompute) and the energy
trajectory every 100 sweeps are stored as JSON text.

Run from the repository root:  python tests/golden/make_chi4_state.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mera_oracle as O  # noqa: E402
from paper_1906_12030_amd import inputs as I  # noqa: E402

CHI, T, SEED, SWEEPS, ITERS = 4, 2, 0, 3000, 30


def main():
    layers, si = I.init_mera(CHI, T, SEED)
    st = O.MeraState(layers, si)
    h, c = O.shifted_hamiltonian()
    O.initial_fixed_point(st, ITERS)
    energies = []
    for k in range(SWEEPS):
        e = O.sweep(st, h, c, iters=ITERS)
        if k % 100 == 99:
            energies.append([k + 1, e])
            print(k + 1, e, flush=True)
    out = {
        "recipe": {"chi": CHI, "transitional_layers": T, "seed": SEED, "sweeps": SWEEPS,
                   "power_iterations": ITERS, "generator": "tests/golden/make_chi4_state.py (oracle only)"},
        "layers": [{"u": u.tolist(), "w": w.tolist()} for u, w in st.layers],
        "si": {"u": st.si[0].tolist(), "w": st.si[1].tolist()},
        "energy_trajectory": energies,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "chi4_state.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
