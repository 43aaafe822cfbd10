"""Write tests/golden/fixed_point_chi24.json: FP64 oracle fixed point and energy of a seeded
chi=24 scale-invariant MERA with the benchmark's layer structure (three transitional layers
2-4-16-24, scale-invariant layer chi=24).

Produced with the FP64 oracle only: seeded tensors (paper_1906_12030_amd/inputs.py
init_mera(24, 3, seed 0); not optimised), rho* by ITERS power-iteration steps
rho <- sym(D(rho)) / tr from the maximally mixed density (Sec. II.B), every D evaluated slice
by slice over its first fine leg (chi^7 intermediates would need 37 GB), then
  * the energy per site tr(h rho_1) + c, rho_1 descended from rho* (Sec. II.B);
  * the fixed-point residual ||D(rho*) - rho*||_F / ||rho*||_F;
  * ||rho*||_F and rho* at NSAMPLE positions drawn with Generator(PCG64(12345)).choice
    (size, NSAMPLE, replace=False), sorted.

Run from the repository root:  python tests/golden/make_fixed_point_chi24.py  (one to two
hours on 8 cores, under 16 GB of memory; each power iteration is 48 slices of the descend).
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

CHI, T, SEED, ITERS, SAMPLE_SEED, NSAMPLE = 24, 3, 0, 8, 12345, 2048


def main():
    layers, si = I.init_mera(CHI, T, SEED)
    st = O.MeraState(layers, si)
    h, c = O.shifted_hamiltonian()
    u, w = st.si
    rho = st.rho_star
    for k in range(ITERS):
        t0 = time.time()
        rho = O.power_iteration_step(u, w, rho, sliced=True)
        print("iteration", k + 1, f"{time.time() - t0:.1f} s", flush=True)
    st.rho_star = rho
    e = O.energy(st, h, c, sliced=True)
    print("energy", e, flush=True)
    resid = O.fixed_point_residual(u, w, rho, sliced=True)
    print("residual", resid, flush=True)
    flat = rho.reshape(-1)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(flat.size, NSAMPLE, replace=False))
    out = {
        "recipe": {"chi": CHI, "transitional_layers": T, "seed": SEED, "power_iterations": ITERS,
                   "rho_start": "maximally mixed", "sample_seed": SAMPLE_SEED, "nsample": NSAMPLE,
                   "generator": "tests/golden/make_fixed_point_chi24.py (oracle only)"},
        "energy": e,
        "residual": resid,
        "rho_fro": float(np.linalg.norm(flat)),
        "rho_sample_index": idx.tolist(),
        "rho_sample": flat[idx].tolist(),
    }
    with open(os.path.join(ROOT, "tests", "golden", "fixed_point_chi24.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
