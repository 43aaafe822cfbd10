"""Finite 16-site binary MERA (Fig. 1b) optimised on the GPU against the oracle.

* Trajectory parity: six sweeps from the same seeded network (chi = 4 and 6),
  GPU (library A/D/env/polar, host top eigenvector) against the oracle's
  finite sweep; energies to 1e-11, tensors to 1e-9.
* The GPU-optimised network's energy equals <psi|H|psi>/16 of its explicit
  2^16-amplitude state (oracle) and lies above the exact E0(16)/16.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mera_oracle as O
from paper_1906_12030_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_12030_amd import finite, ops
    return finite, ops


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.mark.parametrize("chi", [4, 6])
def test_finite_trajectory_matches_oracle(mods, chi):
    finite, ops = mods
    say(f"finite 16-site trajectory chi={chi}")
    layers, top = I.init_finite(chi, 0)
    h_o, c_o = O.shifted_hamiltonian()
    h_g, c_g = ops.tfim_hamiltonian(1.0)
    m = finite.FiniteMera(layers, top)
    ol, ot = layers, top
    for k in range(6):
        ol, ot, e_o = O.finite_sweep(ol, ot, h_o, c_o)
        e_g = finite.sweep(m, h_g, c_g)
        assert abs(e_g - e_o) < 1e-11, (k, e_g, e_o)
    st = m.state_dict()
    for (ug, wg), (uo, wo) in zip(st["layers"], ol):
        assert np.abs(ug - uo).max() < 1e-9
        assert np.abs(wg - wo).max() < 1e-9
    # the top state is an eigenvector: compare the projector (sign-free)
    pg = np.outer(st["top"].reshape(-1), st["top"].reshape(-1))
    po = np.outer(ot.reshape(-1), ot.reshape(-1))
    assert np.abs(pg - po).max() < 1e-9


def test_finite_optimised_network_energy_is_its_state_energy(mods):
    finite, ops = mods
    say("finite 16-site: 40 GPU sweeps, then the explicit state")
    layers, top = I.init_finite(4, 1)
    h_g, c_g = ops.tfim_hamiltonian(1.0)
    m = finite.FiniteMera(layers, top)
    es = [finite.sweep(m, h_g, c_g) for _ in range(40)]
    st = m.state_dict()
    v = O.finite_state(st["layers"], st["top"]).reshape(-1)
    e_brute = float(v @ (O.tfim_periodic_sparse(16) @ v)) / 16
    say(f"  e = {es[-1]:.12f}, <psi|H|psi>/16 = {e_brute:.12f}, exact {finite.exact_energy_per_site():.12f}")
    assert abs(e_brute - es[-1]) < 1e-12
    assert es[-1] > finite.exact_energy_per_site()
    assert abs(finite.energy(m, h_g, c_g) - es[-1]) < 1e-13


def test_tree_network_trajectory_matches_oracle(mods):
    """Identity disentanglers kept fixed (binary tree network): GPU vs oracle sweeps.

    Tolerance 1e-10: the isometry environments of the tree are less well conditioned
    than the MERA's, so the polar factors of the GPU's Newton-Schulz iteration and the
    oracle's SVD differ by a few 1e-12, which the following sweeps amplify (2e-11 after
    three sweeps at seed 2)."""
    finite, ops = mods
    say("tree network trajectory chi=4")
    layers, top = I.init_finite(4, 2, tree=True)
    h_o, c_o = O.shifted_hamiltonian()
    h_g, c_g = ops.tfim_hamiltonian(1.0)
    m = finite.FiniteMera(layers, top)
    ol, ot = layers, top
    for k in range(6):
        ol, ot, e_o = O.finite_sweep(ol, ot, h_o, c_o, update_u_tensors=False)
        e_g = finite.sweep(m, h_g, c_g, disentangle=False)
        assert abs(e_g - e_o) < 1e-10, (k, e_g, e_o)
    for (ug, wg), (uo, wo) in zip(m.state_dict()["layers"], ol):
        assert np.abs(ug - uo).max() == 0.0  # the identity, untouched
        assert np.abs(wg - wo).max() < 1e-8
