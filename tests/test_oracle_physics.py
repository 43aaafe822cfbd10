"""Physics pins of the oracle on an optimised chi = 4 state (Sec. III.A).

The state in tests/golden/chi4_state.json was written by
tests/golden/make_chi4_state.py with the oracle alone (3000 sweeps from seed 0).
Pins: the energy is variational (above the exact -4/pi of Sec. III.A) and
within 1 % of it; the ascending superoperator has the identity eigenvalue
lambda = 1 (Delta = 0) and its next scaling dimension is the Ising sigma,
Delta = 1/8 (Sec. II.B), here within 0.02 at chi = 4; the next one is close to
Delta_epsilon = 1.  The chi = 4 tolerances on the scaling dimensions are this
build's reading (the paper prints no numbers for chi = 4).
"""
import json
import os

import numpy as np
import pytest

from oracle import mera_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def state():
    path = os.path.join(GOLDEN, "chi4_state.json")
    if not os.path.exists(path):
        pytest.skip("golden state not generated")
    g = json.load(open(path))
    layers = [(np.array(l["u"]), np.array(l["w"])) for l in g["layers"]]
    si = (np.array(g["si"]["u"]), np.array(g["si"]["w"]))
    st = O.MeraState(layers, si)
    O.initial_fixed_point(st, 400)
    return st, g


def test_energy_is_variational_and_close_to_exact(state):
    st, g = state
    consts = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    e_exact = consts["exact_energy_density"]["value"]
    h, c = O.shifted_hamiltonian()
    e = O.energy(st, h, c)
    assert e > e_exact
    assert (e - e_exact) / abs(e_exact) < 1e-2
    traj = [x[1] for x in g["energy_trajectory"]]
    assert traj[-1] < traj[0]
    assert abs(traj[-1] - e) < 1e-6  # the stored trajectory ends at this state


def test_fixed_point_of_optimised_state(state):
    st, _ = state
    assert O.fixed_point_residual(*st.si, st.rho_star) < 1e-10


def test_scaling_dimensions_of_optimised_state(state):
    st, _ = state
    consts = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["ising_cft_primary_scaling_dimensions"]
    dims, lam = O.scaling_dimensions(*st.si, k=6)
    assert abs(dims[0] - consts["identity"]) < 1e-10
    assert abs(dims[1] - consts["sigma"]) < 0.02
    assert abs(dims[2] - consts["epsilon"]) < 0.2
