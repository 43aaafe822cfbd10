"""Physics pins of the oracle on an optimised chi = 4 state (Sec. III.A).

The state in tests/golden/chi4_state.json was written by
tests/golden/make_chi4_state.py with the oracle alone (3000 sweeps from seed 0).
Pins: the energy is variational (above the exact -4/pi of Sec. III.A) and
within 1 % of it; the ascending superoperator has the identity eigenvalue
lambda = 1 (Delta = 0) and its next scaling dimension is the Ising sigma,
Delta = 1/8 (Sec. II.B), here within 0.02 at chi = 4; the next one is close to
Delta_epsilon = 1.  The chi = 4 tolerances on the scaling dimensions are this
build's reading (the paper prints no numbers for chi = 4).

Also the finite 16-site network (Fig. 1b) as an optimisation workload: the
top-state energy operator against the window-averaged density, and oracle
sweeps against the energy of the explicit 2^16-amplitude state.
"""
import json
import os

import numpy as np
import pytest

from oracle import mera_oracle as O
from paper_1906_12030_amd import inputs as I

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


# ----------------------------------------------------------------------------
# Finite 16-site network as an optimisation workload
# ----------------------------------------------------------------------------
def test_finite_top_operator_is_the_window_averaged_energy():
    """<t|H_top|t> = tr(h rho_top_avg) for a random top state and a random symmetric h."""
    rng = np.random.default_rng(5)
    for d in (2, 3):
        h = I.random_symmetric(rng, d)
        t = rng.standard_normal((d,) * 4)
        t /= np.linalg.norm(t)
        v = t.reshape(-1)
        lhs = float(v @ O.finite_top_operator(h) @ v)
        rhs = O.trace_product(h, O.finite_top_density(t))
        assert abs(lhs - rhs) < 1e-13
        # the averaged density has unit trace and is symmetric
        r = O.finite_top_density(t).reshape(d ** 3, d ** 3)
        assert abs(np.trace(r) - 1.0) < 1e-13 and np.abs(r - r.T).max() < 1e-15


def test_finite_sweeps_lower_the_energy_of_the_explicit_state():
    """Oracle sweeps of the 16-site network: the energy drops, stays above the exact ground
    energy, and equals <psi|H|psi>/16 of the explicit 2^16-amplitude state."""
    layers, top = I.init_finite(4, 0)
    h, c = O.shifted_hamiltonian()
    exact = O.ising_ground_energy_closed_form(16) / 16
    es = []
    for _ in range(12):
        layers, top, e = O.finite_sweep(layers, top, h, c)
        es.append(e)
    assert es[-1] < es[0] - 0.05
    assert es[-1] > exact
    v = O.finite_state(layers, top).reshape(-1)
    e_brute = float(v @ (O.tfim_periodic_sparse(16) @ v)) / 16
    assert abs(e_brute - es[-1]) < 1e-12


def test_finite_host_helpers_match_oracle():
    """The package's host-side top operator and top density against the oracle's."""
    from paper_1906_12030_amd import finite as F
    rng = np.random.default_rng(6)
    for d in (2, 4):
        h = I.random_symmetric(rng, d)
        t = rng.standard_normal((d,) * 4)
        assert np.abs(F.top_operator(h) - O.finite_top_operator(h)).max() < 1e-13
        assert np.abs(F.top_density(t) - O.finite_top_density(t)).max() < 1e-13
    assert abs(F.exact_energy_per_site(16) - O.ising_ground_energy_closed_form(16) / 16) < 1e-15


def test_tree_network_sweeps():
    """Binary tree network (identity disentanglers, never updated): the disentanglers stay
    the identity, the energy drops and equals the explicit state's, and it stays above the
    exact ground energy."""
    h, c = O.shifted_hamiltonian()
    lt, tt = I.init_finite(4, 0, tree=True)
    es = []
    for _ in range(25):
        lt, tt, et = O.finite_sweep(lt, tt, h, c, update_u_tensors=False)
        es.append(et)
    for u, _ in lt:
        assert np.abs(u.reshape(u.shape[0] ** 2, -1) - np.eye(u.shape[0] ** 2)).max() == 0.0
    v = O.finite_state(lt, tt).reshape(-1)
    assert abs(float(v @ (O.tfim_periodic_sparse(16) @ v)) / 16 - et) < 1e-12
    assert es[-1] < es[0] and es[-1] > O.ising_ground_energy_closed_form(16) / 16
