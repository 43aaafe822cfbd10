"""Pins of the oracle's Hamiltonian, sweep and scale-invariant environment depth (CPU).

* Three-site TFIM density (Sec. II Eq. ham; three-site regrouping of Sec. II.B): with the
  field split evenly over the two bonds of a site, h3 = -X1X2/2 - X2X3/2 - (g/4)Z1
  - (g/2)Z2 - (g/4)Z3 is an open three-site Ising chain.  Its spectrum has the free-fermion
  closed form {+-s1 +- s2 +- s3}, s_k the singular values of the bidiagonal matrix with
  fields (g/4, g/2, g/4) on the diagonal and couplings (1/2, 1/2) above it (Jordan-Wigner
  solution of the open transverse-field chain), so lambda_max = s1 + s2 + s3.  Any other
  split of the field changes the fields and hence the spectrum.
* Sweep (Sec. II.C): the first 100 oracle sweeps from the seeded chi = 4 start reproduce
  the stored trajectory of tests/golden/make_chi4_state.py, whose end state carries the
  physics pins of test_oracle_physics (energy within 1 % of -4/pi, Delta_sigma near 1/8);
  the energy decreases at every sweep and stays above -4/pi (variational, Sec. III.A).
* Scale-invariant environment depth: the scale-invariant tensors appear in every layer
  above the transitional ones.  With rho* a fixed point of D_s, the derivative of
  tr(h D_s^K(rho*)) (rho* held fixed) along a direction of u or w equals twice the inner
  product with sum_{k<K} Env(A_s^k(h), rho*), the sum si_environments_h feeds the sweep.
  Checked by central finite differences.  From the optimised chi = 4 state, K = 3 keeps
  lowering the energy while K = 1 nearly stalls.
"""
import json
import os

import numpy as np
import pytest

from oracle import mera_oracle as O
from paper_1906_12030_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
E_EXACT = -4.0 / np.pi


def _free_fermion_spectrum(g):
    b = np.array([[g / 4, 0.5, 0.0], [0.0, g / 2, 0.5], [0.0, 0.0, g / 4]])
    s = np.linalg.svd(b, compute_uv=False)
    return np.sort([a * s[0] + b_ * s[1] + c * s[2] for a in (1, -1) for b_ in (1, -1) for c in (1, -1)])


@pytest.mark.parametrize("g", [1.0, 0.6, 1.7])
def test_three_site_density_spectrum_is_free_fermion(g):
    lam = np.linalg.eigvalsh(O.tfim_three_site(g))
    assert np.abs(lam - _free_fermion_spectrum(g)).max() < 1e-13
    h, c = O.shifted_hamiltonian(g)
    assert abs(c - _free_fermion_spectrum(g)[-1]) < 1e-13


def test_three_site_density_printed_values():
    # critical field g = 1: spectrum +-1.34067, +-1.16170, +-0.5, +-0.32104 and shift
    # c = 1.3406653 (five and eight significant digits)
    lam = np.linalg.eigvalsh(O.tfim_three_site(1.0))
    ref = np.array([1.34067, 1.16170, 0.5, 0.32104])
    assert np.abs(lam[4:][::-1] - ref).max() < 5e-6
    assert np.abs(lam[:4] + ref).max() < 5e-6
    assert abs(O.shifted_hamiltonian(1.0)[1] - 1.3406653) < 5e-8


def test_sweep_replays_stored_trajectory():
    g = json.load(open(os.path.join(GOLDEN, "chi4_state.json")))
    r = g["recipe"]
    layers, si = I.init_mera(r["chi"], r["transitional_layers"], r["seed"])
    st = O.MeraState(layers, si)
    h, c = O.shifted_hamiltonian()
    O.initial_fixed_point(st, r["power_iterations"])
    es = [O.sweep(st, h, c, iters=r["power_iterations"]) for _ in range(100)]
    first = g["energy_trajectory"][0]
    assert first[0] == 100
    assert abs(es[-1] - first[1]) < 1e-12
    assert np.all(np.diff(es) < 0)
    assert min(es) > E_EXACT
    traj = np.array([e for _, e in g["energy_trajectory"]])
    assert np.all(np.diff(traj) < 0) and traj.min() > E_EXACT


def _tower_energy(u, w, h, rho, levels):
    r = rho
    for _ in range(levels):
        r = O.descend(u, w, r)
    return O.trace_product(h, r)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_si_environment_depth_is_gradient_of_tower(levels):
    rng = np.random.default_rng(3)
    d = 2
    u, w = I.random_layer(rng, d, d)
    h = I.random_symmetric(rng, d)
    rho = O.fixed_point_rho(u, w, O.identity_density(d), 3000)
    assert O.fixed_point_residual(u, w, rho) < 1e-13
    st = O.MeraState([], (u, w), rho)
    hs = O.si_environments_h(st, h, levels)
    assert len(hs) == levels
    env_u = sum(O.env_u(u, w, hk, rho) for hk in hs)
    env_w = sum(O.env_w(u, w, hk, rho) for hk in hs)
    eps = 1e-5
    for _ in range(3):
        du = rng.standard_normal(u.shape)
        dw = rng.standard_normal(w.shape)
        fd_u = (_tower_energy(u + eps * du, w, h, rho, levels)
                - _tower_energy(u - eps * du, w, h, rho, levels)) / (2 * eps)
        fd_w = (_tower_energy(u, w + eps * dw, h, rho, levels)
                - _tower_energy(u, w - eps * dw, h, rho, levels)) / (2 * eps)
        # central differences: truncation eps^2 f'''/6 ~ 1e-9 relative here
        assert abs(fd_u - 2 * np.sum(env_u * du)) < 1e-7 * max(1.0, abs(fd_u))
        assert abs(fd_w - 2 * np.sum(env_w * dw)) < 1e-7 * max(1.0, abs(fd_w))


def test_three_si_levels_keep_descending_where_one_stalls():
    g = json.load(open(os.path.join(GOLDEN, "chi4_state.json")))
    layers = [(np.array(l["u"]), np.array(l["w"])) for l in g["layers"]]
    si = (np.array(g["si"]["u"]), np.array(g["si"]["w"]))
    h, c = O.shifted_hamiltonian()
    out = {}
    for k in (1, 3):
        st = O.MeraState(layers, si)
        O.initial_fixed_point(st, 200)
        e0 = O.energy(st, h, c)
        es = np.array([O.sweep(st, h, c, iters=30, si_levels=k) for _ in range(30)])
        assert es.min() > E_EXACT
        out[k] = (e0, es)
    e0, es3 = out[3]
    _, es1 = out[1]
    assert np.all(np.diff(es3) < 0)
    # K = 3 gains at least ten times as much as K = 1 over the same 30 sweeps
    assert (e0 - es3[-1]) > 10 * (e0 - es1[-1]) > 0
