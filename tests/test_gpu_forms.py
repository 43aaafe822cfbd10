"""Differentiation form and scaling dimensions on the GPU.

* The autograd energy's hand-written backward (environment kernels) against
  the oracle's environments and against central finite differences on 64
  seeded tangent directions (chi = 12, three transitional layers, FP64).
* A Riemannian gradient step lowers the energy like the SVD update does.
* Scaling dimensions from GPU matvecs against the oracle on an optimised
  chi = 4 state (written by tests/golden/make_chi4_state.py).
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import mera_oracle as O
from paper_1906_12030_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "chi4_state.json")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_12030_amd import autograd, ops, scaling, sweep
    return ops, sweep, autograd, scaling


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def _state(chi, T, seed, sweep_mod, ops, iters=60):
    layers, si = I.init_mera(chi, T, seed)
    m = sweep_mod.GpuMera(layers, si)
    sweep_mod.initial_fixed_point(m, iters, "fp64")
    return layers, si, m


def test_autograd_gradients_are_twice_the_oracle_environments(mods):
    ops, sweep, autograd, _ = mods
    say("autograd vs oracle environments chi=4 T=2")
    layers, si, m = _state(4, 2, 3, sweep, ops)
    h1, _ = ops.tfim_hamiltonian(1.0)
    pairs = [(u.clone().requires_grad_(True), w.clone().requires_grad_(True)) for u, w in m.layers]
    e = autograd.energy(pairs, h1, m.rho_star)
    e.backward()
    rho_top = m.rho_star.cpu().numpy()
    h_np, _ = O.shifted_hamiltonian()
    st = O.MeraState(layers, si, rho_top)
    hs = O.ascend_chain(st, h_np)
    rhos = O.descend_chain(st, rho_top)
    assert abs(float(e) - O.trace_product(h_np, rhos[0])) < 1e-12
    for t, (u, w) in enumerate(pairs):
        uo, wo = layers[t]
        ref_u = 2 * O.env_u(uo, wo, hs[t], rhos[t + 1])
        ref_w = 2 * O.env_w(uo, wo, hs[t], rhos[t + 1])
        assert np.abs(u.grad.cpu().numpy() - ref_u).max() < 1e-12 * (1 + np.abs(ref_u).max())
        assert np.abs(w.grad.cpu().numpy() - ref_w).max() < 1e-12 * (1 + np.abs(ref_w).max())


def test_finite_differences_64_tangent_directions(mods):
    """Central differences, step 1e-6, on 64 seeded unit tangent directions (chi=12, T=3)."""
    ops, sweep, autograd, _ = mods
    say("finite differences chi=12 T=3")
    layers, si, m = _state(12, 3, 0, sweep, ops, iters=30)
    h1, _ = ops.tfim_hamiltonian(1.0)
    base = [(u.clone(), w.clone()) for u, w in m.layers]
    pairs = [(u.clone().requires_grad_(True), w.clone().requires_grad_(True)) for u, w in base]
    e0 = autograd.energy(pairs, h1, m.rho_star)
    e0.backward()
    grads = [(u.grad.clone(), w.grad.clone()) for u, w in pairs]
    gen = torch.Generator(device="cpu").manual_seed(0)
    eps = 1e-6
    worst = 0.0
    with torch.no_grad():
        for k in range(64):
            dirs = []
            for (u, w) in base:
                du = autograd.tangent_project(u, torch.randn(u.shape, generator=gen, dtype=torch.float64).cuda())
                dw = autograd.tangent_project(w, torch.randn(w.shape, generator=gen, dtype=torch.float64).cuda())
                dirs.append((du, dw))
            nrm = torch.sqrt(sum((du * du).sum() + (dw * dw).sum() for du, dw in dirs))
            dirs = [(du / nrm, dw / nrm) for du, dw in dirs]
            plus = [(u + eps * du, w + eps * dw) for (u, w), (du, dw) in zip(base, dirs)]
            minus = [(u - eps * du, w - eps * dw) for (u, w), (du, dw) in zip(base, dirs)]
            fd = (float(autograd.energy(plus, h1, m.rho_star)) - float(autograd.energy(minus, h1, m.rho_star))) / (2 * eps)
            an = float(sum((gu * du).sum() + (gw * dw).sum() for (gu, gw), (du, dw) in zip(grads, dirs)))
            worst = max(worst, abs(fd - an))
    say(f"  max |FD - <grad, dir>| = {worst:.3e}")
    assert worst < 1e-8


def test_riemannian_step_lowers_energy(mods):
    ops, sweep, autograd, _ = mods
    say("riemannian descent chi=6")
    layers, si, m = _state(6, 2, 1, sweep, ops)
    h1, c = ops.tfim_hamiltonian(1.0)
    e_start = sweep.energy(m, h1, c)
    es = [e_start]
    for _ in range(5):
        g = autograd.riemannian_descent_step(m, h1, lr=0.02)
        sweep.initial_fixed_point(m, 60, "fp64")
        es.append(sweep.energy(m, h1, c))
    say(f"  energies {es}")
    assert es[-1] < e_start
    # every tensor stays on its isometry manifold
    for u, w in m.layers + [m.si]:
        for x in (u, w):
            xm = x.reshape(-1, x.shape[0] ** 2) if x.dim() == 4 else x.reshape(-1, x.shape[-1])
            eye = torch.eye(xm.shape[1], dtype=torch.float64, device=xm.device)
            assert torch.abs(xm.t() @ xm - eye).max() < 1e-12


def test_autograd_gradients_chi12_are_twice_the_oracle_environments(mods):
    """The differentiation form's configuration (chi = 12, three transitional layers, FP64):
    the backward of the autograd energy against twice the oracle environments of every
    transitional layer (appendix, Fig. A1 caption)."""
    ops, sweep, autograd, _ = mods
    say("autograd vs oracle environments chi=12 T=3")
    layers, si, m = _state(12, 3, 0, sweep, ops, iters=30)
    h1, _ = ops.tfim_hamiltonian(1.0)
    pairs = [(u.clone().requires_grad_(True), w.clone().requires_grad_(True)) for u, w in m.layers]
    e = autograd.energy(pairs, h1, m.rho_star)
    e.backward()
    rho_top = m.rho_star.cpu().numpy()
    h_np, _ = O.shifted_hamiltonian()
    st = O.MeraState(layers, si, rho_top)
    hs = O.ascend_chain(st, h_np)
    rhos = O.descend_chain(st, rho_top)
    assert abs(float(e.detach()) - O.trace_product(h_np, rhos[0])) < 1e-12
    for t, (u, w) in enumerate(pairs):
        uo, wo = layers[t]
        ref_u = 2 * O.env_u(uo, wo, hs[t], rhos[t + 1])
        ref_w = 2 * O.env_w(uo, wo, hs[t], rhos[t + 1])
        eu = np.abs(u.grad.cpu().numpy() - ref_u).max() / (1 + np.abs(ref_u).max())
        ew = np.abs(w.grad.cpu().numpy() - ref_w).max() / (1 + np.abs(ref_w).max())
        say(f"  layer {t}: max grad error u {eu:.2e} w {ew:.2e}")
        assert eu < 1e-12 and ew < 1e-12


def test_riemannian_descent_against_svd_update_chi12(mods):
    """Same seeded chi = 12 state, same number of steps: both lower the energy and stay
    variational; the SVD update, which jumps to the minimiser of the linearised energy, ends
    lower than first-order Riemannian steps."""
    from paper_1906_12030_amd import run
    say("riemannian vs svd chi=12")
    res = run.compare_riemannian(12, 3, 0, 12, lr=0.02, iters=30)
    for k, es in res.items():
        say(f"  {k}: " + " ".join(f"{e:.6f}" for e in es))
        assert es[-1] < es[0], k
        assert min(es) > -4 / np.pi
    assert res["svd"][-1] < res["riemannian"][-1]


def _golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden state missing")
    g = json.load(open(GOLDEN))
    layers = [(np.array(l["u"]), np.array(l["w"])) for l in g["layers"]]
    si = (np.array(g["si"]["u"]), np.array(g["si"]["w"]))
    return layers, si


def test_scaling_dimensions_gpu_vs_oracle(mods):
    ops, sweep, autograd, scaling = mods
    layers, si = _golden()
    say("scaling dimensions chi=4")
    dims_o, lam_o = O.scaling_dimensions(*si, k=12)
    u = torch.from_numpy(si[0]).cuda()
    w = torch.from_numpy(si[1]).cuda()
    dims_g, lam_g, calls = scaling.scaling_dimensions(u, w, k=12)
    say(f"  oracle {np.round(dims_o, 4)}\n  gpu    {np.round(dims_g, 4)} ({calls} matvecs)")
    assert np.abs(np.abs(lam_g) - np.abs(lam_o)).max() < 1e-8
    assert abs(dims_g[0]) < 1e-10
    assert abs(dims_g[1] - 0.125) < 0.02


def test_mfma_peak_microbenchmark(mods):
    """The measured matrix-core throughput is positive and below the published dense peaks."""
    ops = mods[0]
    for kind, published in (("bf16", 2516.6), ("fp32", 157.3), ("fp64", 78.6)):
        tf = ops.mfma_peak(kind)
        say(f"  mfma peak {kind}: {tf:.1f} TFLOP/s (published {published})")
        assert 0.2 * published < tf < 1.05 * published
