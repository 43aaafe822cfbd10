"""Full-size parity of the superoperators and environments with the FP64 oracle.

The ascending and descending superoperators (Sec. II.B, Fig. 4a,b) and the environments of
u and w (Sec. II.C, Fig. 4c,d, appendix figure A1) of one seeded layer, in the LEFT, RIGHT
and AVG placements and in every contraction precision, against oracle values written by
tests/golden/make_superop_env_chi16.py (whole outputs at chi = 16) and
tests/golden/make_slices_chi24.py (one slice of each output at chi = 24, the benchmark's
scale-invariant layer).  At these sizes every chi^9 contraction of the split-bf16 path runs
on the large-tile kernel.

Compared: the output at the stored positions (relative 2-norm of the difference), its
Frobenius norm, its inner products with the seeded Gaussian probes (every entry enters
them; the difference is scaled by the norm of the output, which bounds it through
Cauchy-Schwarz for an error of that relative size), and at chi = 16 the Euler values
<Env_u, u> = 2 e_P and <Env_w, w> = 3 e_P.  AVG is compared with (LEFT + RIGHT)/2 of the
oracle values (the golden files share positions and probes between LEFT and RIGHT).

Tolerances (relative): FP64 1e-12 (the GPU schedule differs from the oracle's only in the
order of summation); FP32 2e-5 and split bf16 1e-4, the bounds of the other parity tests,
derived from the unit roundoff of each arithmetic (2^-24; about 2^-17 per stored split word
and product) times the chain of four to six contractions, with room for the sqrt(K) growth of
K-term sums.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

from paper_1906_12030_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 1e-4}


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_12030_amd import ops as _ops
    return _ops


def _load(name, chi, shapes, nprobe):
    path = os.path.join(GOLDEN, name)
    g = json.load(open(path))
    r = g["recipe"]
    assert r["chi"] == chi
    rng = np.random.default_rng(r["seed"])
    u, w = I.random_layer(rng, chi, chi)
    rho = I.random_density(rng, chi)
    h = I.random_symmetric(rng, chi)
    probe_rng = np.random.default_rng(r["probe_seed"])
    probes = {}
    for q, shape in shapes:  # same draw order as the generator
        probes[q] = [probe_rng.standard_normal(shape) for _ in range(nprobe)]
    return g, (u, w, rho, h), probes


@pytest.fixture(scope="module")
def chi16():
    d = 16
    shapes = [("A", (d,) * 6), ("D", (d,) * 6), ("Env_u", (d,) * 4), ("Env_w", (d, d, d))]
    return _load("superop_env_chi16.json", d, shapes, 2)


@pytest.fixture(scope="module")
def chi24():
    d = 24
    shapes = [("D", (d,) * 5), ("A", (d,) * 5), ("Env_u", (d,) * 3), ("Env_w", (d, d))]
    return _load("slices_chi24.json", d, shapes, 1)


def _compute(ops, q, layer, rho, h, place, prec):
    t = {"D": lambda: ops.descend(layer, rho, place, prec),
         "A": lambda: ops.ascend(layer, h, place, prec),
         "Env_u": lambda: ops.env_u(layer, h, rho, place, prec),
         "Env_w": lambda: ops.env_w(layer, h, rho, place, prec)}[q]()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _reference(g, q, place, key):
    if place == "AVG":
        a, b = g[f"{q}_L"][key], g[f"{q}_R"][key]
        return 0.5 * (np.asarray(a) + np.asarray(b))
    return np.asarray(g[f"{q}_{place[0]}"][key])


def _check(x, g, q, place, probes, prec, label):
    idx = np.asarray(g[f"{q}_L"]["index"])
    ref = _reference(g, q, place, "sample")
    flat = x.reshape(-1)
    e_sample = float(np.linalg.norm(flat[idx] - ref) / np.linalg.norm(ref))
    nrm = float(np.linalg.norm(flat))
    pr = np.atleast_1d(_reference(g, q, place, "probe"))
    e_probe = max(abs(float(np.sum(x * p)) - float(pk)) for p, pk in zip(probes, pr)) / nrm
    out = {"sample": e_sample, "probe": e_probe}
    if place != "AVG":
        fro = g[f"{q}_{place[0]}"]["fro"]
        out["fro"] = abs(nrm - fro) / fro
    say(f"{label} {q} {place} {prec}: " + " ".join(f"{k}={v:.2e}" for k, v in out.items()))
    for k, v in out.items():
        assert v < TOL[prec], (label, q, place, prec, k, v)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("q", ["A", "D", "Env_u", "Env_w"])
def test_chi16_whole_outputs_against_oracle(ops, chi16, q, prec):
    g, (u, w, rho, h), probes = chi16
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    layer = ops.Layer(dev(u), dev(w))
    rho_d, h_d = dev(rho), dev(h)
    say(f"chi=16 {q} {prec}")
    for place in ("L", "R", "AVG"):
        x = _compute(ops, q, layer, rho_d, h_d, place, prec)
        _check(x, g, q, place, probes[q], prec, "chi=16")
        if q in ("Env_u", "Env_w"):
            t = u if q == "Env_u" else w
            k = "euler_u" if q == "Env_u" else "euler_w"
            ref = 0.5 * (g[k + "_L"] + g[k + "_R"]) if place == "AVG" else g[f"{k}_{place[0]}"]
            assert abs(float(np.sum(x * t)) - ref) < TOL[prec] * abs(ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("q", ["D", "A", "Env_u", "Env_w"])
def test_chi24_slices_against_oracle(ops, chi24, q, prec):
    g, (u, w, rho, h), probes = chi24
    k = g["recipe"]["index"]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    layer = ops.Layer(dev(u), dev(w))
    rho_d, h_d = dev(rho), dev(h)
    say(f"chi=24 {q} {prec}")
    for place in ("L", "R", "AVG"):
        x = _compute(ops, q, layer, rho_d, h_d, place, prec)
        x = x[:, :, k] if q == "Env_w" else x[k]
        _check(np.ascontiguousarray(x), g, q, place, probes[q], prec, "chi=24")
