"""Binary tree calls (Fig. 1a; mera_tree_*) against the FP64 oracle's tree network.

The oracle's tree functions are pinned on the CPU to the MERA network with identity
disentanglers and to a separately written tree descent.  Here the GPU schedules are
compared element by element with them, in every placement and precision, at shapes with
din != dout, ragged tile edges (din = 3, 6) and the large-tile sizes (16, 24).  Tolerances
as in the other parity tests: FP64 1e-12 relative Frobenius error, FP32 2e-5, split bf16
1e-4.  At chi = 24 the oracle evaluates the whole tree network (O(chi^7)).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mera_oracle as O
from paper_1906_12030_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_12030_amd import ops as _ops
    return _ops


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


_CASES = {}


def _case(din, dout):
    """Seeded inputs and the oracle's LEFT / RIGHT results (AVG is their mean), once per shape."""
    if (din, dout) not in _CASES:
        rng = np.random.default_rng(700 + 10 * din + dout)
        _, w = I.random_layer(rng, din, dout)
        rho = I.random_density(rng, dout)
        h = I.random_symmetric(rng, din)
        ref = {}
        for p in ("L", "R"):
            ref[("descend", p)] = O.tree_descend(w, rho, p)
            ref[("ascend", p)] = O.tree_ascend(w, h, p)
            ref[("env_w", p)] = O.tree_env_w(w, h, rho, p)
        for k in ("descend", "ascend", "env_w"):
            ref[(k, "AVG")] = 0.5 * (ref[(k, "L")] + ref[(k, "R")])
        _CASES[(din, dout)] = (w, rho, h, ref)
    return _CASES[(din, dout)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("din,dout", [(2, 4), (3, 3), (4, 16), (6, 5), (16, 16), (24, 24)])
def test_tree_calls_match_oracle(ops, din, dout, prec):
    print(f"tree calls din={din} dout={dout} {prec}", file=sys.stderr, flush=True)
    w, rho, h, ref = _case(din, dout)
    wg, rg, hg = gpu(w), gpu(rho), gpu(h)
    errs = {}
    for p in ("L", "R", "AVG"):
        ref_d, ref_a, ref_e = ref[("descend", p)], ref[("ascend", p)], ref[("env_w", p)]
        errs[("descend", p)] = rel(host(ops.tree_descend(wg, rg, p, prec)), ref_d)
        errs[("ascend", p)] = rel(host(ops.tree_ascend(wg, hg, p, prec)), ref_a)
        errs[("env_w", p)] = rel(host(ops.tree_env_w(wg, hg, rg, p, prec)), ref_e)
    worst = max(errs.values())
    print(f"  worst relative error {worst:.2e}", file=sys.stderr, flush=True)
    assert worst < TOL[prec], errs


def test_tree_descend_matches_mera_descend_with_identity(ops):
    """The tree call and the MERA call with u = identity give the same descent (the
    same network, O(chi^7) against O(chi^9) work)."""
    d = 8
    rng = np.random.default_rng(3)
    _, w = I.random_layer(rng, d, d)
    rho = I.random_density(rng, d)
    one = np.eye(d * d).reshape((d,) * 4)
    layer = ops.Layer(gpu(one), gpu(w))
    a = host(ops.tree_descend(gpu(w), gpu(rho), "AVG", "fp64"))
    b = host(ops.descend(layer, gpu(rho), "AVG", "fp64"))
    assert rel(a, b) < 1e-13
