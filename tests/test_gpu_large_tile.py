"""Parity at bond dimensions that reach the large-tile split-bf16 kernel.

The 256-row tile with direct-to-LDS loads takes the chi^9 contractions whose
operands are both contiguous along k and whose innermost k run is a multiple
of 32 with at least 192 output columns: in a MERA layer that is chi = 16, 24,
32, ...  Below that the 128 x 128 kernel runs, so the small-shape parity
tests never reach it.  Here:

* one fine-leg slice of D_L and D_R at chi = 16 and of D_L at chi = 24
  against the oracle's sliced descend (the oracle finishes a 1/chi share of
  the network in seconds);
* A, Env_u and Env_w at chi = 16 in split bf16 against the FP64 GPU path
  (itself pinned to the oracle element by element at smaller shapes);
  Env_u and Env_w run split-k partial sums through the large-tile kernel.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mera_oracle as O
from paper_1906_12030_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_12030_amd import ops as _ops
    return _ops


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _case(chi, seed):
    rng = np.random.default_rng(7000 + chi + seed)
    u, w = I.random_layer(rng, chi, chi)
    rho = I.random_density(rng, chi)
    h = I.random_symmetric(rng, chi)
    return u, w, rho, h


@pytest.mark.parametrize("chi,placement,index", [(16, "L", 3), (16, "R", 11), (24, "L", 7)])
def test_descend_slice_vs_oracle(ops, chi, placement, index):
    u, w, rho, _ = _case(chi, 0)
    say(f"large-tile descend chi={chi} placement={placement} slice {index}")
    ref = O.descend_placement_slice(u, w, rho, placement, index)
    layer = ops.Layer(gpu(u), gpu(w))
    for prec in ("bf16x3",) if chi == 24 else ("bf16x3", "fp32"):
        d = host(ops.descend(layer, gpu(rho), placement, prec))
        got = d[index]  # the slice fixes the first fine leg in both placements
        err = rel(got, ref)
        say(f"  {prec}: rel err {err:.2e}")
        assert err < TOL[prec]
    ops.WORKSPACE.release()


def test_ascend_and_environments_chi16(ops):
    chi = 16
    u, w, rho, h = _case(chi, 1)
    say("large-tile ascend / env_u / env_w chi=16, split bf16 vs FP64")
    layer = ops.Layer(gpu(u), gpu(w))
    hg, rg = gpu(h), gpu(rho)
    for name, fn in (("ascend", lambda p: ops.ascend(layer, hg, "AVG", p)),
                     ("env_u", lambda p: ops.env_u(layer, hg, rg, "AVG", p)),
                     ("env_w", lambda p: ops.env_w(layer, hg, rg, "AVG", p))):
        ref = host(fn("fp64"))
        got = host(fn("bf16x3"))
        err = rel(got, ref)
        say(f"  {name}: rel err {err:.2e}")
        assert err < TOL["bf16x3"]
    ops.WORKSPACE.release()
