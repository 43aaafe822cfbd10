"""The allocation-free descend against the descend with a caller workspace.

mera_descend_noalloc takes its workspace from the library's static device array.  Two
calls in a row, the second on a smaller input, each compared with mera_descend (caller
workspace, same kernels) and with the FP64 oracle (Sec. II.B, Fig. 4b); the first call
(chi = 12, FP64) needs the chi^7 intermediates sliced to fit the array, the second
(chi = 6, split bf16) does not, so the second call runs on an array that still holds the
first call's data.  Tolerances: the parity bounds of the other tests (FP64 1e-12 relative
Frobenius; split bf16 1e-4); against mera_descend, FP64 differs only in the slicing of the
sums (1e-13) and split bf16 takes the same schedule (1e-14).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mera_oracle as O
from paper_1906_12030_amd import _lib
from paper_1906_12030_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_descend_matches_descend(order):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_12030_amd import ops
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    for d, prec, tol_ref, tol_same in ((12, "fp64", 1e-12, 1e-13), (6, "bf16x3", 1e-4, 1e-14)):
        print(f"noalloc descend chi={d} {prec}", file=sys.stderr, flush=True)
        rng = np.random.default_rng(500 + d)
        u, w = I.random_layer(rng, d, d)
        rho = I.random_density(rng, d)
        layer = ops.Layer(torch.from_numpy(u).cuda(), torch.from_numpy(w).cuda())
        rho_d = torch.from_numpy(rho).cuda()
        for place in ("L", "R", "AVG"):
            out = torch.full((d,) * 6, float("nan"), dtype=torch.float64, device="cuda")
            st = _lib.mera_descend_noalloc(layer.c(), rho_d.data_ptr(), out.data_ptr(),
                                           ops.PLACEMENTS[place], ops.PRECISIONS[prec], stream)
            assert st == 0, _lib.load().mera_last_error()
            ref = ops.descend(layer, rho_d, place, prec)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.isfinite(got).all()
            assert rel(got, ref.cpu().numpy()) < tol_same
            assert rel(got, O.apply_placement(O.descend_placement, u, w, rho, place)) < tol_ref
