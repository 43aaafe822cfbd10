"""The contraction engine on its own, through mera_contract, against numpy.einsum (FP64).

Shapes are chosen to reach every kernel and its edge cases: ragged M and N
(tiles cut by the matrix edge), k runs that are not a multiple of the k-tile
(masked loads), permuted multi-leg operands, split-k partial sums with the
fixed-order reduction, beta accumulation, and the large-tile split-bf16
kernel (both operands contiguous along k, k-run a multiple of 32, M >= 256,
N >= 192) in its 256 x 192/256 and 256 x 288 forms, including ragged,
split-k and store-along-m cases (output's innermost leg from the first
operand; vector stores when that leg's extent is a multiple of 4).  Tolerances are relative
Frobenius errors: FP64 1e-12, FP32 2e-5, split bf16 1e-4 (as in the MERA
parity tests).
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 1e-4}

CASES = [
    # spec, sizes, note
    ("mk,kn->mn", dict(m=300, k=70, n=200), "ragged m/n, k not a multiple of the k-tile"),
    ("mk,nk->mn", dict(m=300, k=96, n=200), "both operands k-contiguous, ragged (large tile in bf16x3)"),
    ("mk,nk->mn", dict(m=256, k=32768, n=192), "one output tile, long k: split-k"),
    ("abcd,dcef->aebf", dict(a=5, b=7, c=9, d=11, e=6, f=13), "permuted legs, odd extents"),
    ("abkl,cdkl->abcd", dict(a=16, b=20, k=4, l=8, c=12, d=17), "merged k legs, large tile, ragged n"),
    ("xkl,ylk->yx", dict(x=33, k=5, l=3, y=65), "k legs in different orders"),
    ("mk,nk->nm", dict(m=300, k=96, n=200), "output contiguous along m: 4-row vector stores, ragged"),
    ("abk,nk->nab", dict(a=50, b=6, k=64, n=200), "output contiguous along m, inner leg of 6: element stores"),
    ("mk,nk->mn", dict(m=300, k=2048, n=560), "long k: 256 x 288 tile (4 x 2 waves), ragged m and n"),
    ("mk,nk->nm", dict(m=300, k=2048, n=560), "256 x 288 tile storing along m"),
    ("mk,nk->mn", dict(m=256, k=16384, n=288), "256 x 288 tile, one output tile: split-k"),
]


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_12030_amd import ops as _ops
    return _ops


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("spec,sizes,note", CASES)
def test_contract_matches_einsum(ops, spec, sizes, note, prec):
    print(f"contract {spec} {sizes} {prec}: {note}", flush=True, file=sys.stderr)
    rng = np.random.default_rng(len(spec) * 31 + sum(sizes.values()))
    lhs, lc = spec.split("->")
    la, lb = lhs.split(",")
    a = rng.standard_normal([sizes[ch] for ch in la])
    b = rng.standard_normal([sizes[ch] for ch in lb])
    ref = np.einsum(spec, a, b)
    got = ops.contract(spec, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), prec)
    torch.cuda.synchronize()
    assert rel(got.cpu().numpy(), ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("spec", ["mk,nk->mn", "mk,nk->nm"])
def test_contract_alpha_beta(ops, prec, spec):
    rng = np.random.default_rng(3)
    a = rng.standard_normal((300, 96))
    b = rng.standard_normal((200, 96))
    ab = a @ b.T if spec.endswith("mn") else (a @ b.T).T
    c0 = rng.standard_normal(ab.shape)
    c = torch.from_numpy(c0.copy()).cuda()
    ops.contract(spec, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), prec, 0.5, -1.5, out=c)
    torch.cuda.synchronize()
    assert rel(c.cpu().numpy(), 0.5 * ab - 1.5 * c0) < TOL[prec]
