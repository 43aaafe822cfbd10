"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element by element.

Tolerances: FP64 contractions 1e-12 relative Frobenius error (the schedules
differ from the oracle's in order of summation only); FP32 and split-bf16
paths are checked against bounds derived from their unit roundoff
(FP32: 2^-24 per product, K-term sums; split bf16: about 2^-16 per product).
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


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


SHAPES = [(2, 2), (2, 4), (3, 3), (4, 4), (3, 7), (4, 16), (6, 6), (8, 8)]
PLACE = {"L": "L", "R": "R", "AVG": "AVG"}


def _case(din, dout, seed):
    rng = np.random.default_rng(1000 * din + dout + seed)
    u, w = I.random_layer(rng, din, dout)
    rho = I.random_density(rng, dout)
    h = I.random_symmetric(rng, din)
    return u, w, rho, h


@pytest.mark.parametrize("din,dout", SHAPES)
@pytest.mark.parametrize("placement", ["L", "R", "AVG"])
def test_descend_ascend_fp64(ops, din, dout, placement):
    u, w, rho, h = _case(din, dout, 0)
    say(f"descend/ascend fp64 din={din} dout={dout} placement={placement}")
    layer = ops.Layer(gpu(u), gpu(w))
    d = host(ops.descend(layer, gpu(rho), placement, "fp64"))
    ref = O.apply_placement(O.descend_placement, u, w, rho, placement)
    assert rel(d, ref) < TOL["fp64"]
    a = host(ops.ascend(layer, gpu(h), placement, "fp64"))
    ref = O.apply_placement(O.ascend_placement, u, w, h, placement)
    assert rel(a, ref) < TOL["fp64"]


@pytest.mark.parametrize("din,dout", SHAPES)
@pytest.mark.parametrize("placement", ["L", "R", "AVG"])
def test_environments_fp64(ops, din, dout, placement):
    u, w, rho, h = _case(din, dout, 1)
    say(f"env fp64 din={din} dout={dout} placement={placement}")
    layer = ops.Layer(gpu(u), gpu(w))
    eu = host(ops.env_u(layer, gpu(h), gpu(rho), placement, "fp64"))
    ew = host(ops.env_w(layer, gpu(h), gpu(rho), placement, "fp64"))
    assert rel(eu, O.env_u(u, w, h, rho, placement)) < TOL["fp64"]
    assert rel(ew, O.env_w(u, w, h, rho, placement)) < TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("din,dout", [(3, 3), (4, 16), (8, 8)])
def test_reduced_precision_paths(ops, prec, din, dout):
    u, w, rho, h = _case(din, dout, 2)
    say(f"{prec} din={din} dout={dout}")
    layer = ops.Layer(gpu(u), gpu(w))
    checks = [
        (ops.descend(layer, gpu(rho), "AVG", prec), O.descend(u, w, rho)),
        (ops.ascend(layer, gpu(h), "AVG", prec), O.ascend(u, w, h)),
        (ops.env_u(layer, gpu(h), gpu(rho), "AVG", prec), O.env_u(u, w, h, rho)),
        (ops.env_w(layer, gpu(h), gpu(rho), "AVG", prec), O.env_w(u, w, h, rho)),
    ]
    for g, r in checks:
        err = rel(host(g), r)
        say(f"  rel err {err:.3e}")
        assert err < TOL[prec]


def test_large_chi12_descend(ops):
    """chi = 12: several 128-wide tiles in every GEMM, ragged tails (12^2 = 144)."""
    u, w, rho, h = _case(12, 12, 3)
    say("descend fp64 chi=12")
    layer = ops.Layer(gpu(u), gpu(w))
    d = host(ops.descend(layer, gpu(rho), "AVG", "fp64"))
    assert rel(d, O.descend(u, w, rho)) < TOL["fp64"]
    a = host(ops.ascend(layer, gpu(h), "AVG", "fp64"))
    assert rel(a, O.ascend(u, w, h)) < TOL["fp64"]


@pytest.mark.parametrize("rows,cols", [(4, 4), (16, 4), (16, 16), (64, 8), (81, 81), (256, 16), (576, 24),
                                       (576, 576), (1024, 1024)])
def test_polar_update(ops, rows, cols):
    rng = np.random.default_rng(rows + 7 * cols)
    y = rng.standard_normal((rows, cols))
    say(f"polar rows={rows} cols={cols}")
    out, sv, st = ops.polar_update(gpu(y), rows, cols, want_sv=True)
    got = host(out)
    ref, s = O.polar_update_matrix(y)
    # the polar factor's condition number is about 1/sigma_min (relative)
    cond = s[0] / s[-1]
    assert st == 0
    assert np.abs(got - ref).max() < 1e-13 * cond * max(1.0, np.sqrt(cols))
    assert np.abs(got.T @ got - np.eye(cols)).max() < 1e-13
    # singular values (largest first) against LAPACK: backward-stable eigenvalues of
    # X^T Y are accurate to a few ulps of sigma_max times the order
    assert np.abs(host(sv) - s).max() < 1e-14 * cols * s[0]


def test_polar_rejects_rank_deficient(ops):
    rng = np.random.default_rng(5)
    y = rng.standard_normal((16, 4)) @ np.diag([1.0, 1.0, 1.0, 0.0])
    out, sv, st = ops.polar_update(gpu(y), 16, 4, check=False, want_sv=True)
    assert st == 5  # MERA_ENUMERIC
    # the singular values are still written: the zero one is resolved to the scale of sigma_max
    s = np.linalg.svd(y, compute_uv=False)
    assert np.abs(host(sv) - s).max() < 1e-12 * s[0]
    z = np.zeros((9, 3))
    out, sv, st = ops.polar_update(gpu(z), 9, 3, check=False, want_sv=True)
    assert st == 5
    assert np.all(host(sv) == 0.0) and np.all(host(out) == 0.0)


def _polar_np(a):
    uu, _, vt = np.linalg.svd(a, full_matrices=False)
    return uu @ vt


def test_rank_deficient_update_takes_the_minimiser_closest_to_the_previous_tensor(ops):
    """A disentangler environment of rank 5 < 16 (as the scale-invariant Env_u of an optimised
    chi = 16 state, 107 of its 256 singular values below 1e-12 of the largest): every
    isometry -U_r V_r^T + W, W an isometry between the two null spaces, minimises
    tr(env^T x).  With the previous tensor the update returns the one whose null-space part is
    the polar factor of the previous tensor's null-space block (LAPACK as the comparator)."""
    rng = np.random.default_rng(11)
    d, r = 4, 5
    n = d * d
    env = rng.standard_normal((n, r)) @ rng.standard_normal((r, n))
    prev = _polar_np(rng.standard_normal((n, n)))
    with pytest.raises(Exception):
        ops.update_u(gpu(env.reshape(d, d, d, d)))
    x = host(ops.update_u(gpu(env.reshape(d, d, d, d)), prev=gpu(prev.reshape(d, d, d, d)))).reshape(n, n)
    assert np.abs(x.T @ x - np.eye(n)).max() < 1e-12
    uu, s, vt = np.linalg.svd(env)
    assert abs(np.sum(env * x) + s.sum()) < 1e-9 * s.sum()
    nl, nr = uu[:, r:], vt[r:].T
    expected = -uu[:, :r] @ vt[:r] + nl @ _polar_np(nl.T @ prev @ nr) @ nr.T
    # the zero singular values of env are ~3e-15 |env| after rounding, against the tie-break's
    # 1e-10 |env|: the selected completion differs from the exact one by ~1e-6 (numpy, seeds
    # 11..20: 7.6e-7 .. 5.3e-6)
    assert np.abs(x - expected).max() < 2e-5


def test_polar_update_near_is_the_plain_update_for_a_full_rank_environment(ops):
    """mera_polar_update_near on a full-rank environment (u and w blockings): bitwise the
    output of mera_polar_update; the previous tensor does not enter."""
    rng = np.random.default_rng(12)
    for rows, cols in ((16, 16), (64, 8)):
        env = gpu(rng.standard_normal((rows, cols)))
        prev = gpu(_polar_np(rng.standard_normal((rows, cols))))
        plain = host(ops.polar_update(env, rows, cols)[0])
        near, st = ops.polar_update_near(env, prev, rows, cols)
        assert st == 0
        assert np.array_equal(host(near), plain)


def test_polar_update_near_matches_the_shifted_environment_update(ops):
    """For a rank-deficient environment the call returns the plain update of
    env - t prev, t = tie ||env||_F / ||prev||_F (the shift formed here with numpy)."""
    rng = np.random.default_rng(13)
    rows, cols, r = 36, 6, 3
    env = rng.standard_normal((rows, r)) @ rng.standard_normal((r, cols))
    prev = _polar_np(rng.standard_normal((rows, cols)))
    tie = 1e-8
    near, st = ops.polar_update_near(gpu(env), gpu(prev), rows, cols, tie=tie)
    assert st == 0
    t = tie * np.linalg.norm(env) / np.linalg.norm(prev)
    ref = host(ops.polar_update(gpu(env - t * prev), rows, cols)[0])
    assert np.abs(host(near) - ref).max() < 1e-10
    x = host(near)
    assert np.abs(x.T @ x - np.eye(cols)).max() < 1e-12
    # a zero environment has no tie to break
    _, st0 = ops.polar_update_near(gpu(np.zeros((rows, cols))), gpu(prev), rows, cols, check=False)
    assert st0 == 5  # MERA_ENUMERIC


@pytest.mark.parametrize("d", [2, 3, 4])
def test_fixed_point(ops, d):
    rng = np.random.default_rng(40 + d)
    u, w = I.random_layer(rng, d, d)
    say(f"fixed point d={d}")
    rho0 = O.identity_density(d)
    ref = O.fixed_point_rho(u, w, rho0, 25)
    layer = ops.Layer(gpu(u), gpu(w))
    r = gpu(rho0)
    _, res, st = ops.fixed_point_rho(layer, r, 25, "fp64", want_residual=True)
    assert st == 0
    assert rel(host(r), ref) < 1e-12
    # residual of the returned density, ||D(rho) - rho||_F / ||rho||_F (Sec. II.B)
    want = O.fixed_point_residual(u, w, ref)
    assert abs(host(res)[0] - want) < 1e-12 + 1e-8 * want


def test_energy_and_hamiltonian(ops):
    h_gpu, c = ops.tfim_hamiltonian(1.0)
    h_ref, c_ref = O.shifted_hamiltonian(1.0)
    assert abs(c - c_ref) < 1e-14
    assert np.abs(host(h_gpu) - h_ref).max() < 1e-14
    rng = np.random.default_rng(3)
    for n in (8, 27, 64, 1000):
        a = rng.standard_normal((n, n))
        b = rng.standard_normal((n, n))
        e = host(ops.energy(gpu(a), gpu(b)))[0]
        assert abs(e - np.trace(a @ b)) < 1e-12 * n * n
        # bitwise reproducible
        assert host(ops.energy(gpu(a), gpu(b)))[0] == e


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_refined_fixed_point_reaches_fp64_fixed_point(ops, prec):
    """The reduced-precision fixed point (iterative refinement) converges to the FP64 one."""
    rng = np.random.default_rng(77)
    d = 4
    u, w = I.random_layer(rng, d, d)
    say(f"refined fixed point {prec}")
    layer = ops.Layer(gpu(u), gpu(w))
    r64 = gpu(O.identity_density(d))
    ops.fixed_point_rho(layer, r64, 150, "fp64")
    rlp = gpu(O.identity_density(d))
    ops.fixed_point_rho(layer, rlp, 150, prec)
    ref = O.fixed_point_rho(u, w, O.identity_density(d), 150)
    assert rel(host(r64), ref) < 1e-12
    # plain low-precision power iteration stalls near 1e-6; the refined one does not
    assert rel(host(rlp), ref) < 1e-11


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_sliced_descend_matches_unsliced(ops, prec):
    """With the minimum workspace the chi^7 intermediates are sliced over an open leg."""
    from paper_1906_12030_amd import _lib
    din, dout = 8, 8
    u, w, rho, h = _case(din, dout, 5)
    say(f"sliced descend {prec}")
    layer = ops.Layer(gpu(u), gpu(w))
    full = host(ops.descend(layer, gpu(rho), "AVG", prec))
    q = ops.PRECISIONS[prec]
    nb = _lib.mera_workspace_bytes_min(_lib.MERA_OP_DESCEND, din, dout, q, _lib.MERA_AVG)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) & ~255
    out = torch.empty((din,) * 6, dtype=torch.float64, device="cuda")
    r = gpu(rho)
    st = _lib.mera_descend(layer.c(), r.data_ptr(), out.data_ptr(), _lib.MERA_AVG, q, base, nb,
                           torch.cuda.current_stream().cuda_stream)
    assert st == 0
    sliced = host(out)
    # different slice shapes change the split-bf16 summation order, not the accuracy
    assert rel(sliced, full) < (1e-14 if prec == "fp64" else 1e-5)
    assert rel(sliced, O.descend(u, w, rho)) < TOL[prec]
    # fixed point with its minimum workspace (sliced FP64 refinement residual)
    nf = _lib.mera_workspace_bytes_min(_lib.MERA_OP_FIXED_POINT, din, dout, q, _lib.MERA_AVG)
    ws2 = torch.empty(nf + 256, dtype=torch.uint8, device="cuda")
    base2 = (ws2.data_ptr() + 255) & ~255
    r1 = gpu(O.identity_density(din))
    r2 = gpu(O.identity_density(din))
    ops.fixed_point_rho(layer, r1, 12, prec)
    st = _lib.mera_fixed_point_rho(layer.c(), r2.data_ptr(), 12, 0.0, q, None, base2, nf,
                                   torch.cuda.current_stream().cuda_stream)
    assert st == 0
    # same algorithm, different slice shapes: equal up to the reduced-precision rounding of the
    # correction (far from convergence after 12 steps the correction is not small)
    assert rel(host(r2), host(r1)) < (1e-14 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("frac", [0.0, 0.5])
def test_sliced_descend_large_tile_chi16(ops, frac):
    """Sliced split-bf16 descend at chi = 16, where every chi^8 / chi^9 step runs on the
    large-tile kernel with the sliced leg outermost in its intermediates: workspace at the
    minimum (one fine-leg value per slice) and half-way to the full size."""
    from paper_1906_12030_amd import _lib
    d = 16
    u, w, rho, h = _case(d, d, 7)
    say(f"sliced large-tile descend chi=16 frac={frac}")
    layer = ops.Layer(gpu(u), gpu(w))
    full = ops.descend(layer, gpu(rho), "AVG", "bf16x3")
    ref64 = ops.descend(layer, gpu(rho), "AVG", "fp64")
    q = ops.PRECISIONS["bf16x3"]
    lo = _lib.mera_workspace_bytes_min(_lib.MERA_OP_DESCEND, d, d, q, _lib.MERA_AVG)
    hi = _lib.load().mera_workspace_bytes(_lib.MERA_OP_DESCEND, d, d, q, _lib.MERA_AVG)
    nb = int(lo + frac * (hi - lo))
    assert nb < hi
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) & ~255
    out = torch.empty((d,) * 6, dtype=torch.float64, device="cuda")
    r = gpu(rho)
    st = _lib.mera_descend(layer.c(), r.data_ptr(), out.data_ptr(), _lib.MERA_AVG, q, base, nb,
                           torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    assert float((out - full).norm() / full.norm()) < 1e-5
    assert float((out - ref64).norm() / ref64.norm()) < 1e-5


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_fixed_point_tolerance(ops, prec):
    """tol > 0: the call stops at the first density whose residual is <= tol and returns
    MERA_ENOTCONV when the budget runs out first (Sec. II.B, iterative methods)."""
    rng = np.random.default_rng(91)
    d = 3
    u, w = I.random_layer(rng, d, d)
    say(f"fixed point tolerance {prec}")
    layer = ops.Layer(gpu(u), gpu(w))
    # a budget too small for 1e-12: ENOTCONV, residual of the returned density reported
    r = gpu(O.identity_density(d))
    _, res, st = ops.fixed_point_rho(layer, r, 3, prec, want_residual=True, tol=1e-12, check=False)
    assert st == 6  # MERA_ENOTCONV
    got = host(r)
    assert abs(host(res)[0] - O.fixed_point_residual(u, w, got)) < 1e-12
    assert host(res)[0] > 1e-12
    # a generous budget: stops with the residual at or below tol, and at or below it in the oracle
    r = gpu(O.identity_density(d))
    _, res, st = ops.fixed_point_rho(layer, r, 3000, prec, want_residual=True, tol=1e-10)
    assert st == 0
    got = host(r)
    assert host(res)[0] <= 1e-10
    assert O.fixed_point_residual(u, w, got) <= 1e-10 * (1 + 1e-6) + 1e-15
    assert abs(np.trace(got.reshape(d ** 3, -1)) - 1.0) < 1e-13
    # the same density as the FP64 oracle's after enough plain steps
    ref = O.fixed_point_rho(u, w, O.identity_density(d), 3000)
    assert rel(got, ref) < 1e-8
