"""Host-side tests of the C ABI: exports, argument checks, workspace and flop accounting.

These run without a GPU: every rejected call returns before any HIP call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1906_12030_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmera.so not built")
    return _lib.load()


def test_header_symbols_are_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "mera.h")).read()
    names = set(re.findall(r"\b(mera_[a-z_0-9]+)\s*\(", hdr))
    assert {"mera_ascend", "mera_descend", "mera_env_u", "mera_env_w", "mera_polar_update",
            "mera_fixed_point_rho", "mera_energy"} <= names
    for n in names:
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTED) == names


def test_strerror(lib):
    for st in range(7):
        assert lib.mera_strerror(st)
    assert b"unknown" in lib.mera_strerror(99)
    assert b"reserved" not in lib.mera_strerror(_lib.MERA_ENOTCONV)


def _layer(din, dout, nonnull=True):
    p = 4096 if nonnull else 0
    return _lib.MeraLayer(din, dout, p, p)


def test_invalid_arguments_rejected_before_device(lib):
    fake = 4096  # never dereferenced: validation fails first
    assert _lib.mera_descend(_layer(4, 17), fake, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_ESHAPE
    assert _lib.mera_descend(_layer(4, 4, False), fake, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_descend(_layer(4, 4), fake, fake, 3, 0, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_descend(_layer(4, 4), fake, fake, 2, 7, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_descend(_layer(4, 4), None, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_ascend(_layer(0, 4), fake, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_ESHAPE
    assert _lib.mera_env_u(_layer(3, 3), fake, None, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_env_w(_layer(3, 10), fake, fake, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_ESHAPE
    assert _lib.mera_fixed_point_rho(_layer(3, 4), fake, 5, 0.0, 0, None, fake, 1 << 40, None) == _lib.MERA_ESHAPE
    assert _lib.mera_fixed_point_rho(_layer(3, 3), fake, -1, 0.0, 0, None, fake, 1 << 40, None) == _lib.MERA_EINVAL
    # the tolerance must be a finite number >= 0
    for bad in (-1e-9, float("nan"), float("inf")):
        assert _lib.mera_fixed_point_rho(_layer(3, 3), fake, 5, bad, 0, None, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_polar_update(fake, 4, 9, fake, None, fake, 1 << 40, None) == _lib.MERA_ESHAPE
    assert _lib.mera_polar_update(None, 9, 4, fake, None, fake, 1 << 40, None) == _lib.MERA_EINVAL
    # singular values are limited to the order the device eigensolver handles
    assert _lib.mera_polar_update(fake, 5000, 4100, fake, fake, fake, 1 << 40, None) == _lib.MERA_ESHAPE
    assert b"4080" in lib.mera_last_error()
    assert _lib.mera_energy(fake, fake, 0, fake, None) == _lib.MERA_ESHAPE
    assert lib.mera_last_error()


def test_noalloc_descend_rejects_what_the_static_scratch_cannot_hold(lib):
    fake = 4096  # never dereferenced: the size check fails before any HIP call
    for d, prec in ((14, 0), (15, 1), (13, 2), (15, 2), (24, 2)):
        assert _lib.mera_descend_noalloc(_layer(d, d), fake, fake, 2, prec, None) == _lib.MERA_EWORKSPACE
        assert b"static scratch" in lib.mera_last_error()
    assert _lib.mera_descend_noalloc(_layer(4, 17), fake, fake, 2, 0, None) == _lib.MERA_ESHAPE
    assert _lib.mera_descend_noalloc(_layer(4, 4), None, fake, 2, 0, None) == _lib.MERA_EINVAL
    assert _lib.mera_descend_noalloc(_layer(4, 4), fake, fake, 5, 0, None) == _lib.MERA_EINVAL
    # the limit in the header is the one the library applies
    mib = int(re.search(r"#define MERA_NOALLOC_SCRATCH_MIB (\d+)",
                        open(os.path.join(ROOT, "include", "mera.h")).read()).group(1))
    fits = {(d, prec): _lib.mera_workspace_bytes_min(_lib.MERA_OP_DESCEND, d, d, prec, 2) <= mib << 20
            for d in range(2, 25) for prec in (0, 1, 2)}
    # FP64 up to chi = 13, FP32 up to 14; split bf16 up to 12 and at 14 (at odd chi
    # the slices of its split tensors must start on whole 8-element groups)
    assert [d for d in range(2, 25) if fits[(d, 0)]] == list(range(2, 14))
    assert [d for d in range(2, 25) if fits[(d, 1)]] == list(range(2, 15))
    assert [d for d in range(2, 25) if fits[(d, 2)]] == list(range(2, 13)) + [14]
    for (d, prec), ok in fits.items():
        if not ok:
            assert _lib.mera_descend_noalloc(_layer(d, d), fake, fake, 2, prec, None) == _lib.MERA_EWORKSPACE


def test_workspace_too_small_and_misaligned(lib):
    fake = 4096
    need = _lib.mera_workspace_bytes(_lib.MERA_OP_DESCEND, 4, 4, 0, 2)
    least = _lib.mera_workspace_bytes_min(_lib.MERA_OP_DESCEND, 4, 4, 0, 2)
    assert 0 < least < need
    assert _lib.mera_descend(_layer(4, 4), fake, fake, 2, 0, fake, least - 1, None) == _lib.MERA_EWORKSPACE
    assert _lib.mera_env_u(_layer(4, 4), fake, fake, fake, 2, 0, fake, 1024, None) == _lib.MERA_EWORKSPACE
    fneed = _lib.mera_workspace_bytes_min(_lib.MERA_OP_FIXED_POINT, 4, 4, 2, 2)
    assert 0 < fneed < _lib.mera_workspace_bytes(_lib.MERA_OP_FIXED_POINT, 4, 4, 2, 2)
    # far below the sliced minimum: rejected before any device work
    assert _lib.mera_fixed_point_rho(_layer(4, 4), fake, 3, 0.0, 2, None, fake, fneed // 4, None) == _lib.MERA_EWORKSPACE
    assert _lib.mera_fixed_point_rho(_layer(4, 4), fake, 3, 1e-10, 2, fake, fake, fneed // 4, None) == _lib.MERA_EWORKSPACE
    assert _lib.mera_descend(_layer(4, 4), fake, fake, 2, 0, fake + 8, need, None) == _lib.MERA_EINVAL
    npol = _lib.mera_workspace_bytes(_lib.MERA_OP_POLAR, 16, 4, 0, 0)
    assert _lib.mera_polar_update(fake, 16, 4, fake, fake, fake, npol - 1, None) == _lib.MERA_EWORKSPACE


def test_workspace_grows_with_bond_dimension(lib):
    for op in (_lib.MERA_OP_ASCEND, _lib.MERA_OP_DESCEND, _lib.MERA_OP_ENV_U, _lib.MERA_OP_ENV_W):
        for prec in (0, 1, 2):
            sizes = [_lib.mera_workspace_bytes(op, d, d, prec, 2) for d in (2, 4, 8, 12, 16, 24)]
            assert all(a < b for a, b in zip(sizes, sizes[1:])), (op, prec, sizes)
    # the chi^7 intermediate dominates: FP64 at chi=24 needs about 24^7 * 8 bytes
    ws = _lib.mera_workspace_bytes(_lib.MERA_OP_DESCEND, 24, 24, 0, 2)
    assert 24 ** 7 * 8 < ws < 1.3 * 24 ** 7 * 8
    ws32 = _lib.mera_workspace_bytes(_lib.MERA_OP_DESCEND, 24, 24, 1, 2)
    assert 0.45 < ws32 / ws < 0.6
    assert _lib.mera_workspace_bytes(_lib.MERA_OP_DESCEND, 4, 17, 0, 2) == 0
    assert _lib.mera_workspace_bytes(99, 4, 4, 0, 2) == 0


def test_sliced_workspace_shrinks_as_chi7_over_slices(lib):
    """Slicing the chi^7 intermediates over an open leg: the minimum workspace drops by ~chi."""
    for prec, es in ((0, 8), (2, 4)):
        full = _lib.mera_workspace_bytes(_lib.MERA_OP_DESCEND, 24, 24, prec, 2)
        least = _lib.mera_workspace_bytes_min(_lib.MERA_OP_DESCEND, 24, 24, prec, 2)
        assert full - least > 0.9 * (24 ** 7 - 24 ** 6) * es
    # chi=32 in split bf16 fits a 288 GB device only when sliced for the FP64 refinement
    fp = _lib.mera_workspace_bytes(_lib.MERA_OP_FIXED_POINT, 32, 32, 2, 2)
    fp_min = _lib.mera_workspace_bytes_min(_lib.MERA_OP_FIXED_POINT, 32, 32, 2, 2)
    assert fp > 288e9 > 2 * fp_min


def test_flop_accounting_scales_as_chi9(lib):
    """Executed flops: 8 chi^9 per D or A call (four chi^9 GEMMs) plus lower orders."""
    for chi in (16, 24, 32):
        for op in (_lib.MERA_OP_DESCEND, _lib.MERA_OP_ASCEND):
            f = _lib.mera_flops(op, chi, chi, 2)
            assert 8 * chi ** 9 < f < 8 * chi ** 9 * (1 + 8.0 / chi), (op, chi, f / chi ** 9)
        fu = _lib.mera_flops(_lib.MERA_OP_ENV_U, chi, chi, 2)
        fw = _lib.mera_flops(_lib.MERA_OP_ENV_W, chi, chi, 2)
        assert 16 * chi ** 9 < fu < 16 * chi ** 9 * (1 + 8.0 / chi)
        assert 12 * chi ** 9 < fw < 12 * chi ** 9 * (1 + 8.0 / chi)
        # one placement costs half of the averaged call in the chi^9 terms
        fl = _lib.mera_flops(_lib.MERA_OP_DESCEND, chi, chi, 0)
        assert abs(fl / _lib.mera_flops(_lib.MERA_OP_DESCEND, chi, chi, 2) - 0.5) < 0.06


def test_native_hamiltonian_matches_oracle(lib):
    from oracle import mera_oracle as O
    for g in (1.0, 0.5, 1.7):
        st, h, c = _lib.mera_tfim_hamiltonian(g)
        assert st == 0
        h3 = O.tfim_three_site(g)
        c_ref = np.linalg.eigvalsh(h3)[-1]
        assert abs(c - c_ref) < 1e-14
        assert np.abs(np.array(h).reshape(8, 8) - (h3 - c_ref * np.eye(8))).max() < 1e-14


def test_mfma_peak_argument_checks(lib):
    fake = 4096
    st, _ = _lib.mera_mfma_peak(3, fake, 1 << 21)
    assert st == _lib.MERA_EINVAL
    st, _ = _lib.mera_mfma_peak(0, None, 1 << 21)
    assert st == _lib.MERA_EINVAL
    st, _ = _lib.mera_mfma_peak(0, fake, 1 << 20)
    assert st == _lib.MERA_EWORKSPACE


def test_contract_argument_checks(lib):
    """mera_contract rejects malformed specifications before any HIP call."""
    fake = 4096
    ok = dict(a=fake, b=fake, c=fake, ws=fake, wsb=1 << 30)

    def call(la, lb, lc, labels, sizes, prec=0):
        return _lib.mera_contract(la, ok["a"], lb, ok["b"], lc, ok["c"], labels, sizes, 1.0, 0.0, prec,
                                  ok["ws"], ok["wsb"], None)
    assert call("ab", "bc", "ac", "abc", [2, 3, 4], prec=7) == _lib.MERA_EINVAL
    assert call("ab", "bc", "ac", "abc", [2, 0, 4]) == _lib.MERA_ESHAPE      # empty leg
    assert call("ab", "bc", "ac", "abb", [2, 3, 4]) == _lib.MERA_ESHAPE      # repeated label
    assert call("aab", "bc", "ac", "abc", [2, 3, 4]) == _lib.MERA_ESHAPE     # repeated leg
    assert call("ab", "bc", "abc", "abc", [2, 3, 4]) == _lib.MERA_ESHAPE     # batch leg b
    assert call("ab", "cd", "ac", "abcd", [2, 3, 4, 5]) == _lib.MERA_ESHAPE  # b, d summed in one operand
    assert call("ab", "bc", "ax", "abc", [2, 3, 4]) == _lib.MERA_ESHAPE      # unknown label
    assert call("ab", "bc", "ac", "abc", [1 << 31, 3, 4]) == _lib.MERA_ESHAPE


def _plans(op, d_in, d_out, prec, placement=_lib.MERA_AVG):
    st, lines = _lib.mera_schedule_plan(op, d_in, d_out, prec, placement)
    assert st == _lib.MERA_OK
    out = []
    for ln in lines:
        labels, kern, *rest = ln.split()
        kv = dict(x.split("=") for x in rest)
        out.append((labels, kern, int(kv["m"]), int(kv["n"]), int(kv["k"]), kv["store"], kv.get("tail")))
    return out


def test_schedule_plan_split_bf16_descend_on_large_tile_kernel(lib):
    """Every chi^8 and chi^9 contraction of the split-bf16 descend (the fixed-point
    iteration) is planned on the large-tile kernel, with a column tile that divides
    chi^2 = 576 where that operand is the n side (288 for the long k ranges, 192 for
    the short ones); the intermediates whose innermost leg is an m leg are stored
    along m, the two chi^7 ones (left Y and right T1) as whole 8-column split groups."""
    chi = 24
    plans = _plans(_lib.MERA_OP_DESCEND, chi, chi, _lib.MERA_BF16X3)
    big = [p for p in plans if p[2] * p[3] * p[4] >= chi ** 8]
    assert len(big) == 11  # X1, two copies of X, four chi^9 and four chi^8 chain steps
    for labels, kern, m, n, k, store, tail in big:
        assert kern.startswith("b3x"), (labels, kern)
        if n == chi * chi:
            assert kern == ("b3x288" if k >= 2048 else "b3x192"), labels
        assert store in ("n8", "n4", "m4"), (labels, store)
        if m * n == chi ** 7:
            assert store == "n8", (labels, store)
        # 1296 x 2 tiles of the long-k launches fill ten waves of 256 slots and an eighth
        # of an eleventh: the last 16 tile rows run split eight ways along k
        assert tail == ("16x8" if k == chi ** 3 else None), (labels, tail)
    assert sum(p[5] == "m4" for p in big) >= 6
    # flops: the FP64 schedule is the one mera_flops counts; the split-bf16 one
    # forms two k-contiguous copies of X (one chi^8 contraction more)
    p64 = _plans(_lib.MERA_OP_DESCEND, chi, chi, _lib.MERA_FP64)
    f64 = sum(2.0 * m * n * k for _, _, m, n, k, _, _ in p64)
    assert f64 == _lib.load().mera_flops(_lib.MERA_OP_DESCEND, chi, chi, _lib.MERA_AVG)
    fb3 = sum(2.0 * m * n * k for _, _, m, n, k, _, _ in plans)
    assert fb3 == f64 + 2.0 * chi ** 8
    # the same steps in FP64 and FP32 keep their own kernels
    assert {p[1] for p in p64} == {"f64"}
    assert {p[1] for p in _plans(_lib.MERA_OP_DESCEND, chi, chi, _lib.MERA_FP32)} == {"f32"}


def test_schedule_plan_argument_checks(lib):
    st, _ = _lib.mera_schedule_plan(_lib.MERA_OP_DESCEND, 8, 8, 5, _lib.MERA_AVG)
    assert st == _lib.MERA_EINVAL
    st, _ = _lib.mera_schedule_plan(_lib.MERA_OP_DESCEND, 8, 8, 0, 9)
    assert st == _lib.MERA_EINVAL
    st, _ = _lib.mera_schedule_plan(_lib.MERA_OP_FIXED_POINT, 8, 4, 0, _lib.MERA_AVG)
    assert st == _lib.MERA_ESHAPE
    st, _ = _lib.mera_schedule_plan(_lib.MERA_OP_DESCEND, 2, 5, 0, _lib.MERA_AVG)
    assert st == _lib.MERA_ESHAPE
    st, _ = _lib.mera_schedule_plan(_lib.MERA_OP_POLAR, 8, 8, 0, _lib.MERA_AVG)
    assert st == _lib.MERA_EINVAL
    # truncation: a short buffer holds a NUL-terminated prefix, *needed the full size
    lib_ = _lib.load()
    need = ctypes.c_size_t(0)
    buf = ctypes.create_string_buffer(16)
    assert lib_.mera_schedule_plan(_lib.MERA_OP_ASCEND, 4, 4, 0, 2, buf, 16, ctypes.byref(need)) == 0
    assert len(buf.value) == 15 and need.value > 16


def test_tree_calls_checks_and_cost(lib):
    """Binary tree calls: host-side argument checks, and executed flops growing as din^6 dout
    (against din^6 dout^3 for the MERA cone)."""
    fake = 4096
    assert _lib.mera_tree_descend(4, 17, fake, fake, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_ESHAPE
    assert _lib.mera_tree_descend(4, 4, None, fake, fake, 2, 0, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_tree_ascend(4, 4, fake, fake, None, 2, 0, fake, 1 << 40, None) == _lib.MERA_EINVAL
    assert _lib.mera_tree_env_w(4, 4, fake, fake, fake, fake, 3, 0, fake, 1 << 40, None) == _lib.MERA_EINVAL
    need = _lib.mera_workspace_bytes(_lib.MERA_OP_TREE_ENV_W, 8, 8, 2, 2)
    assert need > 0
    assert _lib.mera_tree_env_w(8, 8, fake, fake, fake, fake, 2, 2, fake, need - 1, None) == _lib.MERA_EWORKSPACE
    for op in (_lib.MERA_OP_TREE_ASCEND, _lib.MERA_OP_TREE_DESCEND, _lib.MERA_OP_TREE_ENV_W):
        r = [_lib.mera_flops(op, d, d, 2) / d ** 7 for d in (16, 32, 64)]
        assert all(3.5 < x < 8 for x in r), (op, r)
        assert r[2] < r[1] < r[0]  # lower orders fade
    assert _lib.mera_flops(_lib.MERA_OP_TREE_DESCEND, 24, 24, 2) < 1e-2 * _lib.mera_flops(_lib.MERA_OP_DESCEND, 24, 24, 2)


def test_every_schedule_is_planned_and_sized(lib):
    """The measuring pass of every call, arithmetic, placement and a range of bond
    dimensions (ragged and sliced shapes included) returns a plan and a workspace size;
    the sliced minimum never exceeds the full size."""
    ops = (_lib.MERA_OP_ASCEND, _lib.MERA_OP_DESCEND, _lib.MERA_OP_ENV_U, _lib.MERA_OP_ENV_W,
           _lib.MERA_OP_FIXED_POINT, _lib.MERA_OP_TREE_ASCEND, _lib.MERA_OP_TREE_DESCEND,
           _lib.MERA_OP_TREE_ENV_W)
    n = 0
    for op in ops:
        for prec in (_lib.MERA_FP64, _lib.MERA_FP32, _lib.MERA_BF16X3):
            for din, dout in ((2, 2), (3, 2), (4, 3), (6, 6), (8, 8), (12, 12), (16, 16), (24, 24)):
                for pl in (_lib.MERA_LEFT, _lib.MERA_RIGHT, _lib.MERA_AVG):
                    if op == _lib.MERA_OP_FIXED_POINT and din != dout:
                        continue
                    st, plan = _lib.mera_schedule_plan(op, din, dout, prec, pl)
                    assert st == _lib.MERA_OK and plan, (op, prec, din, dout, pl)
                    full = _lib.mera_workspace_bytes(op, din, dout, prec, pl)
                    least = _lib.mera_workspace_bytes_min(op, din, dout, prec, pl)
                    assert 0 < least <= full, (op, prec, din, dout, pl, least, full)
                    n += 1
    assert n > 500


def test_polar_update_near_argument_checks(lib):
    fake = 4096
    plain = _lib.mera_workspace_bytes(_lib.MERA_OP_POLAR, 16, 4, 0, 0)
    need = _lib.mera_workspace_bytes(_lib.MERA_OP_POLAR_NEAR, 16, 4, 0, 0)
    assert need == plain + 16 * 4 * 8  # the shifted environment (512 bytes, already aligned)
    assert _lib.mera_workspace_bytes(_lib.MERA_OP_POLAR_NEAR, 4, 16, 0, 0) == 0
    f = _lib.mera_polar_update_near
    assert f(fake, None, 16, 4, 1e-10, fake, None, fake, need, None) == _lib.MERA_EINVAL
    assert f(fake, fake, 16, 4, 0.0, fake, None, fake, need, None) == _lib.MERA_EINVAL
    assert f(fake, fake, 16, 4, float("nan"), fake, None, fake, need, None) == _lib.MERA_EINVAL
    assert f(fake, fake, 4, 16, 1e-10, fake, None, fake, need, None) == _lib.MERA_ESHAPE
    assert f(fake, fake, 16, 4, 1e-10, fake, None, fake, need - 1, None) == _lib.MERA_EWORKSPACE
    assert f(fake, fake, 16, 4, 1e-10, fake, None, fake + 8, need, None) == _lib.MERA_EINVAL
    assert f(None, fake, 16, 4, 1e-10, fake, None, fake, need, None) == _lib.MERA_EINVAL
    st, _ = _lib.mera_schedule_plan(_lib.MERA_OP_POLAR_NEAR, 16, 4, 0, _lib.MERA_AVG)
    assert st == _lib.MERA_EINVAL
