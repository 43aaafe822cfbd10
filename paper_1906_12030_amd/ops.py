"""Torch-facing calls of the MERA hot path.

PyTorch supplies device memory and the stream; every computation happens in
libmera.so (through ``_lib``).  Tensors are float64, contiguous, on a HIP
device.  Outputs and workspaces are allocated here with torch.
"""
from __future__ import annotations

import torch

from . import _lib

PLACEMENTS = {"left": _lib.MERA_LEFT, "right": _lib.MERA_RIGHT, "avg": _lib.MERA_AVG,
              "L": _lib.MERA_LEFT, "R": _lib.MERA_RIGHT, "AVG": _lib.MERA_AVG}
PRECISIONS = {"fp64": _lib.MERA_FP64, "fp32": _lib.MERA_FP32, "bf16x3": _lib.MERA_BF16X3}


def _dev(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if t.dtype != torch.float64:
        raise TypeError("tensors must be float64")
    return t.contiguous()


class Layer:
    """A MERA layer (u: din^4, w: din*din*dout) as device float64 tensors."""

    def __init__(self, u: torch.Tensor, w: torch.Tensor):
        self.u = _dev(u)
        self.w = _dev(w)
        self.din = int(self.w.shape[0])
        self.dout = int(self.w.shape[2])
        if tuple(self.u.shape) != (self.din,) * 4 or tuple(self.w.shape) != (self.din, self.din, self.dout):
            raise ValueError("layer shapes: u must be din^4 and w din x din x dout")

    def c(self) -> _lib.MeraLayer:
        return _lib.MeraLayer(self.din, self.dout, self.u.data_ptr(), self.w.data_ptr())


class Workspace:
    """Grow-only device workspace, reused by calls on the same stream."""

    def __init__(self):
        self.buf: dict = {}

    def get(self, nbytes: int, device) -> tuple[int, int]:
        key = (torch.device(device).index,)
        cur = self.buf.get(key)
        if nbytes == 0:
            return 0, 0
        if cur is None or cur.numel() < nbytes:
            self.buf[key] = None
            cur = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            self.buf[key] = cur
        ptr = cur.data_ptr()
        aligned = (ptr + 255) & ~255
        return aligned, cur.numel() - (aligned - ptr)

    def size(self, device) -> int:
        cur = self.buf.get((torch.device(device).index,))
        return 0 if cur is None else cur.numel()

    def release(self):
        self.buf.clear()

    def for_op(self, op: int, din: int, dout: int, q: int, p: int, device) -> tuple[int, int]:
        """Workspace for one call: the full size when it fits on the device, else as much as
        fits (at least mera_workspace_bytes_min: the chi^7 intermediates are then sliced)."""
        full = _lib.mera_workspace_bytes(op, din, dout, q, p)
        cur = self.size(device)
        if full <= cur:
            return self.get(full, device)
        free, _ = torch.cuda.mem_get_info(device)
        cached = torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device)
        avail = free + cached + cur - (2 << 30)  # keep 2 GiB for the caller's tensors
        if full <= avail:
            return self.get(full, device)
        # sliced: leave a quarter of the device to the caller's chi^6 tensors
        budget = avail - torch.cuda.get_device_properties(device).total_memory // 4
        least = _lib.mera_workspace_bytes_min(op, din, dout, q, p)
        if least > max(budget, avail - (8 << 30)):
            raise MemoryError(f"workspace: {least / 1e9:.1f} GB needed even with slicing, "
                              f"{avail / 1e9:.1f} GB available")
        return self.get(max(least, budget), device)


WORKSPACE = Workspace()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _prec(precision) -> int:
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def _place(placement) -> int:
    return PLACEMENTS[placement] if isinstance(placement, str) else int(placement)


def ascend(layer: Layer, h: torch.Tensor, placement="avg", precision="fp64", out=None):
    """A_P(h): din^6 -> dout^6 (Sec. II.B, Fig. 4a)."""
    h = _dev(h)
    p, q = _place(placement), _prec(precision)
    if out is None:
        out = torch.empty((layer.dout,) * 6, dtype=torch.float64, device=h.device)
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_ASCEND, layer.din, layer.dout, q, p, h.device)
    _lib.check(_lib.mera_ascend(layer.c(), h.data_ptr(), out.data_ptr(), p, q, ws, wsb, _stream(h.device)), "mera_ascend")
    return out


def descend(layer: Layer, rho: torch.Tensor, placement="avg", precision="fp64", out=None):
    """D_P(rho): dout^6 -> din^6 (Sec. II.B, Fig. 4b)."""
    rho = _dev(rho)
    p, q = _place(placement), _prec(precision)
    if out is None:
        out = torch.empty((layer.din,) * 6, dtype=torch.float64, device=rho.device)
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_DESCEND, layer.din, layer.dout, q, p, rho.device)
    _lib.check(_lib.mera_descend(layer.c(), rho.data_ptr(), out.data_ptr(), p, q, ws, wsb, _stream(rho.device)), "mera_descend")
    return out


def env_u(layer: Layer, h: torch.Tensor, rho: torch.Tensor, placement="avg", precision="fp64", out=None):
    """Environment of u (Sec. II.C, Fig. 4d): din^4."""
    h, rho = _dev(h), _dev(rho)
    p, q = _place(placement), _prec(precision)
    if out is None:
        out = torch.empty((layer.din,) * 4, dtype=torch.float64, device=h.device)
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_ENV_U, layer.din, layer.dout, q, p, h.device)
    _lib.check(_lib.mera_env_u(layer.c(), h.data_ptr(), rho.data_ptr(), out.data_ptr(), p, q, ws, wsb, _stream(h.device)), "mera_env_u")
    return out


def env_w(layer: Layer, h: torch.Tensor, rho: torch.Tensor, placement="avg", precision="fp64", out=None):
    """Environment of w (Sec. II.C, Fig. 4c): din x din x dout."""
    h, rho = _dev(h), _dev(rho)
    p, q = _place(placement), _prec(precision)
    if out is None:
        out = torch.empty((layer.din, layer.din, layer.dout), dtype=torch.float64, device=h.device)
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_ENV_W, layer.din, layer.dout, q, p, h.device)
    _lib.check(_lib.mera_env_w(layer.c(), h.data_ptr(), rho.data_ptr(), out.data_ptr(), p, q, ws, wsb, _stream(h.device)), "mera_env_w")
    return out


def _tree_dims(w: torch.Tensor):
    w = _dev(w)
    din, din2, dout = (int(x) for x in w.shape)
    if din2 != din:
        raise ValueError("w must be din x din x dout")
    return w, din, dout


def tree_descend(w: torch.Tensor, rho: torch.Tensor, placement="avg", precision="fp64", out=None):
    """Binary tree descend (Fig. 1a; the MERA with u = identity): dout^6 -> din^6."""
    w, din, dout = _tree_dims(w)
    rho = _dev(rho)
    p, q = _place(placement), _prec(precision)
    if out is None:
        out = torch.empty((din,) * 6, dtype=torch.float64, device=rho.device)
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_TREE_DESCEND, din, dout, q, p, rho.device)
    _lib.check(_lib.mera_tree_descend(din, dout, w.data_ptr(), rho.data_ptr(), out.data_ptr(), p, q, ws, wsb,
                                      _stream(rho.device)), "mera_tree_descend")
    return out


def tree_ascend(w: torch.Tensor, h: torch.Tensor, placement="avg", precision="fp64", out=None):
    """Binary tree ascend: din^6 -> dout^6."""
    w, din, dout = _tree_dims(w)
    h = _dev(h)
    p, q = _place(placement), _prec(precision)
    if out is None:
        out = torch.empty((dout,) * 6, dtype=torch.float64, device=h.device)
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_TREE_ASCEND, din, dout, q, p, h.device)
    _lib.check(_lib.mera_tree_ascend(din, dout, w.data_ptr(), h.data_ptr(), out.data_ptr(), p, q, ws, wsb,
                                     _stream(h.device)), "mera_tree_ascend")
    return out


def tree_env_w(w: torch.Tensor, h: torch.Tensor, rho: torch.Tensor, placement="avg", precision="fp64",
               out=None):
    """Environment of w in the binary tree: din x din x dout."""
    w, din, dout = _tree_dims(w)
    h, rho = _dev(h), _dev(rho)
    p, q = _place(placement), _prec(precision)
    if out is None:
        out = torch.empty((din, din, dout), dtype=torch.float64, device=h.device)
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_TREE_ENV_W, din, dout, q, p, h.device)
    _lib.check(_lib.mera_tree_env_w(din, dout, w.data_ptr(), h.data_ptr(), rho.data_ptr(), out.data_ptr(), p, q,
                                    ws, wsb, _stream(h.device)), "mera_tree_env_w")
    return out


def polar_update(env: torch.Tensor, rows: int, cols: int, out=None, check=True, want_sv=False):
    """-U V^T of env blocked as rows x cols (Sec. II.C, Fig. 5).

    Returns (out, singular values or None, status)."""
    env = _dev(env)
    if out is None:
        out = torch.empty(env.shape, dtype=torch.float64, device=env.device)
    sv = torch.empty(cols, dtype=torch.float64, device=env.device) if want_sv else None
    nb = _lib.mera_workspace_bytes(_lib.MERA_OP_POLAR, rows, cols, 0, 0)
    ws, wsb = WORKSPACE.get(nb, env.device)
    st = _lib.mera_polar_update(env.data_ptr(), rows, cols, out.data_ptr(),
                                sv.data_ptr() if sv is not None else None, ws, wsb, _stream(env.device))
    if check:
        _lib.check(st, "mera_polar_update")
    return out, sv, st


# Relative weight of the previous tensor that breaks the tie of a rank-deficient environment.
TIE_BREAK = 1e-10


def polar_update_near(env: torch.Tensor, prev: torch.Tensor, rows: int, cols: int, tie=TIE_BREAK,
                      out=None, check=True):
    """-U V^T of env, or for a rank-deficient env that of env - t prev with
    t = tie ||env|| / ||prev|| (mera_polar_update_near).  Returns (out, status)."""
    env, prev = _dev(env), _dev(prev)
    if prev.shape != env.shape or prev.device != env.device:
        raise ValueError("prev must have the shape and device of env")
    if out is None:
        out = torch.empty(env.shape, dtype=torch.float64, device=env.device)
    nb = _lib.mera_workspace_bytes(_lib.MERA_OP_POLAR_NEAR, rows, cols, 0, 0)
    ws, wsb = WORKSPACE.get(nb, env.device)
    st = _lib.mera_polar_update_near(env.data_ptr(), prev.data_ptr(), rows, cols, float(tie),
                                     out.data_ptr(), None, ws, wsb, _stream(env.device))
    if check:
        _lib.check(st, "mera_polar_update_near")
    return out, st


def _update(env: torch.Tensor, rows: int, cols: int, prev, check: bool) -> torch.Tensor:
    """-U V^T of env.  When env is rank-deficient the minimiser of tr(env^T x) over isometries
    is not unique; with `prev` (the tensor being updated) the library then takes the update
    of env - t prev, t = TIE_BREAK ||env|| / ||prev||, which selects among those minimisers
    (up to O(t)) the one closest to prev."""
    if prev is None:
        return polar_update(env, rows, cols, check=check)[0]
    return polar_update_near(env, prev, rows, cols, check=check)[0]


def update_u(env: torch.Tensor, check=True, prev=None) -> torch.Tensor:
    d = env.shape[0]
    return _update(env, d * d, d * d, prev, check)


def update_w(env: torch.Tensor, check=True, prev=None) -> torch.Tensor:
    din, _, dout = env.shape
    return _update(env, din * din, dout, prev, check)


def fixed_point_rho(si: Layer, rho: torch.Tensor, iters: int, precision="fp64", want_residual=False,
                    tol: float = 0.0, check=True):
    """In place: at most iters power-iteration steps of the scale-invariant D (Sec. II.B).

    tol > 0 stops at the first density with ||D(rho) - rho||_F / ||rho||_F <= tol.
    Returns (rho, residual of the returned rho as a device tensor or None, status)."""
    if not (rho.is_cuda and rho.dtype == torch.float64 and rho.is_contiguous()):
        raise ValueError("rho must be a contiguous float64 GPU tensor (it is updated in place)")
    q = _prec(precision)
    resid = torch.zeros(1, dtype=torch.float64, device=rho.device) if want_residual else None
    ws, wsb = WORKSPACE.for_op(_lib.MERA_OP_FIXED_POINT, si.din, si.dout, q, _lib.MERA_AVG, rho.device)
    st = _lib.mera_fixed_point_rho(si.c(), rho.data_ptr(), int(iters), float(tol), q,
                                   resid.data_ptr() if resid is not None else None,
                                   ws, wsb, _stream(rho.device))
    if check:
        _lib.check(st, "mera_fixed_point_rho")
    return rho, resid, st


def energy(h: torch.Tensor, rho: torch.Tensor) -> torch.Tensor:
    """tr(h rho) as a one-element device tensor (Sec. II.B)."""
    h, rho = _dev(h), _dev(rho)
    n = int(round(h.numel() ** 0.5))
    if n * n != h.numel() or rho.numel() != h.numel():
        raise ValueError("h and rho must be n x n matrices of the same order")
    e = torch.empty(1, dtype=torch.float64, device=h.device)
    _lib.check(_lib.mera_energy(h.data_ptr(), rho.data_ptr(), n, e.data_ptr(), _stream(h.device)), "mera_energy")
    return e


def tfim_hamiltonian(field: float = 1.0, device="cuda"):
    """Shifted three-site TFIM density (8x8 -> [2]*6) built by the library, and the shift."""
    st, h, c = _lib.mera_tfim_hamiltonian(float(field))
    _lib.check(st, "mera_tfim_hamiltonian")
    return torch.tensor(h, dtype=torch.float64).reshape((2,) * 6).to(device), c


def flops(op: str, din: int, dout: int, placement="avg") -> float:
    ops = {"ascend": _lib.MERA_OP_ASCEND, "descend": _lib.MERA_OP_DESCEND, "env_u": _lib.MERA_OP_ENV_U,
           "env_w": _lib.MERA_OP_ENV_W, "fixed_point_iter": _lib.MERA_OP_FIXED_POINT,
           "tree_ascend": _lib.MERA_OP_TREE_ASCEND, "tree_descend": _lib.MERA_OP_TREE_DESCEND,
           "tree_env_w": _lib.MERA_OP_TREE_ENV_W}
    return _lib.mera_flops(ops[op], din, dout, _place(placement))


def mfma_peak(kind: str = "bf16") -> float:
    """Measured matrix-core throughput (TFLOP/s) of the current device for one
    MFMA shape: "bf16" (16x16x32), "fp32" or "fp64" (16x16x4)."""
    k = {"bf16": 0, "fp32": 1, "fp64": 2}[kind]
    scratch = torch.empty(1 << 19, dtype=torch.float32, device="cuda")
    st, tf = _lib.mera_mfma_peak(k, scratch.data_ptr(), scratch.numel() * 4)
    _lib.check(st, "mera_mfma_peak")
    return tf


def contract(spec: str, a: torch.Tensor, b: torch.Tensor, precision="fp64", alpha=1.0, beta=0.0,
             out: torch.Tensor | None = None) -> torch.Tensor:
    """C = alpha * einsum(spec, a, b) + beta * C through the library's contraction engine
    (spec "ab,bc->ac"; one character per leg; no batch legs)."""
    a, b = _dev(a), _dev(b)
    lhs, lc = spec.replace(" ", "").split("->")
    la, lb = lhs.split(",")
    size = {}
    for lab, t in ((la, a), (lb, b)):
        if len(lab) != t.dim():
            raise ValueError(f"{lab!r} does not match a tensor of rank {t.dim()}")
        for ch, n in zip(lab, t.shape):
            if size.setdefault(ch, int(n)) != int(n):
                raise ValueError(f"leg {ch!r} has two sizes")
    labels = "".join(size)
    if out is None:
        out = torch.zeros([size[ch] for ch in lc], dtype=torch.float64, device=a.device)
    na, nb, nc = a.numel(), b.numel(), out.numel()
    need = 8 * (na + nb) + 8 * min(16 * nc, 1 << 24) + 4096
    ws, wsb = WORKSPACE.get(need, a.device)
    _lib.check(_lib.mera_contract(la, a.data_ptr(), lb, b.data_ptr(), lc, out.data_ptr(), labels,
                                  [size[ch] for ch in labels], float(alpha), float(beta), _prec(precision),
                                  ws, wsb, _stream(a.device)), "mera_contract")
    return out
