"""Scaling dimensions from the scale-invariant ascending superoperator (Sec. II.B, Sec. III.A).

The eigenvalues lambda of A (translation-averaged, scale-invariant layer) on
the d^6-dimensional space of three-site operators give Delta = -log2|lambda|.
The Krylov iteration (ARPACK, implicitly restarted Arnoldi) runs on the host;
every matrix-vector product is one mera_ascend call on the GPU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg
import torch

from . import ops


def scaling_dimensions(u: torch.Tensor, w: torch.Tensor, k: int = 12, precision="fp64", tol=1e-10,
                       progress=None):
    """The k eigenvalues of A with largest modulus and Delta = -log2|lambda|, sorted by |lambda|.
    progress (optional) is called with the number of matrix-vector products every 25 of them."""
    layer = ops.Layer(u, w)
    d = layer.din
    if layer.dout != d:
        raise ValueError("the scale-invariant layer has din == dout")
    n = d ** 6
    dev = u.device
    calls = [0]

    def mv(x):
        calls[0] += 1
        if progress is not None and calls[0] % 25 == 0:
            progress(calls[0])
        xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev).reshape((d,) * 6)
        y = ops.ascend(layer, xt, "avg", precision)
        return y.reshape(-1).cpu().numpy()

    op = scipy.sparse.linalg.LinearOperator((n, n), matvec=mv, dtype=np.float64)
    ncv = min(n - 1, max(2 * k + 1, 30))
    v0 = np.ones(n) / np.sqrt(n)  # deterministic start
    lam = scipy.sparse.linalg.eigs(op, k=k, which="LM", ncv=ncv, tol=tol, v0=v0,
                                   return_eigenvectors=False)
    lam = lam[np.argsort(-np.abs(lam))]
    return -np.log2(np.abs(lam)), lam, calls[0]
