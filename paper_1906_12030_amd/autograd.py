"""Energy of a MERA as a differentiable function, with environments as the adjoint.

The appendix of the paper notes that the environments of w and u (Fig. A1) can
be obtained by automatic differentiation.  Here the converse is built: a
``torch.autograd.Function`` whose forward is the descending chain plus the
FP64 trace, and whose hand-written backward is made of the environment
kernels (mera_env_u / mera_env_w) and the ascending superoperator.

    e(theta, rho_top) = tr(h_1 D_1(D_2(... D_T(rho_top))))

with D the translation-averaged descending superoperator and no
renormalisation of rho (so e is a polynomial in every tensor and finite
differences off the isometry manifold are well defined).  For real symmetric
h and rho, the derivative with respect to all copies of a tensor in layer t is
twice its environment:

    de/du_t = 2 Env_u(h_t, rho_{t+1}),  de/dw_t = 2 Env_w(h_t, rho_{t+1}),
    h_t = A_{t-1}(... A_1(h_1)),  rho_{t+1} = D_{t+1}(... D_T(rho_top)),
    de/drho_top = h_{T+1}^T.

The forward keeps no intermediate density: the backward recomputes the rho_t
top-down (one descend per layer) and ascends h bottom-up.
"""
from __future__ import annotations

import torch

from . import ops


def _layers(flat):
    return [ops.Layer(flat[2 * i], flat[2 * i + 1]) for i in range(len(flat) // 2)]


class MeraEnergy(torch.autograd.Function):
    """e = tr(h1 rho_1) for layers (u_1, w_1, ..., u_T, w_T) and a top density."""

    @staticmethod
    def forward(ctx, h1, rho_top, precision, *flat):
        layers = _layers(flat)
        rho = rho_top.contiguous()
        for lay in reversed(layers):
            rho = ops.descend(lay, rho, "avg", precision)
        e = ops.energy(h1, rho)
        ctx.precision = precision
        ctx.save_for_backward(h1, rho_top, *flat)
        return e.reshape(())

    @staticmethod
    def backward(ctx, ge):
        h1, rho_top, *flat = ctx.saved_tensors
        prec = ctx.precision
        layers = _layers(flat)
        T = len(layers)
        # recompute rho_{t+1} for t = T..1 (top-down), kept only for this backward
        rhos = [None] * (T + 1)
        rhos[T] = rho_top.contiguous()
        for t in reversed(range(T)):
            if t > 0:
                rhos[t] = ops.descend(layers[t], rhos[t + 1], "avg", prec)
        grads = []
        h = h1.contiguous()
        for t in range(T):
            gu = ops.env_u(layers[t], h, rhos[t + 1], "avg", prec).mul_(2.0)
            gw = ops.env_w(layers[t], h, rhos[t + 1], "avg", prec).mul_(2.0)
            grads += [gu * ge, gw * ge]
            h = ops.ascend(layers[t], h, "avg", prec)
        d = h.shape[0]
        n = d ** 3
        g_rho = h.reshape(n, n).t().contiguous().reshape(h.shape) * ge
        g_h1 = None
        if ctx.needs_input_grad[0]:
            rho1 = rhos[1] if T > 1 else rho_top
            rho1 = ops.descend(layers[0], rho1, "avg", prec)
            g_h1 = rho1.reshape(h1.numel() // int(round(h1.numel() ** 0.5)), -1).t().reshape(h1.shape) * ge
        return (g_h1, g_rho, None, *grads)


def energy(layers, h1, rho_top, precision="fp64"):
    """Differentiable energy; `layers` is [(u, w), ...] of tensors (requires_grad as needed)."""
    flat = [x for pair in layers for x in pair]
    return MeraEnergy.apply(h1, rho_top, precision, *flat)


# ---------------------------------------------------------------------------
# Riemannian gradient steps on the isometry manifolds
# ---------------------------------------------------------------------------
def _as_matrix(x):
    if x.dim() == 4:
        d = x.shape[0]
        return x.reshape(d * d, d * d)
    din, _, dout = x.shape
    return x.reshape(din * din, dout)


def tangent_project(x, g):
    """Project an ambient gradient onto the tangent space of {X : X^T X = I} at x:
    G - X sym(X^T G), with the products on the library's contraction engine (FP64)."""
    xm, gm = _as_matrix(x).contiguous(), _as_matrix(g).contiguous()
    sym = ops.contract("ab,ac->bc", xm, gm, alpha=0.5)                 # (X^T G) / 2
    ops.contract("ab,ac->bc", gm, xm, alpha=0.5, beta=1.0, out=sym)    # + (G^T X) / 2
    out = gm.clone()
    ops.contract("ab,bc->ac", xm, sym, alpha=-1.0, beta=1.0, out=out)  # G - X sym
    return out.reshape(x.shape)


def retract(x, step):
    """Polar retraction: the isometry closest to x + step (computed by mera_polar_update)."""
    y = (x + step).contiguous()
    rows, cols = _as_matrix(y).shape
    # mera_polar_update returns -U V^T of its input: pass -y to obtain +U V^T
    out, _, _ = ops.polar_update(-y, rows, cols)
    return out


def riemannian_descent_step(m, h1, lr=0.05, precision="fp64", si_levels=1):
    """One Riemannian gradient step on every tensor of a GpuMera, then rho* is refreshed.

    Transitional layers use the autograd energy with rho* held fixed; the
    scale-invariant tensors use twice their environment (first SI layer, as in
    the SVD sweep).  Returns the Riemannian gradient norm.
    """
    from . import sweep as _sweep

    pairs = [(u.detach().clone().requires_grad_(True), w.detach().clone().requires_grad_(True))
             for u, w in m.layers]
    e = energy(pairs, h1, m.rho_star, precision)
    e.backward()
    hs = _sweep.ascend_chain(m, h1, precision)
    si = m.si_layer()
    g_su = ops.env_u(si, hs[-1], m.rho_star, "avg", precision).mul_(2.0)
    g_sw = ops.env_w(si, hs[-1], m.rho_star, "avg", precision).mul_(2.0)
    gnorm2 = 0.0
    new_layers = []
    for (u, w) in pairs:
        ru = tangent_project(u.detach(), u.grad)
        rw = tangent_project(w.detach(), w.grad)
        gnorm2 += float((ru * ru).sum() + (rw * rw).sum())
        new_layers.append([retract(u.detach(), -lr * ru), retract(w.detach(), -lr * rw)])
    ru = tangent_project(m.si[0], g_su)
    rw = tangent_project(m.si[1], g_sw)
    gnorm2 += float((ru * ru).sum() + (rw * rw).sum())
    m.si = [retract(m.si[0], -lr * ru), retract(m.si[1], -lr * rw)]
    m.layers = new_layers
    return gnorm2 ** 0.5
