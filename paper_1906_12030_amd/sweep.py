"""Scale-invariant binary MERA optimisation sweep on the GPU (Sec. II.C).

Host-side orchestration only: every contraction, update, fixed-point step and
trace runs in libmera.so through ``ops``.

Sweep order (the paper fixes "scale-invariant layer first, then transitional
layers layer by layer"; the rest is this implementation's reading):
  1. ascend h through the transitional layers with the current tensors;
  2. scale-invariant layer: u <- -polar(Env_u(h_{T+1}, rho*)), then
     w <- -polar(Env_w(h_{T+1}, rho*)) with the new u;
  3. rho* <- ``iters`` power-iteration steps of the scale-invariant D,
     warm-started from the previous rho*;
  4. transitional layers top-down: u then w from (h_t, rho_{t+1}), then
     rho_t = D_t(rho_{t+1}) with the updated tensors;
  5. energy per site tr(h_1 rho_1) + shift.
Contractions run in ``precision``; polar updates, the fixed-point residual and
renormalisation (iterative refinement, see mera_fixed_point_rho), the descent
of rho* through the transitional layers and the energy are FP64 in every mode.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs, ops


class GpuMera:
    """Transitional layers, scale-invariant layer and rho* as device tensors."""

    def __init__(self, layers, si, rho_star=None, device="cuda"):
        self.device = torch.device(device)
        self.layers = [self._pair(u, w) for u, w in layers]
        self.si = self._pair(*si)
        d = self.si[0].shape[0]
        if rho_star is None:
            n = d ** 3
            rho_star = torch.eye(n, dtype=torch.float64, device=self.device).div_(n).reshape((d,) * 6)
        self.rho_star = torch.as_tensor(rho_star, dtype=torch.float64).to(self.device).contiguous()

    def _pair(self, u, w):
        u = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous()
        w = torch.as_tensor(w, dtype=torch.float64).to(self.device).contiguous()
        return [u, w]

    @classmethod
    def seeded(cls, chi: int, n_transitional: int, seed: int, device="cuda"):
        layers, si = inputs.init_mera(chi, n_transitional, seed)
        return cls(layers, si, device=device)

    def layer(self, t: int) -> ops.Layer:
        u, w = self.layers[t]
        return ops.Layer(u, w)

    def si_layer(self) -> ops.Layer:
        return ops.Layer(*self.si)

    def dims(self):
        return [int(u.shape[0]) for u, _ in self.layers] + [int(self.si[0].shape[0])]

    def state_dict(self):
        return {"layers": [(u.cpu().numpy(), w.cpu().numpy()) for u, w in self.layers],
                "si": (self.si[0].cpu().numpy(), self.si[1].cpu().numpy()),
                "rho_star": self.rho_star.cpu().numpy()}


def ascend_chain(m: GpuMera, h1: torch.Tensor, precision="fp64"):
    hs = [h1]
    for t in range(len(m.layers)):
        hs.append(ops.ascend(m.layer(t), hs[-1], "avg", precision))
    return hs


def descend_chain(m: GpuMera):
    """rho_t for every level, descended from rho* in FP64 (the transitional
    descends are a few per cent of a sweep, so every mode keeps them exact)."""
    rhos = [m.rho_star]
    for t in reversed(range(len(m.layers))):
        rhos.append(ops.descend(m.layer(t), rhos[-1], "avg", "fp64"))
    return rhos[::-1]


def energy(m: GpuMera, h1: torch.Tensor, shift: float) -> float:
    """Energy per site of the current state (rho* as stored), FP64 descent and trace."""
    rho1 = descend_chain(m)[0]
    return float(ops.energy(h1, rho1).item()) + shift


def initial_fixed_point(m: GpuMera, iters=30, precision="fp64"):
    ops.fixed_point_rho(m.si_layer(), m.rho_star, iters, precision)


def _si_operators(m: GpuMera, h_top, si_levels, precision):
    hs = [h_top]
    for _ in range(si_levels - 1):
        hs.append(ops.ascend(m.si_layer(), hs[-1], "avg", precision))
    return hs


def sweep(m: GpuMera, h1: torch.Tensor, shift: float, iters=30, precision="fp64", si_levels=1,
          timings: dict | None = None, env_precision: str | None = None):
    """One optimisation sweep; returns the energy per site (device tensor + shift).

    ``precision`` selects the contractions of every step; ``env_precision`` (default:
    the same) overrides it for the ascent of h and the environments, so that e.g. only
    the fixed-point iteration runs in split bf16 while the update directions are FP64."""
    envp = precision if env_precision is None else env_precision
    ev = {}

    def mark(name):
        if timings is not None:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            ev[name] = e

    mark("start")
    hs = ascend_chain(m, h1, envp)
    mark("ascend")
    h_si = _si_operators(m, hs[-1], si_levels, envp)
    si = m.si_layer()
    eu = None
    for hk in h_si:
        e = ops.env_u(si, hk, m.rho_star, "avg", envp)
        eu = e if eu is None else eu.add_(e)
    m.si[0] = ops.update_u(eu, prev=m.si[0])
    si = m.si_layer()
    ew = None
    for hk in h_si:
        e = ops.env_w(si, hk, m.rho_star, "avg", envp)
        ew = e if ew is None else ew.add_(e)
    m.si[1] = ops.update_w(ew, prev=m.si[1])
    mark("si_update")
    ops.fixed_point_rho(m.si_layer(), m.rho_star, iters, precision)
    mark("fixed_point")
    rho = m.rho_star
    for t in reversed(range(len(m.layers))):
        lay = m.layer(t)
        m.layers[t][0] = ops.update_u(ops.env_u(lay, hs[t], rho, "avg", envp), prev=m.layers[t][0])
        lay = m.layer(t)
        m.layers[t][1] = ops.update_w(ops.env_w(lay, hs[t], rho, "avg", envp), prev=m.layers[t][1])
        lay = m.layer(t)
        rho = ops.descend(lay, rho, "avg", "fp64")
    mark("transitional")
    e = ops.energy(h1, rho)
    mark("end")
    if timings is not None:
        torch.cuda.synchronize()
        names = list(ev)
        for a, b in zip(names, names[1:]):
            timings[b] = timings.get(b, 0.0) + ev[a].elapsed_time(ev[b]) / 1e3
    return e, shift


def sweep_flops(dims_in_out, iters=30, si_levels=1) -> dict:
    """Executed contraction flops of one sweep, by phase (from the library's own counter).

    dims_in_out: [(din, dout) for each transitional layer] + [(d, d)] for the SI layer.
    """
    trans, (d, _) = dims_in_out[:-1], dims_in_out[-1]
    f = {"ascend": sum(ops.flops("ascend", a, b) for a, b in trans),
         "si_env": si_levels * (ops.flops("env_u", d, d) + ops.flops("env_w", d, d))
         + (si_levels - 1) * ops.flops("ascend", d, d),
         "fixed_point": iters * ops.flops("fixed_point_iter", d, d),
         "transitional": sum(ops.flops("env_u", a, b) + ops.flops("env_w", a, b) + ops.flops("descend", a, b)
                             for a, b in trans)}
    f["total"] = sum(f.values())
    return f


def layer_dims(m: GpuMera):
    out = [(int(w.shape[0]), int(w.shape[2])) for _, w in m.layers]
    d = int(m.si[1].shape[0])
    return out + [(d, d)]


def optimize(chi: int, n_transitional: int, sweeps: int, seed=0, iters=30, precision="fp64",
             si_levels=3, callback=None, device="cuda"):
    """Seeded initial state, initial fixed point, then `sweeps` sweeps; returns (state, energies)."""
    m = GpuMera.seeded(chi, n_transitional, seed, device)
    h1, shift = ops.tfim_hamiltonian(1.0, device)
    initial_fixed_point(m, iters, precision)
    es = []
    for k in range(sweeps):
        e, c = sweep(m, h1, shift, iters, precision, si_levels)
        es.append(float(e.item()) + c)
        if callback is not None:
            callback(k, es[-1], m)
    return m, np.array(es)
