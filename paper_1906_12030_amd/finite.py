"""Finite periodic binary MERA on 16 sites (Fig. 1b) as an optimisation workload, and
the binary tree network (Fig. 1a) as its special case with identity disentanglers.

Two layers (16 -> 8 -> 4 sites) under a 4-site periodic top state.  Each
three-site window of the top ring has its own causal cone below it, so the
layer superoperators, environments and polar updates are exactly those of the
infinite network (`ops`), applied to densities averaged over the windows of a
level.  The sweep follows Sec. II.C with the top state in place of the
scale-invariant layer: ascend h through the layers; replace the top state by
the lowest eigenvector of its energy operator; then, top-down, update u and w
of each layer from their environments and descend the density.

The top state has d^4 amplitudes (d = the top bond dimension, 4 or 8): its
energy operator (a d^4 x d^4 matrix) and its lowest eigenvector are formed on
the host in FP64 (numpy); every contraction of the layers runs in the library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ops

N_SITES = 16


def top_operator(h_top: np.ndarray) -> np.ndarray:
    """d^4 x d^4 matrix H with <t|H|t> = average over s of <t| h_top on (s, s+1, s+2) mod 4 |t>."""
    d = h_top.shape[0]
    hm = h_top.reshape(d ** 3, d ** 3)
    n = d ** 4
    # h on the first three of four sites, as (d^3 x d^3) kron 1_d
    h0 = np.kron(hm, np.eye(d)).reshape((d,) * 8)
    out = np.zeros((n, n))
    for s in range(4):
        # ring rotation: site q of the rotated operator acts on site (q + s) mod 4
        order = [(q - s) % 4 for q in range(4)]
        out += np.transpose(h0, order + [4 + q for q in order]).reshape(n, n)
    return out / 4.0


def top_density(top: np.ndarray) -> np.ndarray:
    """Average over the four three-site windows of the top ring of tr_rest |t><t|."""
    d = top.shape[0]
    acc = np.zeros((d ** 3, d ** 3))
    for s in range(4):
        t = np.transpose(top, [(s + q) % 4 for q in range(4)]).reshape(d ** 3, d)
        acc += t @ t.T
    return (acc / 4.0).reshape((d,) * 6)


class FiniteMera:
    """Two layers [(u, w)] (bottom first, FP64 on the device) and the top state (host)."""

    def __init__(self, layers, top, device="cuda"):
        self.layers = [[torch.as_tensor(np.asarray(u), dtype=torch.float64, device=device).contiguous(),
                        torch.as_tensor(np.asarray(w), dtype=torch.float64, device=device).contiguous()]
                       for u, w in layers]
        self.top = np.array(top, dtype=np.float64)
        self.device = device

    def layer(self, t: int) -> ops.Layer:
        return ops.Layer(self.layers[t][0], self.layers[t][1])

    def top_rho(self) -> torch.Tensor:
        return torch.from_numpy(top_density(self.top)).to(self.device)

    def state_dict(self):
        return {"layers": [(u.cpu().numpy(), w.cpu().numpy()) for u, w in self.layers], "top": self.top.copy()}


def descend_chain(m: FiniteMera, precision="fp64") -> list:
    rhos = [m.top_rho()]
    for t in reversed(range(len(m.layers))):
        rhos.insert(0, ops.descend(m.layer(t), rhos[0], "avg", precision))
    return rhos


def energy(m: FiniteMera, h1: torch.Tensor, shift: float) -> float:
    """Energy per site tr(h1 rho_1) + shift."""
    return float(ops.energy(h1, descend_chain(m)[0]).item()) + shift


def sweep(m: FiniteMera, h1: torch.Tensor, shift: float, precision="fp64", disentangle=True) -> float:
    """One sweep; returns the energy per site after it.  disentangle=False is the binary
    tree network of Fig. 1a: the disentanglers are left out (the layers' u must be the
    identity) and the layers run on the tree calls (mera_tree_*), which contract the
    cone of isometries alone."""
    hs = [h1]
    for t in range(len(m.layers)):
        if disentangle:
            hs.append(ops.ascend(m.layer(t), hs[-1], "avg", precision))
        else:
            hs.append(ops.tree_ascend(m.layers[t][1], hs[-1], "avg", precision))
    vals, vecs = np.linalg.eigh(top_operator(hs[-1].cpu().numpy()))
    d = hs[-1].shape[0]
    m.top = vecs[:, 0].reshape((d,) * 4)
    rho = m.top_rho()
    for t in reversed(range(len(m.layers))):
        if disentangle:
            m.layers[t][0] = ops.update_u(ops.env_u(m.layer(t), hs[t], rho, "avg", precision),
                                          prev=m.layers[t][0])
            m.layers[t][1] = ops.update_w(ops.env_w(m.layer(t), hs[t], rho, "avg", precision),
                                          prev=m.layers[t][1])
            rho = ops.descend(m.layer(t), rho, "avg", "fp64")
        else:
            m.layers[t][1] = ops.update_w(ops.tree_env_w(m.layers[t][1], hs[t], rho, "avg", precision),
                                          prev=m.layers[t][1])
            rho = ops.tree_descend(m.layers[t][1], rho, "avg", "fp64")
    return float(ops.energy(h1, rho).item()) + shift


def exact_energy_per_site(nsite: int = N_SITES) -> float:
    """Critical Ising ring, free-fermion ground energy per site: -2 / (N sin(pi / 2N))."""
    return -2.0 / (nsite * np.sin(np.pi / (2 * nsite)))
