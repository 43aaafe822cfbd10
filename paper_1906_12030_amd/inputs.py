"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws random numbers and shapes them into valid inputs.  It
holds none of the method's arithmetic (no superoperator, environment, update or
energy), so the oracle and the GPU path can both take their inputs from here
without sharing any computation.

Conventions (binary MERA, Sec. II.A, Eqs. iso and unitarity):
  * disentangler ``u[a, b, c, d]``: (a, b) are the two lower legs (finer
    lattice), (c, d) the two upper legs; sum_{ab} u[ab,cd] u[ab,c'd'] = delta.
  * isometry ``w[a, b, c]``: (a, b) lower legs, c the upper (coarse) leg;
    sum_{ab} w[ab,c] w[ab,c'] = delta.
  * three-site operators and densities are (d^3 x d^3) matrices stored as
    ``[i1, i2, i3, j1, j2, j3]`` (row = ket legs, column = bra legs).
"""
from __future__ import annotations

import numpy as np


def bond_dims(chi: int, n_transitional: int) -> list[int]:
    """Dimensions d_1 .. d_{T+1} of the levels between transitional layers.

    The physical level holds a spin-1/2 (d_1 = 2); each layer coarse-grains two
    sites into one and keeps at most ``chi`` states: d_{t+1} = min(chi, d_t^2).
    The scale-invariant layer then has all legs of dimension d_{T+1}.
    """
    dims = [2]
    for _ in range(n_transitional):
        dims.append(min(chi, dims[-1] ** 2))
    return dims


def random_isometry_matrix(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Q factor of a QR of an N(0,1) rows x cols matrix, signs fixed by diag(R) > 0."""
    if cols > rows:
        raise ValueError("an isometry needs rows >= cols")
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def random_layer(rng: np.random.Generator, din: int, dout: int) -> tuple[np.ndarray, np.ndarray]:
    """Disentangler then isometry of one layer, drawn in that order."""
    u = random_isometry_matrix(rng, din * din, din * din).reshape(din, din, din, din)
    w = random_isometry_matrix(rng, din * din, dout).reshape(din, din, dout)
    return u, w


def init_mera(chi: int, n_transitional: int, seed: int):
    """Seeded initial tensors: transitional layers 1..T, then the scale-invariant layer.

    Returns ``(layers, si)`` with ``layers[t] = (u, w)`` for t = 0..T-1 and
    ``si = (u_s, w_s)``.  Draw order: for each layer bottom-up, u then w.
    """
    rng = np.random.default_rng(seed)
    dims = bond_dims(chi, n_transitional)
    layers = []
    for t in range(n_transitional):
        layers.append(random_layer(rng, dims[t], dims[t + 1]))
    d = dims[-1]
    si = random_layer(rng, d, d)
    return layers, si


def init_finite(chi: int, seed: int, tree: bool = False):
    """Seeded 16-site network: layers (2 -> d2), (d2 -> d3) with d2 = min(chi, 4),
    d3 = min(chi, d2^2), drawn bottom-up (u then w), then a unit-norm top state of
    shape (d3,)*4 from standard_normal.  tree=True replaces every disentangler by
    the identity u[a,b,c,d] = delta_ac delta_bd (same draws, so the isometries and
    the top state are those of the MERA start)."""
    rng = np.random.default_rng(seed)
    d2 = min(chi, 4)
    d3 = min(chi, d2 * d2)
    layers = [random_layer(rng, 2, d2), random_layer(rng, d2, d3)]
    top = rng.standard_normal((d3,) * 4)
    if tree:
        layers = [(np.eye(u.shape[0] ** 2).reshape(u.shape), w) for u, w in layers]
    return layers, top / np.linalg.norm(top)


def random_density(rng: np.random.Generator, d: int, rank: int = 64) -> np.ndarray:
    """Positive semidefinite unit-trace three-site density: G G^T / tr, G in R^{d^3 x rank}."""
    n = d ** 3
    g = rng.standard_normal((n, min(rank, n) if rank > 0 else n))
    rho = g @ g.T
    rho /= np.trace(rho)
    return rho.reshape((d,) * 6)


def random_symmetric(rng: np.random.Generator, d: int) -> np.ndarray:
    """Real symmetric three-site operator with N(0,1) entries (before symmetrisation)."""
    n = d ** 3
    g = rng.standard_normal((n, n))
    return (0.5 * (g + g.T)).reshape((d,) * 6)


def random_general(rng: np.random.Generator, shape) -> np.ndarray:
    """Plain N(0,1) array of the given shape (environments, polar inputs)."""
    return rng.standard_normal(shape)


def reflection_symmetric_layer(rng: np.random.Generator, d: int):
    """Layer whose tensors are invariant under reversal of the lattice.

    u[a,b,c,d] = u[b,a,d,c] and w[a,b,c] = w[b,a,c]; built from the symmetric /
    antisymmetric two-site subspaces so that both stay isometric.
    """
    n = d * d
    swap = np.zeros((n, n))
    for a in range(d):
        for b in range(d):
            swap[a * d + b, b * d + a] = 1.0
    # orthonormal bases of the +1 and -1 eigenspaces of the swap
    evals, evecs = np.linalg.eigh(swap)
    plus = evecs[:, evals > 0]
    minus = evecs[:, evals < 0]
    # u commutes with swap: block-diagonal random orthogonal in the (+, -) basis
    qp = random_isometry_matrix(rng, plus.shape[1], plus.shape[1])
    qm = random_isometry_matrix(rng, minus.shape[1], minus.shape[1])
    umat = plus @ qp @ plus.T + minus @ qm @ minus.T
    u = umat.reshape(d, d, d, d)
    # w's columns live in the symmetric subspace
    if d > plus.shape[1]:
        raise ValueError("symmetric subspace too small for an isometry")
    qw = random_isometry_matrix(rng, plus.shape[1], d)
    w = (plus @ qw).reshape(d, d, d)
    return u, w
