"""Command-line driver: optimise a scale-invariant binary MERA for the critical Ising chain.

    python -m paper_1906_12030_amd.run --chi 8 --layers 3 --sweeps 500 --precision fp64 \
        [--seed 0] [--iters 30] [--save state.npz] [--resume state.npz] [--grow-from small.npz]
        [--dims 12] [--log run.jsonl] [--compare-precisions fp64,fp32,bf16x3]

Prints one JSON line per reporting interval (energy per site, error against
the exact -4/pi of Sec. III.A, seconds per sweep) and, with --dims k, the k
lowest scaling dimensions of the final scale-invariant layer (Sec. III.A).
Checkpoints hold every tensor, rho*, the sweep index and the settings; a
resumed run continues the same trajectory.  --grow-from pads a converged
smaller-chi state to --chi (zero padding of every leg, seeded N(0, 1e-3)
noise, re-projection onto isometries) as a warm start.  --compare-precisions
recomputes rho*, the energy and (with --dims) the scaling dimensions of the final
tensors with each listed contraction precision and reports the differences from
the first.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import autograd, inputs, ops, scaling, sweep

EXACT = -4.0 / math.pi


def save_state(path, m: sweep.GpuMera, meta: dict, with_rho=True):
    """Tensors (and rho*, unless with_rho is False: it is chi^6 doubles and is recomputed
    by the fixed-point iteration when such a state is resumed) as an .npz file."""
    st = m.state_dict()
    arrays = {"si_u": st["si"][0], "si_w": st["si"][1]}
    if with_rho:
        arrays["rho_star"] = st["rho_star"]
    for t, (u, w) in enumerate(st["layers"]):
        arrays[f"u{t}"] = u
        arrays[f"w{t}"] = w
    np.savez(path, meta=json.dumps(meta), **arrays)


def load_state(path, device="cuda"):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    T = sum(1 for k in z.files if k.startswith("u"))
    layers = [(z[f"u{t}"], z[f"w{t}"]) for t in range(T)]
    rho = z["rho_star"] if "rho_star" in z.files else None
    meta["has_rho"] = rho is not None
    return sweep.GpuMera(layers, (z["si_u"], z["si_w"]), rho, device), meta


def pad_with_noise(small_layers, small_si, chi, n_transitional, seed, noise=1e-3):
    """Warm-start input for a larger bond dimension chi (host; seeded random numbers only):
    every leg of the smaller state's tensors zero-padded to the new dimensions, plus seeded
    N(0, noise^2) entries.  Layers beyond the small state's depth start from its
    scale-invariant tensors.  Returns (layers, si) before the projection onto isometries."""
    rng = np.random.default_rng(seed)
    dims = inputs.bond_dims(chi, n_transitional)
    src = list(small_layers) + [small_si] * (n_transitional - len(small_layers))
    out = []
    for t in range(n_transitional + 1):
        din = dims[t] if t < n_transitional else dims[-1]
        dout = dims[t + 1] if t < n_transitional else dims[-1]
        u0, w0 = src[t] if t < n_transitional else small_si
        u = np.zeros((din,) * 4)
        w = np.zeros((din, din, dout))
        a, b = min(din, u0.shape[0]), min(dout, w0.shape[2])
        u[:a, :a, :a, :a] = u0[:a, :a, :a, :a]
        w[:a, :a, :b] = w0[:a, :a, :b]
        u += noise * rng.standard_normal(u.shape)
        w += noise * rng.standard_normal(w.shape)
        out.append((u, w))
    return out[:-1], out[-1]


def grow(small_layers, small_si, chi, n_transitional, seed, noise=1e-3, device="cuda"):
    """Pad a smaller state to bond dimension chi (pad_with_noise), then replace every tensor
    by the nearest isometry, U V^T of its SVD, with the library's polar update on the GPU."""
    layers, si = pad_with_noise(small_layers, small_si, chi, n_transitional, seed, noise)

    def nearest_isometry(x, rows, cols):
        y = torch.from_numpy(np.ascontiguousarray(x)).to(device)
        out, _, _ = ops.polar_update(-y, rows, cols)  # -polar(-y) = +U V^T of y
        return out.cpu().numpy()

    def proj(u, w):
        din, dout = w.shape[0], w.shape[2]
        return (nearest_isometry(u, din * din, din * din), nearest_isometry(w, din * din, dout))

    return [proj(u, w) for u, w in layers], proj(*si)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--chi", type=int, default=8)
    ap.add_argument("--layers", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--env-precision", default=None, choices=["fp64", "fp32", "bf16x3"],
                    help="contractions of the ascent and the environments (default: --precision)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--si-levels", type=int, default=3,
                    help="scale-invariant layers whose environments update the scale-invariant "
                         "tensors (1 = the first layer only, which stalls near convergence)")
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--save", default=None)
    ap.add_argument("--save-without-rho", action="store_true",
                    help="leave rho* out of the saved state (recomputed on --resume)")
    ap.add_argument("--resume", default=None)
    ap.add_argument("--grow-from", default=None)
    ap.add_argument("--dims", type=int, default=0)
    ap.add_argument("--log", default=None)
    ap.add_argument("--compare-sweeps", type=int, default=0,
                    help="with --compare-precisions: also run this many sweeps from the final state in each "
                         "precision and compare the FP64-evaluated energies (optimisation outcome)")
    ap.add_argument("--compare-precisions", default=None,
                    help="comma list, e.g. fp64,fp32,bf16x3: at the final state, rho* (30 warm-started "
                         "iterations), energy and (with --dims) scaling dimensions in each precision; "
                         "for --compare-sweeps an entry a/b runs the fixed point in a and the "
                         "environments in b")
    ap.add_argument("--compare-riemannian", type=int, default=0,
                    help="instead of optimising: this many SVD-update sweeps and this many Riemannian "
                         "gradient steps (step --lr) from the same seeded state, energy after each")
    ap.add_argument("--lr", type=float, default=0.02)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("a GPU is required")
    if a.compare_riemannian > 0:
        res = compare_riemannian(a.chi, a.layers, a.seed, a.compare_riemannian, a.lr, a.iters)
        for method, es in res.items():
            print(json.dumps({"method": method, "chi": a.chi, "lr": a.lr if method == "riemannian" else None,
                              "energy": es, "rel_error": [(e - EXACT) / abs(EXACT) for e in es]}), flush=True)
        return res
    start = 0
    if a.resume:
        m, meta = load_state(a.resume)
        start = int(meta.get("sweep", 0))
    elif a.grow_from:
        small, _ = load_state(a.grow_from)
        st = small.state_dict()
        layers, si = grow(st["layers"], st["si"], a.chi, a.layers, a.seed)
        m = sweep.GpuMera(layers, si)
    else:
        m = sweep.GpuMera.seeded(a.chi, a.layers, a.seed)
    h1, shift = ops.tfim_hamiltonian(1.0)
    if not a.resume or not meta.get("has_rho", True):
        sweep.initial_fixed_point(m, a.iters, a.precision)
    log = open(a.log, "a") if a.log else None
    t0 = time.perf_counter()
    e = float("nan")
    for k in range(start, start + a.sweeps):
        ek, c = sweep.sweep(m, h1, shift, a.iters, a.precision, a.si_levels, env_precision=a.env_precision)
        if (k + 1) % a.every == 0 or k + 1 == start + a.sweeps:
            e = float(ek.item()) + c
            dt = (time.perf_counter() - t0) / (k + 1 - start)
            rec = {"sweep": k + 1, "energy": e, "rel_error": (e - EXACT) / abs(EXACT), "s_per_sweep": dt,
                   "chi": a.chi, "precision": a.precision,
                   "peak_gb": round(torch.cuda.max_memory_allocated() / 1e9, 2)}
            line = json.dumps(rec)
            print(line, flush=True)
            if log:
                log.write(line + "\n")
                log.flush()
    if a.save:
        save_state(a.save, m, {"sweep": start + a.sweeps, "chi": a.chi, "layers": a.layers,
                               "seed": a.seed, "iters": a.iters, "precision": a.precision},
                   with_rho=not a.save_without_rho)
    if a.dims > 0 and not a.compare_precisions:
        d, lam, calls = scaling.scaling_dimensions(m.si[0], m.si[1], k=a.dims)
        print(json.dumps({"scaling_dimensions": [round(float(x), 6) for x in d], "matvecs": calls}), flush=True)
    if a.compare_precisions:
        compare_precisions(m, h1, shift, a.compare_precisions.split(","), a.iters, a.dims, a.compare_sweeps,
                           a.si_levels)
    return e


def compare_riemannian(chi, n_transitional, seed, nsteps, lr=0.02, iters=30):
    """Energy per step of the SVD update (Sec. II.C, Fig. 5) and of Riemannian gradient
    descent with the autograd environments (appendix, Fig. A1 caption) from the same seeded
    state, FP64.  One SVD step is a sweep; one Riemannian step moves every tensor along its
    projected gradient by lr and retracts with the polar update, then refreshes rho* with
    `iters` power iterations.  Returns {"svd": [...], "riemannian": [...]}."""
    h1, shift = ops.tfim_hamiltonian(1.0)
    out = {}
    for method in ("svd", "riemannian"):
        m = sweep.GpuMera.seeded(chi, n_transitional, seed)
        sweep.initial_fixed_point(m, iters, "fp64")
        es = []
        for _ in range(nsteps):
            if method == "svd":
                e, c = sweep.sweep(m, h1, shift, iters, "fp64")
                es.append(float(e.item()) + c)
            else:
                autograd.riemannian_descent_step(m, h1, lr=lr)
                sweep.initial_fixed_point(m, iters, "fp64")
                es.append(sweep.energy(m, h1, shift))
        out[method] = es
        del m
    return out


def _copy(m):
    return sweep.GpuMera([(u.clone(), w.clone()) for u, w in m.layers], (m.si[0].clone(), m.si[1].clone()),
                         m.rho_star.clone())


def compare_precisions(m, h1, shift, precisions, iters, dims, nsweeps=0, si_levels=1):
    """Energy, rho* and scaling dimensions of the same tensors in several contraction
    precisions; differences against the first one listed.  With nsweeps > 0, also the
    optimisation outcome: nsweeps sweeps (si_levels scale-invariant environment levels)
    from the same state in each precision, the resulting tensors evaluated in FP64 (rho* by
    iters warm-started FP64 iterations, FP64 descent and trace)."""
    if nsweeps > 0:
        eref = None
        for prec in precisions:
            mm = _copy(m)
            fp, _, ep = prec.partition("/")  # "bf16x3/fp64": fixed point in bf16x3, environments in FP64
            for _ in range(nsweeps):
                sweep.sweep(mm, h1, shift, iters, fp, si_levels, env_precision=ep or None)
            sweep.initial_fixed_point(mm, iters, "fp64")
            e = sweep.energy(mm, h1, shift)
            rec = {"precision": prec, "sweeps_from_state": nsweeps, "energy_fp64_eval": e}
            if eref is None:
                eref = e
            else:
                rec["dE"] = abs(e - eref)
            print(json.dumps(rec), flush=True)
            del mm
            torch.cuda.empty_cache()
    ref = None
    for prec in [p for p in precisions if "/" not in p]:
        mm = _copy(m)
        sweep.initial_fixed_point(mm, iters, prec)
        e = sweep.energy(mm, h1, shift)
        d = None
        if dims > 0:
            d, _, _ = scaling.scaling_dimensions(
                mm.si[0], mm.si[1], k=dims, precision=prec,
                progress=lambda n: print(f"# {prec}: {n} ascends", file=sys.stderr, flush=True))
            d = np.asarray(d)
        rec = {"precision": prec, "energy": e}
        if d is not None:
            rec["scaling_dimensions"] = [round(float(x), 9) for x in d]
        if ref is None:
            ref = (e, mm.rho_star.clone(), d)
        else:
            rec["dE"] = abs(e - ref[0])
            rec["rho_rel_err"] = float((mm.rho_star - ref[1]).norm() / ref[1].norm())
            if d is not None:
                rec["max_dDelta"] = float(np.abs(d - ref[2]).max())
        print(json.dumps(rec), flush=True)
        del mm
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main(sys.argv[1:])
