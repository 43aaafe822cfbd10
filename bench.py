"""Benchmark: scale-invariant binary MERA sweep for the critical Ising chain at chi = 24.

One step = one optimisation sweep (ascend h, scale-invariant u/w updates, 30
power iterations for rho*, transitional-layer updates, energy) on seeded
synthetic tensors.  In the timed ("mixed") sweeps the fixed-point iteration runs
on split-bf16 contractions in iterative-refinement form (--precision) and the
ascent and environments on FP64 contractions (--env-precision); polar updates,
renormalisation and energy are FP64.  The same sweep in plain FP64 is timed
beside it for the mixed-vs-FP64 ratio, and the forms with FP32 environments,
with every contraction in split bf16 and with FP32 contractions are timed once
each with their energy difference after one sweep.

Prints one JSON line (see the keys below).  Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM traffic per chi^9 split-bf16 launch at chi=24, from the FETCH_SIZE / WRITE_SIZE
# counter runs summarised in profiles/b3_contraction_traffic_chi24.md (copy-calibrated).
# Valid only for the kernel sources it was measured on (hash of csrc/*).
TRAFFIC_RECORD = {"source_hash": "75dc436f58aa05ea", "bytes_per_launch": 28.68e9}


def kernel_source_hash() -> str:
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1906_12030_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


PEAK = {  # MI355X published dense peaks, TFLOP/s
    "fp64": 78.6,
    "fp32": 157.3,
    "bf16": 2516.6,
}


def env_rates(recs, code, ops, lib, precision):
    """Environment contraction launches (mera_env_u / mera_env_w) of the timed sweeps, against
    the roof of their own arithmetic: FP64 / FP32 MFMA peak, or for split bf16 the useful roof
    (bf16 peak / 3) and the bf16 peak itself for the executed products (three per useful one)."""
    env_ops = (lib.MERA_OP_ENV_U, lib.MERA_OP_ENV_W)
    sel = [r for r in recs if r[4] in env_ops and r[1] == code]
    if not sel:
        return None
    f = sum(r[2] for r in sel)
    ms = sum(r[3] for r in sel)
    tf = f / (ms / 1e3) / 1e12
    out = {"precision": precision, "launches": len(sel), "flops": f, "launch_ms": round(ms, 3),
           "tflops": round(tf, 3)}
    if precision == "bf16x3":
        out["frac_of_bf16x3_useful_roof"] = round(tf / (PEAK["bf16"] / 3.0), 4)
        out["frac_of_bf16_mfma_peak_executed"] = round(3.0 * tf / PEAK["bf16"], 4)
    else:
        out[f"frac_of_{precision}_mfma_peak"] = round(tf / PEAK[precision], 4)
    return out


def env_call_rates(m, h1, precision, ops, sweep, lib):
    """One mera_env_u and one mera_env_w call on the scale-invariant layer at the
    current tensors: whole-call time (HIP events on the stream, conversions included)
    and the contraction launches inside, against the FP32 MFMA peak."""
    import torch

    h = sweep.ascend_chain(m, h1, "fp64")[-1]
    si = m.si_layer()
    d = si.din
    torch.cuda.synchronize()
    out = {"precision": precision}
    tot_f, tot_s = 0.0, 0.0
    for name, fn in (("env_u", ops.env_u), ("env_w", ops.env_w)):
        lib.mera_profile_begin()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn(si, h, m.rho_star, "avg", precision)
        b.record()
        torch.cuda.synchronize()
        _, recs = lib.mera_profile_end()
        f = ops.flops(name, d, d)
        s_call = a.elapsed_time(b) / 1e3
        s_launch = sum(r[3] for r in recs) / 1e3
        out[name] = {"flops": f, "call_ms": round(1e3 * s_call, 3), "call_tflops": round(f / s_call / 1e12, 3),
                     "launch_tflops": round(f / s_launch / 1e12, 3)}
        tot_f += f
        tot_s += s_call
    out["call_tflops"] = round(tot_f / tot_s / 1e12, 3)
    out["frac_of_fp32_mfma_peak"] = round(tot_f / tot_s / 1e12 / PEAK["fp32"], 4)
    return out


def layer_update_times(m, h1, ops, sweep):
    """One update of the scale-invariant layer at the current tensors, FP64, split into
    contractions and polar (SVD) updates: the MERA (ascend, Env_u, Env_w, descend; polar of
    u and of w) against the binary tree network (Fig. 1a: ascend, Env_w, descend of the tree
    calls; polar of w).  Sec. III.B compares these shares (rho* about 40 times the u-SVD
    for the MERA at chi = 16, about 3 for a tree)."""
    import torch

    h = sweep.ascend_chain(m, h1, "fp64")[-1]
    si = m.si_layer()
    u, w = m.si
    din = int(w.shape[0])
    torch.cuda.synchronize()

    def timed(fn, reps=3):
        best = None
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            out = fn()
            b.record()
            torch.cuda.synchronize()
            t = a.elapsed_time(b) / 1e3
            best = t if best is None else min(best, t)
        return best, out

    t_asc, _ = timed(lambda: ops.ascend(si, h, "avg", "fp64"))
    t_eu, eu = timed(lambda: ops.env_u(si, h, m.rho_star, "avg", "fp64"))
    t_ew, ew = timed(lambda: ops.env_w(si, h, m.rho_star, "avg", "fp64"))
    t_d, _ = timed(lambda: ops.descend(si, m.rho_star, "avg", "fp64"))
    t_pu, _ = timed(lambda: ops.update_u(eu))
    t_pw, _ = timed(lambda: ops.update_w(ew))
    tt_asc, _ = timed(lambda: ops.tree_ascend(w, h, "avg", "fp64"))
    tt_ew, tew = timed(lambda: ops.tree_env_w(w, h, m.rho_star, "avg", "fp64"))
    tt_d, _ = timed(lambda: ops.tree_descend(w, m.rho_star, "avg", "fp64"))
    tt_pw, _ = timed(lambda: ops.update_w(tew))
    mera_c = t_asc + t_eu + t_ew + t_d
    tree_c = tt_asc + tt_ew + tt_d
    return {"chi": din, "precision": "fp64",
            "mera": {"contractions_s": round(mera_c, 5), "polar_s": round(t_pu + t_pw, 5),
                     "polar_u_s": round(t_pu, 5), "contractions_over_polar": round(mera_c / (t_pu + t_pw), 2)},
            "tree": {"contractions_s": round(tree_c, 5), "polar_s": round(tt_pw, 5),
                     "contractions_over_polar": round(tree_c / tt_pw, 2)},
            "mera_over_tree_contractions": round(mera_c / tree_c, 1)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chi", type=int, default=24)
    ap.add_argument("--layers", type=int, default=3)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="plain FP64 sweeps timed from the same state (their median is the ratio's denominator)")
    ap.add_argument("--env-precision", default="fp64", choices=["fp32", "bf16x3", "fp64"],
                    help="contractions of the ascent and the environments in the timed sweeps (the "
                         "fixed-point iteration uses --precision)")
    ap.add_argument("--all-reduced-steps", type=int, default=1,
                    help="sweeps timed with every contraction in --precision (environments included)")
    ap.add_argument("--fp32-steps", type=int, default=1,
                    help="sweeps timed with FP32-MFMA contractions (the other reduced-precision form)")
    ap.add_argument("--fp32-env-steps", type=int, default=1,
                    help="sweeps timed with the fixed point in --precision and the ascent and environments "
                         "on FP32 MFMA (FP64 kept for polar, renormalisation, transitional descents, energy)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + timed sweeps only (for external profilers)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one split-bf16 descend at --chi plus a 1 GiB device copy (for HBM counters)")
    return ap.parse_args()


def _host_info():
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:  # pragma: no cover
        pass
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        blas = ", ".join(f"{d.get('internal_api')} {d.get('version')}" for d in info
                         if d.get("user_api") == "blas") or None
        threads = max((int(d.get("num_threads", 1)) for d in info), default=os.cpu_count())
    except Exception:  # pragma: no cover
        blas, threads = None, os.cpu_count()
    return cpu_model, blas, threads


def _oracle_inputs(chi, seed):
    import numpy as np

    from paper_1906_12030_amd import inputs as I

    rng = np.random.default_rng(seed)
    u, w = I.random_layer(rng, chi, chi)
    rho = I.random_density(rng, chi)
    h = I.random_symmetric(rng, chi)
    return u, w, rho, h


def cpu_baseline(chi: int, seed: int, dims, iters: int, si_levels: int = 1) -> dict:
    """The FP64 oracle on the host cores: measured on a bounded sample of the workload (one
    1/chi slice of the left-window descend at chi), and its seconds per sweep extrapolated
    from per-call times: a whole descend at chi = 2 chi slices (left and right windows); the
    other calls at chi from their cost relative to the descend, measured on whole calls at
    chi/2 (all AVG); the transitional layers' calls by the ratio of their executed flops to
    the scale-invariant call's (the GPU schedule's own count)."""
    from oracle import mera_oracle as O
    from paper_1906_12030_amd import ops

    u, w, rho, h = _oracle_inputs(chi, seed)
    t0 = time.perf_counter()
    O.descend_placement_slice(u, w, rho, "L", 0)
    t_slice = time.perf_counter() - t0
    del u, w, rho, h
    flops = ops.flops("descend", chi, chi, "L") / chi  # that sample in the GPU schedule's count
    chi0 = chi // 2
    u0, w0, rho0, h0 = _oracle_inputs(chi0, seed)
    calls0 = {}
    for name, fn in (("ascend", lambda: O.ascend(u0, w0, h0)), ("descend", lambda: O.descend(u0, w0, rho0)),
                     ("env_u", lambda: O.env_u(u0, w0, h0, rho0)), ("env_w", lambda: O.env_w(u0, w0, h0, rho0))):
        t0 = time.perf_counter()
        fn()
        calls0[name] = time.perf_counter() - t0
    t_descend = 2 * chi * t_slice
    per_call = {k: t_descend * v / calls0["descend"] for k, v in calls0.items()}  # SI-layer calls at chi

    def call(op, din, dout):
        return per_call[op] * ops.flops(op, din, dout) / ops.flops(op, chi, chi)

    trans = dims[:-1]
    sweep_s = {"ascend": sum(call("ascend", a, b) for a, b in trans),
               "si_update": si_levels * (per_call["env_u"] + per_call["env_w"])
               + (si_levels - 1) * per_call["ascend"],
               "fixed_point": iters * per_call["descend"],
               "transitional": sum(call("env_u", a, b) + call("env_w", a, b) + call("descend", a, b)
                                   for a, b in trans)}
    cpu_model, blas, threads = _host_info()
    return {"value": flops / t_slice / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "seconds": round(t_slice, 3), "nproc": os.cpu_count(), "cpu_model": cpu_model, "blas": blas,
            "sample": f"oracle D_L at chi={chi} with the first fine leg fixed to one value "
                      f"(1/{chi} of a left-window descend, {flops:.3e} flop in the GPU schedule's count)",
            "sweep_s_extrapolated": round(sum(sweep_s.values()), 1),
            "sweep_s_extrapolated_by_phase": {k: round(v, 1) for k, v in sweep_s.items()},
            "per_call_s_extrapolated": {k: round(v, 2) for k, v in per_call.items()},
            "extrapolation": f"descend at chi={chi} = 2 x {chi} slices of {t_slice:.2f} s; ascend, env_u, env_w "
                             f"from their time relative to the descend at chi={chi0} (ascend {calls0['ascend']:.2f} s, "
                             f"descend {calls0['descend']:.2f} s, env_u {calls0['env_u']:.2f} s, env_w "
                             f"{calls0['env_w']:.2f} s); sweep = {iters} descends + the SI environments + the "
                             f"transitional layers scaled by executed flops"}


def cpu_thread_scan(chi: int, seed: int) -> list:
    """Oracle throughput on one host thread and on all of them: the 1/chi slice of D_L at
    the benchmark's chi (Sec. III.B compares thread counts; the paper used 1/16/32/64)."""
    from threadpoolctl import threadpool_limits

    from oracle import mera_oracle as O
    from paper_1906_12030_amd import ops

    u, w, rho, _ = _oracle_inputs(chi, seed)
    flops = ops.flops("descend", chi, chi, "L") / chi
    out = []
    for threads in (1, os.cpu_count()):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            O.descend_placement_slice(u, w, rho, "L", 0)
            dt = time.perf_counter() - t0
        out.append({"threads": threads, "chi": chi, "seconds": round(dt, 3),
                    "TFLOP/s": round(flops / dt / 1e12, 4)})
    return out


def traffic_probe(args):
    """Kernels for the FETCH_SIZE / WRITE_SIZE counter runs: one descend call in the
    benchmark precision (its chi^9 launches are the dominant kernel) and a plain
    copy of a known size (2^27 doubles) that calibrates the counters."""
    import torch

    from paper_1906_12030_amd import inputs, ops

    import numpy as np

    chi = args.chi
    u, w = inputs.random_layer(np.random.default_rng(args.seed), chi, chi)
    lay = ops.Layer(torch.from_numpy(u).cuda(), torch.from_numpy(w).cuda())
    rho = torch.from_numpy(inputs.random_density(np.random.default_rng(args.seed + 1), chi)).cuda()
    out = ops.descend(lay, rho, "avg", args.precision)
    torch.cuda.synchronize()
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_probe": True, "chi": chi, "precision": args.precision,
                      "copy_bytes": 8 << 27, "check": float(out.reshape(-1)[0].item())}))


def evaluation_vs_oracle(args, h1, shift, sweep, prec):
    """Energy of the seeded chi = 24 state (the benchmark's initial tensors) after the power
    iterations the stored oracle value used (from the maximally mixed density; FP64 descent
    and trace), computed by the mixed pipeline (fixed point in `prec` with FP64 refinement) and
    by plain FP64, against the FP64 oracle value of tests/golden/fixed_point_chi24.json
    (written by the oracle alone)."""
    path = os.path.join(ROOT, "tests", "golden", "fixed_point_chi24.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    r = g["recipe"]
    if (r["chi"], r["transitional_layers"], r["seed"]) != (args.chi, args.layers, args.seed):
        return None
    iters = int(r["power_iterations"])
    out = {"oracle_energy": g["energy"], "power_iterations": iters}
    for p in (prec, "fp64"):
        mm = sweep.GpuMera.seeded(args.chi, args.layers, args.seed)
        sweep.initial_fixed_point(mm, iters, p)
        e = sweep.energy(mm, h1, shift)
        out[f"energy_{p}"] = e
        out[f"dE_{p}"] = abs(e - g["energy"])
        del mm
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the sharded multi-GPU path is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1906_12030_amd import _lib, ops, sweep

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.traffic_probe:
        traffic_probe(args)
        return
    chi, T = args.chi, args.layers
    m = sweep.GpuMera.seeded(chi, T, args.seed)
    h1, shift = ops.tfim_hamiltonian(1.0)
    prec = args.precision
    flops = sweep.sweep_flops(sweep.layer_dims(m), args.iters)
    print(f"# chi={chi} T={T} dims={sweep.layer_dims(m)} precision={prec} sweep flops={flops['total']:.3e}",
          file=sys.stderr, flush=True)
    sweep.initial_fixed_point(m, args.iters, prec)
    torch.cuda.synchronize()
    envp = args.env_precision
    for k in range(args.warmup):
        sweep.sweep(m, h1, shift, args.iters, prec, env_precision=envp)
        torch.cuda.synchronize()
        print(f"# warmup sweep {k} done", file=sys.stderr, flush=True)
    start_state = m.state_dict()

    # ---- timed mixed-precision sweeps (per-launch events recorded by the library) ----
    _lib.mera_profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_mixed = None
    e_first = None
    phases = {}
    each = []
    for k in range(args.steps):
        tk = time.perf_counter()
        e, c = sweep.sweep(m, h1, shift, args.iters, prec, timings=phases, env_precision=envp)  # synchronises
        each.append(time.perf_counter() - tk)
        e_mixed = e
        if k == 0:
            e_first = e
    torch.cuda.synchronize()
    e_first = float(e_first.item()) + shift
    t_mixed = (time.perf_counter() - t0) / args.steps
    st, recs = _lib.mera_profile_end()
    e_mixed = float(e_mixed.item()) + shift
    print(f"# mixed sweeps: {t_mixed:.3f} s/sweep, e = {e_mixed:.12f}", file=sys.stderr, flush=True)
    if args.profile_only:
        return

    # dominant kernel: the chi^9 contraction launches (four per descend / ascend call) in the
    # benchmark precision; the FP64 refinement descends inside the mixed fixed point are
    # contraction launches too, but of another kernel and arithmetic
    code = ops.PRECISIONS[prec]
    top = max(x[2] for x in recs if x[1] == code)
    big = [r for r in recs if r[1] == code and r[2] >= 0.5 * top]
    big_f = sum(r[2] for r in big)
    big_ms = sum(r[3] for r in big)
    all_ms = sum(r[3] for r in recs)
    all_f = sum(r[2] for r in recs)

    # per-step totals of the timed sweeps (stderr only)
    steps = {}
    for r in recs:
        e = steps.setdefault((r[0], r[1], r[4]), [0, 0.0, 0.0])
        e[0] += 1
        e[1] += r[3]
        e[2] += r[2]
    print("# top contraction steps over the timed sweeps (labels, arith, op): count, total ms, TFLOP/s",
          file=sys.stderr)
    for (lab, ar, op), (n, ms, f) in sorted(steps.items(), key=lambda kv: -kv[1][1])[:30]:
        print(f"#   {lab:28s} a={ar} op={op} {n:5d} {ms:10.2f} {f / (ms / 1e3) / 1e12:8.1f}", file=sys.stderr)
    sys.stderr.flush()

    def timed_from_start(nsteps, precision, env_precision=None, profile=False):
        """nsteps sweeps from the common starting state: per-sweep seconds, the energy after
        the first sweep, and the profile records when asked for."""
        mm = sweep.GpuMera(start_state["layers"], start_state["si"], start_state["rho_star"])
        if profile:
            _lib.mera_profile_begin()
        torch.cuda.synchronize()
        times, e_one = [], None
        for k in range(nsteps):
            tk = time.perf_counter()
            e, c = sweep.sweep(mm, h1, shift, args.iters, precision, env_precision=env_precision)
            e = float(e.item()) + shift  # synchronises
            times.append(time.perf_counter() - tk)
            if k == 0:
                e_one = e
        recs_ = _lib.mera_profile_end()[1] if profile else None
        del mm
        return times, e_one, recs_

    # ---- plain FP64 sweeps from the same starting state, for the ratio (median) ----
    t_fp64, e_fp64, fp64_each = None, None, []
    if args.fp64_steps > 0:
        fp64_each, e_fp64, _ = timed_from_start(args.fp64_steps, "fp64")
        t_fp64 = float(np.median(fp64_each))
        print(f"# fp64 sweeps: {fp64_each} s, e = {e_fp64:.12f}", file=sys.stderr, flush=True)

    # ---- the FP32-contraction form of the sweep from the same state (time and energy) ----
    t_fp32, e_fp32 = None, None
    if args.fp32_steps > 0 and prec != "fp32":
        ts, e_fp32, _ = timed_from_start(args.fp32_steps, "fp32")
        t_fp32 = float(np.median(ts))
        print(f"# fp32 sweep: {t_fp32:.3f} s/sweep, e = {e_fp32:.12f}", file=sys.stderr, flush=True)

    # ---- fixed point in the benchmark precision, ascent and environments on FP32 MFMA ----
    t_f32env, e_f32env, env_f32_sweep = None, None, None
    if args.fp32_env_steps > 0 and envp != "fp32":
        ts, e_f32env, recs_f = timed_from_start(args.fp32_env_steps, prec, "fp32", profile=True)
        t_f32env = float(np.median(ts))
        env_f32_sweep = env_rates(recs_f, ops.PRECISIONS["fp32"], ops, _lib, "fp32")
        print(f"# fixed point {prec}, environments fp32: {t_f32env:.3f} s/sweep, e = {e_f32env:.12f}",
              file=sys.stderr, flush=True)

    # ---- every contraction in the benchmark precision (environments included) ----
    t_red, e_red, env = None, None, None
    if args.all_reduced_steps > 0 and envp != prec:
        ts, e_red, recs_red = timed_from_start(args.all_reduced_steps, prec, profile=True)
        t_red = float(np.median(ts))
        env = env_rates(recs_red, code, ops, _lib, prec)
        print(f"# all contractions {prec}: {t_red:.3f} s/sweep, e = {e_red:.12f}", file=sys.stderr, flush=True)
    else:
        env = env_rates(recs, code, ops, _lib, prec)

    # ---- evaluation parity at chi = 24 against the FP64 oracle (seeded state) ----
    oracle_eval = evaluation_vs_oracle(args, h1, shift, sweep, prec)
    if oracle_eval is not None:
        print(f"# chi={chi} evaluation vs oracle: {oracle_eval}", file=sys.stderr, flush=True)

    # ---- energy evaluation at the final tensors: mixed pipeline vs FP64 pipeline ----
    def eval_energy(precision):
        mm = sweep.GpuMera([(u.clone(), w.clone()) for u, w in m.layers], (m.si[0].clone(), m.si[1].clone()),
                           m.rho_star.clone())
        sweep.initial_fixed_point(mm, args.iters, precision)
        return sweep.energy(mm, h1, shift)

    e_eval_mixed = eval_energy(prec)
    e_eval_fp64 = eval_energy("fp64")
    # both evaluations: rho* by args.iters steps from the same warm start (the
    # mixed one in FP64 iterative-refinement form), FP64 descent and trace
    print(f"# energy at final tensors: mixed {e_eval_mixed:.15f}  fp64 {e_eval_fp64:.15f}", file=sys.stderr, flush=True)

    env_fp32 = env_call_rates(m, h1, "fp32", ops, sweep, _lib)
    print(f"# environment calls in fp32: {env_fp32}", file=sys.stderr, flush=True)
    layer_times = layer_update_times(m, h1, ops, sweep)
    fp_share = None
    if phases.get("fixed_point"):
        fp_share = round(phases["fixed_point"] / args.steps / layer_times["mera"]["polar_u_s"], 1)
    print(f"# layer update MERA vs tree: {layer_times}; fixed point / u polar {fp_share}", file=sys.stderr,
          flush=True)

    cpu = None
    scan = None
    if args.cpu_baseline:
        cpu = cpu_baseline(chi, args.seed, sweep.layer_dims(m), args.iters)
        print(f"# cpu baseline: {cpu}", file=sys.stderr, flush=True)
        scan = cpu_thread_scan(chi, args.seed)
        print(f"# oracle thread scan: {scan}", file=sys.stderr, flush=True)

    value = flops["total"] / t_mixed / 1e12
    roof_peak = PEAK["bf16"] / 3.0 if prec == "bf16x3" else PEAK[prec]
    # the same roof measured on this card: pure-MFMA loops, no memory traffic
    kind = {"bf16x3": "bf16", "fp32": "fp32", "fp64": "fp64"}[prec]
    peak_measured = ops.mfma_peak(kind) / (3.0 if prec == "bf16x3" else 1.0)
    traffic = None
    if prec == "bf16x3" and chi == 24 and kernel_source_hash() == TRAFFIC_RECORD["source_hash"]:
        traffic = TRAFFIC_RECORD["bytes_per_launch"]
    achieved = big_f / (big_ms / 1e3) / 1e12
    out = {
        "metric": "MERA sweep s & env-contraction TFLOP/s at chi=24, mixed vs FP64, |dE|<=1e-9",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_mixed, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec if envp == prec else f"{prec}/{envp}",
        "data": "synthetic (seeded QR-of-Gaussian MERA tensors, exact TFIM h=1)",
        "config": {"workload": f"scale-invariant binary MERA sweep, critical TFIM, chi={chi}, "
                               f"{T} transitional layers ({'-'.join(str(a) for a, _ in sweep.layer_dims(m)[:-1])}-{chi}) "
                               f"+ SI layer, {args.iters} power iterations, seed {args.seed}; fixed-point "
                               f"contractions {prec} (FP64 refinement), ascent and environments {envp}",
                   "chi": chi, "transitional_layers": T, "power_iterations": args.iters,
                   "fixed_point_precision": prec, "environment_precision": envp},
        "sweep_s_mixed": round(t_mixed, 4),
        "sweep_s_mixed_each": [round(x, 4) for x in each],
        "sweep_s_mixed_median": round(float(np.median(each)), 4),
        "sweep_s_mixed_min": round(min(each), 4),
        "sweep_s_fp64": round(t_fp64, 4) if t_fp64 else None,
        "sweep_s_fp64_each": [round(x, 4) for x in fp64_each],
        "speedup_mixed_vs_fp64": round(t_fp64 / float(np.median(each)), 3) if t_fp64 else None,
        "speedup_note": "median FP64 sweep / median mixed sweep, same starting state",
        "sweep_s_fp32_environments": round(t_f32env, 4) if t_f32env else None,
        "speedup_fp32_environments_vs_fp64": round(t_fp64 / t_f32env, 3) if (t_f32env and t_fp64) else None,
        "dE_one_sweep_fp32_environments_vs_fp64": abs(e_f32env - e_fp64) if (e_f32env is not None and e_fp64 is not None) else None,
        "env_contraction_fp32_in_sweep": env_f32_sweep,
        "evaluation_vs_oracle_chi24": oracle_eval,
        "layer_update_mera_vs_tree": layer_times,
        "fixed_point_over_u_polar": fp_share,
        "sweep_s_all_contractions_reduced": round(t_red, 4) if t_red else None,
        "speedup_all_reduced_vs_fp64": round(t_fp64 / t_red, 3) if (t_red and t_fp64) else None,
        "dE_one_sweep_all_reduced_vs_fp64": abs(e_red - e_fp64) if (e_red is not None and e_fp64 is not None) else None,
        "sweep_s_fp32_contractions": round(t_fp32, 4) if t_fp32 else None,
        "speedup_fp32_vs_fp64": round(t_fp64 / t_fp32, 3) if (t_fp32 and t_fp64) else None,
        "dE_one_sweep_fp32_vs_fp64": abs(e_fp32 - e_fp64) if (e_fp32 is not None and e_fp64 is not None) else None,
        "sweep_flops": flops,
        "sweep_phase_s": {k: round(v / args.steps, 4) for k, v in phases.items()},
        "contraction_tflops_all_launches": round(all_f / (all_ms / 1e3) / 1e12, 3),
        "env_contraction": env,
        "env_contraction_fp32": env_fp32,
        "energy_after_mixed_sweeps": e_mixed,
        "energy_after_one_sweep_mixed": e_first,
        "energy_after_one_sweep_fp64": e_fp64,
        "dE_one_sweep_same_start": abs(e_first - e_fp64) if e_fp64 is not None else None,
        "energy_eval_final_tensors_mixed": e_eval_mixed,
        "energy_eval_final_tensors_fp64": e_eval_fp64,
        "dE_eval": abs(e_eval_mixed - e_eval_fp64),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": round(roof_peak, 1),
                     "unit": "TFLOP/s", "frac": round(achieved / roof_peak, 4), "traffic": traffic,
                     "peak_measured": round(peak_measured, 1), "frac_of_measured": round(achieved / peak_measured, 4),
                     "traffic_unit": "bytes per launch (HBM, copy-calibrated FETCH_SIZE + WRITE_SIZE)",
                     "kernel": f"chi^9 contraction launches ({prec}), {len(big)} launches, "
                               f"{big_f / len(big):.3e} flop each, avg {big_ms / len(big):.3f} ms",
                     "note": "split-bf16 peak = bf16 dense MFMA peak / 3 (three bf16 products per useful multiply-add)"
                     if prec == "bf16x3" else ""},
        "cpu_baseline": cpu,
        "oracle_thread_scan": scan,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
