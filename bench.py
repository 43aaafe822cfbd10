"""Benchmark: scale-invariant binary MERA sweep for the critical Ising chain at chi = 24.

One step = one optimisation sweep (ascend h, scale-invariant u/w updates, 30
power iterations for rho*, transitional-layer updates, energy) on seeded
synthetic tensors, with the contractions in split-bf16 ("mixed") precision and
polar updates, fixed-point renormalisation and energy in FP64.  The same sweep
in plain FP64 is timed beside it for the mixed-vs-FP64 ratio.

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
TRAFFIC_RECORD = {"source_hash": "260e3cf427d6c309", "bytes_per_launch": 30.94e9}


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


def env_rates(recs, code, ops, lib):
    """Environment contraction launches (mera_env_u / mera_env_w) of the timed sweeps."""
    env_ops = (lib.MERA_OP_ENV_U, lib.MERA_OP_ENV_W)
    sel = [r for r in recs if r[4] in env_ops and r[1] == code]
    if not sel:
        return None
    f = sum(r[2] for r in sel)
    ms = sum(r[3] for r in sel)
    tf = f / (ms / 1e3) / 1e12
    return {"launches": len(sel), "flops": f, "launch_ms": round(ms, 3), "tflops": round(tf, 3),
            "frac_of_fp32_mfma_peak": round(tf / PEAK["fp32"], 4)}


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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chi", type=int, default=24)
    ap.add_argument("--layers", type=int, default=3)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--env-precision", default="fp64", choices=["fp32", "bf16x3", "fp64"],
                    help="contractions of the ascent and the environments in the timed sweeps (the "
                         "fixed-point iteration uses --precision)")
    ap.add_argument("--all-reduced-steps", type=int, default=1,
                    help="sweeps timed with every contraction in --precision (environments included)")
    ap.add_argument("--fp32-steps", type=int, default=1,
                    help="sweeps timed with FP32-MFMA contractions (the other reduced-precision form)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + timed sweeps only (for external profilers)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one split-bf16 descend at --chi plus a 1 GiB device copy (for HBM counters)")
    return ap.parse_args()


def cpu_baseline(chi: int, seed: int) -> dict:
    """The FP64 oracle on a bounded sample of the same workload, on the host cores."""
    import numpy as np

    from oracle import mera_oracle as O
    from paper_1906_12030_amd import inputs as I

    rng = np.random.default_rng(seed)
    u, w = I.random_layer(rng, chi, chi)
    g = rng.standard_normal((chi ** 3, 64))
    rho = (g @ g.T)
    rho /= np.trace(rho)
    rho = rho.reshape((chi,) * 6)
    t0 = time.perf_counter()
    flops = 0.0
    O.descend_placement_slice(u, w, rho, "L", 0)
    dt = time.perf_counter() - t0
    # the work of that sample in the GPU schedule's own flop count (1/chi of a left-window descend)
    from paper_1906_12030_amd import ops
    flops = ops.flops("descend", chi, chi, "L") / chi
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(d.get("num_threads", 1)) for d in threadpool_info()) if threadpool_info() else os.cpu_count()
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:  # pragma: no cover
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = ", ".join(f"{d.get('internal_api')} {d.get('version')}" for d in threadpool_info()
                         if d.get("user_api") == "blas") or None
    except Exception:  # pragma: no cover
        blas = None
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "seconds": dt, "nproc": os.cpu_count(), "cpu_model": cpu_model, "blas": blas,
            "sample": f"oracle D_L at chi={chi} with the first fine leg fixed to one value "
                      f"(1/{chi} of a left-window descend, {flops:.3e} flop in the GPU schedule's count)"}


def cpu_thread_scan(chi: int, seed: int) -> list:
    """Oracle throughput on one host thread and on all of them (the same 1/chi slice of
    D_L at a smaller chi, so that the single-thread run stays short)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import mera_oracle as O
    from paper_1906_12030_amd import inputs as I
    from paper_1906_12030_amd import ops

    rng = np.random.default_rng(seed)
    u, w = I.random_layer(rng, chi, chi)
    g = rng.standard_normal((chi ** 3, 64))
    rho = (g @ g.T) / np.trace(g @ g.T)
    rho = rho.reshape((chi,) * 6)
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of this build",
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

    # ---- plain FP64 sweep(s) from the same starting state, for the ratio ----
    t_fp64 = None
    e_fp64 = None
    if args.fp64_steps > 0:
        m64 = sweep.GpuMera(start_state["layers"], start_state["si"], start_state["rho_star"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.fp64_steps):
            e, c = sweep.sweep(m64, h1, shift, args.iters, "fp64")
            if k == 0:
                e_fp64_first = float(e.item()) + shift
        torch.cuda.synchronize()
        t_fp64 = (time.perf_counter() - t0) / args.fp64_steps
        e_fp64 = e_fp64_first
        print(f"# fp64 sweep: {t_fp64:.3f} s/sweep, e = {e_fp64:.12f}", file=sys.stderr, flush=True)
        del m64

    # ---- the FP32-contraction form of the sweep from the same state (time and energy) ----
    t_fp32 = None
    e_fp32 = None
    if args.fp32_steps > 0 and prec != "fp32":
        m32 = sweep.GpuMera(start_state["layers"], start_state["si"], start_state["rho_star"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.fp32_steps):
            e, c = sweep.sweep(m32, h1, shift, args.iters, "fp32")
            if k == 0:
                e_fp32 = float(e.item()) + shift
        torch.cuda.synchronize()
        t_fp32 = (time.perf_counter() - t0) / args.fp32_steps
        print(f"# fp32 sweep: {t_fp32:.3f} s/sweep, e = {e_fp32:.12f}", file=sys.stderr, flush=True)
        del m32

    # ---- every contraction in the benchmark precision (environments included) ----
    t_red = None
    e_red = None
    env = None
    if args.all_reduced_steps > 0 and envp != prec:
        mr = sweep.GpuMera(start_state["layers"], start_state["si"], start_state["rho_star"])
        _lib.mera_profile_begin()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.all_reduced_steps):
            e, c = sweep.sweep(mr, h1, shift, args.iters, prec)
            if k == 0:
                e_red = float(e.item()) + shift
        torch.cuda.synchronize()
        t_red = (time.perf_counter() - t0) / args.all_reduced_steps
        _, recs_red = _lib.mera_profile_end()
        env = env_rates(recs_red, code, ops, _lib)
        print(f"# all contractions {prec}: {t_red:.3f} s/sweep, e = {e_red:.12f}", file=sys.stderr, flush=True)
        del mr
    else:
        env = env_rates(recs, code, ops, _lib)

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

    cpu = None
    scan = None
    if args.cpu_baseline:
        cpu = cpu_baseline(chi, args.seed)
        print(f"# cpu baseline: {cpu}", file=sys.stderr, flush=True)
        scan = cpu_thread_scan(16, args.seed)
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
        "speedup_mixed_vs_fp64": round(t_fp64 / t_mixed, 3) if t_fp64 else None,
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
