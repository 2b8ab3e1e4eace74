"""Benchmark of the SR-MRA EM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision P]

Workload (default): Lh 64, K 2, Ll 32, N = 100000 observations, sigma = 1,
seeded synthetic smooth image, Dirichlet(1) shift distributions.  A "step" is
one full EM iteration (pack x + score/log-sum-exp pass + combine +
posterior/back-projection pass + FP64 M-step), with the observation stack and
its per-job preparation already resident in HBM.  The main form is timed and
the plain FP32 (vector ALU) form is timed beside it on the same inputs.

Prints ONE JSON line.  Also reports:
 * roofline of the dominant kernel (the posterior/back-projection pass), its
   duration measured with HIP events recorded by the library on the step's
   stream, against the MI355X FP32 matrix peak (157.3 TFLOP/s) or, for the
   vector-ALU form, the non-packed FP32 vector peak (78.6 TFLOP/s);
 * cpu_baseline: the FP64 oracle on a bounded prefix of the observations, timed
   on this host, and the GPU's relative error against it on that prefix.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "EM obs×shift pairs/s vs plain FP32 at rel err ≤1e-4; p50/p99 solve latency"
PEAK = {  # MI355X published dense peaks
    "fp32_mfma": ("mfma", 157.3e12), "fp32_plain": ("alu", 78.6e12),
    "bf16_split3": ("mfma", 2516.6e12),
}
KNAME = {"fp32_mfma": "mfma", "fp32_plain": "valu", "bf16_split3": "bf16"}
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE + WRITE_SIZE for the
# dominant kernel at the default workload (None until counters are taken for
# the current kernel version).
TRAFFIC = {}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lh64_k2_n100000")
    ap.add_argument("--precision", default="fp32_mfma")
    ap.add_argument("--baseline-precision", default="fp32_plain")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="observations in the oracle sample (0 = sized for ~15 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the timed region, run one device-to-device copy of this many MiB "
                         "(reference kernel of known traffic for hardware-counter calibration)")
    return ap.parse_args()


def run_form(inst, precision, steps, warmup):
    """Time `steps` EM iterations of one precision form; returns a dict."""
    import torch
    from paper_2204_04754_amd import binding as B
    from paper_2204_04754_amd.em import EMJob

    job = EMJob(inst.y, inst.K, inst.sigma, inst.x0, inst.log_rho0, precision=precision)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for e in evs:
        e.record()
    torch.cuda.synchronize()

    def one(profile):
        a, b = job.cur, 1 - job.cur
        if profile:
            B.srmra_em_step_profiled(job.y, job.prep, job.N, job.Ll, job.K, job.x[a],
                                     job.log_rho[a], job.sigma, job.x[b], job.rho,
                                     job.log_rho[b], job.loglik, job.precision, job.workspace,
                                     evs)
        else:
            B.srmra_em_step_prepared(job.y, job.prep, job.N, job.Ll, job.K, job.x[a],
                                     job.log_rho[a], job.sigma, job.x[b], job.rho,
                                     job.log_rho[b], job.loglik, job.precision, job.workspace)
        job.cur = b

    for _ in range(warmup):
        one(False)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    phase = np.zeros(5)
    t0.record()
    for _ in range(steps):
        one(True)
    t1.record()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    # events hold the last step's phase boundaries
    for k in range(5):
        phase[k] = evs[k].elapsed_time(evs[k + 1])
    # average per-phase durations over a second profiled sweep, one step at a time
    acc = np.zeros(5)
    n_prof = max(1, min(steps, 5))
    for _ in range(n_prof):
        one(True)
        torch.cuda.synchronize()
        acc += [evs[k].elapsed_time(evs[k + 1]) for k in range(5)]
    phase = acc / n_prof
    ll = float(job.loglik.item())
    return dict(ms_per_step=total_ms / steps, phase_ms=phase.tolist(), loglik=ll, job=job)


def cpu_baseline(inst, n_sample, precision):
    """FP64 oracle on the first n_sample observations; the GPU runs the same
    prefix for the error figure."""
    import torch
    from oracle import em_oracle as O
    from paper_2204_04754_amd import synth
    from tests.gpu_helpers import gpu_step, rel

    ys = inst.y[:n_sample]
    cores = len(os.sched_getaffinity(0))
    t = time.perf_counter()
    ref = O.em_step(ys, inst.x0, inst.log_rho0, inst.sigma, inst.K)
    dt = time.perf_counter() - t
    pairs = n_sample * inst.Lh * inst.Lh
    g = gpu_step(ys, inst.x0, inst.log_rho0, inst.sigma, inst.K, precision, debug=False)
    err = dict(x=rel(g["x_new"], ref["x_new"]), rho=rel(g["rho_new"], ref["rho_new"]),
               loglik=abs(g["loglik"] - ref["loglik"]) / abs(ref["loglik"]))
    threads = os.environ.get("OMP_NUM_THREADS")
    return dict(value=pairs / dt, unit="obs×shift pairs/s", cores=cores, kind="oracle",
                sample=f"first {n_sample} observations of the workload, one EM step "
                       f"({dt:.1f} s, FP64 NumPy, BLAS threads={threads or 'default'})"), err


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2204_04754_amd import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    t = time.perf_counter()
    inst = synth.workload(args.workload)
    print(f"[bench] workload {args.workload} generated in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)

    main_r = run_form(inst, args.precision, args.steps, args.warmup)
    print(f"[bench] {args.precision}: {main_r['ms_per_step']:.2f} ms/step phases "
          f"{np.round(main_r['phase_ms'], 3).tolist()}", file=sys.stderr, flush=True)
    pairs = inst.pairs_per_step
    value = pairs / (main_r["ms_per_step"] * 1e-3)
    forms = {args.precision: dict(pairs_per_s=value, ms_per_step=main_r["ms_per_step"],
                                  phase_ms=main_r["phase_ms"])}
    del main_r["job"]
    if not args.no_plain and args.baseline_precision != args.precision:
        base_steps = max(2, args.steps // 4)
        br = run_form(inst, args.baseline_precision, base_steps, 1)
        del br["job"]
        forms[args.baseline_precision] = dict(
            pairs_per_s=pairs / (br["ms_per_step"] * 1e-3), ms_per_step=br["ms_per_step"],
            phase_ms=br["phase_ms"])
        print(f"[bench] {args.baseline_precision}: {br['ms_per_step']:.2f} ms/step",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    # roofline of the dominant kernel: posterior + back-projection pass (phase 3)
    Ll2 = inst.Ll * inst.Ll
    bound, peak = PEAK[args.precision]
    k_ms = main_r["phase_ms"][3]
    alg_flop = 2.0 * Ll2 * pairs          # back-projection contraction, 2 Ll^2 per pair
    issued_flop = 4.0 * Ll2 * pairs       # + the recomputed score contraction
    achieved = alg_flop / (k_ms * 1e-3)
    roof = {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": TRAFFIC.get((args.workload, args.precision)),
            "kernel": f"k_backproject_{KNAME[args.precision]}<{inst.Ll}>",
            "kernel_ms": k_ms, "issued_frac": issued_flop / (k_ms * 1e-3) / peak,
            "score_pass": {"kernel_ms": main_r["phase_ms"][1],
                           "frac": 2.0 * Ll2 * pairs / (main_r["phase_ms"][1] * 1e-3) / peak}}

    out = {"metric": METRIC, "value": value, "unit": "obs×shift pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": forms[args.precision]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp32_mfma": "f32", "fp32_plain": "f32", "bf16_split3": "bf16x3"}[args.precision],
           "data": "synthetic",
           "config": {"workload": args.workload, "L_high": inst.Lh, "K": inst.K, "L_low": inst.Ll,
                      "N": inst.N, "sigma": inst.sigma, "precision": args.precision,
                      "pairs_per_step": pairs},
           "roofline": roof, "forms": forms}
    if args.baseline_precision in forms and args.baseline_precision != args.precision:
        out["speedup_vs_plain_fp32"] = value / forms[args.baseline_precision]["pairs_per_s"]
    if args.copy_probe > 0:
        nb = args.copy_probe << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nb
        del src, dst
    if not args.no_cpu:
        n = args.cpu_sample or max(64, int(15.0 * 1.0e7 / (inst.Lh * inst.Lh * inst.Ll * inst.Ll / 16)))
        n = min(n, inst.N)
        cb, err = cpu_baseline(inst, n, args.precision)
        out["cpu_baseline"] = cb
        out["rel_err_vs_oracle_on_sample"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
