"""Benchmark of the SR-MRA EM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision P]

Workload (default): the precision study, Lh 128, K 4, Ll 32, N = 200000
observations, sigma 0.5, seeded synthetic smooth image, Dirichlet(1) shift
distributions; main form the BF16 split with three products.  A "step" is
one full EM iteration (pack x + score/log-sum-exp pass + combine +
posterior/back-projection pass + FP64 M-step), with the observation stack and
its per-job preparation already resident in HBM.  Plain FP32 (vector ALU),
FP32 MFMA, the FFT route and the 4-product split are timed beside it on the
same inputs, and the single-instance workload (Lh 64, K 2, N 100000, FP32
MFMA, one pass) is reported as a secondary line.

Prints ONE JSON line.  Also reports:
 * roofline of the dominant kernel (the single pass, or for two-pass shapes
   the posterior/back-projection pass) and of the score pass, their
   durations measured with HIP events recorded by the library on the step's
   stream, against the MI355X peak of the form's arithmetic (BF16 dense
   2516.6 TFLOP/s, FP32 matrix 157.3 TFLOP/s, or the non-packed FP32 vector
   rate 78.6 TFLOP/s): algorithmic work (4 Ll^2 flop per observation x shift
   pair) and issued work (with the score recompute and the split's products);
 * cpu_baseline: the FP64 oracle on the first 2000 observations, timed on
   this host, and every GPU form's relative error against it on that subset;
 * batched and serving: the 64-instance mix in the batched form (main
   precision, every class on the FFT route, FP32 MFMA, plain FP32) and a short
   Poisson serving run (60 jobs at 50 jobs/s), compact (--no-mix skips them;
   --mode batched / serve run the full sweeps).
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
    "bf16_split3": ("mfma", 2516.6e12), "bf16_split4": ("mfma", 2516.6e12),
    "fp32_fft": ("alu", 78.6e12),
}
KNAME = {"fp32_mfma": "mfma", "fp32_plain": "valu", "bf16_split3": "bf16", "bf16_split4": "bf16",
         "fp32_fft": "fft"}
PRODUCTS = {"bf16_split3": 3, "bf16_split4": 4}   # BF16 products per multiply-add
DTYPE = {"fp32_mfma": "f32", "fp32_plain": "f32", "bf16_split3": "bf16x3", "bf16_split4": "bf16x4",
         "fp32_fft": "f32"}
HBM_PEAK = 8.0e12   # B/s
# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE (x 2.0)
# and WRITE_SIZE (x 1.0), keyed by (workload, precision, kernel), with a hash of
# the kernel's sources at the time the counters were taken: a changed kernel
# reports null until its counters are taken again.
_MFMA_SRC = ("srmra_common.h", "srmra_mfma_impl.h", "srmra_mfma.hip")
_BF16_SRC = ("srmra_common.h", "srmra_bf16_impl.h", "srmra_bf16.hip")
_BF16W_SRC = ("srmra_common.h", "srmra_bf16_impl.h", "srmra_bf16w_impl.h", "srmra_bf16.hip")
TRAFFIC = {
    ("lh64_k2_n100000", "fp32_mfma", "k_fused_mfma<32>"):
        dict(bytes=428054630, src=_MFMA_SRC, sha="5fe9b8ec41a003f1"),
    ("lh128_k4_n200000_s0.5", "bf16_split3", "k_fused16_bf16<32, 3>"):
        dict(bytes=15727274189, src=_BF16_SRC, sha="74937274c8f678c3"),
    ("lh256_k4_n20000", "bf16_split3", "b16w::k_backproject<64, 3>"):
        dict(bytes=7369647616, src=_BF16W_SRC, sha="f7205148b449a689"),
}


def traffic_bytes(key):
    import hashlib
    e = TRAFFIC.get(key)
    if e is None:
        return None
    m = hashlib.sha256()
    for f in e["src"]:
        with open(os.path.join(ROOT, "paper_2204_04754_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return e["bytes"] if m.hexdigest()[:16] == e["sha"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lh128_k4_n200000_s0.5")
    ap.add_argument("--precision", default="bf16_split3")
    ap.add_argument("--baseline-precision", default="fp32_plain")
    ap.add_argument("--cpu-sample", type=int, default=2000,
                    help="observations in the oracle sample (0 = sized for --cpu-seconds)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target oracle time on the host for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--extra-forms", default="fp32_mfma,fp32_fft,bf16_split4",
                    help="comma-separated forms also timed beside the main one (single mode)")
    ap.add_argument("--secondary-workload", default="lh64_k2_n100000",
                    help="single mode: a second workload timed in --secondary-precision ('' = none)")
    ap.add_argument("--secondary-precision", default="fp32_mfma")
    ap.add_argument("--mode", default="single",
                    choices=["single", "batched", "serve", "errors", "projected", "moments"],
                    help="single: one instance (default); batched: 64-instance mix, 20 iterations "
                         "captured as a HIP graph; serve: Poisson job arrivals, continuous batching")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--outer", type=int, default=4, help="projected mode: outer iterations in the graph")
    ap.add_argument("--error-obs", type=int, default=2000,
                    help="errors mode: observations in the subset the oracle runs on")
    ap.add_argument("--no-tune", action="store_true", help="batched mode: skip the autotuned runs")
    ap.add_argument("--per-class", action="store_true",
                    help="batched mode: also time each (L_low, K) class of the mix alone, in the main form")
    ap.add_argument("--iterations", type=int, default=20)
    ap.add_argument("--rates", default="5,50,200")
    ap.add_argument("--jobs", type=int, default=200,
                    help="serve mode: jobs per arrival rate for the BF16 forms")
    ap.add_argument("--jobs-fp32", type=int, default=24,
                    help="serve mode: jobs per arrival rate for the FP32 forms (about 10x slower)")
    ap.add_argument("--budget-gb", type=float, default=4.0,
                    help="serve mode: HBM budget of the extra footprint-admission point (0: none)")
    ap.add_argument("--serve-precisions", default="",
                    help="serve mode: comma-separated forms (default: --precision, fp32_mfma, "
                         "fp32_plain); '<form>+fft' runs jobs at an L_low the FFT route supports "
                         "through it and the rest in <form>")
    ap.add_argument("--no-mix", action="store_true",
                    help="single mode: skip the compact batched-mix and serving summaries")
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

    # a0: the per-job preparation, re-run on the resident stack (HBM-bound; its
    # algorithmic bytes are one read of y plus the prepared buffer written)
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    prep_ms = []
    for _ in range(3):
        pe[0].record()
        B.srmra_prepare_observations(job.y, job.N, job.Ll, job.K, job.precision, job.prep)
        pe[1].record()
        torch.cuda.synchronize()
        prep_ms.append(pe[0].elapsed_time(pe[1]))
    # two reads of y (the offset mu, then the centred norms / planes) + the buffer written
    prep_bytes = 8.0 * job.N * job.Ll * job.Ll + B.srmra_prepared_bytes(job.N, job.Ll, job.K, job.precision)
    prep = dict(ms=min(prep_ms), bytes=prep_bytes, gb_per_s=prep_bytes / (min(prep_ms) * 1e-3) / 1e9,
                hbm_frac=prep_bytes / (min(prep_ms) * 1e-3) / HBM_PEAK)
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
    return dict(ms_per_step=total_ms / steps, phase_ms=phase.tolist(), loglik=ll, job=job, prep=prep)


def oracle_sample_size(inst, seconds):
    """Observations the oracle gets through in about `seconds` on this host,
    from an untimed calibration step on the first 64 observations."""
    from oracle import em_oracle as O
    n0 = min(64, inst.N)
    t = time.perf_counter()
    O.em_step(inst.y[:n0], inst.x0, inst.log_rho0, inst.sigma, inst.K)
    per_obs = (time.perf_counter() - t) / n0
    return max(n0, int(seconds / max(per_obs, 1e-9)))


def cpu_baseline(inst, n_sample, forms):
    """FP64 oracle on the first n_sample observations, timed on this host; every
    GPU form runs the same subset for its error figure (x', rho' norm-wise,
    loglik relative), flagged against the 1e-4 target."""
    from oracle import em_oracle as O
    from tests.gpu_helpers import gpu_step, rel

    ys = np.ascontiguousarray(inst.y[:n_sample])
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
                   or [1])
    except Exception:   # threadpoolctl missing: report the environment's setting
        blas = int(os.environ.get("OMP_NUM_THREADS", "1"))
    t = time.perf_counter()
    ref = O.em_step(ys, inst.x0, inst.log_rho0, inst.sigma, inst.K)
    dt = time.perf_counter() - t
    pairs = n_sample * inst.Lh * inst.Lh
    errs = {}
    for prec in forms:
        g = gpu_step(ys, inst.x0, inst.log_rho0, inst.sigma, inst.K, prec, debug=False)
        e = dict(x=rel(g["x_new"], ref["x_new"]), rho=rel(g["rho_new"], ref["rho_new"]),
                 loglik=abs(g["loglik"] - ref["loglik"]) / abs(ref["loglik"]))
        e["within_1e-4"] = bool(e["x"] <= 1e-4 and e["rho"] <= 1e-4)
        errs[prec] = e
    return dict(value=pairs / dt, unit="obs×shift pairs/s", cores=blas, kind="oracle",
                sample=f"first {n_sample} observations of the workload, one EM step from its seeded "
                       f"start ({dt:.1f} s; FP64 NumPy: the loop over shifts in one thread, the "
                       f"M-step products on {blas} BLAS threads; {cores} host cores visible)"), errs


def roofline(inst, precision, phase_ms, workload):
    """Roofline of the dominant kernel (phase 3: the single pass, else the
    posterior / back-projection pass) and, for two passes, of the score pass
    (phase 1).  Algorithmic work: 2 Ll^2 flop per pair for the score and as
    much for the back-projection; issued work adds the pass-2 recompute of the
    scores and the split's products per multiply-add."""
    import math
    from paper_2204_04754_amd import binding as B
    pairs = inst.pairs_per_step
    Ll2 = inst.Ll * inst.Ll
    bound, peak = PEAK[precision]
    n_pass = B.srmra_em_step_passes(inst.N, inst.Ll, inst.K, precision)
    prod = float(PRODUCTS.get(precision, 1))
    targ = f"<{inst.Ll}, {PRODUCTS[precision]}>" if precision in PRODUCTS else f"<{inst.Ll}>"
    k_ms = phase_ms[3]
    s_name = None
    if precision == "fp32_fft":
        # pass 2: an inverse and a forward complex 2-D FFT of Ll^2 points per
        # (observation, component) pair, 5 n log2 n flop each
        kname = f"k_fft_pass2<{inst.Ll}>"
        alg_flop = inst.N * inst.K * inst.K * 2 * 5.0 * Ll2 * math.log2(Ll2)
        issued_flop = alg_flop
    elif n_pass == 1:
        # the BF16 split's single pass at 4 < K^2 <= 16 is its own kernel
        wide = precision in PRODUCTS and inst.K * inst.K > 4
        kname = f"k_fused{'16' if wide else ''}_{KNAME[precision]}{targ}"
        alg_flop = 4.0 * Ll2 * pairs
        issued_flop = alg_flop * prod
    elif precision in PRODUCTS and inst.Ll >= 48:   # BF16 split with 2 x 2 tiles
        kname = f"b16w::k_backproject{targ}"
        s_name = f"b16w::k_score_lse{targ}"
        alg_flop = 2.0 * Ll2 * pairs
        issued_flop = 4.0 * Ll2 * pairs * prod
    else:
        kname = f"k_backproject_{KNAME[precision]}{targ}"
        s_name = f"k_score_lse_{KNAME[precision]}{targ}"
        alg_flop = 2.0 * Ll2 * pairs
        issued_flop = 4.0 * Ll2 * pairs * prod
    traffic = traffic_bytes((workload, precision, kname))
    roof = {"bound": bound, "achieved": alg_flop / (k_ms * 1e-3) / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": alg_flop / (k_ms * 1e-3) / peak, "traffic": traffic,
            # the same kernel against the HBM roofline (counter bytes / duration / 8 TB/s)
            "hbm_frac": None if traffic is None else traffic / (k_ms * 1e-3) / HBM_PEAK,
            "kernel": kname, "kernel_ms": k_ms, "passes": n_pass,
            "issued_frac": issued_flop / (k_ms * 1e-3) / peak}
    if n_pass == 2:
        s_ms = phase_ms[1]
        if precision == "fp32_fft":   # one inverse complex FFT per (observation, component)
            s_flop = inst.N * inst.K * inst.K * 5.0 * Ll2 * math.log2(Ll2)
            s_issued = s_flop
            s_name = f"k_fft_pass1<{inst.Ll}>"
        else:
            s_flop = 2.0 * Ll2 * pairs
            s_issued = s_flop * prod
        st = traffic_bytes((workload, precision, s_name)) if s_name else None
        roof["score_pass"] = {"kernel": s_name, "kernel_ms": s_ms,
                              "achieved": s_flop / (s_ms * 1e-3) / 1e12,
                              "frac": s_flop / (s_ms * 1e-3) / peak,
                              "issued_frac": s_issued / (s_ms * 1e-3) / peak, "traffic": st,
                              "hbm_frac": None if st is None else st / (s_ms * 1e-3) / HBM_PEAK}
    return roof


def bench_batched(args):
    """64 instances of the uneven mix (Lh in {32,48,64,96}, K in {2,3,4}, N in
    [5000, 50000], sigma in [0.3, 2]) advanced together; `iterations` EM steps
    captured as one HIP graph and replayed."""
    import torch
    from paper_2204_04754_amd import synth
    from paper_2204_04754_amd.batch import BatchedEM

    t = time.perf_counter()
    mix = synth.mixed_batch(args.instances)
    ins = []
    for d in mix:
        inst = synth.make_instance(**d)
        ins.append(dict(y=inst.y, K=inst.K, sigma=inst.sigma, x0=inst.x0, log_rho0=inst.log_rho0))
    print(f"[bench] {len(ins)} instances generated in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    forms = {}
    tuning = {}
    # each form with the library's default partition; the main form with every
    # class on the FFT route (a table sending each (L_low, K) there); then the
    # main form and FP32 MFMA with the autotuner's table, the main form also
    # with the FFT route among the tuner's candidates (tuned on this batch;
    # tuning time reported apart from the timed graph replays)
    from paper_2204_04754_amd import binding as B
    fft_table = [dict(precision=B._prec(args.precision), L_low=ll, K=k, form=B.SRMRA_FP32_FFT, item_obs=0)
                 for (ll, k) in sorted({(d["Lh"] // d["K"], d["K"]) for d in mix})]
    runs = [(args.precision, args.iterations, None, False), ("fp32_mfma", args.iterations, None, False),
            ("fp32_plain", 2, None, False), (args.precision, args.iterations, fft_table, False)]
    if not args.no_tune:
        runs += [(args.precision, args.iterations, "auto", False), ("fp32_mfma", args.iterations, "auto", False),
                 (args.precision, args.iterations, "auto", True)]
    for prec, iters, tune, fft in runs:
        key = prec + ("+fft_all" if isinstance(tune, list) else "") + ("+tuned" if tune == "auto" else "") + \
            ("+fft" if fft else "")
        if key in forms:
            continue
        be = BatchedEM(ins, precision=prec, tuning=tune, fft=fft)
        pairs = be.pairs_per_step
        g = be.capture(iters)
        g.replay()                                   # warm-up replay
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / iters
        forms[key] = dict(pairs_per_s=pairs / (ms * 1e-3), ms_per_step=ms, iterations_in_graph=iters)
        if tune == "auto":
            forms[key]["tune_seconds"] = be.tune_seconds
            tuning[key] = [dict(L_low=t["L_low"], K=t["K"], form=t["form"], item_obs=t["item_obs"], tile=t.get("tile", 0))
                           for t in be.tuning]
        print(f"[bench] batched {key}: {ms:.2f} ms/step", file=sys.stderr, flush=True)
        del g, be
        torch.cuda.empty_cache()
    # each (L_low, K) class alone, in its own plan (the mix runs them concurrently)
    classes = []
    if args.per_class:
        groups = {}
        for d, e in zip(mix, ins):
            groups.setdefault((d["Lh"] // d["K"], d["K"]), []).append((d, e))
        def time_class(members, tuning):
            be = BatchedEM(members, precision=args.precision, tuning=tuning)
            g = be.capture(2)
            g.replay()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            ms, pairs = e0.elapsed_time(e1) / 2, be.pairs_per_step
            del g, be
            torch.cuda.empty_cache()
            return ms, pairs

        for (ll, k) in sorted(groups):
            members = [e for _, e in groups[(ll, k)]]
            ms, pairs = time_class(members, None)
            ms_fft, _ = time_class(members, [t for t in fft_table if (t["L_low"], t["K"]) == (ll, k)])
            # the class's algorithmic work (4 L_low^2 flop per pair) at the form's peak, issued
            # with its products per multiply-add (3 or 4 for the BF16 split)
            ideal = pairs * 4 * ll * ll * PRODUCTS.get(args.precision, 1) / PEAK[args.precision][1] * 1e3
            classes.append(dict(L_low=ll, K=k, instances=len(members), pairs=pairs, ms_per_step=ms,
                                ideal_ms=ideal, frac=ideal / ms, fft_ms_per_step=ms_fft))
            print(f"[bench] class L_low {ll} K {k}: {len(members)} instances, {ms:.2f} ms/step, "
                  f"{100 * ideal / ms:.0f}% of its peak-rate time {ideal:.2f} ms; FFT route {ms_fft:.2f} ms/step",
                  file=sys.stderr, flush=True)
    # the headline batched figure is the main form at its best table
    best = min((k for k in forms if k.split("+")[0] == args.precision), key=lambda k: forms[k]["ms_per_step"])
    main_p = args.precision
    out = {"metric": METRIC, "value": forms[best]["pairs_per_s"], "unit": "obs×shift pairs/s",
           "n_gpus": 1, "steps": args.iterations, "warmup": args.iterations,
           "ms_per_step": forms[best]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           # classes the table sends to the FFT route compute in FP32
           "dtype": DTYPE[main_p] + ("+f32" if "fft" in best else ""), "data": "synthetic",
           "config": {"workload": f"batched_mix_{args.instances}", "instances": args.instances,
                      "pairs_per_step": sum(d['N'] * d['Lh'] ** 2 for d in mix),
                      "precision": main_p, "table": best[len(main_p) + 1:] or "default",
                      "graph_iterations": args.iterations},
           "forms": forms, "tuning": tuning, "classes": classes,
           "speedup_vs_plain_fp32": forms[best]["pairs_per_s"] / forms["fp32_plain"]["pairs_per_s"]}
    print(json.dumps(out), flush=True)


def _time_batched(ins, precision, tuning, iters):
    """ms per step of one plan over the instances (`iters` EM steps captured as
    one HIP graph, one warm-up replay, one timed replay) and its pairs per step."""
    import torch
    from paper_2204_04754_amd.batch import BatchedEM
    be = BatchedEM(ins, precision=precision, tuning=tuning)
    pairs = be.pairs_per_step
    g = be.capture(iters)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    del g, be
    torch.cuda.empty_cache()
    return ms, pairs


def mix_summary(precision: str) -> dict:
    """The batched form on the 64-instance mix, compact (the default run's
    record of it): the main precision with the library's default table and
    with every class on the FFT route (a fixed table, no tuning), FP32 MFMA
    and plain FP32 with fewer iterations per graph."""
    from paper_2204_04754_amd import binding as B
    from paper_2204_04754_amd import synth
    t = time.perf_counter()
    mix = synth.mixed_batch(64)
    ins = []
    for d in mix:
        inst = synth.make_instance(**d)
        ins.append(dict(y=inst.y, K=inst.K, sigma=inst.sigma, x0=inst.x0, log_rho0=inst.log_rho0))
    fft_table = [dict(precision=B._prec(precision), L_low=ll, K=k, form=B.SRMRA_FP32_FFT, item_obs=0)
                 for (ll, k) in sorted({(d["Lh"] // d["K"], d["K"]) for d in mix})]
    tables = {}
    for key, prec, tab, iters in ((precision, precision, None, 20),
                                  (precision + "+fft_all", precision, fft_table, 20),
                                  ("fp32_mfma", "fp32_mfma", None, 2), ("fp32_plain", "fp32_plain", None, 2)):
        ms, pairs = _time_batched(ins, prec, tab, iters)
        tables[key] = dict(ms_per_step=ms, pairs_per_s=pairs / (ms * 1e-3), iterations_in_graph=iters)
    plain = tables["fp32_plain"]["pairs_per_s"]
    for v in tables.values():
        v["speedup_vs_plain_fp32"] = v["pairs_per_s"] / plain
    out = {"workload": "batched_mix_64", "instances": 64, "pairs_per_step": pairs, "tables": tables,
           "seconds": time.perf_counter() - t}
    print(f"[bench] batched mix: " + ", ".join(f"{k} {v['ms_per_step']:.1f} ms/step" for k, v in tables.items()),
          file=sys.stderr, flush=True)
    return out


def serve_summary(precision: str, rate: float = 50.0, jobs: int = 60, iterations: int = 20) -> dict:
    """A short serving run (Poisson arrivals at `rate` jobs/s of `jobs`
    20-iteration jobs from the serving pool), the main precision with the FFT
    route inside the plan and alone: solves/s and p50 / p99 latency."""
    import torch
    from paper_2204_04754_amd import synth
    from paper_2204_04754_amd.serve import GPUExecutor, Job, serve
    t = time.perf_counter()
    pool_shapes = synth.mixed_batch(11, config=4) + [dict(Lh=256, K=4, N=20000, sigma=1.0,
                                                            config=4, instance=999)]
    pool = [synth.make_instance(**d) for d in pool_shapes]
    r = np.random.default_rng(int(rate * 1000) + 7)
    arr = np.cumsum(r.exponential(1.0 / rate, size=jobs))
    pick = [11 if r.random() < 0.1 else int(r.integers(0, 11)) for _ in range(jobs)]
    res = {}
    for key, fft in ((precision + "+fftplan", "plan"), (precision, False)):
        js = [Job(k, pool[pick[k]].y, pool[pick[k]].K, pool[pick[k]].sigma, pool[pick[k]].x0,
                  pool[pick[k]].log_rho0, iterations=iterations, arrival=float(arr[k])) for k in range(jobs)]
        ex = GPUExecutor(precision=precision, fft=fft)
        summ = serve(js, ex, hbm_budget=200 << 30, max_slots=64).summary()
        res[key] = {k: summ[k] for k in ("jobs", "done", "failed", "solves_per_s", "p50_latency_s",
                                         "p99_latency_s")}
        del ex
        torch.cuda.empty_cache()
    out = {"workload": "serve_poisson_mix", "rate_jobs_per_s": rate, "jobs": jobs,
           "iterations_per_job": iterations, "results": res, "seconds": time.perf_counter() - t}
    print(f"[bench] serving at {rate:g} jobs/s: " + ", ".join(
        f"{k} {v['solves_per_s']:.1f} solves/s p50 {v['p50_latency_s']:.2f} s p99 {v['p99_latency_s']:.2f} s"
        for k, v in res.items()), file=sys.stderr, flush=True)
    return out


def bench_projected(args):
    """Projected EM (Alg. 2): F = 5 EM steps then the Gaussian-smoothing
    projection and the noise-level decay, `outer` outer iterations captured as
    one HIP graph; throughput over the EM steps with the projections inside
    the timed region, and the projection's own time."""
    import torch
    from paper_2204_04754_amd import binding as B
    from paper_2204_04754_amd import synth
    from paper_2204_04754_amd.projected import ProjectedEM

    inst = synth.workload(args.workload)
    F, T = 5, args.outer
    pe = ProjectedEM(inst.y, inst.K, inst.sigma, inst.x0, inst.log_rho0, precision=args.precision, F=F)
    g = pe.capture(T)
    g.replay()                                        # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_outer = e0.elapsed_time(e1) / T
    # the projection alone (50 calls on the current iterate's copy)
    x = pe.x.clone()
    st = torch.ones(1, dtype=torch.float32, device="cuda")
    e0.record()
    for _ in range(50):
        B.srmra_project_gaussian(x, x, inst.Lh, st, 1.0, pe.pws)
    e1.record()
    torch.cuda.synchronize()
    ms_proj = e0.elapsed_time(e1) / 50
    ms_step = ms_outer / F
    # reconstruction quality (the paper's shift-invariant error against the
    # true image) after the 2 T outer iterations run so far, beside plain EM
    # for the same number of steps from the same start
    from paper_2204_04754_amd.em import EMJob
    ws_e = B.empty_bytes(B.srmra_shift_error_workspace_bytes(inst.Lh))
    err = torch.empty(1, dtype=torch.float64, device="cuda")
    xt = torch.as_tensor(inst.x_true).cuda()
    B.srmra_shift_error(pe.x, xt, inst.Lh, err, None, ws_e)
    err_proj = float(err.item())
    plain = EMJob(inst.y, inst.K, inst.sigma, inst.x0, inst.log_rho0, precision=args.precision)
    for _ in range(2 * T * F):
        plain.step()
    B.srmra_shift_error(plain.x_current, xt, inst.Lh, err, None, ws_e)
    err_plain = float(err.item())
    out = {"metric": METRIC, "value": inst.pairs_per_step / (ms_step * 1e-3), "unit": "obs×shift pairs/s",
           "n_gpus": 1, "steps": F * T, "warmup": F * T, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.precision], "data": "synthetic",
           "config": {"workload": args.workload, "algorithm": "projected EM", "F": F,
                      "outer_iterations_in_graph": T, "projection": "gaussian, s_1 = 1, decay 2^-1/10",
                      "precision": args.precision},
           "ms_per_outer_iteration": ms_outer, "projection_ms": ms_proj,
           "reconstruction_error": {"em_steps": 2 * T * F, "projected": err_proj, "plain_em": err_plain},
           "sigma_after": float(pe.sigma_state.item())}
    print(json.dumps(out), flush=True)


def bench_moments(args):
    """Empirical moments M1, M2 of the workload's observation stack (one pass,
    FP32 matrix cores for the Gram matrix): time per call and the Gram
    kernel's rate against the FP32 matrix peak (algorithmic flops N P (P + 1)
    for the symmetric product, P = Ll^2)."""
    import torch
    from paper_2204_04754_amd import binding as B
    from paper_2204_04754_amd import synth

    inst = synth.workload(args.workload)
    N, Ll = inst.N, inst.Ll
    P = Ll * Ll
    y = torch.as_tensor(inst.y).cuda()
    m1 = torch.empty(P, dtype=torch.float64, device="cuda")
    m2 = torch.empty((P, P), dtype=torch.float64, device="cuda")
    ws = B.empty_bytes(B.srmra_moments_workspace_bytes(N, Ll))
    for _ in range(args.warmup):
        B.srmra_moments(y, N, Ll, m1, m2, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        B.srmra_moments(y, N, Ll, m1, m2, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    T = (P + 127) // 128
    alg = float(N) * P * (P + 1)
    issued = 2.0 * N * (T * (T + 1) // 2) * 128 * 128
    out = {"metric": "empirical moments (eq. empiric_MOM) per second", "value": 1e3 / ms, "unit": "calls/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": args.workload, "N": N, "L_low": Ll, "P": P},
           "roofline": {"bound": "mfma", "achieved": alg / (ms * 1e-3) / 1e12, "peak": 157.3,
                        "unit": "TFLOP/s", "frac": alg / (ms * 1e-3) / 157.3e12,
                        "issued_frac": issued / (ms * 1e-3) / 157.3e12, "traffic": None,
                        "kernel": "whole call (Gram tiles + FP64 reductions)"}}
    print(json.dumps(out), flush=True)


def bench_errors(args):
    """Error table: one EM step of every precision form against the FP64 oracle
    on the first `error_obs` observations of the precision-study workloads
    (sigma 0.5 and 2; and the [0, 1]-image variant with and without centring),
    from the initial iterate and from the true image and prior.  Relative
    norm-wise errors of x' (all pixels, and components with at least one
    observation's posterior mass), rho', loglik, and the mean absolute error of
    the per-observation log-likelihood terms."""
    from oracle import em_oracle as O
    from paper_2204_04754_amd import synth
    from tests.gpu_helpers import gpu_step, rel

    cases = [("lh128_k4_n200000_s0.5", True), ("lh128_k4_n200000_s2", True),
             ("lh128_k4_n200000_unit_s0.25", True), ("lh128_k4_n200000_unit_s0.25", False)]
    precs = ["fp32_plain", "fp32_mfma", "bf16_split3", "bf16_split4", "fp32_fft"]
    rows = []
    cores = len(os.sched_getaffinity(0))
    for name, centre in cases:
        t = time.perf_counter()
        inst = synth.workload(name)
        y = np.ascontiguousarray(inst.y[:args.error_obs])
        K, sig, Lh = inst.K, inst.sigma, inst.Lh
        starts = {"init": (inst.x0, inst.log_rho0),
                  "truth": (inst.x_true, np.log(np.stack([inst.rho1, inst.rho2])).astype(np.float32))}
        for sname, (x, lr) in starts.items():
            ref = O.em_step(y, x, lr, sig, K, return_details=True)
            keep = ref["a"] >= 1.0
            print(f"[bench] errors {name} centre={centre} start={sname}: oracle done "
                  f"({time.perf_counter() - t:.0f} s)", file=sys.stderr, flush=True)
            for prec in precs:
                g = gpu_step(y, x, lr, sig, K, prec, centre=centre)
                rows.append(dict(workload=name, centre=centre, start=sname, precision=prec,
                                 x=rel(g["x_new"], ref["x_new"]),
                                 x_mass1=rel(g["x_new"][keep], ref["x_new"][keep]),
                                 mass1_frac=float(keep.mean()),
                                 rho=rel(g["rho_new"], ref["rho_new"]),
                                 loglik=abs(g["loglik"] - ref["loglik"]) / abs(ref["loglik"]),
                                 lse_mean_abs=float(np.mean(np.abs(g["ll_obs"] - ref["lse"])))))
    out = {"metric": "relative error vs FP64 oracle (one EM step)", "value": None, "unit": "",
           "n_gpus": 1, "data": "synthetic", "config": {"workload": "precision study subsets",
                                                        "observations": args.error_obs,
                                                        "oracle_cores": cores},
           "rows": rows}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson arrivals of 20-iteration jobs (90% drawn from the batched mix,
    10% Lh 256, K 4, N 20000), swept over arrival rates; solves/s and p50/p99
    latency (arrival -> completion) per rate and precision.  The BF16 forms
    serve `jobs` jobs per rate, the FP32 forms `jobs_fp32`; one more point runs
    the main form with a small HBM budget so that admission by footprint
    holds jobs back."""
    import torch
    from paper_2204_04754_amd import synth
    from paper_2204_04754_amd.serve import GPUExecutor, Job, serve

    pool_shapes = synth.mixed_batch(11, config=4) + [dict(Lh=256, K=4, N=20000, sigma=1.0,
                                                            config=4, instance=999)]
    t = time.perf_counter()
    pool = [synth.make_instance(**d) for d in pool_shapes]
    print(f"[bench] job pool generated in {time.perf_counter() - t:.1f} s", file=sys.stderr,
          flush=True)
    rates = [float(r) for r in args.rates.split(",")]
    results = {}

    def sequence(rate, n):
        # one job sequence per (rate, count): the same jobs and arrival times
        # for every precision that serves that many jobs
        r = np.random.default_rng(int(rate * 1000) + 7)
        arr = np.cumsum(r.exponential(1.0 / rate, size=n))
        pick = [11 if r.random() < 0.1 else int(r.integers(0, 11)) for _ in range(n)]
        return arr, pick

    def run(prec, rate, n, budget, key):
        arr, pick = sequence(rate, n)
        jobs = []
        for k in range(n):
            inst = pool[pick[k]]
            jobs.append(Job(k, inst.y, inst.K, inst.sigma, inst.x0, inst.log_rho0,
                            iterations=args.iterations, arrival=float(arr[k])))
        # "<precision>+fft": jobs at an L_low the FFT route supports take it by
        # their own steps; "<precision>+fftplan": inside the plan, as FFT classes
        base, _, extra = prec.partition("+")
        ex = GPUExecutor(precision=base, fft={"fft": True, "fftplan": "plan"}.get(extra, False))
        rep = serve(jobs, ex, hbm_budget=budget, max_slots=64)
        summ = rep.summary()
        summ.update(jobs_served=n, hbm_budget_gb=budget / 2 ** 30)
        results[key] = summ
        print(f"[bench] serve {key}: {summ}", file=sys.stderr, flush=True)
        del ex
        torch.cuda.empty_cache()

    precs = [p for p in args.serve_precisions.split(",") if p] or \
        [args.precision + "+fftplan", args.precision + "+fft", args.precision, "fp32_mfma", "fp32_plain"]
    for prec in dict.fromkeys(precs):
        n = args.jobs_fp32 if prec.split("+")[0].startswith("fp32") else args.jobs
        for rate in rates:
            run(prec, rate, n, 200 << 30, f"{prec}@{rate:g}")
    if args.budget_gb > 0:
        rate = rates[len(rates) // 2]
        run(precs[0], rate, args.jobs, int(args.budget_gb * 2 ** 30),
            f"{precs[0]}@{rate:g}@budget{args.budget_gb:g}GB")
    main_key = f"{precs[0]}@{rates[-1]:g}"
    out = {"metric": METRIC, "value": results[main_key]["solves_per_s"], "unit": "solves/s",
           "n_gpus": 1, "steps": args.jobs, "warmup": 0, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.precision], "data": "synthetic",
           "config": {"workload": "serve_poisson_mix", "jobs_per_rate": args.jobs,
                      "jobs_per_rate_fp32": args.jobs_fp32,
                      "iterations_per_job": args.iterations, "rates": rates, "main": precs[0]},
           "p50_latency_s": results[main_key]["p50_latency_s"],
           "p99_latency_s": results[main_key]["p99_latency_s"], "per_rate": results}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library and this benchmark run on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.mode == "batched":
        return bench_batched(args)
    if args.mode == "errors":
        return bench_errors(args)
    if args.mode == "projected":
        return bench_projected(args)
    if args.mode == "moments":
        return bench_moments(args)
    if args.mode == "serve":
        return bench_serve(args)
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
                                  phase_ms=main_r["phase_ms"], obs_prep=main_r["prep"])}
    del main_r["job"]
    if not args.no_plain and args.baseline_precision != args.precision:
        base_steps = max(2, args.steps // 4)
        br = run_form(inst, args.baseline_precision, base_steps, 1)
        del br["job"]
        forms[args.baseline_precision] = dict(
            pairs_per_s=pairs / (br["ms_per_step"] * 1e-3), ms_per_step=br["ms_per_step"],
            phase_ms=br["phase_ms"], obs_prep=br["prep"])
        print(f"[bench] {args.baseline_precision}: {br['ms_per_step']:.2f} ms/step",
              file=sys.stderr, flush=True)
    from paper_2204_04754_amd import binding as B
    for extra in [f for f in args.extra_forms.split(",") if f]:
        if extra in forms or B.srmra_em_step_workspace_bytes(inst.N, inst.Ll, inst.K, extra) == 0:
            continue
        er = run_form(inst, extra, max(2, args.steps // 2), 1)
        del er["job"]
        forms[extra] = dict(pairs_per_s=pairs / (er["ms_per_step"] * 1e-3), ms_per_step=er["ms_per_step"],
                            phase_ms=er["phase_ms"], obs_prep=er["prep"])
        print(f"[bench] {extra}: {er['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    roof = roofline(inst, args.precision, main_r["phase_ms"], args.workload)

    out = {"metric": METRIC, "value": value, "unit": "obs×shift pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": forms[args.precision]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.precision],
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
    fastest = min(forms, key=lambda k: forms[k]["ms_per_step"])
    out["fastest_form"] = {"precision": fastest, "pairs_per_s": forms[fastest]["pairs_per_s"],
                           "ms_per_step": forms[fastest]["ms_per_step"]}
    if args.secondary_workload:
        t = time.perf_counter()
        inst2 = synth.workload(args.secondary_workload)
        sr = run_form(inst2, args.secondary_precision, args.steps, args.warmup)
        del sr["job"]
        out["secondary"] = {
            "workload": args.secondary_workload, "precision": args.secondary_precision,
            "L_high": inst2.Lh, "K": inst2.K, "L_low": inst2.Ll, "N": inst2.N, "sigma": inst2.sigma,
            "ms_per_step": sr["ms_per_step"],
            "pairs_per_s": inst2.pairs_per_step / (sr["ms_per_step"] * 1e-3),
            "roofline": roofline(inst2, args.secondary_precision, sr["phase_ms"], args.secondary_workload)}
        print(f"[bench] secondary {args.secondary_workload} {args.secondary_precision}: "
              f"{sr['ms_per_step']:.2f} ms/step ({time.perf_counter() - t:.1f} s)",
              file=sys.stderr, flush=True)
        del inst2
    if not args.no_mix:
        # the batched (64-instance mix) and serving forms, compact, so that the
        # default run records them too (full sweeps: --mode batched / serve)
        out["batched"] = mix_summary(args.precision)
        out["serving"] = serve_summary(args.precision)
    if not args.no_cpu:
        n = args.cpu_sample or oracle_sample_size(inst, args.cpu_seconds)
        n = min(n, inst.N)
        t = time.perf_counter()
        cb, err = cpu_baseline(inst, n, list(forms))
        out["cpu_baseline"] = cb
        out["rel_err_vs_oracle_on_sample"] = err
        print(f"[bench] cpu baseline and errors ({time.perf_counter() - t:.1f} s)", file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
