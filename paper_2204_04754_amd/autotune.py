"""Autotuner of the batched form.

For every (L_low, K) class of a batch it times candidate settings of the plan's
tuning table (srmra_tuning in the C ABI) on the class's own problems and keeps
the fastest:

* the form: in a BF16 split plan, the BF16 kernels or FP32 MFMA (both meet the
  accuracy target; which is faster depends on the shape), otherwise the plan's
  own precision; with fft, also the FFT route where it covers the L_low (its
  candidates run on FFT preparations of the class's problems, made for the
  trials);
* observations per work item, as multiples of the library's default (about
  2^28 multiply-adds per item, down to 2^24 where that gives a problem fewer
  than 128 chunks): smaller items balance the persistent launch
  better, larger ones write fewer per-chunk partials;
* the block layout where the form and shape offer a choice (SRMRA_TILE_* of
  srmra.h): for the BF16 split the matrix-core tile shape at L_low 48 (3 x 3
  tiles of 16x16 in one pass, or 2 x 2 tiles of 32x32 in two passes), the
  observations and waves per workgroup at L_low 24 and 32 (a single pass over
  8 observations x 4 components with 4 waves, or 4 observations x 16
  components with 8 waves, or two passes) and the component slots at L_low 16
  (a workgroup of 32 / WC observations x 4 WC components, WC in {1, 2, 4});
  for FP32 MFMA the single pass or two passes; timed at the default item size
  before the item sizes are swept at the best layout.

Timing runs one EM step of the class alone per candidate, on scratch copies of
the iterates (the problems' own iterates are left unchanged), with HIP events
on the stream.  Marshalling and timing only: every step runs the library's
kernels.
"""
from __future__ import annotations

from collections import OrderedDict
from typing import Dict, List, Sequence, Tuple

import torch

from . import binding as B

SCALES = (0.25, 0.5, 1.0, 2.0, 4.0)


def candidate_forms(precision: int, L_low: int, fft: bool = False) -> List[int]:
    base = B.srmra_plan_form(precision, L_low)
    if base < 0:
        raise B.SrmraError(B.SRMRA_EUNSUPPORTED, "autotune")
    forms = [base, B.SRMRA_FP32_MFMA] if base in (B.SRMRA_BF16_SPLIT3, B.SRMRA_BF16_SPLIT4) else [base]
    if fft and B.srmra_em_step_workspace_bytes(1024, L_low, 1, "fp32_fft") > 0:
        forms.append(B.SRMRA_FP32_FFT)
    return forms


def candidate_tiles(form: int, L_low: int, K: int) -> List[int]:
    """Block layouts the form offers at this (L_low, K) ([0]: the default only)."""
    KK = K * K
    if form in (B.SRMRA_BF16_SPLIT3, B.SRMRA_BF16_SPLIT4):
        if L_low in (8, 12):
            ncw = 4 if L_low == 8 else 8   # components per block of the packed tiles
            return [0, B.SRMRA_TILE_TWO_PASS] if (KK + ncw - 1) // ncw <= 4 else [0]
        if L_low == 16:
            return [1, 2, 4]
        if L_low in (24, 32):
            tiles = [B.SRMRA_TILE_FUSED_8OBS] if KK <= 4 else []
            tiles += [B.SRMRA_TILE_FUSED_4OBS] if KK <= 16 else []
            return tiles + [B.SRMRA_TILE_TWO_PASS] if tiles else [0]
        if L_low == 48 and KK <= 4:
            return [B.SRMRA_TILE_16X16, B.SRMRA_TILE_TWO_PASS]
    if form == B.SRMRA_FP32_MFMA and B.srmra_em_step_passes(1024, L_low, K, "fp32_mfma") == 1:
        return [0, B.SRMRA_TILE_TWO_PASS]
    return [0]


def _scratch(pr: dict, form: int, stream=None) -> dict:
    """The problem with its own observations, a preparation for `form` (its own
    when that serves the form) and fresh iterate buffers (copies of the current
    iterate)."""
    d = dict(pr)
    if (form == B.SRMRA_FP32_FFT) != (pr.get("prep_form") == B.SRMRA_FP32_FFT):
        pb = B.srmra_prepared_bytes(pr["N"], pr["L_low"], pr["K"], form)
        d["prep"] = B.empty_bytes(pb, pr["y"].device)
        B.srmra_prepare_observations(pr["y"], pr["N"], pr["L_low"], pr["K"], form, d["prep"], stream)
    d["x"] = pr["x"].clone()
    d["log_rho"] = pr["log_rho"].clone()
    d["x_new"] = torch.empty_like(pr["x"])
    d["log_rho_new"] = torch.empty_like(pr["log_rho"])
    d["rho_new"] = torch.empty_like(pr["rho_new"])
    d["loglik"] = torch.empty_like(pr["loglik"])
    return d


def _time_plan(problems, precision, entry, reps, warmup, stream) -> float:
    plan = B.Plan(problems, precision, tuning=[entry])
    ws = B.empty_bytes(plan.workspace_bytes, problems[0]["y"].device)
    plan.upload(ws, stream)
    for _ in range(warmup):
        plan.execute(ws, stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    s = stream if stream is not None else torch.cuda.current_stream()
    ev[0].record(s)
    for _ in range(reps):
        plan.execute(ws, stream)
    ev[1].record(s)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    plan.close()
    return ms


def tune(problems: Sequence[dict], precision, scales=SCALES, reps: int = 3, warmup: int = 1,
         stream=None, fft: bool = False) -> Tuple[List[dict], List[dict]]:
    """problems: the batch (dicts with y, prep, prep_form, N, L_low, K, sigma, x,
    log_rho, rho_new, loglik, as for binding.Plan); a BF16 preparation also
    serves FP32 MFMA, and FFT candidates get preparations of their own.
    Returns (table, report): one srmra_tuning entry per class, and every timing."""
    p = B._prec(precision)
    groups: Dict[Tuple[int, int], List[int]] = OrderedDict()
    for i, pr in enumerate(problems):
        groups.setdefault((int(pr["L_low"]), int(pr["K"])), []).append(i)
    table, report = [], []
    for (Ll, K), idx in groups.items():
        n_max = max(int(problems[i]["N"]) for i in idx)
        best = None
        for form in candidate_forms(p, Ll, fft):
            scratch = [_scratch(problems[i], form, stream) for i in idx]
            base = B.srmra_plan_default_item_obs(n_max, Ll, K, form)
            seen = set()

            def trial(item, tile):
                nonlocal best
                entry = dict(precision=p, L_low=Ll, K=K, form=form, item_obs=item, tile=tile)
                ms = _time_plan(scratch, p, entry, reps, warmup, stream)
                report.append(dict(entry, ms=ms, problems=len(idx)))
                if best is None or ms < best[0]:
                    best = (ms, entry)
                return ms

            tiles = candidate_tiles(form, Ll, K)
            tile = tiles[0]
            if len(tiles) > 1:
                tile = min(tiles, key=lambda t: trial(base, t))
                seen.add(base)
            for sc in scales:
                item = max(1, int(round(base * sc)))
                if item in seen:
                    continue
                seen.add(item)
                trial(item, tile)
        table.append(best[1])
    return table, report
