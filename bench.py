"""Benchmark of the DSG-NLM forward on one MI355X.

Workload: 64 synthetic piecewise-smooth images of uneven sizes (sides from
{128, ..., 1024}, square or 2:1, about 17 Mpx in total), search half-width
S = 10 (21 x 21 window), patch half-width P = 3 (7 x 7 patches), h = 1.2
sigma_n per image, FP32.  One step = the DSG-NLM forward y = W(x) x of every
image of the batch (inputs resident in HBM).

Prints one JSON line: Mpixel/s of the forward, the dominant kernel's roofline
fraction (its device time measured with HIP events on its launch stream), the
forward+backward / forward time ratio, and the FP64 oracle timed on the host
cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak rates of one MI355X used for the roofline (derivation in the design notes):
# 256 CUs x 64 FP32 lanes x 2.4 GHz = 39.3e12 non-packed FP32 VALU lane-ops/s;
# a transcendental (v_exp_f32) occupies 4 lane-op slots.
VALU_LANE_OPS_PER_S = 256 * 64 * 2.4e9
EXP_SLOTS = 4
# Algorithmic work per (pixel, in-window shift), in lane-op slots:
#   weight: diff 1 + square 1 + separable sliding box 4 + exponent 1 + exp2 (4)
#   pass A adds 1 (accumulate omega); pass B adds 2 (two FMAs)
OPS_PASS_A = 8 + EXP_SLOTS
OPS_PASS_B = 9 + EXP_SLOTS


def window_pairs(n1: int, n2: int, S: int) -> int:
    """Number of (pixel, shift) pairs with both pixels in the image."""
    def axis(n):
        tot = 0
        for i in range(n):
            tot += min(n - 1, i + S) - max(0, i - S) + 1
        return tot
    return axis(n1) * axis(n2)


def cpu_baseline(images, S, P, budget_s: float = 20.0):
    """FP64 oracle (shift-loop route) on crops of the first images until about
    budget_s seconds of host time have been spent."""
    import torch
    from oracle import dsnlm_ref
    crop = 192
    done_px = 0
    t0 = time.perf_counter()
    used = 0
    for it in images:
        x = it.noisy[:crop, :crop]
        dsnlm_ref.dsnlm_shifts(x, x, S, P, it.h)
        done_px += x.size
        used += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=done_px / dt / 1e6, unit="Mpixel/s", cores=torch.get_num_threads(),
                kind="oracle",
                sample=f"{used} crops of up to {crop}x{crop} px from the batch, S={S}, P={P}, "
                       f"{done_px} px in {dt:.1f} s (FP64 shift loop, torch CPU)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["batched", "perimage"], default="batched")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--count", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the batch would shard image by image; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_06110_amd as M
    from paper_1901_06110_amd import _lib
    import synth

    S, P = 10, 3
    lib = _lib.get()
    images = synth.config2_batch(count=args.count)
    xs = [torch.as_tensor(it.noisy).cuda() for it in images]
    ys = [torch.empty_like(x) for x in xs]
    hs = [it.h for it in images]
    total_px = sum(x.numel() for x in xs)
    pairs = sum(window_pairs(x.shape[0], x.shape[1], S) for x in xs)

    if args.mode == "batched":
        def step():
            M.dsnlm_forward_batched(list(zip(xs, xs, hs)), S, P, outs=ys)
    else:
        handles = []
        for x, y, h in zip(xs, ys, hs):
            _, w = M.dsnlm_forward(x, None, S, P, h, y=y, keep=True)
            handles.append(w)

        def step():
            for x, y, h, w in zip(xs, ys, hs, handles):
                M.dsnlm_forward(x, None, S, P, h, y=y, weights=w)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1) / args.steps

    # per-kernel device time of the sweeps, on their launch stream
    lib.dsnlm_profile_reset()
    lib.dsnlm_profile_enable(1)
    prof_steps = max(2, min(args.steps, 5))
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    import ctypes as C
    tot = {}
    for name, kind in [("pass_a", _lib.K_PASS_A), ("pass_b", _lib.K_PASS_B),
                       ("epilogue", _lib.K_EPILOGUE)]:
        t = C.c_double()
        n = C.c_int()
        lib.dsnlm_profile_query(kind, C.byref(t), C.byref(n))
        tot[name] = (t.value, n.value)
    lib.dsnlm_profile_enable(0)
    pb_ms, pb_n = tot["pass_b"]
    launches_per_step = pb_n / prof_steps
    pb_avg_ms = pb_ms / max(pb_n, 1)
    ops_per_launch = OPS_PASS_B * pairs / launches_per_step
    achieved = ops_per_launch / (pb_avg_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS_PER_S / 1e12

    out = {
        "metric": "DSG-NLM Mpixel/s @21x21 search, 7x7 patch (forward)",
        "value": total_px / (ms * 1e-3) / 1e6,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched DSG-NLM forward, {len(xs)} uneven piecewise-smooth images "
                        f"({total_px} px), S=10 (21x21), P=3 (7x7), h=1.2 sigma_n",
            "images": len(xs), "pixels": total_px, "S": S, "P": P, "mode": args.mode,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_sweep pass B (step-S2 row sums, B', max m)",
            "achieved": achieved,
            "peak": peak,
            "unit": "Tops/s",
            "frac": achieved / peak,
            "traffic": None,
            "ops_per_pair": OPS_PASS_B,
            "pairs_per_launch": pairs / launches_per_step,
            "avg_launch_ms": pb_avg_ms,
        },
        "kernel_ms_per_step": {k: v[0] / prof_steps for k, v in tot.items()},
        "forward_roofline_frac": (OPS_PASS_A + OPS_PASS_B) * pairs / (ms * 1e-3) / VALU_LANE_OPS_PER_S,
        "wall_s_timed": wall,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(images, S, P)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
