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

# Peak rate of one MI355X used for the roofline: 256 CUs x 64 FP32 lanes x
# 2.4 GHz = 39.3e12 non-packed FP32 VALU lane-ops/s (the library is built
# without packed FP32 ops).  A v_exp_f32 occupies EXP_SLOTS lane-op slots;
# the value is measured on the device by dsnlm_peak_probe (4 = quarter rate
# is the fallback when the probe is unavailable).
VALU_LANE_OPS_PER_S = 256 * 64 * 2.4e9
EXP_SLOTS_FALLBACK = 4.0
# The sweeps evaluate each unordered pair {s, s + d} once (half window, the
# weight is symmetric) and add it to both pixels.  Algorithmic FP32 VALU ops
# per evaluated pair, the transcendental apart:
#   weight: diff 1 + square 1 + separable sliding box 4 + exponent 1 (+ 1 exp)
#   pass A adds 2 (omega at s and at s + d); pass B adds 4 (two FMAs at each)
VALU_PASS_A = 9
VALU_PASS_B = 11
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_half_b_batched64_S10P3.md")
TRAFFIC_SOURCE = os.path.join(ROOT, "paper_1901_06110_amd", "csrc", "dsnlm_half.hip")


def measured_traffic(kind: str):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel source changed after the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
        src = open(TRAFFIC_SOURCE, "rb").read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith(("|", "#")))
    if vals.get("source_sha256_dsnlm_half.hip", "").strip() != hashlib.sha256(src).hexdigest():
        return None
    v = vals.get(f"traffic_bytes_per_launch_{kind}")
    return float(v) if v else None


def window_pairs(n1: int, n2: int, S: int) -> int:
    """Number of ordered (pixel, shift) pairs with both pixels in the image
    (d = 0 included); the unordered pairs with d != 0 are (this - n1 n2) / 2."""
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


def fwd_bwd_ratio(M, xs, hs, S, P, steps):
    """Time the batched forward alone and the batched forward + backward
    (input, guide and h gradients of every image); return the ratio."""
    import torch
    imgs = [(x, x, h) for x, h in zip(xs, hs)]
    outs = M.dsnlm_forward_batched(imgs, S, P)
    ybars = [2.0 * (y - x) for x, y in zip(xs, outs)]

    def fwd():
        M.dsnlm_forward_batched(imgs, S, P, outs=outs)

    def fwd_bwd():
        fwd()
        M.dsnlm_backward_batched(ybars)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    tf = timed(fwd)
    tfb = timed(fwd_bwd)
    return {"fwd_ms": tf, "fwd_bwd_ms": tfb, "ratio": tfb / tf,
            "fwd_bwd_mpx_s": sum(x.numel() for x in xs) / (tfb * 1e-3) / 1e6,
            "note": "batched launches, %d images, S=%d, P=%d; backward = d/dx, d/dguide, d/dh"
                    % (len(xs), S, P)}


def ladmm_sr_timing(M, S, P):
    """2x super-resolution of a 512x512 synthetic image: 50 iterations of
    Algorithm 1, weights rebuilt for 5 iterations then frozen (graph-captured)."""
    import numpy as np
    import torch
    import synth
    cfg = synth.config1_inputs(512)
    b = np.exp(-np.arange(-4, 5) ** 2 / 2.0)
    taps = (b / b.sum()).astype(np.float32)
    op = M.SROperator(n1=512, n2=512, taps=taps, factor=2, y=None, boundary=0)
    xc = torch.as_tensor(cfg["clean"]).cuda()
    y = M.ladmm_apply_forward(op, xc) + torch.as_tensor(cfg["lr_noise"]).cuda()
    op.y = y
    x0 = torch.as_tensor(synth.bicubic_upsample(y.cpu().numpy(), 2)).cuda()
    gamma = 1.0 / M.ladmm_operator_norm2(op, 300)
    prm = M.LadmmParams(lam=cfg["lam"], rho=cfg["rho"], gamma=gamma, S=S, P=P, h=cfg["h"],
                        freeze_after=cfg["freeze_after"], iters=cfg["iters"])
    res = torch.zeros((cfg["iters"], 2), device="cuda")
    st = torch.cuda.Stream()
    times = []
    for rep in range(3):
        x, v, u = x0.clone(), x0.clone(), torch.zeros_like(x0)
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            M.ladmm_solve(op, prm, x, v, u, residuals=res)
            e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    err0 = float(torch.sqrt(torch.mean((x0 - xc) ** 2)))
    err = float(torch.sqrt(torch.mean((x - xc) ** 2)))
    return {"ms_per_solve": min(times), "iters": cfg["iters"], "freeze_after": cfg["freeze_after"],
            "rmse_bicubic": err0, "rmse_ladmm": err,
            "final_primal_residual": float(res[-1, 0]), "final_dual_residual": float(res[-1, 1]),
            "note": "includes weight rebuilds (5), frozen applies (45), graph capture and one "
                    "host synchronisation per solve"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["batched", "perimage"], default="batched")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--no-ladmm", action="store_true", help="skip the LADMM solve timing")
    ap.add_argument("--no-fb", action="store_true", help="skip the forward+backward timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(a batch would shard image by image across GPUs, with no communication)", file=sys.stderr)
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
                       ("prep_and_gather", _lib.K_HALF_AUX), ("epilogue", _lib.K_EPILOGUE)]:
        t = C.c_double()
        n = C.c_int()
        lib.dsnlm_profile_query(kind, C.byref(t), C.byref(n))
        tot[name] = (t.value, n.value)
    lib.dsnlm_profile_enable(0)
    # ---- measured peak rates of this device (context for the roofline)
    probes = {}
    for kind, name in [(0, "fp32_fma_flop_s"), (1, "exp_per_s"), (2, "hbm_copy_bytes_s")]:
        r = C.c_double()
        if lib.dsnlm_peak_probe(kind, C.byref(r), C.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0:
            probes[name] = r.value
    if "fp32_fma_flop_s" in probes and "exp_per_s" in probes:
        probes["exp_cost_in_fma_slots"] = probes["fp32_fma_flop_s"] / 2 / probes["exp_per_s"]

    exp_slots = probes.get("exp_cost_in_fma_slots", EXP_SLOTS_FALLBACK)
    pb_ms, pb_n = tot["pass_b"]
    launches_per_step = pb_n / prof_steps
    pb_avg_ms = pb_ms / max(pb_n, 1)
    ops_pair_b = VALU_PASS_B + exp_slots
    ops_pair_a = VALU_PASS_A + exp_slots
    half_pairs = (pairs - total_px) / 2  # pairs the sweeps evaluate
    ops_per_launch = ops_pair_b * half_pairs / launches_per_step
    achieved = ops_per_launch / (pb_avg_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS_PER_S / 1e12

    # ---- forward + backward vs forward, per-image launches over the batch
    fb = None if args.no_fb else fwd_bwd_ratio(M, xs, hs, S, P, steps=max(1, min(args.steps, 3)))

    # ---- linearized PnP-ADMM super-resolution solve (512x512, 50 iterations)
    lad = ladmm_sr_timing(M, S, P) if not args.no_ladmm else None

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
            "kernel": "k_half pass B (half-window step-S2 sums at both pixels of each pair)",
            "achieved": achieved,
            "peak": peak,
            "unit": "Tops/s",
            "frac": achieved / peak,
            "frac_vs_packed_fp32_peak": achieved / (2 * peak),
            "traffic": measured_traffic("pass_b"),
            "ops_per_pair": ops_pair_b,
            "exp_slots": exp_slots,
            "pairs_evaluated_per_launch": half_pairs / launches_per_step,
            "avg_launch_ms": pb_avg_ms,
        },
        "kernel_ms_per_step": {k: v[0] / prof_steps for k, v in tot.items()},
        "measured_peaks": probes,
        "fwd_bwd_over_fwd": fb["ratio"] if fb else None,
        "fwd_bwd": fb,
        "ladmm_sr_512": lad,
        "forward_roofline_frac": (ops_pair_a + ops_pair_b) * half_pairs / (ms * 1e-3) / VALU_LANE_OPS_PER_S,
        "wall_s_timed": wall,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(images, S, P)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
