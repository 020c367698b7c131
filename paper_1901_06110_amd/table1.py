"""Table 1 on synthetic data: brute-force vs fast DSG-NLM timings.

The paper times a 256 x 256 image with a fixed window N_s = 21 and patch
sides N_p = 11, 17, 23, 29 (Table 1), on a CPU.  Here both implementations run
on the GPU: the brute-force comparator sums every patch distance over its N_p^2
offsets (`dsnlm_forward_brute`), the fast path uses box sums whose cost does
not depend on N_p (`dsnlm_forward`: the register-resident half-window sweeps
for P <= 5, the wide-patch passes for P > 5).  The window is taken both ways
the paper can be read: 21 x 21 (S = 10) and 43 x 43 (S = 21).  N_p runs over
3, 5, 7, 9, 11 and the paper's 17, 23, 29.  Each fast time is the median of 20
runs after 3 warm-ups, each brute-force time the median of 5; inputs resident.
Usage: python -m paper_1901_06110_amd.table1
"""
from __future__ import annotations

import json
import os
import sys

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

from . import api as M  # noqa: E402


def _median_ms(fn, reps: int = 20, warm: int = 3) -> float:
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def main() -> None:
    _, noisy = synth.piecewise_smooth(256, 256, seed=1001, sigma_n=0.05)
    x = torch.as_tensor(noisy).cuda()
    y = torch.empty_like(x)
    rows = []
    for S in (10, 21):
        for P in (1, 2, 3, 4, 5, 8, 11, 14):
            h = 0.1
            _, w = M.dsnlm_forward(x, None, S, P, h, y=y, keep=True)
            fast = _median_ms(lambda: M.dsnlm_forward(x, None, S, P, h, y=y, weights=w))
            brute = _median_ms(lambda: M.dsnlm_forward_brute(x, None, S, P, h, y=y), reps=5, warm=1)
            rows.append(dict(window=2 * S + 1, Np=2 * P + 1, brute_ms=brute, fast_ms=fast, ratio=brute / fast))
            print(f"window {2 * S + 1:2d}  N_p {2 * P + 1:2d}  brute {brute:9.3f} ms  fast {fast:7.3f} ms  "
                  f"ratio {brute / fast:7.1f}", flush=True)
    print(json.dumps(rows))


if __name__ == "__main__":
    main()
