"""Pick the tile shape, records staged per thread, block width of the lock-step walk and depth-segment length
of the batched step by measured replay time.

Every candidate computes the same forward bit for bit (the per-pair arithmetic is fixed and records are
culled only where they provably do not contribute) and the same gradients up to the order of the float
atomic additions (and, for the segment length, the FP32 association of the transmittance product), so the
choice changes speed only.  Results are cached in a JSON file keyed by the GPU
architecture, the resolution class, the Gaussian-count band and the SH degree.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import binding as B

# (tile_w, tile_h, records staged per thread, block width of the lock-step walk, depth-segment length;
# -1 = never split).  The first is the default: another candidate is chosen only if it is faster by more than
# TIE (measurement noise would otherwise flip between near-equal ones from run to run).
CANDIDATES: List[Tuple[int, int, int, int, int]] = [
    (16, 8, 1, 4, 512), (16, 16, 1, 4, 512), (16, 16, 1, 4, 1024), (16, 8, 1, 4, 1024), (16, 8, 1, 8, 512),
    (16, 8, 2, 4, 512), (8, 8, 1, 4, 512), (32, 8, 1, 4, 512), (16, 16, 1, 8, -1), (16, 16, 1, 2, 512)]
TIE = 0.02

_CACHE = os.environ.get("GS_AUTOTUNE_CACHE",
                        os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".scene_cache",
                                     "autotune.json"))


def cache_key(n: int, cams: Sequence, sh_degree: int) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    px = sum(c.width * c.height for c in cams)
    return f"{arch}|views{len(cams)}|px2^{round(math.log2(max(px, 1)))}|n2^{round(math.log2(max(n, 1)))}|deg{sh_degree}"


def _load() -> Dict[str, list]:
    try:
        with open(_CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict[str, list]) -> None:
    try:
        os.makedirs(os.path.dirname(_CACHE), exist_ok=True)
        with open(_CACHE + ".tmp", "w") as f:
            json.dump(d, f, indent=1)
        os.replace(_CACHE + ".tmp", _CACHE)
    except OSError:
        pass


def tune_batched(make_step, n: int, cams: Sequence, sh_degree: int, replays: int = 8,
                 candidates: Sequence[Tuple[int, int, int, int, int]] = CANDIDATES, use_cache: bool = True,
                 log=None):
    """make_step(opts) -> a BatchedStep.  Returns (best (tile_w, tile_h, depth, block_w, seg_len),
    {candidate: ms})."""
    key = cache_key(n, cams, sh_degree)
    cache = _load() if use_cache else {}
    if key in cache:
        return tuple(cache[key][0]), {}
    times = {}
    for tw, th, dp, bw, sg in candidates:
        opts = B.default_opts(tile_w=tw, tile_h=th, batch_depth=dp, block_w=bw, seg_len=sg)
        step = make_step(opts)
        step.capture()
        step.run()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(replays):
            step.run()
        e.record()
        e.synchronize()
        ms = s.elapsed_time(e) / replays
        step.finish()
        if step.replans:
            ms = float("inf")  # the capacity was re-planned inside the timed replays
        times[(tw, th, dp, bw, sg)] = ms
        if log:
            log(f"  autotune {tw}x{th} depth {dp} block {bw} seg_len {sg}: {ms:.3f} ms")
        del step
        torch.cuda.empty_cache()
    fastest = min(times.values())
    best = next(c for c in times if times[c] <= fastest * (1.0 + TIE))
    if use_cache:
        cache[key] = [list(best), {f"{a}x{b}/d{c}/b{d}/L{e}": v for (a, b, c, d, e), v in times.items()}]
        _store(cache)
    return best, times
