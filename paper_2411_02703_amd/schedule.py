"""Training policies of LVI-GS mapping on top of the batched step (Sections III-C, III-D, III-E).

These decide, per iteration, which keyframes and pyramid levels are optimised, with which SH degree, and when
a keyframe's LiDAR points join the map.  They are host-side bookkeeping (seeded, deterministic); every step
they select runs in the HIP library through `BatchedStep`.

* KeyframeQueue (Sec. III-E): a newly received keyframe is optimised once as a submap; afterwards each iteration
  shuffles the keyframe sequence and picks keyframes at random.  Every keyframe has an upper limit on its
  optimisation iterations and leaves the sequence when it reaches it.
* DelayBuffer (Sec. III-C): a keyframe's colourised LiDAR points are integrated into the map (initialise
  Gaussians) only after `delay` newer keyframes have arrived, so that Gaussians of one frame are not pruned
  before later viewpoints have observed them.
* PyramidSchedule (Sec. III-D): coarse to fine.  A keyframe's first iterations use its coarsest pyramid level;
  after every `iters_per_level` of its iterations the level steps one finer, ending at full resolution.
* SHSchedule (Sec. III-E): the SH degree starts at 0 and grows by one every `every` iterations, capped at 3.

Readings where the paper gives no numbers: the iteration caps, the delay length, the per-level iteration count
and the SH period are parameters; "select one frame at random" after a shuffle is a uniform pick, and picking
`batch` keyframes per iteration (several keyframes in one batched step) draws them without replacement.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field
from typing import Dict, Hashable, List, Optional, Sequence

import numpy as np


@dataclass
class KeyframeQueue:
    """The keyframe sequence of Sec. III-E with per-keyframe iteration caps."""

    cap: int = 100
    batch: int = 1
    seed: int = 0
    counts: Dict[Hashable, int] = field(default_factory=dict)
    order: List[Hashable] = field(default_factory=list)  # active keyframes, in arrival order
    fresh: deque = field(default_factory=deque)          # received but not yet optimised once
    retired: List[Hashable] = field(default_factory=list)

    def __post_init__(self):
        if self.cap < 1 or self.batch < 1:
            raise ValueError("cap and batch must be >= 1")
        self.rng = np.random.default_rng(self.seed)

    def add(self, kf: Hashable) -> None:
        if kf in self.counts:
            raise ValueError(f"keyframe {kf!r} already received")
        self.counts[kf] = 0
        self.order.append(kf)
        self.fresh.append(kf)

    @property
    def active(self) -> List[Hashable]:
        return list(self.order)

    def select(self) -> List[Hashable]:
        """The keyframes of the next iteration: fresh keyframes first (each optimised once as a submap), then
        random picks from the shuffled sequence; counts advance and capped keyframes retire."""
        picked: List[Hashable] = []
        while self.fresh and len(picked) < self.batch:
            picked.append(self.fresh.popleft())
        rest = [k for k in self.order if k not in picked]
        if len(picked) < self.batch and rest:
            perm = self.rng.permutation(len(rest))
            picked += [rest[i] for i in perm[:self.batch - len(picked)]]
        for k in picked:
            self.counts[k] += 1
            if self.counts[k] >= self.cap:
                self.order.remove(k)
                self.retired.append(k)
                if k in self.fresh:
                    self.fresh.remove(k)
        return picked


@dataclass
class DelayBuffer:
    """Keyframes wait until `delay` newer keyframes have arrived before their points join the map."""

    delay: int = 2
    waiting: deque = field(default_factory=deque)

    def push(self, kf: Hashable) -> List[Hashable]:
        """Receive a keyframe; returns the keyframes released into the map by its arrival."""
        self.waiting.append(kf)
        out = []
        while len(self.waiting) > self.delay:
            out.append(self.waiting.popleft())
        return out

    def flush(self) -> List[Hashable]:
        out = list(self.waiting)
        self.waiting.clear()
        return out


@dataclass
class PyramidSchedule:
    """Coarse-to-fine level of a keyframe from the number of iterations it has taken (level 0 = full
    resolution, levels - 1 = coarsest)."""

    levels: int = 3
    iters_per_level: int = 10

    def level(self, iters_done: int) -> int:
        return max(0, self.levels - 1 - iters_done // self.iters_per_level)

    def weights(self, iters_done: int, weight: float = 1.0) -> List[float]:
        """Loss weight of each level (one-hot on the scheduled level)."""
        lv = self.level(iters_done)
        return [weight if l == lv else 0.0 for l in range(self.levels)]


@dataclass
class SHSchedule:
    """SH degree after `it` iterations: 0, rising by one every `every` iterations, capped at `max_degree`."""

    every: int = 1000
    max_degree: int = 3

    def degree(self, it: int) -> int:
        return min(self.max_degree, it // self.every)
