"""Autotuner for the synthesis tile shapes.

For a workload (L, nside, nmaps, eps) it builds one plan per candidate tile
shape (rings per lane of the Legendre waves, workgroup size of the ring FFT)
and times full syntheses on the GPU with events on the execution stream,
keeping the fastest.  Results are cached per process and, optionally, in a
JSON file.  Timing runs the library's kernels only; nothing here computes
any part of the transform.
"""
from __future__ import annotations

import json
import os

import torch

from . import sht

RINGS_PER_LANE = (1, 2, 4)
RING_THREADS = (256, 512, 1024)

_cache: dict = {}


def _key(L, nside, nmaps, eps):
    return f"{L}/{nside}/{nmaps}/{eps:g}"


def time_synthesis(plan, nmaps, *, steps=5, warmup=2, path=sht.PATH_AUTO, seed=0):
    """Mean milliseconds of one synthesis of nmaps random maps."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    alm = torch.complex(torch.randn(plan.nalm, nmaps, generator=g, dtype=torch.float64),
                        torch.randn(plan.nalm, nmaps, generator=g, dtype=torch.float64)).cuda()
    out = torch.empty((nmaps, plan.npix), dtype=torch.float64, device="cuda")
    ws = plan.workspace(nmaps, path=path)
    for _ in range(warmup):
        plan.synthesis(alm, out, path=path, workspace=ws)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        plan.synthesis(alm, out, path=path, workspace=ws)
    end.record()
    end.synchronize()
    return start.elapsed_time(end) / steps


def tune(L, nside, nmaps, eps=0.0, *, steps=5, cache_file=None, verbose=False):
    """Best {"rings_per_lane", "ring_threads", "ms"} for this workload."""
    key = _key(L, nside, nmaps, eps)
    if key in _cache:
        return _cache[key]
    if cache_file and os.path.exists(cache_file):
        try:
            disk = json.load(open(cache_file))
        except ValueError:
            disk = {}
        if key in disk:
            _cache[key] = disk[key]
            return disk[key]
    best = None
    for r in RINGS_PER_LANE:
        for t in RING_THREADS:
            plan = sht.Plan(L, nside, eps, rings_per_lane=r, ring_threads=t)
            ms = time_synthesis(plan, nmaps, steps=steps)
            plan.close()
            if verbose:
                print(f"[autotune] L={L} nside={nside} B={nmaps} R={r} T={t}: {ms:.4f} ms")
            if best is None or ms < best["ms"]:
                best = {"rings_per_lane": r, "ring_threads": t, "ms": ms}
    _cache[key] = best
    if cache_file:
        disk = {}
        if os.path.exists(cache_file):
            try:
                disk = json.load(open(cache_file))
            except ValueError:
                disk = {}
        disk[key] = best
        with open(cache_file, "w") as fh:
            json.dump(disk, fh, indent=1)
    return best


def tuned_plan(L, nside, nmaps, eps=0.0, plan_eps=None, plan_kw=None, **kw):
    """A plan built with the tuned tile shape for (L, nside, nmaps, eps).

    plan_eps (default eps) and plan_kw (e.g. store_fp32) apply to the plan
    that is returned; the tile shapes are those tuned at eps, so a butterfly
    plan can reuse shapes tuned on the brute-force path."""
    best = tune(L, nside, nmaps, eps, **kw)
    return sht.Plan(L, nside, eps if plan_eps is None else plan_eps, rings_per_lane=best["rings_per_lane"],
                    ring_threads=best["ring_threads"], **(plan_kw or {}))
