"""Autotuner for the synthesis tile shapes and the butterfly cost model.

For a workload (L, nside, nmaps, eps) and an execution path and precision it
builds one plan per candidate and times full syntheses on the GPU with events
on the execution stream, keeping the fastest:

  brute force  rings per lane of the Legendre waves x workgroup size of the
               ring FFT;
  butterfly    the cost model's rho (Sec. 3.4: stored interpolation entries
               against residual recurrence elements; FP32 level products
               stream half the bytes, so their best rho differs from FP64's),
               with the ring shape tuned on the brute-force path (the ring
               stage is the same launch on both paths).

Results are cached per process and, optionally, in a JSON file, under a key
that names the GPU architecture, the path and the precision.  Timing runs the
library's kernels only; nothing here computes any part of the transform.
"""
from __future__ import annotations

import json
import os

import torch

from . import sht

RINGS_PER_LANE = (1, 2, 4)
RING_THREADS = (256, 512, 1024)
BF_RHO = (2.0, 4.0, 6.0)

_cache: dict = {}
_PATHS = {sht.PATH_BRUTE: "brute", sht.PATH_BUTTERFLY: "butterfly"}
_PRECS = {sht.PREC_FP64: "fp64", sht.PREC_FP32: "fp32"}


def arch() -> str:
    """GPU architecture of device 0 (e.g. "gfx950"), "none" without a GPU."""
    if not torch.cuda.is_available():
        return "none"
    name = getattr(torch.cuda.get_device_properties(0), "gcnArchName", "") or "unknown"
    return name.split(":")[0]


def _resolve(eps, path, precision):
    if path == sht.PATH_AUTO:
        path = sht.PATH_BUTTERFLY if eps > 0 else sht.PATH_BRUTE
    if path not in _PATHS:
        raise ValueError(f"no tuning for path {path}")
    if path == sht.PATH_BRUTE:
        precision = sht.PREC_FP64  # the brute-force recurrence runs in FP64 only
    if precision not in _PRECS:
        raise ValueError(f"unknown precision {precision}")
    if path == sht.PATH_BUTTERFLY and not eps > 0:
        raise ValueError("the butterfly path needs eps > 0")
    return path, precision


def _key(L, nside, nmaps, eps, path=sht.PATH_BRUTE, precision=sht.PREC_FP64):
    return f"{arch()}/{_PATHS[path]}/{_PRECS[precision]}/{L}/{nside}/{nmaps}/{eps:g}"


def candidates(path, ring_shape=None):
    """Plan keyword sets swept for a path (ring_shape: the tuned brute-force
    ring shape, which the butterfly candidates keep)."""
    if path == sht.PATH_BRUTE:
        return [{"rings_per_lane": r, "ring_threads": t} for r in RINGS_PER_LANE for t in RING_THREADS]
    base = dict(ring_shape or {})
    return [dict(base, rho=rho) for rho in BF_RHO]


def time_synthesis(plan, nmaps, *, steps=5, warmup=2, path=sht.PATH_AUTO, precision=sht.PREC_FP64, seed=0):
    """Mean milliseconds of one synthesis of nmaps random maps."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    alm = torch.complex(torch.randn(plan.nalm, nmaps, generator=g, dtype=torch.float64),
                        torch.randn(plan.nalm, nmaps, generator=g, dtype=torch.float64)).cuda()
    out = torch.empty((nmaps, plan.npix), dtype=torch.float64, device="cuda")
    ws = plan.workspace(nmaps, path=path, precision=precision)
    for _ in range(warmup):
        plan.synthesis(alm, out, path=path, workspace=ws, precision=precision)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        plan.synthesis(alm, out, path=path, workspace=ws, precision=precision)
    end.record()
    end.synchronize()
    return start.elapsed_time(end) / steps


def _load_disk(cache_file):
    if cache_file and os.path.exists(cache_file):
        try:
            return json.load(open(cache_file))
        except ValueError:
            return {}
    return {}


def tune(L, nside, nmaps, eps=0.0, *, path=sht.PATH_AUTO, precision=sht.PREC_FP64, plan_kw=None, steps=5,
         cache_file=None, verbose=False):
    """Best plan keywords for this workload, path and precision, with the time
    in ms: {"rings_per_lane", "ring_threads", "ms"} on the brute-force path,
    those plus "rho" on the butterfly path.  plan_kw (e.g. store_fp32, needed
    to time FP32 level products) is passed to every candidate plan."""
    path, precision = _resolve(eps, path, precision)
    key = _key(L, nside, nmaps, eps, path, precision)
    if key in _cache:
        return _cache[key]
    disk = _load_disk(cache_file)
    if key in disk:
        _cache[key] = disk[key]
        return disk[key]
    ring_shape = None
    if path == sht.PATH_BUTTERFLY:
        shape = tune(L, nside, nmaps, 0.0, path=sht.PATH_BRUTE, steps=steps, cache_file=cache_file, verbose=verbose)
        ring_shape = {k: v for k, v in shape.items() if k != "ms"}
    kw = dict(plan_kw or {})
    if path == sht.PATH_BUTTERFLY and precision == sht.PREC_FP32:
        kw["store_fp32"] = True
    best = None
    for cand in candidates(path, ring_shape):
        plan = sht.Plan(L, nside, eps, **cand, **kw)
        ms = time_synthesis(plan, nmaps, steps=steps, path=path, precision=precision)
        plan.close()
        if verbose:
            print(f"[autotune] {key} {cand}: {ms:.4f} ms")
        if best is None or ms < best["ms"]:
            best = dict(cand, ms=ms)
    _cache[key] = best
    if cache_file:
        disk = _load_disk(cache_file)
        disk[key] = best
        with open(cache_file, "w") as fh:
            json.dump(disk, fh, indent=1)
    return best


def tuned_plan(L, nside, nmaps, eps=0.0, plan_eps=None, plan_kw=None, *, path=sht.PATH_AUTO,
               precision=sht.PREC_FP64, **kw):
    """A plan built with the keywords tuned for (L, nside, nmaps, eps, path,
    precision).

    plan_eps (default eps) and plan_kw (e.g. store_fp32) apply to the plan
    that is returned; with plan_eps > 0 and a brute-force tuning (eps = 0)
    the butterfly part keeps the default cost model."""
    best = tune(L, nside, nmaps, eps, path=path, precision=precision, plan_kw=plan_kw, **kw)
    knobs = {k: v for k, v in best.items() if k != "ms"}
    pkw = dict(plan_kw or {})
    if _resolve(eps, path, precision) == (sht.PATH_BUTTERFLY, sht.PREC_FP32):
        pkw["store_fp32"] = True
    return sht.Plan(L, nside, eps if plan_eps is None else plan_eps, **knobs, **pkw)
