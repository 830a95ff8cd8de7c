#!/usr/bin/env python
"""Throughput of HEALPix spherical harmonic synthesis on one MI355X.

Workload: L = 4095, nside = 2048 (50.3M pixels, 8191 rings), 4 maps with
seeded complex Gaussian a_lm (C_l = 1/(l+1)^2, seeds 400..403), FP64
brute-force path: Legendre phase kernel + ring FFT kernel per step.

Prints one JSON line.  `value` is maps/s of the whole step with inputs
resident in HBM.  The roofline object covers the dominant kernel (the
Legendre recurrence, FP64 vector ALU bound): algorithmic flops per launch
(5 per recurrence step + 4 per map per step, over the plan's (l, ring) pairs
above the cutoff) divided by its mean duration, measured with HIP events
recorded on the execution stream around that stage during the timed steps.
The CPU baseline times the oracle on a random sample of rings.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "L=4095 synthesis maps/s: butterfly vs brute-force, FP64 vs FP32-MFMA, max rel err"
FP64_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 FP64 flops/clk (vector FMA)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
LEGENDRE_SRC = os.path.join(ROOT, "paper_1110_4874_amd", "csrc", "legendre.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha():
    with open(LEGENDRE_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(L, nside, nmaps):
    """HBM bytes per Legendre launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and workload."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except ValueError:
        return None
    if rec.get("source_sha256") != kernel_source_sha():
        return None
    if (rec.get("L"), rec.get("nside"), rec.get("nmaps")) != (L, nside, nmaps):
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=4095)
    ap.add_argument("--nside", type=int, default=2048)
    ap.add_argument("--maps", type=int, default=4)
    ap.add_argument("--cpu-rings", type=int, default=900, help="rings in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip timing the adjoint")
    ap.add_argument("--rings-per-lane", type=int, default=0, help="Legendre kernel tile (1, 2, 4; 0 = plan default)")
    ap.add_argument("--ring-threads", type=int, default=0, help="ring kernel workgroup size (256, 512, 1024; 0 = default)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus} GPUs, WORLD_SIZE={world}); "
              "the transform is not sharded across GPUs in this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1110_4874_amd import sht
    from paper_1110_4874_amd.synthetic import alm_gaussian

    L, N, B = args.L, args.nside, args.maps
    seeds = [400 + b for b in range(B)]
    log(f"[bench] L={L} nside={N} maps={B}: drawing inputs")
    alm = alm_gaussian(L, seeds)
    log("[bench] building plan")
    t0 = time.perf_counter()
    plan = sht.Plan(L, N, rings_per_lane=args.rings_per_lane, ring_threads=args.ring_threads)
    info = plan.info()
    log(f"[bench] plan built in {time.perf_counter() - t0:.1f}s: n_step={info['n_step']:.4e} "
        f"exec={info['n_step_exec']:.4e} dd_rings={info['n_dd_rings']}")

    dev = torch.device("cuda:0")
    d_alm = torch.from_numpy(alm).to(dev)
    out = torch.empty((B, plan.npix), dtype=torch.float64, device=dev)
    ws = plan.workspace(B, dev)
    stream = torch.cuda.current_stream()

    def new_events():
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * sht.NSTAGES)]
        for e in evs:
            e.record(stream)  # materialise the HIP event
        return evs

    ev_sets = [new_events() for _ in range(args.steps)]
    torch.cuda.synchronize()

    for i in range(args.warmup):
        plan.synthesis(d_alm, out, workspace=ws)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps); timing {args.steps} steps")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        plan.synthesis(d_alm, out, workspace=ws, events=ev_sets[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    value = B * args.steps / elapsed

    leg_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev_sets]))
    ring_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in ev_sets]))
    flops = info["n_step"] * (5 + 4 * B)
    achieved = flops / (leg_ms * 1e-3) / 1e12
    log(f"[bench] {ms_per_step:.3f} ms/step, legendre {leg_ms:.3f} ms, ring {ring_ms:.3f} ms")

    # the hand-written adjoint on the same workload (reported beside the metric)
    adj = None
    if not args.no_adjoint:
        y = out.clone()
        g = torch.empty((plan.nalm, B), dtype=torch.complex128, device=dev)
        for i in range(args.warmup):
            plan.adjoint(y, g, workspace=ws)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for k in range(args.steps):
            plan.adjoint(y, g, workspace=ws, events=ev_sets[k])
        torch.cuda.synchronize()
        adj_elapsed = time.perf_counter() - ta
        ra_ms = float(np.mean([e[4].elapsed_time(e[5]) for e in ev_sets]))
        la_ms = float(np.mean([e[6].elapsed_time(e[7]) for e in ev_sets]))
        adj = {"maps_per_s": round(B * args.steps / adj_elapsed, 3),
               "ms_per_step": round(1e3 * adj_elapsed / args.steps, 4),
               "stages_ms": {"ring_analysis": round(ra_ms, 4), "legendre_adjoint": round(la_ms, 4)},
               "legendre_adjoint_tflops": round(flops / (la_ms * 1e-3) / 1e12, 3)}
        log(f"[bench] adjoint {adj['ms_per_step']:.3f} ms/step, ring analysis {ra_ms:.3f} ms, "
            f"legendre adjoint {la_ms:.3f} ms")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).normal_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {nbytes} bytes read + {nbytes} bytes written")

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"HEALPix synthesis L={L} nside={N}, {B} maps per step, brute-force FP64 "
                        "(Legendre recurrence + ring FFT)",
            "L": L, "nside": N, "maps": B, "path": "brute", "precision": "fp64",
            "spectrum": "C_l=1/(l+1)^2", "seeds": seeds,
        },
        "stages_ms": {"legendre": round(leg_ms, 4), "ring_fft": round(ring_ms, 4)},
        "roofline": {
            "kernel": "k_legendre (brute-force Legendre phase)",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": measured_traffic(L, N, B),
            "flops_per_launch": flops,
        },
    }
    if adj is not None:
        line["adjoint"] = adj

    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(0)
        nr = plan.nrings
        k = min(args.cpu_rings, nr)
        rings = np.sort(rng.choice(np.arange(1, nr + 1), size=k, replace=False))
        log(f"[bench] CPU baseline: FP64 oracle on {k} of {nr} rings, {oracle.num_threads()} threads")
        tc = time.perf_counter()
        oracle.synthesis_rings(L, N, alm, rings)
        tcpu = time.perf_counter() - tc
        full = tcpu * nr / k
        line["cpu_baseline"] = {
            "value": round(B / full, 6),
            "unit": "maps/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{k} of {nr} rings drawn uniformly (seed 0), all {B} maps, FP64 oracle "
                      f"(one-step Legendre recurrence + direct per-ring DFT); {tcpu:.1f}s measured, "
                      f"scaled by {nr}/{k}",
        }
        # accuracy of this GPU result on a few rings against the long-double oracle
        chk = [1, 2, 100, 1000, 2 * N, 2 * N + 1, 3 * N, nr]
        ref = oracle.synthesis_rings(L, N, alm, chk, ld=True)
        f = out.cpu().numpy()
        fmax = np.max(np.abs(f), axis=1)
        worst = 0.0
        for ring, r in zip(chk, ref):
            _, _, J, _, off = oracle.ring_info(N, ring)
            worst = max(worst, float(np.max(np.max(np.abs(f[:, off:off + J] - r), axis=1) / fmax)))
        line["max_rel_err"] = float(f"{worst:.3e}")
        line["max_rel_err_sample"] = f"rings {chk}, all maps, vs long-double oracle, relative to max|f| per map"
        log(f"[bench] cpu baseline {line['cpu_baseline']['value']:.4f} maps/s; max rel err {worst:.3e}")

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
