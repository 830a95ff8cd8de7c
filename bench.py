#!/usr/bin/env python
"""Throughput of HEALPix spherical harmonic synthesis on one MI355X.

Workload: L = 4095, nside = 2048 (50.3M pixels, 8191 rings), 4 maps with
seeded complex Gaussian a_lm (C_l = 1/(l+1)^2, seeds 400..403).  One plan
(eps = 1e-12) holds both Legendre forms; each step is one synthesis of the
4 maps (Legendre phase + ring FFT) with inputs resident in HBM:
  brute      FP64 two-step recurrence over every (l, ring) above the cutoff
  bf64       butterfly-compressed operator, FP64 products
  bf32       butterfly-compressed operator, FP32 matrix-core products
The headline `value` is the fastest FP64 path (maps/s over exactly --steps
steps bracketed by device synchronisation); the other paths are timed the
same way and reported under "paths".  Under "adjoint", every path is also
timed on the map-fitting gradient: forward + backward of
||synthesis(a) - d||^2 through autograd, whose backward is the hand-written
adjoint of the same path, and on the adjoint alone.  Under "analysis", every
path runs the quadrature analysis (weight 4 pi / Npix) of the synthesized maps,
without and with 3 Jacobi refinement steps.  The roofline object covers the
dominant kernel of the headline path, measured with HIP events recorded on
the execution stream around its stage.  The CPU baseline times the oracle on
a random sample of rings; max_rel_err compares each path with the oracle's
long-double mode on sampled rings.
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
FP64_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz (vector FMA)
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters.json")
CSRC = os.path.join(ROOT, "paper_1110_4874_amd", "csrc")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _code_only(text):
    """Source text without comments and blank space, so that editing a
    comment does not count as changing a kernel."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.strip() for line in text.splitlines() if line.strip())


def source_sha(src):
    """Hash of a kernel source file together with every header of the
    library (its constants and shared device code), comments excluded."""
    if not src or not os.path.exists(os.path.join(CSRC, src)):
        return None
    names = [src] + sorted(n for n in os.listdir(CSRC) if n.endswith(".h"))
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(CSRC, n)) as fh:
            h.update(n.encode() + b"\0" + _code_only(fh.read()).encode() + b"\0")
    return h.hexdigest()


def _profile_record(path, kernel, L, nside, nmaps, t_entries=None):
    """The record of `kernel` in a committed rocprofv3 summary, if it was
    taken on the current kernel source and workload (and, for butterfly
    kernels, on a plan with the same number of dense entries)."""
    if not os.path.exists(path):
        return None
    try:
        recs = json.load(open(path)).get("records", [])
    except (ValueError, AttributeError):
        return None
    for rec in recs:
        if not rec.get("kernel", "").startswith(kernel):
            continue
        if rec.get("source_sha256") != source_sha(rec.get("source", "")):
            return None
        if (rec.get("L"), rec.get("nside"), rec.get("nmaps")) != (L, nside, nmaps):
            return None
        if t_entries is not None and rec.get("plan_T_entries") not in (None, t_entries):
            return None
        return rec
    return None


def measured_traffic(kernel, L, nside, nmaps, t_entries=None):
    """HBM bytes per launch of `kernel` (FETCH_SIZE and WRITE_SIZE, scaled by
    the same counters' reading of a 1 GiB copy)."""
    rec = _profile_record(TRAFFIC_FILE, kernel, L, nside, nmaps, t_entries)
    return rec.get("bytes_per_launch") if rec else None


def measured_counters(kernel, L, nside, nmaps, t_entries=None):
    """FP64 rate and matrix-core use of `kernel` from the committed counter
    pass (FP64 VALU and MFMA instruction counts, MFMA busy cycles)."""
    rec = _profile_record(COUNTERS_FILE, kernel, L, nside, nmaps, t_entries)
    if not rec:
        return None
    return {k: rec.get(k) for k in ("mean_duration_ms", "fp64_tflops", "fp64_frac", "mfma_busy_frac",
                                    "fp64_valu_flops", "fp64_mfma_flops", "fp32_mfma_flops")}


def batch_bench(np, torch, sht, steps):
    """64 queued syntheses of mixed L in {127, 255, 511, 1023}, nside =
    (L+1)/2, 1-8 maps each (seed 500): one batch call (and its captured HIP
    graph) against 64 sequential calls, with tuned plans: FP64 brute force
    (tuned tile shapes), then butterfly plans (eps 1e-12, depth from the cost
    model with rho tuned per precision) with FP64 and FP32 matrix-core level
    products."""
    from paper_1110_4874_amd import autotune
    from paper_1110_4874_amd.synthetic import alm_gaussian, mixed_requests

    queue = mixed_requests(seed=500, n=64)
    inputs = []
    for (L, N, B, seeds) in queue:
        alm = torch.from_numpy(alm_gaussian(L, seeds)).cuda()
        out = torch.empty((B, 12 * N * N), dtype=torch.float64, device="cuda")
        inputs.append((L, N, alm, out))
    nmaps = sum(x[2].shape[1] for x in inputs)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - ts) / k

    def run_config(plans, path, prec):
        reqs = [(plans[(L, N)], alm, out) for (L, N, alm, out) in inputs]
        wss = {id(p): p.workspace(max(r[1].shape[1] for r in reqs if r[0] is p), path=path, precision=prec)
               for p in plans.values()}
        batch = sht.Batch(reqs, path=path, precision=prec)

        def seq():
            for p, a, o in reqs:
                p.synthesis(a, o, workspace=wss[id(p)], path=path, precision=prec)

        t_seq = timed(seq, steps)
        t_batch = timed(batch.run, steps)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            batch.run(stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            batch.run(stream=torch.cuda.current_stream())
        t_graph = timed(g.replay, steps)
        # the graph's results equal the sequential calls'
        ref = [o.clone() for _, _, o in reqs]
        seq()
        torch.cuda.synchronize()
        same = all(torch.equal(o, r) for (_, _, o), r in zip(reqs, ref))
        return {"sequential_maps_per_s": round(nmaps / t_seq, 2), "batch_maps_per_s": round(nmaps / t_batch, 2),
                "graph_maps_per_s": round(nmaps / t_graph, 2),
                "graph_speedup_vs_sequential": round(t_seq / t_graph, 3), "graph_matches_sequential": bool(same)}

    def run_queue(plans, path=sht.PATH_BRUTE, prec=sht.PREC_FP64):
        # work-queue form: on the brute-force path one persistent Legendre
        # launch per wave shape over every request's items; on the butterfly
        # path one launch per stage and map-group width over every request;
        # then one ring launch per ring size class; replayed as a graph.  The
        # tile shape (rings per lane, ring workgroup size) is swept and the
        # fastest graph is reported.
        reqs = [(plans[(L, N)], alm, out) for (L, N, alm, out) in inputs]
        seq_ref = []
        for p, a, o in reqs:
            p.synthesis(a, o, path=path, precision=prec)
            seq_ref.append(o.clone())
        rpls = (1, 2, 4) if path == sht.PATH_BRUTE else (2,)
        sweep, best = {}, None
        for rpl in rpls:
            for thr in (256, 512, 1024):
                qb = sht.QueueBatch(reqs, path=path, precision=prec, rings_per_lane=rpl, ring_threads=thr)
                t_run = timed(qb.run, steps)
                s = torch.cuda.Stream()
                s.wait_stream(torch.cuda.current_stream())
                g = torch.cuda.CUDAGraph()
                with torch.cuda.stream(s):
                    with torch.cuda.graph(g, stream=s):
                        qb.run(stream=s)
                torch.cuda.current_stream().wait_stream(s)
                t_graph = timed(g.replay, steps)
                torch.cuda.synchronize()
                # the ring stage's twiddle stepping depends on the workgroup
                # size, so shapes other than the plans' agree to rounding
                diff = max(float((o - r).abs().max() / r.abs().max()) for (_, _, o), r in zip(reqs, seq_ref))
                st = qb.stats()
                qb.close()
                del g
                key = f"rpl{rpl}_t{thr}" if path == sht.PATH_BRUTE else f"t{thr}"
                sweep[key] = round(nmaps / t_graph, 1)
                r = {"run_maps_per_s": round(nmaps / t_run, 2), "graph_maps_per_s": round(nmaps / t_graph, 2),
                     "work_items": st["items"], "launches_per_run": st["launches"],
                     "max_rel_diff_vs_sequential": diff, "rings_per_lane": rpl, "ring_threads": thr}
                if path == sht.PATH_BRUTE:
                    r["persistent_waves"] = st["waves"]
                if not diff <= 1e-12:
                    raise RuntimeError(f"work-queue batch {key} differs from the sequential calls by {diff:.3e}")
                if best is None or r["graph_maps_per_s"] > best["graph_maps_per_s"]:
                    best = r
        best["sweep_graph_maps_per_s"] = sweep
        return best

    # tile shapes and cost model tuned per path and precision at 4 maps per
    # request (the ring shape on the brute-force path, rho on the butterfly
    # path for FP64 and FP32 level products separately)
    t0 = time.perf_counter()
    shapes = sorted({(L, N) for (L, N, _, _) in inputs})
    plans = {(L, N): autotune.tuned_plan(L, N, 4) for (L, N) in shapes}
    bf_plans = {prec: {(L, N): autotune.tuned_plan(L, N, 4, 1e-12, path=sht.PATH_BUTTERFLY, precision=prec,
                                                   plan_kw={"store_fp32": True}) for (L, N) in shapes}
                for prec in (sht.PREC_FP64, sht.PREC_FP32)}
    tune_s = time.perf_counter() - t0

    def shape(L, N, eps=0.0, path=sht.PATH_BRUTE, prec=sht.PREC_FP64):
        return {k: v for k, v in autotune.tune(L, N, 4, eps, path=path, precision=prec).items() if k != "ms"}

    res = {"requests": len(inputs), "maps": nmaps, "tuning_seconds": round(tune_s, 1), "arch": autotune.arch(),
           "tile_shapes": {f"{L}": {"brute_fp64": shape(L, N),
                                    "butterfly_fp64": shape(L, N, 1e-12, sht.PATH_BUTTERFLY, sht.PREC_FP64),
                                    "butterfly_fp32": shape(L, N, 1e-12, sht.PATH_BUTTERFLY, sht.PREC_FP32)}
                           for (L, N) in shapes},
           "brute_fp64": run_config(plans, sht.PATH_BRUTE, sht.PREC_FP64)}
    res["queue_brute_fp64"] = run_queue(plans)
    log(f"[bench] batching queue_brute_fp64: run {res['queue_brute_fp64']['run_maps_per_s']} maps/s, graph "
        f"{res['queue_brute_fp64']['graph_maps_per_s']} ({res['queue_brute_fp64']['launches_per_run']} launches)")
    res["butterfly_depth_hist"] = {f"{L}": p.info()["bf_depth_hist"][:6]
                                   for (L, _), p in bf_plans[sht.PREC_FP64].items()}
    res["butterfly_fp64"] = run_config(bf_plans[sht.PREC_FP64], sht.PATH_BUTTERFLY, sht.PREC_FP64)
    res["butterfly_fp32"] = run_config(bf_plans[sht.PREC_FP32], sht.PATH_BUTTERFLY, sht.PREC_FP32)
    for k, prec in (("queue_butterfly_fp64", sht.PREC_FP64), ("queue_butterfly_fp32", sht.PREC_FP32)):
        res[k] = run_queue(bf_plans[prec], sht.PATH_BUTTERFLY, prec)
        log(f"[bench] batching {k}: run {res[k]['run_maps_per_s']} maps/s, graph {res[k]['graph_maps_per_s']} "
            f"({res[k]['launches_per_run']} launches)")
    for p in list(plans.values()) + [q for d in bf_plans.values() for q in d.values()]:
        p.close()
    for k in ("brute_fp64", "butterfly_fp64", "butterfly_fp32"):
        log(f"[bench] batching {k}: sequential {res[k]['sequential_maps_per_s']} maps/s, "
            f"batch {res[k]['batch_maps_per_s']}, graph {res[k]['graph_maps_per_s']}")
    return res


def level_roofline(info, nlev, sz, B, levels_ms, L, N):
    """Roofline of the butterfly level launches (levels >= 2; level 1 runs
    fused with the fold).  Algorithmic bytes per launch are what the method
    must stream once per pass: the dense interpolation entries of the level
    (sz bytes each) plus their index data (a 64-byte record and 2 n int16
    column positions per pair node).  The vectors passed between levels
    (child vectors read, parent vectors written, 2 B values per column) are
    an artefact of running one launch per level and are reported apart as
    intermediate_bytes_per_launch."""
    lvls = range(2, nlev + 1)
    nl = max(nlev - 1, 1)
    alg = sum(info["bf_level_T"][i] * sz + 64 * info["bf_level_nodes"][i] + 4 * info["bf_level_units"][i]
              for i in lvls) / nl
    inter = sum(2 * info["bf_level_units"][i] * 2 * B * sz for i in lvls) / nl
    launch_ms = levels_ms / nl
    achieved = alg / (launch_ms * 1e-3) / 1e9
    nb = 8 if B >= 8 else 4 if B >= 4 else 2 if B >= 2 else 1
    kern = "void sht::k_bf_level<%d, %s, true>(" % (nb, "double" if sz == 8 else "float")
    return {"kernel": f"k_bf_level ({nl} launches per pass, one per level 2..{nlev})", "bound": "hbm",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kern, L, N, B, info["bf_T_entries"]),
            "counters": measured_counters(kern, L, N, B, info["bf_T_entries"]),
            "bytes_per_launch": int(alg),
            "intermediate_bytes_per_launch": int(inter), "launch_ms": round(launch_ms, 4),
            "with_intermediate_GBs": round((alg + inter) / (launch_ms * 1e-3) / 1e9, 1)}


def rms_err(np, y, x):
    """RMS relative error of Sec. 4.2 (Eq. 24), worst over maps (rows)."""
    return max(float(np.sqrt(np.sum((y[b] - x[b]) ** 2) / np.sum(x[b] ** 2))) for b in range(x.shape[0]))


def sampled_errors(np, oracle, L, N, alm, maps_by_path, rings):
    """max rel and RMS error of each path on the listed rings against the
    long-double oracle (relative to the oracle's max on the same rings)."""
    ref = np.concatenate(oracle.synthesis_rings(L, N, alm, rings, ld=True), axis=1)
    out = {}
    for name, f in maps_by_path.items():
        y = np.concatenate([f[:, oracle.ring_info(N, r)[4]:oracle.ring_info(N, r)[4] + oracle.ring_info(N, r)[2]]
                            for r in rings], axis=1)
        mx = max(float(np.max(np.abs(y[b] - ref[b])) / np.max(np.abs(ref[b]))) for b in range(ref.shape[0]))
        out[name] = {"max_rel_err": float(f"{mx:.3e}"), "rms_eps": float(f"{rms_err(np, y, ref):.3e}")}
    return out


def timed_paths(np, torch, sht, plan, d_alm, paths, steps, warmup):
    """Synthesis of every path over `steps` steps with stage events; returns
    per-path timings and the last output maps (host)."""
    B = d_alm.shape[1]
    dev = d_alm.device
    out = torch.empty((B, plan.npix), dtype=torch.float64, device=dev)
    big = max(plan.workspace_bytes(B, path=p, precision=q) for _, p, q in paths)
    ws = torch.empty(big, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    evs = []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2 * sht.NSTAGES)]
        for x in e:
            x.record(stream)
        evs.append(e)
    res, maps = {}, {}
    for name, path, prec in paths:
        for _ in range(warmup):
            plan.synthesis(d_alm, out, path=path, precision=prec, workspace=ws)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(steps):
            plan.synthesis(d_alm, out, path=path, precision=prec, workspace=ws, events=evs[k])
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        r = {"maps_per_s": round(B * steps / el, 3), "ms_per_step": round(1e3 * el / steps, 4),
             "legendre_ms": round(float(np.mean([e[0].elapsed_time(e[1]) for e in evs])), 4),
             "ring_ms": round(float(np.mean([e[2].elapsed_time(e[3]) for e in evs])), 4)}
        if path == sht.PATH_BUTTERFLY:
            s8, s10 = 2 * sht.STAGE_BF_RESIDUAL, 2 * sht.STAGE_BF_LEVELS
            r["residual_ms"] = round(float(np.mean([e[s8].elapsed_time(e[s8 + 1]) for e in evs])), 4)
            r["levels_ms"] = round(float(np.mean([e[s10].elapsed_time(e[s10 + 1]) for e in evs])), 4)
        res[name] = r
        maps[name] = out.cpu().numpy()
    del ws, out
    return res, maps


def many_map_bench(np, torch, sht, plan, info, args, ref_maps):
    """Many maps per step at the headline size (the many-transform regime of
    Sec. 3.4): one pass of the butterfly kernels takes up to 64 maps in
    groups of 8, so the interpolation matrices stream from HBM once per pass
    instead of once per 8 maps.  Seeds 400.. (the first four maps are the
    headline's, and must come out identical to it)."""
    from paper_1110_4874_amd.synthetic import alm_gaussian
    L, N = plan.L, plan.nside
    nlev = max([d for d, c in enumerate(info["bf_depth_hist"]) if c > 0] + [0])
    out = {}
    for B in args.many_maps:
        need = max(plan.workspace_bytes(B, path=sht.PATH_BUTTERFLY), plan.workspace_bytes(B, path=sht.PATH_BRUTE)) \
            + B * (plan.npix * 8 + plan.nalm * 16)
        free = torch.cuda.mem_get_info()[0]
        if need > 0.85 * free:
            out[str(B)] = {"skipped": f"needs {need / 1e9:.1f} GB of device memory, {free / 1e9:.1f} GB free"}
            log(f"[bench] many maps B={B}: skipped ({out[str(B)]['skipped']})")
            continue
        d_alm = torch.from_numpy(alm_gaussian(L, [400 + b for b in range(B)])).cuda()
        paths = [("brute", sht.PATH_BRUTE, sht.PREC_FP64), ("bf64", sht.PATH_BUTTERFLY, sht.PREC_FP64),
                 ("bf32", sht.PATH_BUTTERFLY, sht.PREC_FP32)]
        steps = max(2, min(args.steps, 5))
        res, maps = timed_paths(np, torch, sht, plan, d_alm, paths, steps, 1)
        passes = -(-B // 64)
        for name in res:
            r = res[name]
            r["speedup_vs_brute"] = round(r["maps_per_s"] / res["brute"]["maps_per_s"], 3)
            if name in ref_maps:
                k = min(B, ref_maps[name].shape[0])
                r["first_maps_equal_headline"] = bool(np.array_equal(maps[name][:k], ref_maps[name][:k]))
            if name != "brute":
                sz = 8 if name == "bf64" else 4
                r["interp_bytes_per_map"] = int(info["bf_T_entries"] * sz * passes / B)
                if nlev >= 2 and B <= 64:
                    r["level_roofline"] = level_roofline(info, nlev, sz, B, r["levels_ms"], L, N)
        out[str(B)] = {"maps": B, "steps": steps, "passes": passes, "paths": res}
        log(f"[bench] many maps B={B}: " + ", ".join(f"{n} {res[n]['maps_per_s']:.1f} maps/s" for n in res))
        del d_alm, maps
        torch.cuda.empty_cache()
    return out


def config3_bench(np, torch, sht, args):
    """16 maps at L = 2047, nside = 1024 (seeds 300..315): brute FP64 and the
    butterfly as a multi-map product in FP64 and FP32 (eps 1e-12), with the
    errors of each against the long-double oracle on sampled rings."""
    import oracle
    from paper_1110_4874_amd.synthetic import alm_gaussian
    L, N, B = 2047, 1024, 16
    plan = sht.cached_plan(L, N, 1e-12, store_fp32=True, log=log)
    info = plan.info()
    alm = alm_gaussian(L, list(range(300, 300 + B)))
    d_alm = torch.from_numpy(alm).cuda()
    paths = [("brute", sht.PATH_BRUTE, sht.PREC_FP64), ("bf64", sht.PATH_BUTTERFLY, sht.PREC_FP64),
             ("bf32", sht.PATH_BUTTERFLY, sht.PREC_FP32)]
    res, maps = timed_paths(np, torch, sht, plan, d_alm, paths, args.steps, args.warmup)
    errs = sampled_errors(np, oracle, L, N, alm, maps, [1, 2, 120, 400, N, 2 * N, 3 * N, 4 * N - 1])
    nlev = max([d for d, c in enumerate(info["bf_depth_hist"]) if c > 0] + [0])
    for name in res:
        res[name].update(errs[name])
        res[name]["speedup_vs_brute"] = round(res[name]["maps_per_s"] / res["brute"]["maps_per_s"], 3)
        if name != "brute" and nlev >= 2:
            res[name]["level_roofline"] = level_roofline(info, nlev, 8 if name == "bf64" else 4, B,
                                                         res[name]["levels_ms"], L, N)
    log("[bench] L=2047 B=16: " + ", ".join(f"{n} {res[n]['maps_per_s']:.1f} maps/s (err {res[n]['max_rel_err']:.1e})"
                                          for n in res))
    out = {"workload": "HEALPix synthesis L=2047 nside=1024, 16 maps per step", "steps": args.steps,
           "T_entries": info["bf_T_entries"], "depth_hist": info["bf_depth_hist"][:6], "paths": res}
    plan.close()
    del d_alm
    torch.cuda.empty_cache()
    return out


def interp_bench(np, torch, sht, args, d_alm, alm, brute):
    """The interpolation form of Sec. 3.3 at the headline size: the Legendre
    phase at the roots of P~_N^m (about a third of the brute-force chain
    steps), then the exact interpolation to the rings (Eq. 23) as a Cauchy
    product on the FP64 matrix cores; timed like the other paths, with its
    error against the long-double oracle on sampled rings."""
    import oracle
    L, N = 4095, 2048
    if d_alm.shape[0] != (L + 1) * (L + 2) // 2:
        return None
    plan = sht.cached_plan(L, N, 0.0, interp=True, log=log)
    info = plan.info()
    res, maps = timed_paths(np, torch, sht, plan, d_alm, [("interp", sht.PATH_INTERP, sht.PREC_FP64)],
                            args.steps, args.warmup)
    r = res["interp"]
    r.update(sampled_errors(np, oracle, L, N, alm, maps, [1, 2, 100, 250, 251, 1000, 2 * N, 2 * N + 1, 3 * N,
                                                          4 * N - 1])["interp"])
    r["speedup_vs_brute"] = round(r["maps_per_s"] / brute["maps_per_s"], 3)
    r["node_steps"] = info["ip_steps"]
    r["brute_steps"] = info["n_step"]
    r["nodes"] = info["ip_nodes"]
    r["precompute_seconds"] = round(info["ip_build_seconds"], 1)
    log(f"[bench] interp: {r['maps_per_s']:.1f} maps/s ({r['speedup_vs_brute']}x brute), legendre "
        f"{r['legendre_ms']:.3f} ms, error {r['max_rel_err']:.2e}")
    plan.close()
    torch.cuda.empty_cache()
    return r


def pol_bench(np, torch, sht, plan, args):
    """Polarized synthesis (the Discussion's reduction to scalar transforms)
    with the headline plan: E and B of band limit L - 1 (seeds 900, 901, the
    headline spectrum), one polarized map per step = six scalar maps through
    one Legendre phase plus Q and U through the ring stage; brute force and
    FP64 butterfly, with the error against the long-double oracle on sampled
    rings (the polar caps on both sides of the direct-recurrence threshold)."""
    import oracle
    from paper_1110_4874_amd.synthetic import alm_gaussian
    L, N = plan.L, plan.nside
    E = alm_gaussian(L - 1, [900])
    B = alm_gaussian(L - 1, [901])
    dE, dB = torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda()
    npol = plan.info()["pol_rings"]
    rings = sorted(set(r for r in [1, 2, npol, npol + 1, N // 2, N, 2 * N, 3 * N, 4 * N - 1 - npol, 4 * N - 1]
                       if 1 <= r <= 4 * N - 1))
    t0 = time.perf_counter()
    rq, ru = oracle.pol_synthesis_rings(L - 1, N, E, B, rings, ld=True)
    log(f"[bench] polarization oracle (long double) on {len(rings)} rings: {time.perf_counter() - t0:.1f} s")
    res = {"band_limit": L - 1, "polar_rings": npol, "rings_checked": rings}
    paths = [("brute", sht.PATH_BRUTE)] + ([("bf64", sht.PATH_BUTTERFLY)] if plan.info()["bf_built"] else [])
    for name, path in paths:
        ws = torch.empty(plan.pol_workspace_bytes(1, path), dtype=torch.uint8, device="cuda")
        out = torch.empty((2, 1, plan.npix), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            plan.pol_synthesis(dE, dB, out, path=path, workspace=ws)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(args.steps):
            plan.pol_synthesis(dE, dB, out, path=path, workspace=ws)
        torch.cuda.synchronize()
        el = (time.perf_counter() - ts) / args.steps
        f = out.cpu().numpy()
        ys = np.concatenate([np.concatenate([f[c][:, oracle.ring_info(N, r)[4]:oracle.ring_info(N, r)[4] +
                                                   oracle.ring_info(N, r)[2]] for r in rings], axis=1)
                             for c in (0, 1)], axis=1)
        xs = np.concatenate([np.concatenate(rq, axis=1), np.concatenate(ru, axis=1)], axis=1)
        err = float(np.max(np.abs(ys - xs)) / np.max(np.abs(xs)))
        res[name] = {"pol_maps_per_s": round(1.0 / el, 3), "ms_per_step": round(1e3 * el, 4),
                     "max_rel_err": err}
        log(f"[bench] polarization {name}: {1e3 * el:.3f} ms per Q/U map pair, error {err:.2e}")
        del ws, out
    torch.cuda.empty_cache()
    return res


def gradient_bench(np, torch, sht, plan, info, paths, d_alm, f_true, ws, ev_sets, args, flops):
    """Forward + backward of the map-fitting loss ||synthesis(a) - d||^2 per path.

    d = synthesis(a_true) + white noise of sigma = 0.1 rms (seeds 410..),
    evaluated at a = a_true + 0.1 * (draw of seed 420, same spectrum); the
    backward is the hand-written adjoint of the same path and precision
    (autograd through synthesis_fn).  Also times the adjoint alone with its
    two stages, and compares each path's gradient with the brute-force one.
    """
    from paper_1110_4874_amd.synthetic import alm_gaussian, gaussian_map
    B = f_true.shape[0]
    L, dev = plan.L, d_alm.device
    sig = 0.1 * np.sqrt(np.mean(f_true ** 2, axis=1))
    d = torch.from_numpy(f_true + gaussian_map(plan.npix, [410 + b for b in range(B)], sig)).to(dev)
    pert = torch.from_numpy(alm_gaussian(L, [420] * B)).to(dev)
    a0 = (d_alm + 0.1 * pert).detach()
    out = {"loss_at_zero": None, "paths": {}}
    with torch.no_grad():
        out["loss_at_zero"] = float((d ** 2).sum())
    grads = {}
    g = torch.empty((plan.nalm, B), dtype=torch.complex128, device=dev)
    for name, path, prec in paths:
        a = a0.clone().requires_grad_(True)

        def step():
            a.grad = None
            f = sht.synthesis_fn(plan, a, path=path, precision=prec)
            loss = ((f - d) ** 2).sum()
            loss.backward()
            return loss

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(args.steps):
            loss = step()
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        grads[name] = a.grad.detach().cpu().numpy()
        # adjoint alone, with stage events
        y = d.clone()
        for _ in range(args.warmup):
            plan.adjoint(y, g, workspace=ws, path=path, precision=prec)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for k in range(args.steps):
            plan.adjoint(y, g, workspace=ws, path=path, precision=prec, events=ev_sets[k])
        torch.cuda.synchronize()
        adj_el = time.perf_counter() - ta
        ra_ms = float(np.mean([e[4].elapsed_time(e[5]) for e in ev_sets]))
        la_ms = float(np.mean([e[6].elapsed_time(e[7]) for e in ev_sets]))
        rec = {"fwd_bwd_ms_per_step": round(1e3 * el / args.steps, 4),
               "fwd_bwd_maps_per_s": round(B * args.steps / el, 3),
               "loss": float(loss),
               "adjoint_ms_per_step": round(1e3 * adj_el / args.steps, 4),
               "adjoint_maps_per_s": round(B * args.steps / adj_el, 3),
               "adjoint_stages_ms": {"ring_analysis": round(ra_ms, 4), "legendre_adjoint": round(la_ms, 4)}}
        if name == "brute":
            rec["legendre_adjoint_tflops"] = round(flops / (la_ms * 1e-3) / 1e12, 3)
        out["paths"][name] = rec
        log(f"[bench] gradient {name}: fwd+bwd {rec['fwd_bwd_ms_per_step']:.3f} ms/step, adjoint "
            f"{rec['adjoint_ms_per_step']:.3f} ms (ring analysis {ra_ms:.3f}, Legendre {la_ms:.3f})")
    gb = grads["brute"]
    for name in grads:
        if name == "brute":
            continue
        err = max(float(np.max(np.abs(grads[name][:, b] - gb[:, b])) / np.max(np.abs(gb[:, b])))
                  for b in range(B))
        out["paths"][name]["grad_max_rel_vs_brute"] = float(f"{err:.3e}")
        out["paths"][name]["adjoint_speedup_vs_brute"] = round(
            out["paths"]["brute"]["adjoint_ms_per_step"] / out["paths"][name]["adjoint_ms_per_step"], 3)
    return out


def analysis_bench(np, torch, sht, plan, paths, d_alm, f_true, args):
    """Quadrature analysis with Jacobi refinement (sht_analysis_ex) per path.

    The maps are the benchmark's own syntheses of a_true, so the error against
    a_true shows what the Jacobi steps recover on a band-limited map at
    L = 2 nside - 1.  Timed with iterations = 0 (one adjoint) and 3."""
    B = f_true.shape[0]
    dev = d_alm.device
    f = torch.from_numpy(f_true).to(dev)
    a_true = d_alm.cpu().numpy()
    steps = max(1, min(args.steps, 5))
    out = {"weight": "4 pi / Npix", "steps": steps, "paths": {}}
    for name, path, prec in paths:
        ws = plan.analysis_workspace(B, dev, path, prec)
        a = torch.empty((plan.nalm, B), dtype=torch.complex128, device=dev)
        rec = {}
        for iters in (0, 3):
            plan.analysis(f, a, iterations=iters, path=path, precision=prec, workspace=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.analysis(f, a, iterations=iters, path=path, precision=prec, workspace=ws)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            an = a.cpu().numpy()
            err = max(float(np.max(np.abs(an[:, b] - a_true[:, b])) / np.max(np.abs(a_true[:, b])))
                      for b in range(B))
            rec[f"iterations_{iters}"] = {"ms": round(1e3 * el, 3), "maps_per_s": round(B / el, 3),
                                          "max_rel_err_vs_alm": float(f"{err:.3e}")}
        out["paths"][name] = rec
        log(f"[bench] analysis {name}: {rec['iterations_0']['ms']:.3f} ms (no refinement, error "
            f"{rec['iterations_0']['max_rel_err_vs_alm']:.2e}), {rec['iterations_3']['ms']:.3f} ms with 3 Jacobi "
            f"steps (error {rec['iterations_3']['max_rel_err_vs_alm']:.2e})")
        del ws
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=4095)
    ap.add_argument("--nside", type=int, default=2048)
    ap.add_argument("--maps", type=int, default=4)
    ap.add_argument("--eps", type=float, default=1e-12, help="butterfly tolerance (0: brute force only)")
    ap.add_argument("--rho", type=float, default=0.0, help="butterfly depth cost ratio (0: plan default)")
    ap.add_argument("--cpu-rings", type=int, default=900, help="rings in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip timing the adjoint")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-request batching measurement")
    ap.add_argument("--no-analysis", action="store_true", help="skip timing the quadrature analysis")
    ap.add_argument("--many-maps", type=int, nargs="*", default=[16, 64],
                    help="also time these map counts at the headline size (one pass of up to 64 maps)")
    ap.add_argument("--no-config3", action="store_true", help="skip the 16-map L=2047 measurement")
    ap.add_argument("--no-interp", action="store_true", help="skip the interpolation-form measurement")
    ap.add_argument("--no-pol", action="store_true", help="skip the polarized-synthesis measurement")
    ap.add_argument("--rings-per-lane", type=int, default=0, help="Legendre kernel tile (1, 2, 4; 0 = plan default)")
    ap.add_argument("--ring-threads", type=int, default=0, help="ring kernel workgroup size (256, 512, 1024; 0 = default)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus} GPUs, WORLD_SIZE={world}); "
              "the library does not shard a transform across GPUs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1110_4874_amd import sht
    from paper_1110_4874_amd.synthetic import alm_gaussian

    L, N, B = args.L, args.nside, args.maps
    seeds = [400 + b for b in range(B)]
    log(f"[bench] L={L} nside={N} maps={B}: drawing inputs")
    alm = alm_gaussian(L, seeds)
    log(f"[bench] plan (eps={args.eps}): from the plan cache, else built (untimed, as the paper excludes "
        "loading its precomputed data)")
    t0 = time.perf_counter()
    # the transposed matrix copy serves the adjoint of the gradient measurement
    kw = {k: v for k, v in (("rings_per_lane", args.rings_per_lane), ("ring_threads", args.ring_threads),
                            ("rho", args.rho)) if v}
    plan = sht.cached_plan(L, N, args.eps, store_fp32=args.eps > 0,
                           store_transpose=args.eps > 0 and not args.no_adjoint, log=log, **kw)
    info = plan.info()
    log(f"[bench] plan ready in {time.perf_counter() - t0:.1f}s: n_step={info['n_step']:.4e} "
        f"dd_rings={info['n_dd_rings']} butterfly={info['bf_built']} T={info['bf_T_entries']:.4e} "
        f"residual={info['bf_res_elems']:.4e} device={info['device_bytes'] / 1e9:.2f} GB")

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

    paths = [("brute", sht.PATH_BRUTE, sht.PREC_FP64)]
    if info["bf_built"]:
        paths += [("bf64", sht.PATH_BUTTERFLY, sht.PREC_FP64), ("bf32", sht.PATH_BUTTERFLY, sht.PREC_FP32)]

    results, maps_out = {}, {}
    for name, path, prec in paths:
        for _ in range(args.warmup):
            plan.synthesis(d_alm, out, path=path, precision=prec, workspace=ws)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(args.steps):
            plan.synthesis(d_alm, out, path=path, precision=prec, workspace=ws, events=ev_sets[k])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - ts
        leg_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev_sets]))
        ring_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in ev_sets]))
        results[name] = {"maps_per_s": B * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
                         "legendre_ms": leg_ms, "ring_ms": ring_ms}
        if path == sht.PATH_BUTTERFLY and info["bf_nbatch"] == 1:
            # the residual launch and the level launches, bracketed inside the stage
            s8, s10 = 2 * sht.STAGE_BF_RESIDUAL, 2 * sht.STAGE_BF_LEVELS
            results[name]["residual_ms"] = float(np.mean([e[s8].elapsed_time(e[s8 + 1]) for e in ev_sets]))
            results[name]["levels_ms"] = float(np.mean([e[s10].elapsed_time(e[s10 + 1]) for e in ev_sets]))
        maps_out[name] = out.cpu().numpy()
        log(f"[bench] {name}: {results[name]['ms_per_step']:.3f} ms/step, legendre {leg_ms:.3f} ms, "
            f"ring {ring_ms:.3f} ms")

    flops = info["n_step"] * (5 + 4 * B)
    q_bytes = (L + 1) * plan.nrings * B * 16
    alm_bytes = plan.nalm * B * 16

    # level launches per pass: one per depth that any (m, parity) reaches
    nlev = max([d for d, c in enumerate(info["bf_depth_hist"]) if c > 0] + [0]) if info["bf_built"] else 0

    def path_roofline(name):
        r = results[name]
        if name == "brute":
            achieved = flops / (r["legendre_ms"] * 1e-3) / 1e12
            return {"kernel": "k_legendre (brute-force Legendre phase, one launch)", "bound": "alu",
                    "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                    "traffic": measured_traffic("void sht::k_legendre<", L, N, B),
                    "counters": measured_counters("void sht::k_legendre<", L, N, B), "flops_per_launch": flops}
        sz = 8 if name == "bf64" else 4
        if "levels_ms" not in r or nlev == 0:
            nbytes = info["bf_T_entries"] * sz + alm_bytes + q_bytes
            achieved = nbytes / (r["legendre_ms"] * 1e-3) / 1e9
            return {"kernel": "butterfly stage (k_bf_residual + k_bf_level + k_bf_fold)", "bound": "hbm",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": nbytes}
        if r["levels_ms"] >= r["residual_ms"]:
            return level_roofline(info, nlev, sz, B, r["levels_ms"], L, N)
        rflops = info["bf_res_elems"] * (5 + 4 * B)
        achieved = rflops / (r["residual_ms"] * 1e-3) / 1e12
        return {"kernel": "k_bf_residual (one launch)", "bound": "alu", "achieved": round(achieved, 3),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": measured_traffic("void sht::k_bf_residual<%d, %s>(" % (
                    min(B, 8), "double" if sz == 8 else "float"), L, N, B, info["bf_T_entries"]),
                "counters": measured_counters("void sht::k_bf_residual<%d, %s>(" % (
                    min(B, 8), "double" if sz == 8 else "float"), L, N, B, info["bf_T_entries"]),
                "flops_per_launch": rflops, "launch_ms": round(r["residual_ms"], 4)}

    fp64 = [n for n in results if n != "bf32"]
    head = max(fp64, key=lambda n: results[n]["maps_per_s"])
    hr = results[head]
    log(f"[bench] headline path: {head}")

    many = None
    if info["bf_built"] and args.many_maps:
        many = many_map_bench(np, torch, sht, plan, info, args, maps_out)

    adj = None
    if not args.no_adjoint:
        adj = gradient_bench(np, torch, sht, plan, info, paths, d_alm, maps_out["brute"], ws, ev_sets, args, flops)

    ana = None
    if not args.no_analysis:
        ana = analysis_bench(np, torch, sht, plan, paths, d_alm, maps_out["brute"], args)

    if not args.no_batch:
        line_batch = batch_bench(np, torch, sht, args.steps)
    else:
        line_batch = None

    cfg3 = None if args.no_config3 else config3_bench(np, torch, sht, args)
    pol = None if args.no_pol else pol_bench(np, torch, sht, plan, args)
    ipl = None if args.no_interp else interp_bench(np, torch, sht, args, d_alm, alm, results["brute"])

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
        "value": round(hr["maps_per_s"], 3),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hr["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"HEALPix synthesis L={L} nside={N}, {B} maps per step, FP64 "
                        f"({'butterfly eps=%g' % args.eps if head != 'brute' else 'brute-force recurrence'}"
                        " + ring FFT)",
            "L": L, "nside": N, "maps": B, "path": head, "precision": "fp64", "eps": args.eps,
            "spectrum": "C_l=1/(l+1)^2", "seeds": seeds,
        },
        "stages_ms": {"legendre": round(hr["legendre_ms"], 4), "ring_fft": round(hr["ring_ms"], 4)},
        "roofline": path_roofline(head),
    }
    line["paths"] = {}
    for name in results:
        r = results[name]
        line["paths"][name] = {
            "maps_per_s": round(r["maps_per_s"], 3), "ms_per_step": round(r["ms_per_step"], 4),
            "legendre_ms": round(r["legendre_ms"], 4), "ring_ms": round(r["ring_ms"], 4),
            "speedup_vs_brute": round(r["maps_per_s"] / results["brute"]["maps_per_s"], 3),
            **({"residual_ms": round(r["residual_ms"], 4), "levels_ms": round(r["levels_ms"], 4)}
               if "levels_ms" in r else {}),
            "roofline": path_roofline(name),
        }
    if info["bf_built"]:
        line["butterfly_plan"] = {"eps": args.eps, "T_entries": info["bf_T_entries"],
                                  "residual_elements": info["bf_res_elems"],
                                  "residual_lane_steps": info["bf_res_exec"], "nodes": info["bf_nodes"],
                                  "depth_hist": info["bf_depth_hist"][:8],
                                  "build_seconds": round(info["bf_build_seconds"], 1),
                                  "device_gb": round(info["device_bytes"] / 1e9, 2)}
    if adj is not None:
        line["adjoint"] = adj
    if ana is not None:
        line["analysis"] = ana
    if line_batch is not None:
        line["batching"] = line_batch
    if many is not None:
        line["many_maps"] = many
    if cfg3 is not None:
        line["L2047_16maps"] = cfg3
    if ipl is not None:
        line["interp"] = ipl
    if pol is not None:
        line["polarization"] = pol

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
        cores = oracle.num_threads()
        line["cpu_baseline"] = {
            "value": round(B / full, 6),
            "unit": "maps/s",
            "cores": cores,
            "cpu_model": cpu_model(),
            "cpu_seconds_per_transform": round(full * cores / B, 1),
            "kind": "oracle",
            "sample": f"{k} of {nr} rings drawn uniformly (seed 0), all {B} maps, FP64 oracle "
                      f"(one-step Legendre recurrence + direct per-ring DFT); {tcpu:.1f}s measured, "
                      f"scaled by {nr}/{k}",
        }
        # accuracy of each GPU path on a few rings against the long-double oracle
        chk = [1, 2, 100, 250, 251, 1000, 2 * N, 2 * N + 1, 3 * N, nr]
        errs = sampled_errors(np, oracle, L, N, alm, maps_out, chk)
        for name in maps_out:
            line["paths"][name].update(errs[name])
        line["max_rel_err"] = line["paths"][head]["max_rel_err"]
        line["rms_eps"] = line["paths"][head]["rms_eps"]
        line["max_rel_err_sample"] = (f"rings {chk}, all maps, vs long-double oracle, relative to the oracle's "
                                      "max on those rings per map; rms_eps is Eq. 24 on the same sample")
        log(f"[bench] cpu baseline {line['cpu_baseline']['value']:.4f} maps/s; errors "
            + ", ".join(f"{n} {line['paths'][n]['max_rel_err']:.2e}" for n in maps_out))

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
