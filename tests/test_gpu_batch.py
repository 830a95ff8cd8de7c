"""Batched synthesis (many requests in one call; many-transform regime of
Sec. 3.4): results equal the per-request calls exactly, and a captured HIP
graph of one batch replays correctly several times with eager work between
the replays."""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_4874_amd import sht
from paper_1110_4874_amd.synthetic import alm_gaussian, mixed_requests

pytestmark = pytest.mark.gpu


def _requests(n, seed, gpu, eps=0.0, max_maps=5, store_fp32=False):
    plans = {}
    reqs = []
    for (L, N, B, seeds) in mixed_requests(seed=seed, n=n, lmax_choices=(31, 63, 127, 255), max_maps=max_maps):
        key = (L, N)
        if key not in plans:
            plans[key] = gpu.Plan(L, N, eps, max_levels=2 if eps else -1, store_fp32=store_fp32)
        alm = torch.from_numpy(alm_gaussian(L, seeds)).cuda()
        out = torch.full((B, 12 * N * N), float("nan"), dtype=torch.float64, device="cuda")
        reqs.append((plans[key], alm, out))
    return plans, reqs


@pytest.mark.parametrize("eps,nstreams", [(0.0, 4), (0.0, 1), (1e-12, 3)])
def test_batch_equals_individual_calls(gpu, eps, nstreams):
    plans, reqs = _requests(12, 77, gpu, eps)
    batch = sht.Batch(reqs, nstreams=nstreams)
    batch.run()
    torch.cuda.synchronize()
    for plan, alm, out in reqs:
        ref = plan.synthesis(alm)
        assert torch.equal(out, ref)


def test_batch_against_oracle(gpu):
    plans, reqs = _requests(6, 78, gpu)
    sht.Batch(reqs).run()
    torch.cuda.synchronize()
    for plan, alm, out in reqs:
        ref = oracle.synthesis(plan.L, plan.nside, alm.cpu().numpy())
        f = out.cpu().numpy()
        err = max(np.max(np.abs(f[b] - ref[b])) / np.max(np.abs(ref[b])) for b in range(ref.shape[0]))
        assert err <= 1e-12


def test_batch_graph_replay(gpu):
    plans, reqs = _requests(10, 79, gpu)
    batch = sht.Batch(reqs)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(stream=s)  # eager warm-up (kernel attributes, internal streams)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    eager = [out.clone() for _, _, out in reqs]
    g = torch.cuda.CUDAGraph()
    for _, _, out in reqs:
        out.fill_(float("nan"))
    with torch.cuda.graph(g):
        batch.run(stream=torch.cuda.current_stream())
    for rep in range(3):
        for _, _, out in reqs:
            out.fill_(float("nan"))
        x = torch.randn(1 << 20, device="cuda")  # eager work between replays
        (x * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, out), ref in zip(reqs, eager):
            assert torch.equal(out, ref), f"replay {rep}"


@pytest.mark.parametrize("rpl,threads", [(0, 0), (1, 256), (4, 1024)])
def test_queue_batch_equals_individual_calls(gpu, rpl, threads):
    # the work-queue form: one persistent Legendre launch over every request's
    # items, longest first, and one ring launch per ring size class
    plans, reqs = _requests(12, 80, gpu)
    qb = sht.QueueBatch(reqs, rings_per_lane=rpl, ring_threads=threads)
    st = qb.stats()
    assert st["items"] > 0 and st["launches"] <= 1 + 5 + 8
    qb.run()
    torch.cuda.synchronize()
    for plan, alm, out in reqs:
        ref = plan.synthesis(alm, path=sht.PATH_BRUTE)
        assert torch.equal(out, ref)
    # a second run (counter reset by the run itself) gives the same maps
    for _, _, out in reqs:
        out.fill_(float("nan"))
    qb.run()
    torch.cuda.synchronize()
    for plan, alm, out in reqs:
        assert torch.equal(out, plan.synthesis(alm, path=sht.PATH_BRUTE))


@pytest.mark.parametrize("prec", [sht.PREC_FP64, sht.PREC_FP32])
def test_queue_batch_butterfly_equals_individual_calls(gpu, prec):
    # butterfly path: one launch per stage and map-group width over every
    # request's passes (widths 8, 4, 2, 1 all occur with up to 11 maps)
    plans, reqs = _requests(12, 83, gpu, eps=1e-12, max_maps=11, store_fp32=True)
    assert any(a.shape[1] >= 8 for _, a, _ in reqs)
    qb = sht.QueueBatch(reqs, path=sht.PATH_BUTTERFLY, precision=prec)
    assert qb.stats()["items"] > 0
    for rep in range(2):
        for _, _, out in reqs:
            out.fill_(float("nan"))
        qb.run()
        torch.cuda.synchronize()
        for plan, alm, out in reqs:
            ref = plan.synthesis(alm, path=sht.PATH_BUTTERFLY, precision=prec)
            assert torch.equal(out, ref), f"run {rep}, L={plan.L}, maps={alm.shape[1]}"


def test_queue_batch_graph_replay(gpu):
    plans, reqs = _requests(10, 81, gpu)
    qb = sht.QueueBatch(reqs)
    qb.run()
    torch.cuda.synchronize()
    eager = [out.clone() for _, _, out in reqs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            qb.run(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for _, _, out in reqs:
            out.fill_(float("nan"))
        x = torch.randn(1 << 20, device="cuda")  # eager work between replays
        (x * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, out), ref in zip(reqs, eager):
            assert torch.equal(out, ref), f"replay {rep}"


def test_queue_batch_rejects_bad_arguments(gpu):
    plans, reqs = _requests(2, 82, gpu)
    lib = sht.load()
    with pytest.raises(sht.ShtError):
        sht.QueueBatch(reqs, rings_per_lane=3)
    o = sht.BatchOpts()
    lib.sht_batch_opts_default(o)
    o.path = sht.PATH_BUTTERFLY
    r = (sht.Request * 1)()
    r[0].plan = reqs[0][0]._h
    r[0].nmaps = reqs[0][1].shape[1]
    r[0].alm = reqs[0][1].data_ptr()
    r[0].map = reqs[0][2].data_ptr()
    assert not lib.sht_batch_create(r, 1, o)
    assert lib.sht_last_status() == sht.SHT_EUNSUPPORTED
