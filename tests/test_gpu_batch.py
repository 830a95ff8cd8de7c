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


def _requests(n, seed, gpu, eps=0.0):
    plans = {}
    reqs = []
    for (L, N, B, seeds) in mixed_requests(seed=seed, n=n, lmax_choices=(31, 63, 127, 255), max_maps=5):
        key = (L, N)
        if key not in plans:
            plans[key] = gpu.Plan(L, N, eps, max_levels=2 if eps else -1)
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
