"""The synthesis entry point that allocates nothing (sht_synthesis_noalloc),
called through the C ABI and checked against sht_synthesis_ex on the same
inputs: the two run the same kernels on the same data, so the maps must be
identical bit for bit.  Two calls in a row, the second with a smaller
transform, show that the shared fixed scratch carries nothing from one call
into the next; a transform larger than the scratch is refused before
anything runs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1110_4874_amd import sht
from paper_1110_4874_amd.synthetic import alm_gaussian

pytestmark = pytest.mark.gpu


def _noalloc(plan, alm, out, path, prec):
    lib = sht.load()
    x = plan._exec(alm.shape[1], path=path, precision=prec)
    return lib.sht_synthesis_noalloc(plan._h, ctypes.byref(x), ctypes.c_void_p(alm.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()))


def _case(plan, L, seeds, path, prec):
    alm = torch.from_numpy(alm_gaussian(L, seeds)).cuda()
    ref = plan.synthesis(alm, path=path, precision=prec)
    out = torch.full_like(ref, float("nan"))
    torch.cuda.synchronize()
    assert _noalloc(plan, alm, out, path, prec) == sht.SHT_OK, sht.load().sht_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_matches_synthesis_ex(gpu):
    lib = sht.load()
    assert lib.sht_noalloc_scratch_bytes() == 64 << 20
    big = gpu.Plan(511, 256, 1e-12, max_levels=3, store_fp32=True)
    small = gpu.Plan(127, 64, 1e-12, max_levels=2)
    # first call: a transform filling most of the scratch (24 / 60 / 46 MiB), then a smaller one
    for seeds, path, prec in (([11, 12, 13], sht.PATH_BRUTE, sht.PREC_FP64),
                              ([18, 19], sht.PATH_BUTTERFLY, sht.PREC_FP64)):
        _case(big, 511, seeds, path, prec)
        _case(small, 127, [14], path, prec)
    _case(big, 511, [15, 16, 20], sht.PATH_BUTTERFLY, sht.PREC_FP32)
    _case(small, 127, [17], sht.PATH_BRUTE, sht.PREC_FP64)


def test_noalloc_refuses_transforms_beyond_the_scratch(gpu):
    p = gpu.Plan(511, 256)
    need = p.workspace_bytes(9)
    assert need > sht.load().sht_noalloc_scratch_bytes()
    alm = torch.zeros((p.nalm, 9), dtype=torch.complex128, device="cuda")
    out = torch.full((9, p.npix), 7.0, dtype=torch.float64, device="cuda")
    assert _noalloc(p, alm, out, sht.PATH_BRUTE, sht.PREC_FP64) == sht.SHT_ENOMEM
    assert "scratch" in sht.load().sht_last_error().decode()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing ran
