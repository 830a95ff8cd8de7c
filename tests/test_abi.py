"""C-ABI contract and host-side plan logic (no GPU needed).

The library must load and export every function include/sht.h declares; a
host-only plan exposes the recurrence tables and chain start values, which
are checked here against the paper's recurrence algebra and the oracle.
"""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "sht.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(sht_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def sht():
    from paper_1110_4874_amd import sht as mod
    mod.load()
    return mod


def test_exports_every_declared_symbol(sht):
    names = _header_functions()
    assert "sht_plan" in names and "sht_synthesis" in names
    lib = sht.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sht.EXPORTS), set(names) ^ set(sht.EXPORTS)


def test_invalid_arguments(sht):
    lib = sht.load()
    assert not lib.sht_plan(-1, 4, 0.0)
    assert "L must be" in lib.sht_last_error().decode()
    assert not lib.sht_plan(10, 0, 0.0)
    assert not lib.sht_plan(10, 4096, 0.0)
    assert not lib.sht_plan(10, 4, -1.0)
    assert not lib.sht_plan(10, 4, 0.5)
    assert "eps must be below" in lib.sht_last_error().decode()
    o = sht.PlanOpts()
    lib.sht_plan_opts_default(o)
    o.max_levels = 11
    assert not lib.sht_plan_ex(10, 4, 1e-12, o)
    assert "max_levels" in lib.sht_last_error().decode()


def test_host_only_plan_cannot_execute(sht):
    p = sht.Plan(15, 8, host_only=True)
    lib = sht.load()
    x = sht.ExecOpts()
    lib.sht_exec_opts_default(x)
    rc = lib.sht_synthesis_ex(p._h, x, None, None)
    assert rc == sht.SHT_EDEVICE
    info = p.info()
    assert info["L"] == 15 and info["nrings"] == 31 and info["device_bytes"] == 0


def _a(l, m):
    return math.sqrt((l * l - m * m) / (4.0 * l * l - 1.0)) if l > m else 0.0


@pytest.mark.parametrize("L,m", [(40, 0), (40, 1), (40, 17), (40, 39), (300, 123)])
def test_recurrence_coefficients_match_one_step_algebra(sht, L, m):
    # App. A.2: c_l = a_{l+1} a_{l+2} and d_l = a_{l+1}^2 + a_l^2 with
    # a_l = sqrt((l^2 - m^2)/(4 l^2 - 1)); the plan uses the paper's closed
    # forms for c and d, so this ties them to the ordinary recurrence.
    p = sht.Plan(L, 8, host_only=True)
    cf = p.coef(m)
    for e, (beta, ab, gam) in enumerate(cf):
        l = m + e
        c = _a(l + 1, m) * _a(l + 2, m)
        d = _a(l + 1, m) ** 2 + _a(l, m) ** 2
        cm2 = _a(l - 1, m) * _a(l, m) if l - 2 >= m else 0.0
        assert beta == pytest.approx(1.0 / c, rel=1e-14)
        assert ab == pytest.approx(-d / c, rel=1e-14)
        assert gam == pytest.approx(-cm2 / c, rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("L,N", [(63, 32), (200, 16)])
def test_chain_start_values_match_oracle(sht, L, N):
    import oracle
    p = sht.Plan(L, N, host_only=True, cutoff=1e-30)
    rng = np.random.default_rng(0)
    for _ in range(60):
        m = int(rng.integers(0, L + 1))
        k = int(rng.integers(0, 2 * N))
        col = oracle.plm_ring(L, m, N, k + 1, ld=True)
        for t in (0, 1):
            idx, (v0, v1) = p.start(m, t, k)
            chain = col[t::2]
            if idx >= len(chain):
                # dead chain: every value stays below the cutoff
                assert np.all(np.abs(chain) < 1e-30)
                continue
            assert idx % 8 == 0
            assert np.all(np.abs(chain[:idx]) < 1e-30)
            assert v0 == pytest.approx(chain[idx], rel=1e-15, abs=0)
            if idx + 1 < len(chain):
                assert v1 == pytest.approx(chain[idx + 1], rel=1e-15, abs=0)
            # the first value at or above the cutoff is inside the first chunk
            above = np.flatnonzero(np.abs(chain) >= 1e-30)
            assert above[0] < idx + 8


def test_plan_info_work_count(sht):
    # with no cutoff skip possible (tiny L) the step count is the full
    # (l, ring) product over the north rings
    L, N = 7, 4
    p = sht.Plan(L, N, host_only=True)
    assert p.info()["n_step"] == (L + 1) * (L + 2) // 2 * (2 * N) - sum(
        1 for m in range(L + 1) if (L - m) % 2 == 0) * 0 - _odd_equator_steps(L, N)


def _odd_equator_steps(L, N):
    # odd chains vanish identically on the equator ring (z = 0)
    return sum((L - m - 1) // 2 + 1 for m in range(L + 1) if L - m - 1 >= 0)


def test_workspace_sizes(sht):
    # the analysis workspace is the synthesis workspace plus one residual map
    # set (Npix B doubles) and one alm set (nalm B complex); on a butterfly
    # plan the synthesis workspace also holds the level vectors
    lib = sht.load()
    for eps, path in ((0.0, sht.PATH_BRUTE), (1e-10, sht.PATH_BUTTERFLY)):
        p = sht.Plan(63, 32, eps, host_only=True, max_levels=1 if eps else -1)
        for B in (1, 3, 8, 9):
            x = sht.ExecOpts()
            lib.sht_exec_opts_default(x)
            x.nmaps, x.path = B, path
            ws = lib.sht_workspace_bytes(p._h, x)
            wa = lib.sht_analysis_workspace_bytes(p._h, x)
            q = (p.L + 1) * p.nrings * B * 16
            assert ws >= q and (eps > 0 or ws == q)
            assert wa == ws + 12 * 32 * 32 * B * 8 + p.nalm * B * 16
