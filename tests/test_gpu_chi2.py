"""GPU check of the chi^2 monitor (plan flag WF_FLAG_CHI2) against the oracle's
chi^2 of every iterate (Sect. 3's convergence monitor, at lambda = 1).

The oracle runs the same sweeps and reports each iterate (s_WF map, s_lm) through
its callback; oracle.messenger.chi2 evaluates the definition. Bars: 1e-10 relative
for FP64 (the sums are FP64 atomics: only the order of additions differs), 1e-5
for the FP32 path.
"""
import sys

import numpy as np
import pytest

from oracle import messenger
from tests.helpers import small_band_inputs

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1211_0585_amd import mwf
    mwf.lib()
    return torch


def _oracle_history(d, c, lams, nside, lmax):
    out = []

    def cb(k, s_map, s_alm):
        out.append(messenger.chi2(s_map, s_alm, d, c["ninv"], c["cl"], lmax))
    messenger.solve(d, c["ninv"], c["cl"], lams, nside, lmax, callback=cb)
    return np.array(out)


@pytest.mark.parametrize("name,dt,tol", [("f64", 0, 1e-10), ("f32", 1, 1e-5)])
@pytest.mark.parametrize("nside,lmax", [(8, 16), (16, 32)])
def test_chi2_history_matches_oracle(torch_dev, name, dt, tol, nside, lmax):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nm = 3
    cs = [small_band_inputs(nside, lmax, seed=40 + i) for i in range(nm)]
    c = cs[0]
    lams = np.geomspace(1e3, 1.0, 14)
    rt = np.float64 if dt == 0 else np.float32
    D = np.stack([x["d"] for x in cs]).astype(rt)
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=dt, max_batch=nm, flags=mwf.WF_FLAG_CHI2) as p:
        p.solve(torch.from_numpy(D).cuda(), lams)
        last = p.last_stats.chi2_last
        hist = p.chi2(nm, len(lams))
    for i in range(nm):
        ref = _oracle_history(D[i].astype(np.float64), c, lams, nside, lmax)
        e = np.max(np.abs(hist[i] - ref) / np.abs(ref))
        _log(f"chi2 {name} Nside {nside} map {i}: first {hist[i][0]:.6g} last {hist[i][-1]:.6g} "
             f"(oracle {ref[-1]:.6g}), max rel diff {e:.2e}")
        assert e <= tol
    assert last == hist[0][-1]


def test_chi2_requires_flag_and_sizes(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c = small_band_inputs(8, 16, seed=1)
    d = torch.from_numpy(c["d"]).cuda()
    with mwf.Plan(8, 16, c["cl"], c["ninv"]) as p:
        p.solve(d, np.ones(3))
        assert p.last_stats.chi2_last == 0.0
        with pytest.raises(mwf.WFError):
            p.chi2(1, 3)
    with mwf.Plan(8, 16, c["cl"], c["ninv"], flags=mwf.WF_FLAG_CHI2 | mwf.WF_FLAG_TIMING) as p:
        p.solve(d, np.ones(3))
        assert p.last_stats.timed == 1 and p.last_stats.chi2_last > 0
        with pytest.raises(mwf.WFError):
            p.chi2(1, 4)
        p.solve(d, np.ones(5))   # a longer schedule grows the history
        assert p.chi2(1, 5).shape == (1, 5)


@pytest.mark.parametrize("name,dt,tol", [("f64", 0, 1e-10), ("f32", 1, 1e-5)])
def test_chi2_batch_after_adaptive_solve(torch_dev, name, dt, tol):
    """The history buffer is laid out per solve: an adaptive solve (one map, a long
    sweep cap) followed by a 3-map batch on the same plan records the batch's history
    as a fresh plan does, and as the oracle evaluates it; a shorter batch after that
    (fewer sweeps, fewer maps) too."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax, nm = 8, 16, 3
    cs = [small_band_inputs(nside, lmax, seed=60 + i) for i in range(nm)]
    c = cs[0]
    rt = np.float64 if dt == 0 else np.float32
    D = np.stack([x["d"] for x in cs]).astype(rt)
    lams = np.geomspace(1e3, 1.0, 14)
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=dt, max_batch=nm, flags=mwf.WF_FLAG_CHI2) as p:
        _, _, info = p.solve_adaptive(torch.from_numpy(D[0]).cuda(), 300)
        assert len(info["chi2"]) > len(lams)
        p.solve(torch.from_numpy(D).cuda(), lams)
        hist = p.chi2(nm, len(lams))
        p.solve(torch.from_numpy(D[1:2].copy()).cuda(), lams[:5])
        hist_short = p.chi2(1, 5)
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=dt, max_batch=nm, flags=mwf.WF_FLAG_CHI2) as q:
        q.solve(torch.from_numpy(D).cuda(), lams)
        fresh = q.chi2(nm, len(lams))
    e_fresh = np.max(np.abs(hist - fresh) / np.abs(fresh))
    worst = 0.0
    for i in range(nm):
        ref = _oracle_history(D[i].astype(np.float64), c, lams, nside, lmax)
        worst = max(worst, np.max(np.abs(hist[i] - ref) / np.abs(ref)))
    ref_short = _oracle_history(D[1].astype(np.float64), c, lams[:5], nside, lmax)
    e_short = np.max(np.abs(hist_short[0] - ref_short) / np.abs(ref_short))
    _log(f"chi2 {name} batch after adaptive ({len(info['chi2'])} sweeps): vs fresh plan {e_fresh:.2e}, "
         f"vs oracle {worst:.2e}; shorter batch vs oracle {e_short:.2e}")
    assert e_fresh <= tol and worst <= tol and e_short <= tol
