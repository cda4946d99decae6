"""wf_solve_batch_static (work buffers in the per-device static workspace, no
allocation) against wf_solve_batch on the same plans, through the C ABI.

Two calls in a row per dtype, the second on a smaller plan and fewer maps, so the
second runs on a workspace that still holds the first call's larger contents. FP64
results are also checked against the oracle (<= 1e-10).
"""
import sys

import numpy as np
import pytest

from oracle import healpix, messenger, sht
from paper_1211_0585_amd import synth
from tests.helpers import rel_l2

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


def _case(nside, lmax, nmaps):
    theta, _ = healpix.pixel_angles(nside)
    c = synth.small_band_case(theta, lmax, seed=0)
    ds = []
    for i in range(nmaps):
        ci = synth.small_band_case(theta, lmax, seed=i)
        ds.append(sht.alm2map(ci["signal_alm"], nside, lmax) + ci["noise"])
    return c, np.stack(ds)


def _run_pair(torch, mwf, nside, lmax, nmaps, dtype, sched, oracle=False):
    c, d = _case(nside, lmax, nmaps)
    tdt = torch.float64 if dtype == mwf.WF_F64 else torch.float32
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=dtype, max_batch=nmaps) as p:
        dd = torch.from_numpy(d).to("cuda", tdt)
        _log(f"static solve: nside {nside} lmax {lmax} maps {nmaps} dtype {dtype}")
        s_st, a_st = p.solve(dd, sched, static=True)
        torch.cuda.synchronize()
        p.sync()
        s_pl, a_pl = p.solve(dd, sched)
        torch.cuda.synchronize()
        p.sync()
        s_st, s_pl = s_st.cpu().numpy(), s_pl.cpu().numpy()
        a_st, a_pl = a_st.cpu().numpy(), a_pl.cpu().numpy()
    em = rel_l2(s_st, s_pl)
    ea = rel_l2(a_st, a_pl)
    _log(f"  static vs plan buffers: map {em:.2e} alm {ea:.2e} bitwise {np.array_equal(s_st, s_pl)}")
    bar = 1e-12 if dtype == mwf.WF_F64 else 1e-6
    assert em <= bar and ea <= bar
    if oracle:
        for i in range(nmaps):
            ref, _ = messenger.solve(d[i], c["ninv"], c["cl"], sched, nside, lmax)
            e = rel_l2(s_st[i], ref)
            _log(f"  map {i} vs oracle {e:.2e}")
            assert e <= 1e-10


def test_static_solve_fp64_two_calls(torch_dev):
    from paper_1211_0585_amd import mwf
    sched = synth.geometric_schedule(1e4, 4, 3)
    _run_pair(torch_dev, mwf, 64, 128, 2, mwf.WF_F64, sched, oracle=True)
    _run_pair(torch_dev, mwf, 16, 32, 1, mwf.WF_F64, sched, oracle=True)


def test_static_solve_fp32_two_calls(torch_dev):
    from paper_1211_0585_amd import mwf
    sched = synth.geometric_schedule(1e4, 3, 2)
    _run_pair(torch_dev, mwf, 64, 128, 5, mwf.WF_F32, sched)
    _run_pair(torch_dev, mwf, 32, 64, 2, mwf.WF_F32, sched)


def test_static_solve_rejects_oversized(torch_dev):
    """Two FP32 maps at Nside 512 / lmax 1024 need 137 MiB of workspace: WF_EINVAL with
    the need in the message; one map (69 MiB) runs."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 512, 1024
    npix = 12 * nside * nside
    cl = synth.cl_power_law(lmax)
    ninv = np.full(npix, 1.0)
    with mwf.Plan(nside, lmax, cl, ninv, dtype=mwf.WF_F32, max_batch=2) as p:
        d = torch.zeros((2, npix), dtype=torch.float32, device="cuda")
        with pytest.raises(mwf.WFError) as ei:
            p.solve(d, [1.0], static=True)
        assert ei.value.code == mwf.WF_EINVAL and "MiB" in str(ei.value)
        s, _ = p.solve(d[0], [1.0], static=True)
        torch.cuda.synchronize()
        p.sync()
        assert float(s.abs().max()) == 0.0
