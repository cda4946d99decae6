"""The matrix-core analysis with 4 and 8 column tiles per workgroup (the first four
waves generate the Legendre values of a 256-pair block once for 64 or 128 columns;
every wave contracts its own tile), selected with a launch-shape cache line as
wf_autotune records it, against the FP64 oracle and against the 2-tile shape,
through the C ABI.

Bars: transforms and solves <= 1e-5 for FP32 and bf16x6 against the oracle (bf16x3:
transforms 1e-5, solves its stated 5e-5); tile shapes agree to FP32 summation order
(the block partial sums are the same sums; <= 1e-6).
"""
import sys

import numpy as np
import pytest

from oracle import messenger, sht
from tests.helpers import alm_rel_l2, rel_l2, small_band_inputs

pytestmark = pytest.mark.gpu

MODES = [("f32", 1, 1e-5), ("bf16x6", 3, 1e-5), ("bf16x3", 2, 5e-5)]


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


def _cache(tmp_path, dt, nside, lmax, nmaps, ct):
    path = tmp_path / f"tune_{dt}_{nside}_{lmax}_{nmaps}_{ct}.txt"
    path.write_text(f"d{dt}_n{nside}_l{lmax}_c{2 * nmaps} {ct} 2 0\n")
    return str(path)


def _map2alm(torch, mwf, tmp_path, dt, nside, lmax, maps, ct):
    nmaps = maps.shape[0]
    cl = np.ones(lmax + 1)
    ninv = np.ones(12 * nside * nside)
    with mwf.Plan(nside, lmax, cl, ninv, dtype=dt, max_batch=nmaps,
                  tune_cache=_cache(tmp_path, dt, nside, lmax, nmaps, ct)) as p:
        a = p.map2alm(torch.from_numpy(maps.astype(np.float32)).cuda())
        p.sync()
        return a.to(torch.complex128).cpu().numpy()


@pytest.mark.parametrize("name,dt,tol", MODES)
@pytest.mark.parametrize("nside,lmax,nmaps", [(4, 12, 1), (16, 32, 3), (32, 64, 33), (64, 128, 64), (128, 256, 5)])
@pytest.mark.parametrize("ct", [4, 8])
def test_analysis_tiles_map2alm(torch_dev, tmp_path, name, dt, tol, nside, lmax, nmaps, ct):
    """Analysis of random maps (the tile shape under test) against the oracle and the 2-tile shape."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    if ct == 8 and dt != mwf.WF_F32:
        pytest.skip("8 column tiles (16 waves) are an FP32 shape")
    rng = np.random.default_rng(100 + nmaps)
    maps = rng.standard_normal((nmaps, 12 * nside * nside))
    got = _map2alm(torch, mwf, tmp_path, dt, nside, lmax, maps, ct)
    ref2 = _map2alm(torch, mwf, tmp_path, dt, nside, lmax, maps, 2)
    errs = [alm_rel_l2(got[i], sht.map2alm(maps[i].astype(np.float32).astype(np.float64), nside, lmax), lmax)
            for i in range(nmaps)]
    e_shape = max(alm_rel_l2(got[i], ref2[i], lmax) for i in range(nmaps))
    _log(f"analysis {ct} tiles {name} Nside {nside} lmax {lmax} x{nmaps}: vs oracle max {max(errs):.2e}, "
         f"vs 2 tiles {e_shape:.2e}")
    assert max(errs) <= 1e-5 and e_shape <= 1e-6


@pytest.mark.parametrize("name,dt,tol", MODES)
@pytest.mark.parametrize("ct", [4, 8])
def test_analysis_tiles_solve(torch_dev, tmp_path, name, dt, tol, ct):
    """Full solves of a 6-map batch with the tile shape under test against the oracle."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    if ct == 8 and dt != mwf.WF_F32:
        pytest.skip("8 column tiles (16 waves) are an FP32 shape")
    nside, lmax, nmaps = 32, 64, 6
    cases = [small_band_inputs(nside, lmax, seed=s) for s in range(nmaps)]
    c0 = cases[0]
    d = np.stack([c["d"] for c in cases])
    sched = np.concatenate([np.geomspace(1e4, 1.0, 12), np.ones(10)])
    with mwf.Plan(nside, lmax, c0["cl"], c0["ninv"], dtype=dt, max_batch=nmaps,
                  tune_cache=_cache(tmp_path, dt, nside, lmax, nmaps, ct)) as p:
        s, a = p.solve(torch.from_numpy(d.astype(np.float32)).cuda(), sched)
        p.sync()
        s, a = s.double().cpu().numpy(), a.to(torch.complex128).cpu().numpy()
    worst = 0.0
    for i in range(nmaps):
        ref_s, ref_a = messenger.solve(d[i].astype(np.float32).astype(np.float64), c0["ninv"], c0["cl"], sched,
                                       nside, lmax)
        worst = max(worst, rel_l2(s[i], ref_s), alm_rel_l2(a[i], ref_a, lmax))
    _log(f"analysis {ct} tiles {name}: {len(sched)}-sweep solve of {nmaps} maps, worst vs oracle {worst:.2e}")
    assert worst <= tol
