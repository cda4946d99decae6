"""The wide matrix-core synthesis (256 ring pairs and 64 columns per workgroup, 32 x 32
tiles with the Legendre operand taken from registers) against the FP64 oracle and
against the per-wave synthesis, through the C ABI. The kernel is selected with a
launch-shape cache file (its fourth field), as wf_autotune records it.

Bars as for the other reduced-precision tests: transforms and solves <= 1e-5 for
FP32 and bf16x6 against the oracle (bf16x3: transforms 1e-5, solves its stated 5e-5);
wide and per-wave kernels agree to FP32 summation order (<= 1e-5).
"""
import os
import sys

import numpy as np
import pytest

from oracle import messenger, sht
from tests.helpers import alm_rel_l2, random_alm, rel_l2, small_band_inputs

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


def _cache(tmp_path, dt, nside, lmax, nmaps, wide):
    path = tmp_path / f"tune_{dt}_{nside}_{lmax}_{nmaps}_{wide}.txt"
    path.write_text(f"d{dt}_n{nside}_l{lmax}_c{2 * nmaps} 2 2 {wide}\n")
    return str(path)


@pytest.mark.parametrize("name,dt,tol", MODES)
@pytest.mark.parametrize("nside,lmax,nmaps,nt", [(4, 12, 1, 1), (16, 32, 3, 1), (32, 64, 33, 1), (64, 128, 64, 1),
                                                 (128, 256, 5, 1), (4, 12, 1, 2), (32, 64, 33, 2), (64, 128, 64, 2)])
def test_wide_synthesis_alm2map(torch_dev, tmp_path, name, dt, tol, nside, lmax, nmaps, nt):
    """Synthesis of random alm (the wide kernel alone) against the oracle, every map."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    alms = np.stack([random_alm(lmax, 10 + i) for i in range(nmaps)])
    cl = np.ones(lmax + 1)
    ninv = np.ones(12 * nside * nside)
    out = {}
    for wide in (nt, 0):
        with mwf.Plan(nside, lmax, cl, ninv, dtype=dt, max_batch=nmaps,
                      tune_cache=_cache(tmp_path, dt, nside, lmax, nmaps, wide)) as p:
            mp = p.alm2map(torch.from_numpy(alms.astype(np.complex64)).cuda())
            p.sync()
            out[wide] = mp.double().cpu().numpy()
    errs = [rel_l2(out[nt][i], sht.alm2map(alms[i].astype(np.complex64).astype(np.complex128), nside, lmax))
            for i in range(nmaps)]
    e_kern = rel_l2(out[nt], out[0])
    _log(f"wide synthesis ({nt} column tiles) {name} Nside {nside} lmax {lmax} x{nmaps}: vs oracle max {max(errs):.2e}, "
         f"vs per-wave kernel {e_kern:.2e}")
    assert max(errs) <= 1e-5 and e_kern <= 1e-5


@pytest.mark.parametrize("name,dt,tol", MODES)
@pytest.mark.parametrize("nt", [1, 2])
def test_wide_synthesis_solve(torch_dev, tmp_path, name, dt, tol, nt):
    """Full solves of a 6-map batch with the wide kernel against the oracle."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax, nmaps = 32, 64, 6
    cases = [small_band_inputs(nside, lmax, seed=s) for s in range(nmaps)]
    c0 = cases[0]
    d = np.stack([c["d"] for c in cases])
    sched = np.concatenate([np.geomspace(1e4, 1.0, 12), np.ones(10)])
    with mwf.Plan(nside, lmax, c0["cl"], c0["ninv"], dtype=dt, max_batch=nmaps,
                  tune_cache=_cache(tmp_path, dt, nside, lmax, nmaps, nt)) as p:
        s, a = p.solve(torch.from_numpy(d.astype(np.float32)).cuda(), sched)
        p.sync()
        s, a = s.double().cpu().numpy(), a.to(torch.complex128).cpu().numpy()
    worst = 0.0
    for i in range(nmaps):
        ref_s, ref_a = messenger.solve(d[i].astype(np.float32).astype(np.float64), c0["ninv"], c0["cl"], sched,
                                       nside, lmax)
        worst = max(worst, rel_l2(s[i], ref_s), alm_rel_l2(a[i], ref_a, lmax))
    _log(f"wide synthesis {name}: {len(sched)}-sweep solve of {nmaps} maps, worst vs oracle {worst:.2e}")
    assert worst <= tol
