"""GPU parity of the band-limited and adaptive solves (Sect. 3: adaptive cooling of
lambda, transforms cut at l_iter + margin) against the oracle.

  * wf_solve_banded vs oracle.adaptive.solve_banded on the same data and schedule:
    s_WF map and alm (full layout) within 1e-10 (FP64) / 1e-5 (FP32, bf16x6), the
    chi^2 history within 1e-10 / 1e-5; band limits from 0 to lmax, including
    jumps; Nside 16 and the Nside-512 plan with band limits up to 200.
  * wf_solve_adaptive vs oracle.adaptive.solve_adaptive (FP64, Nside 16 and 32):
    the same levels, band limits and sweep count (the decisions are FP64 on both
    sides), chi^2 and the result within 1e-10. FP32 plans take their decisions
    on FP32 chi^2, so their schedule is compared with the oracle's replay of it.
  * At Nside 512 (default options: l_iter from 20, margin 100): the adaptive
    result equals wf_solve_banded replaying the schedule it took, the lambdas are
    those of the level table, and the band limits only rise.
"""
import sys

import numpy as np
import pytest

from oracle import adaptive, healpix, sht
from tests.helpers import alm_rel_l2, rel_l2, small_band_inputs

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


TOL = {0: 1e-10, 1: 1e-5, 3: 1e-5}
RT = {0: np.float64, 1: np.float32, 3: np.float32}


def _gpu_banded(torch, mwf, nside, lmax, c, d, lams, bands, dt):
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=dt, flags=mwf.WF_FLAG_CHI2) as p:
        s, a = p.solve_banded(torch.from_numpy(d.astype(RT[dt])).cuda(), lams, bands)
        hist = p.chi2(1, len(lams))[0]
        last = p.last_stats.chi2_last
        p.sync()
        return s.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.complex128), hist, last


@pytest.mark.parametrize("name,dt", [("f64", 0), ("f32", 1), ("bf16x6", 3)])
@pytest.mark.parametrize("bands", [[0, 3, 3, 6, 6, 12, 20, 32, 32, 32],
                                   [6, 6, 32, 32, 32, 32, 32, 32, 32, 32],
                                   [2, 2, 2, 2, 2, 2, 2, 2, 2, 9]])
def test_banded_parity_nside16(torch_dev, name, dt, bands):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 16, 32
    c = small_band_inputs(nside, lmax, seed=11)
    d = c["d"].astype(RT[dt]).astype(np.float64)
    lams = np.geomspace(300.0, 1.0, len(bands))
    _log(f"banded {name} Nside {nside} bands {bands}")
    m_ref, a_ref, chi_ref = adaptive.solve_banded(d, c["ninv"], c["cl"], lams, bands, nside, lmax)
    m, a, hist, last = _gpu_banded(torch, mwf, nside, lmax, c, d, lams, bands, dt)
    e_map, e_alm = rel_l2(m, m_ref), alm_rel_l2(a, a_ref, lmax)
    e_chi = float(np.max(np.abs(hist - chi_ref) / np.abs(chi_ref)))
    _log(f"  map {e_map:.2e} alm {e_alm:.2e} chi2 {e_chi:.2e}")
    assert e_map <= TOL[dt] and e_alm <= TOL[dt] and e_chi <= TOL[dt]
    assert last == hist[-1]
    # nothing above the last band limit
    top = bands[-1]
    ell = sht.alm_ell(lmax)
    assert np.all(a[ell > top] == 0)


def test_banded_rejects_bad_schedules(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 8, 16
    c = small_band_inputs(nside, lmax, seed=1)
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"]) as p:
        d = torch.from_numpy(c["d"]).cuda()
        for bands in ([4, 2], [4, 17], [-1, 3]):
            with pytest.raises(mwf.WFError) as e:
                p.solve_banded(d, [10.0, 1.0], bands)
            assert e.value.code == mwf.WF_EINVAL
        with pytest.raises(mwf.WFError) as e:
            p.solve_adaptive(d, 0)
        assert e.value.code == mwf.WF_EINVAL
        with pytest.raises(mwf.WFError) as e:
            p.solve_adaptive(d, 10, l_pad=-2)
        assert e.value.code == mwf.WF_EINVAL
        # the plan still works after the rejected calls
        s, _ = p.solve_banded(d, [10.0, 1.0], [4, 16])
        p.sync()
        assert np.isfinite(s.cpu().numpy()).all()


ADAPT = [
    # (nside, lmax, seed, options, max_sweeps)
    (16, 32, 0, dict(l_iter0=2, l_pad=4), 300),
    (16, 32, 3, dict(l_iter0=2, l_pad=4, plateau_tol=0.2, max_level_sweeps=6), 300),
    (32, 64, 1, dict(l_iter0=4, l_pad=8), 400),
    (16, 32, 0, dict(l_iter0=2, l_pad=4, full_band=1), 300),
    (16, 32, 0, dict(l_iter0=2, l_pad=4), 1),
    (16, 32, 0, dict(l_iter0=2, l_pad=4), 2),
    (16, 32, 0, dict(l_iter0=2, l_pad=4), 7),
]


@pytest.mark.parametrize("nside,lmax,seed,opts,max_sweeps", ADAPT)
def test_adaptive_parity_f64(torch_dev, nside, lmax, seed, opts, max_sweeps):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c = small_band_inputs(nside, lmax, seed=seed)
    ao = mwf.adaptive_opts(**opts)
    o = {k: getattr(ao, k) for k, _ in ao._fields_}
    _log(f"adaptive f64 Nside {nside} seed {seed} opts {o} max {max_sweeps}")
    m_ref, a_ref, info = adaptive.solve_adaptive(c["d"], c["ninv"], c["cl"], nside, lmax, max_sweeps,
                                                 l_iter0=o["l_iter0"], l_pad=o["l_pad"],
                                                 full_band=bool(o["full_band"]),
                                                 max_level_sweeps=o["max_level_sweeps"],
                                                 plateau_tol=o["plateau_tol"], stop_tol=o["stop_tol"])
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"]) as p:
        s, a, got = p.solve_adaptive(torch.from_numpy(c["d"]).cuda(), max_sweeps, **opts)
        p.sync()
        hist = p.chi2(1, len(got["chi2"]))[0]
        m, a = s.cpu().numpy(), a.cpu().numpy()
    _log(f"  sweeps {len(got['chi2'])} (oracle {len(info['chi2'])}), bands {sorted(set(got['lmax_sht']))}, "
         f"converged {got['converged']}")
    assert list(got["lmax_sht"]) == list(info["lmax_sht"])
    assert np.allclose(got["lambdas"], info["lambdas"], rtol=1e-14, atol=0)
    assert got["converged"] == info["converged"]
    e_chi = float(np.max(np.abs(got["chi2"] - info["chi2"]) / info["chi2"]))
    e_map, e_alm = rel_l2(m, m_ref), alm_rel_l2(a, a_ref, lmax)
    _log(f"  map {e_map:.2e} alm {e_alm:.2e} chi2 {e_chi:.2e}")
    assert e_map <= 1e-10 and e_alm <= 1e-10 and e_chi <= 1e-10
    assert np.array_equal(hist, got["chi2"])


def test_adaptive_f32_matches_oracle_replay(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 16, 32
    c = small_band_inputs(nside, lmax, seed=0)
    d32 = c["d"].astype(np.float32)
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=mwf.WF_F32) as p:
        s, a, got = p.solve_adaptive(torch.from_numpy(d32).cuda(), 300, l_iter0=2, l_pad=4)
        p.sync()
        m, a = s.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.complex128)
    m_ref, a_ref, chi_ref = adaptive.solve_banded(d32.astype(np.float64), c["ninv"], c["cl"], got["lambdas"],
                                                  got["lmax_sht"], nside, lmax)
    e_map, e_alm = rel_l2(m, m_ref), alm_rel_l2(a, a_ref, lmax)
    e_chi = float(np.max(np.abs(got["chi2"] - chi_ref) / np.abs(chi_ref)))
    _log(f"adaptive f32 Nside 16: {len(got['chi2'])} sweeps, map {e_map:.2e} alm {e_alm:.2e} chi2 {e_chi:.2e}")
    assert len(set(got["lmax_sht"])) > 2
    assert e_map <= 1e-5 and e_alm <= 1e-5 and e_chi <= 1e-5


def _case512_plan_inputs():
    """Nside-512 satellite recipe (C_l, N^-1, mask of the lmax-1024 case); the data
    map is the seeded signal cut at l <= 64 (oracle synthesis) plus the seeded
    noise, so that the oracle can run the band-limited sweeps."""
    from paper_1211_0585_amd import synth
    theta, phi = healpix.pixel_angles(512)
    c = synth.satellite_case(theta, phi, 1024, seed=0)
    sig = sht.alm2map(_cut_alm(c["signal_alm"], 1024, 64), 512, 64)
    c["d"] = sig + c["noise"]
    return c


def _cut_alm(alm, lmax, L):
    from oracle.legendre import alm_index, n_alm
    out = np.zeros(n_alm(L), dtype=np.complex128)
    for m in range(L + 1):
        out[alm_index(L, m, m):alm_index(L, L, m) + 1] = alm[alm_index(lmax, m, m):alm_index(lmax, L, m) + 1]
    return out


@pytest.fixture(scope="module")
def sat512():
    return _case512_plan_inputs()


@pytest.mark.parametrize("name,dt", [("f64", 0), ("f32", 1)])
def test_banded_parity_nside512(torch_dev, sat512, name, dt):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c = sat512
    lams = [400.0, 150.0, 150.0, 20.0]
    bands = [48, 64, 64, 200]
    d = c["d"].astype(RT[dt]).astype(np.float64)
    _log(f"banded {name} Nside 512 lmax 1024 bands {bands}")
    m_ref, a_ref, chi_ref = adaptive.solve_banded(d, c["ninv"], c["cl"], lams, bands, 512, 1024)
    m, a, hist, _ = _gpu_banded(torch, mwf, 512, 1024, c, d, lams, bands, dt)
    e_map, e_alm = rel_l2(m, m_ref), alm_rel_l2(a, a_ref, 1024)
    e_chi = float(np.max(np.abs(hist - chi_ref) / np.abs(chi_ref)))
    _log(f"  map {e_map:.2e} alm {e_alm:.2e} chi2 {e_chi:.2e}")
    assert e_map <= TOL[dt] and e_alm <= TOL[dt] and e_chi <= TOL[dt]


def test_adaptive_nside512_replays_as_banded(torch_dev, sat512):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c = sat512
    with mwf.Plan(512, 1024, c["cl"], c["ninv"]) as p:
        d = torch.from_numpy(c["d"]).cuda()
        s, a, got = p.solve_adaptive(d, 160)
        s2, a2 = p.solve_banded(d, got["lambdas"], got["lmax_sht"])
        p.sync()
        lv = mwf.adaptive_levels(1024, c["cl"], p.tau, healpix.pixel_area(512))
        m, a, m2, a2 = s.cpu().numpy(), a.cpu().numpy(), s2.cpu().numpy(), a2.cpu().numpy()
    bands = list(got["lmax_sht"])
    _log(f"adaptive Nside 512: {len(bands)} sweeps, levels {lv}, bands {sorted(set(bands))}, "
         f"chi2 first {got['chi2'][0]:.6g} last {got['chi2'][-1]:.6g}, converged {got['converged']}")
    assert bands == sorted(bands) and bands[0] == lv[0][1]
    for lam, band in zip(got["lambdas"], bands):
        assert any(abs(lam - x) <= 1e-14 * x and band == b for x, b in lv)
    assert np.array_equal(m, m2) and np.array_equal(a, a2)
    assert got["chi2"][-1] < got["chi2"][0]
