"""Polarised (T, Q, U) path on the GPU against the polarised oracle, through the C ABI.

Transforms (spin-0 T with spin-2 E/B) at Nside 1..64 including ragged band limits
and lmax up to 4 Nside - 1 (aliasing on every polar ring): <= 1e-12. Solves of the
small polarised case (TE-coupled spectra, 3x3 pixel noise with Q-U correlations,
separate T and P masks): <= 1e-10 on s_WF and on the alm, alone and in a batch (each
batch member equal to its solo run). Special cases: the uniform full-sky closed form,
T observed with Q/U masked everywhere and no TE (E = B = 0), a general 3x3 noise with
T-P correlations, and band limits with no E/B modes at all.
"""
import sys

import numpy as np
import pytest

from oracle import healpix, polar, sht
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


def _alm_err(x, ref, lmax):
    w = sht.alm_weights(lmax)
    return rel_l2(np.asarray(x), np.asarray(ref), np.broadcast_to(w, np.shape(ref)))


def _rand_alm(lmax, seed):
    rs = np.random.default_rng(seed)
    nalm = (lmax + 1) * (lmax + 2) // 2
    a = rs.standard_normal((3, nalm)) + 1j * rs.standard_normal((3, nalm))
    a[:, :lmax + 1] = a[:, :lmax + 1].real
    ell = sht.alm_ell(lmax)
    a[1:, ell < 2] = 0.0
    return a


def _plan_inputs(nside, lmax, seed=0):
    theta, _ = healpix.pixel_angles(nside)
    c = synth.pol_small_case(theta, lmax, seed=seed)
    return c


@pytest.mark.parametrize("nside,lmax", [(1, 0), (1, 3), (2, 7), (4, 9), (8, 16), (8, 31), (16, 33), (32, 64),
                                        (64, 128), (64, 255)])
def test_pol_sht_pair(torch_dev, nside, lmax):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c = _plan_inputs(nside, lmax)
    npix = 12 * nside * nside
    a = _rand_alm(lmax, 1)
    f = np.random.default_rng(2).standard_normal((3, npix))
    _log(f"pol SHT nside {nside} lmax {lmax}")
    with mwf.PolPlan(nside, lmax, c["cl4"], c["ninv6"], mask=c["mask"]) as p:
        m_gpu = p.alm2map(torch.from_numpy(a).cuda()).cpu().numpy()
        a_gpu = p.map2alm(torch.from_numpy(f).cuda()).cpu().numpy()
        p.sync()
    m_ref = polar.alm2map(a, nside, lmax)
    a_ref = polar.map2alm(f, nside, lmax)
    e1, e2 = rel_l2(m_gpu, m_ref), _alm_err(a_gpu, a_ref, lmax)
    _log(f"  alm2map {e1:.2e} map2alm {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12


def _solve_case(torch, nside, lmax, sched, nmaps=1, seeds=None, cl4=None, ninv6=None, mask=None):
    from paper_1211_0585_amd import mwf
    c = _plan_inputs(nside, lmax)
    cl4 = c["cl4"] if cl4 is None else cl4
    ninv6 = c["ninv6"] if ninv6 is None else ninv6
    mask = c["mask"] if mask is None else mask
    theta, _ = healpix.pixel_angles(nside)
    ds = []
    for s in (seeds or list(range(nmaps))):
        ci = synth.pol_small_case(theta, lmax, seed=s)
        ds.append(polar.alm2map(ci["signal_alm"], nside, lmax) + ci["noise"])
    d = np.stack(ds)
    with mwf.PolPlan(nside, lmax, cl4, ninv6, mask=mask, max_batch=len(ds)) as p:
        s_wf, s_alm = p.solve(torch.from_numpy(d).cuda(), sched)
        torch.cuda.synchronize()
        p.sync()
        return d, s_wf.cpu().numpy(), s_alm.cpu().numpy(), (cl4, ninv6, mask)


@pytest.mark.parametrize("nside,lmax,ncool,nfin", [(4, 8, 3, 2), (8, 16, 10, 10), (16, 32, 40, 100), (32, 64, 6, 4)])
def test_pol_solve_parity(torch_dev, nside, lmax, ncool, nfin):
    sched = synth.geometric_schedule(1e4, ncool, nfin)
    _log(f"pol solve nside {nside} lmax {lmax} sweeps {len(sched)}")
    d, s_wf, s_alm, (cl4, ninv6, mask) = _solve_case(torch_dev, nside, lmax, sched)
    ref_map, ref_alm = polar.solve(d[0], ninv6, cl4, sched, nside, lmax, mask=mask)
    e1, e2 = rel_l2(s_wf[0], ref_map), _alm_err(s_alm[0], ref_alm, lmax)
    _log(f"  s_WF {e1:.2e} alm {e2:.2e}")
    assert e1 <= 1e-10 and e2 <= 1e-10


def test_pol_batch_equals_alone(torch_dev):
    nside, lmax = 16, 32
    sched = synth.geometric_schedule(1e4, 5, 3)
    d, s_wf, s_alm, (cl4, ninv6, mask) = _solve_case(torch_dev, nside, lmax, sched, seeds=[0, 1, 2])
    for i in range(3):
        _, s1, a1, _ = _solve_case(torch_dev, nside, lmax, sched, seeds=[i])
        assert np.array_equal(s1[0], s_wf[i]) and np.array_equal(a1[0], s_alm[i])
        ref_map, _ = polar.solve(d[i], ninv6, cl4, sched, nside, lmax, mask=mask)
        e = rel_l2(s_wf[i], ref_map)
        _log(f"  batch member {i} vs oracle {e:.2e} (bitwise equal to its solo run)")
        assert e <= 1e-10


def test_pol_uniform_fullsky_closed_form(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 32, 64
    npix = 12 * nside * nside
    cl4 = synth.cl_pol(synth.cl_power_law(lmax))
    d = np.random.default_rng(9).standard_normal((1, 3, npix)) * 30.0
    n6 = np.zeros((6, npix))
    n6[:3] = 1.0 / 900.0
    sched = [300.0, 20.0, 1.7]
    with mwf.PolPlan(nside, lmax, cl4, n6) as p:
        s_wf, s_alm = p.solve(torch.from_numpy(d).cuda(), sched)
        torch.cuda.synchronize()
        s_alm = s_alm.cpu().numpy()[0]
    F = polar.harmonic_filter(cl4, 1.7, 900.0, healpix.pixel_area(nside))
    ref = polar.apply_filter(F, polar.map2alm(d[0], nside, lmax), lmax)
    e = _alm_err(s_alm, ref, lmax)
    _log(f"uniform full-sky closed form: {e:.2e}")
    assert e <= 1e-13


def test_pol_no_polarisation_data_gives_no_eb(torch_dev):
    """Q/U masked everywhere and TE = 0: E = B = 0 exactly, T equals the oracle."""
    nside, lmax = 16, 32
    c = _plan_inputs(nside, lmax)
    cl4 = c["cl4"].copy()
    cl4[3] = 0.0
    mask = (c["mask"] & 1).astype(np.uint8)
    sched = synth.geometric_schedule(1e3, 4, 3)
    d, s_wf, s_alm, _ = _solve_case(torch_dev, nside, lmax, sched, cl4=cl4, mask=mask)
    assert np.all(s_alm[0, 1:] == 0.0)
    ref_map, _ = polar.solve(d[0], c["ninv6"], cl4, sched, nside, lmax, mask=mask)
    assert rel_l2(s_wf[0], ref_map) <= 1e-10


def test_pol_general_3x3_noise(torch_dev):
    """T-Q and T-U noise correlations (a full 3x3 N^-1 per pixel)."""
    nside, lmax = 8, 16
    npix = 12 * nside * nside
    rs = np.random.default_rng(11)
    A = rs.standard_normal((npix, 3, 3))
    N = A @ np.transpose(A, (0, 2, 1)) + 0.5 * np.eye(3)
    Ni = np.linalg.inv(N) * 1e-3
    n6 = np.stack([Ni[:, 0, 0], Ni[:, 1, 1], Ni[:, 2, 2], Ni[:, 0, 1], Ni[:, 0, 2], Ni[:, 1, 2]])
    sched = synth.geometric_schedule(1e4, 8, 6)
    d, s_wf, s_alm, (cl4, _, mask) = _solve_case(torch_dev, nside, lmax, sched, ninv6=n6)
    ref_map, ref_alm = polar.solve(d[0], n6, cl4, sched, nside, lmax, mask=mask)
    e1, e2 = rel_l2(s_wf[0], ref_map), _alm_err(s_alm[0], ref_alm, lmax)
    _log(f"general 3x3 noise: s_WF {e1:.2e} alm {e2:.2e}")
    assert e1 <= 1e-10 and e2 <= 1e-10


@pytest.mark.parametrize("lmax", [0, 1, 2])
def test_pol_low_band_limits(torch_dev, lmax):
    nside = 4
    sched = [100.0, 1.0]
    d, s_wf, s_alm, (cl4, ninv6, mask) = _solve_case(torch_dev, nside, lmax, sched)
    ref_map, ref_alm = polar.solve(d[0], ninv6, cl4, sched, nside, lmax, mask=mask)
    assert rel_l2(s_wf[0], ref_map) <= 1e-10
    if lmax < 2:
        assert np.all(s_alm[0, 1:] == 0.0)


def test_pol_rejects_bad_inputs(torch_dev):
    from paper_1211_0585_amd import mwf
    nside, lmax = 4, 8
    c = _plan_inputs(nside, lmax)
    bad = c["cl4"].copy()
    bad[3, 5] = 2.0 * np.sqrt(bad[0, 5] * bad[1, 5])        # |TE| > sqrt(TT EE)
    with pytest.raises(mwf.WFError):
        mwf.PolPlan(nside, lmax, bad, c["ninv6"])
    bad = c["cl4"].copy()
    bad[1, 1] = 1.0                                          # EE at l = 1
    with pytest.raises(mwf.WFError):
        mwf.PolPlan(nside, lmax, bad, c["ninv6"])
    n6 = c["ninv6"].copy()
    n6[5] = 2.0 * np.sqrt(n6[1] * n6[2])                     # indefinite Q-U block
    with pytest.raises(mwf.WFError):
        mwf.PolPlan(nside, lmax, c["cl4"], n6)
    with pytest.raises(mwf.WFError):                         # nside not a power of two
        mwf.PolPlan(3, 4, np.zeros((4, 5)), np.ones((6, 108)) * [[1], [1], [1], [0], [0], [0]])


GOLDEN_POL = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.abspath(__file__)),
                                        "golden", "nside512_pol.npz")


def _field_errs(g, prefix, maps, alm, lmax, nside):
    """Per field: sampled pixels and alm, norms, worst ring and worst m of the seeded
    per-ring / per-m projections (norms floored at 1e-6 of the largest)."""
    ri = healpix.ring_info(nside)
    v = np.random.default_rng(99).standard_normal(maps.shape[1])
    u = (np.random.default_rng(98).standard_normal(alm.shape[1])
         + 1j * np.random.default_rng(97).standard_normal(alm.shape[1]))
    mstart = np.array([m * (2 * lmax + 1 - m) // 2 + m for m in range(lmax + 1)])
    w = sht.alm_weights(lmax)[g[prefix + "alm_idx"]]
    out = {}
    for f in range(3):
        k, ka = prefix + "TQU"[f] + "_", prefix + "TEB"[f] + "_"
        rp = np.add.reduceat(v * maps[f], ri["start"])
        rn = np.maximum(g[k + "ring_norm"], 1e-6 * g[k + "ring_norm"].max())
        mp = np.add.reduceat(u * alm[f], mstart)
        mn = np.maximum(g[ka + "m_norm"], 1e-6 * g[ka + "m_norm"].max())
        out["TQU"[f]] = max(rel_l2(maps[f][g[prefix + "pix_idx"]], g[k + "pix_val"]),
                            abs(np.linalg.norm(maps[f]) - g[k + "map_norm"]) / g[k + "map_norm"],
                            float(np.max(np.abs(rp - g[k + "ring_proj"]) / rn)) / 10)
        out["TEB"[f]] = max(rel_l2(alm[f][g[prefix + "alm_idx"]], g[ka + "alm_val"], w),
                            float(np.max(np.abs(mp - g[ka + "m_proj"]) / mn)) / 10)
    return out


def test_pol_nside512_vs_stored_oracle(torch_dev):
    """The satellite-scale polarised case (Nside 512, lmax 1024, 3-sweep schedule) against
    the oracle's stored solve (tests/golden/make_golden_pol.py): <= 1e-10 per field on
    sampled pixels and alm and norms, and <= 1e-9 on the worst ring / m projection."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    import os
    if not os.path.exists(GOLDEN_POL):
        pytest.skip("golden file missing (python tests/golden/make_golden_pol.py)")
    g = dict(np.load(GOLDEN_POL))
    nside, lmax = 512, 1024
    theta, phi = healpix.pixel_angles(nside)
    c = synth.pol_satellite_case(theta, phi, lmax, seed=0)
    with mwf.PolPlan(nside, lmax, c["cl4"], c["ninv6"], mask=c["mask"]) as p:
        d = p.alm2map(torch.from_numpy(c["signal_alm"]).cuda()) + torch.from_numpy(c["noise"]).cuda()
        a_d = p.map2alm(d)
        p.sync()
        e_in = _field_errs(g, "d_", d.cpu().numpy(), a_d.cpu().numpy(), lmax, nside)
        _log(f"Nside 512 polarised data map and its alm vs oracle: {e_in}")
        assert max(e_in.values()) <= 1e-12
        s, a = p.solve(d, g["schedule"])
        p.sync()
        e = _field_errs(g, "sol_", s.cpu().numpy(), a.cpu().numpy(), lmax, nside)
    _log(f"Nside 512 polarised solve, {len(g['schedule'])} sweeps vs oracle: {e}")
    assert max(e.values()) <= 1e-10
