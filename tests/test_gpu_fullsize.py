"""Full-size GPU parity: the satellite-scale solve (Nside 512, lmax 1024) in the
launch configurations the benchmark times, and the Nside-1024 / lmax-2048
precision variant.

Nside 512: the FP64 oracle's solve of the seed-0 case is stored in
tests/golden/nside512_satellite.npz (written by tests/golden/make_golden.py from
the oracle alone: sampled pixels and alm, norms, projections on seeded random
vectors, and per ring and per m a projection, checked as the worst ring and worst m
within 10 times the bar). The GPU builds the same data map with its FP64 synthesis, checked
against the oracle's map through the stored norm, head and projections, then
solves: plain FP64 one map (<= 1e-10), and the 64-map matrix-core batch with
the case as map 0 (FP32 and bf16x6 <= 1e-5; bf16x3 <= 5e-5, its stated accuracy, below
the 1e-5 bar), plus batch
composition: maps solved alone equal their batch results (<= 1e-6).

Nside 1024: the FP64 oracle's solve of the seed-0 precision case (satellite recipe,
N_obs / 4) under a 4-sweep schedule ending at lambda = 1 is stored in
tests/golden/nside1024_satellite.npz (tests/golden/make_golden_1024.py, oracle only):
FP64 <= 1e-10, FP32 and bf16x6 <= 1e-5 on sampled pixels, sampled alm, norms,
projections and the worst ring and worst m of per-ring / per-m projections. Besides:
sampled outputs the oracle computes directly (whole m columns of the analysis, the
synthesis of alm restricted to those columns at every pixel), the full-sky
uniform-noise closed form of the solve on those columns, and the agreement of the
reduced-precision 80-sweep solves with the FP64 one.
"""
import os
import sys

import numpy as np
import pytest

from oracle import healpix, messenger, sht
from oracle.legendre import alm_index
from paper_1211_0585_amd import synth
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nside512_satellite.npz")
GOLDEN10 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nside1024_satellite.npz")
N5, L5 = 512, 1024
N10, L10 = 1024, 2048
MS = [0, 1, 2, 255, 1023, 1024, 2000, 2047, 2048]
# Solve bars against the FP64 oracle: FP32 and bf16x6 meet the 1e-5 bar. bf16x3 (two bf16
# pieces, three products) does not: its pieces leave ~2^-18 of each operand unrepresented
# and it drops lo*lo, so a full 80-sweep solve lands at ~2-4e-5; it is checked against
# that stated accuracy, 5e-5, and is not counted as meeting the bar.
SOLVE_TOL = {1: 1e-5, 3: 1e-5, 2: 5e-5}
MODES = [("f32", 1), ("bf16x6", 3), ("bf16x3", 2)]


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


@pytest.fixture(scope="module")
def case512(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing (python tests/golden/make_golden.py)")
    g = dict(np.load(GOLDEN))
    theta, phi = healpix.pixel_angles(N5)
    c = synth.satellite_case(theta, phi, L5, seed=0)
    with mwf.Plan(N5, L5, c["cl"], c["ninv"], mask=~c["mask"]) as p:
        sig = p.alm2map(torch.from_numpy(c["signal_alm"]).cuda())
        d = (sig + torch.from_numpy(c["noise"]).cuda()).cpu().numpy()
    proj = np.random.default_rng(77).standard_normal((4, d.size))
    e_in = max(abs(np.linalg.norm(d) - g["d_norm"]) / g["d_norm"], rel_l2(d[:64], g["d_head"]),
               rel_l2(proj @ d, g["d_proj"]))
    _log(f"Nside 512 input: GPU synthesis vs oracle data map {e_in:.2e}")
    assert e_in <= 1e-12
    return c, d, g, proj


def _assert_vs_golden(e, tol):
    """The sampled, norm and projection errors within tol; the worst ring and worst m
    (when the stored values hold per-ring / per-m projections) within 10 tol: a projection
    on a random vector changes by about the local error norm, so a factor 10 above the bar
    still flags any ring or m with a local error near it."""
    assert max(e[k] for k in ("pix", "alm", "norm", "proj")) <= tol
    if "worst_ring" in e:
        assert e["worst_ring"] <= 10 * tol and e["worst_m"] <= 10 * tol


def test_plain_f64_nside512_vs_oracle(torch_dev, case512):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c, d, g, proj = case512
    sched = c["schedule"]
    with mwf.Plan(N5, L5, c["cl"], c["ninv"], mask=~c["mask"]) as p:
        dt = torch.from_numpy(d).cuda()
        for prefix, lam in (("two_", sched[:2]), ("full_", sched)):
            s, a = p.solve(dt, lam)
            p.sync()
            e = _vs_golden_full(prefix, g, s.cpu().numpy(), a.cpu().numpy(), L5, N5)
            _log(f"plain FP64 Nside 512, {len(lam)} sweeps vs oracle: {e}")
            _assert_vs_golden(e, 1e-10)


@pytest.mark.parametrize("name,dt", MODES)
def test_batched64_nside512_vs_oracle_and_alone(torch_dev, case512, name, dt):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c, d, g, proj = case512
    B = 64
    model = {k: c[k] for k in ("cl", "sigma2", "mask", "ninv", "schedule", "lmax")}
    alms = np.stack([synth.draw(model, s)["signal_alm"] for s in range(1, B)]).astype(np.complex64)
    noise = np.stack([synth.draw(model, s)["noise"] for s in range(1, B)]).astype(np.float32)
    with mwf.Plan(N5, L5, c["cl"], c["ninv"], mask=~c["mask"], dtype=dt, max_batch=B) as p:
        rest = p.alm2map(torch.from_numpy(alms).cuda()) + torch.from_numpy(noise).cuda()
        D = torch.cat([torch.from_numpy(d.astype(np.float32)).cuda()[None], rest]).contiguous()
        s, a = p.solve(D, c["schedule"])
        p.sync()
        s0, a0 = s[0].double().cpu().numpy(), a[0].to(torch.complex128).cpu().numpy()
        e = _vs_golden_full("full_", g, s0, a0, L5, N5)
        _log(f"batched {name} x{B} Nside 512, map 0 vs oracle: {e}")
        _assert_vs_golden(e, SOLVE_TOL[dt])
    with mwf.Plan(N5, L5, c["cl"], c["ninv"], mask=~c["mask"], dtype=dt, max_batch=1) as p1:
        for i in (0, 37):
            si, _ = p1.solve(D[i].contiguous(), c["schedule"], want_alm=False)
            p1.sync()
            e = rel_l2(si.cpu().numpy(), s[i].cpu().numpy())
            _log(f"batched {name}: map {i} alone vs in the batch {e:.2e} (bitwise {bool(torch.equal(si, s[i]))})")
            assert e <= 1e-6


def _vs_golden_full(prefix, g, s_map, s_alm, lmax, nside):
    """Sampled pixels and alm, the map norm and four projections against the stored values,
    plus the worst ring and worst m (when stored): per-ring / per-m projections on seeded
    random vectors against the stored ones, relative to that ring's / m's norm."""
    rs = np.random.default_rng(77)
    proj = rs.standard_normal((4, s_map.size))
    w = sht.alm_weights(lmax)[g[prefix + "alm_idx"]]
    out = {"pix": rel_l2(s_map[g[prefix + "pix_idx"]], g[prefix + "pix_val"]),
           "alm": rel_l2(s_alm[g[prefix + "alm_idx"]], g[prefix + "alm_val"], w),
           "norm": abs(np.linalg.norm(s_map) - g[prefix + "map_norm"]) / g[prefix + "map_norm"],
           "proj": rel_l2(proj @ s_map, g[prefix + "map_proj"])}
    if prefix + "ring_proj" in g:
        ri = healpix.ring_info(nside)
        v = np.random.default_rng(99).standard_normal(s_map.size)
        rp = np.add.reduceat(v * s_map, ri["start"])
        # relative to each ring's (m's) norm, floored at 1e-6 of the largest: columns of
        # almost no power (the highest m, where the GPU leaves out values below 2^-448)
        # are compared at the precision they contribute to the whole
        rn = np.maximum(g[prefix + "ring_norm"], 1e-6 * g[prefix + "ring_norm"].max())
        out["worst_ring"] = float(np.max(np.abs(rp - g[prefix + "ring_proj"]) / rn))
        u = np.random.default_rng(98).standard_normal(s_alm.size) + 1j * np.random.default_rng(97).standard_normal(
            s_alm.size)
        mp = np.add.reduceat(u * s_alm, np.array([alm_index(lmax, m, m) for m in range(lmax + 1)]))
        mn = np.maximum(g[prefix + "m_norm"], 1e-6 * g[prefix + "m_norm"].max())
        out["worst_m"] = float(np.max(np.abs(mp - g[prefix + "m_proj"]) / mn))
    return out


@pytest.fixture(scope="module")
def case1024(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    if not os.path.exists(GOLDEN10):
        pytest.skip("golden file missing (python tests/golden/make_golden_1024.py)")
    g = dict(np.load(GOLDEN10))
    theta, phi = healpix.pixel_angles(N10)
    model = synth.satellite_model(theta, phi, L10, nobs_scale=0.25)
    dr = synth.draw(model, 0)
    with mwf.Plan(N10, L10, model["cl"], model["ninv"], mask=~model["mask"]) as p:
        d = (p.alm2map(torch.from_numpy(dr["signal_alm"]).cuda()) + torch.from_numpy(dr["noise"]).cuda()).cpu().numpy()
    proj = np.random.default_rng(77).standard_normal((4, d.size))
    e_in = max(abs(np.linalg.norm(d) - g["d_norm"]) / g["d_norm"], rel_l2(d[:64], g["d_head"]),
               rel_l2(proj @ d, g["d_proj"]))
    _log(f"Nside 1024 input: GPU synthesis vs oracle data map {e_in:.2e}")
    assert e_in <= 1e-12
    return model, d, g


@pytest.mark.parametrize("name,dt", [("f64", 0)] + MODES)
def test_nside1024_solve_vs_oracle(torch_dev, case1024, name, dt):
    """The precision workload (Nside 1024, lmax 2048) per dtype against the oracle's solve."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    model, d, g = case1024
    tol = 1e-10 if dt == 0 else SOLVE_TOL[dt]
    dd = torch.from_numpy(d if dt == 0 else d.astype(np.float32)).cuda()
    with mwf.Plan(N10, L10, model["cl"], model["ninv"], mask=~model["mask"], dtype=dt) as p:
        s, a = p.solve(dd, g["schedule"])
        p.sync()
        e = _vs_golden_full("sol_", g, s.double().cpu().numpy(), a.to(torch.complex128).cpu().numpy(), L10, N10)
    _log(f"Nside 1024 lmax 2048 {name}, {len(g['schedule'])} sweeps vs oracle: {e}")
    _assert_vs_golden(e, tol)


@pytest.fixture(scope="module")
def columns1024():
    rs = np.random.default_rng(1024)
    f = rs.standard_normal(healpix.npix(N10))
    ana = sht.map2alm_columns(f, N10, L10, MS)
    cols = {m: rs.standard_normal(L10 - m + 1) + 1j * rs.standard_normal(L10 - m + 1) for m in MS}
    cols[0] = cols[0].real.astype(np.complex128)
    syn = sht.alm2map_columns(cols, N10, L10)
    return f, ana, cols, syn


def _packed(cols, lmax):
    a = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    for m, v in cols.items():
        i0 = alm_index(lmax, m, m)
        a[i0:i0 + lmax - m + 1] = v
    return a


@pytest.mark.parametrize("name,dt,tol", [("f64", 0, 1e-12), ("f32", 1, 1e-5), ("bf16x6", 3, 1e-5),
                                         ("bf16x3", 2, 1e-5)])
def test_sht_nside1024_columns_vs_oracle(torch_dev, columns1024, name, dt, tol):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    f, ana, cols, syn = columns1024
    rt, ct = (np.float64, np.complex128) if dt == 0 else (np.float32, np.complex64)
    with mwf.Plan(N10, L10, np.ones(L10 + 1), np.ones(healpix.npix(N10)), dtype=dt) as p:
        alm = p.map2alm(torch.from_numpy(f.astype(rt)).cuda()).cpu().numpy()
        mp = p.alm2map(torch.from_numpy(_packed(cols, L10).astype(ct)).cuda()).cpu().numpy()
        p.sync()
    ref_f = f.astype(rt).astype(np.float64)
    ana_ref = ana if dt == 0 else sht.map2alm_columns(ref_f, N10, L10, MS)
    e_ana = max(rel_l2(alm[alm_index(L10, m, m):alm_index(L10, m, m) + L10 - m + 1], ana_ref[m]) for m in MS)
    syn_ref = syn if dt == 0 else sht.alm2map_columns(
        {m: v.astype(ct).astype(np.complex128) for m, v in cols.items()}, N10, L10)
    e_syn = rel_l2(mp, syn_ref)
    _log(f"Nside 1024 lmax 2048 {name}: analysis columns {e_ana:.2e}, synthesis of the columns {e_syn:.2e}")
    assert e_ana <= tol and e_syn <= tol


@pytest.mark.parametrize("name,dt,tol", [("f64", 0, 1e-12), ("f32", 1, 1e-5)])
def test_uniform_fullsky_closed_form_nside1024(torch_dev, name, dt, tol):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    npix = healpix.npix(N10)
    rs = np.random.default_rng(77)
    cl = synth.cl_satellite(L10)
    d = rs.standard_normal(npix) * 40.0
    ninv = np.full(npix, 1.0 / 30.0 ** 2)
    lams = np.geomspace(1e3, 2.0, 3)
    rt = np.float64 if dt == 0 else np.float32
    d_in = d.astype(rt)
    with mwf.Plan(N10, L10, cl, ninv, dtype=dt) as p:
        _, s_alm = p.solve(torch.from_numpy(d_in).cuda(), lams)
        p.sync()
        s_alm = s_alm.cpu().numpy()
    tau = messenger.tau_of(ninv)
    f_l = messenger.harmonic_filter(cl, lams[-1], tau, healpix.pixel_area(N10))
    ref = sht.map2alm_columns(d_in.astype(np.float64), N10, L10, MS)
    e = max(rel_l2(s_alm[alm_index(L10, m, m):alm_index(L10, m, m) + L10 - m + 1],
                   f_l[m:] * ref[m]) for m in MS if np.any(f_l[m:] > 0))
    _log(f"Nside 1024 uniform full sky {name}: solve alm vs closed form on sampled columns {e:.2e}")
    assert e <= tol


def test_precision_paths_nside1024_vs_fp64(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    theta, phi = healpix.pixel_angles(N10)
    model = synth.satellite_model(theta, phi, L10, nobs_scale=0.25)
    dr = synth.draw(model, 0)
    with mwf.Plan(N10, L10, model["cl"], model["ninv"], mask=~model["mask"]) as p:
        d = p.alm2map(torch.from_numpy(dr["signal_alm"]).cuda()) + torch.from_numpy(dr["noise"]).cuda()
        ref_w, ref_a = p.solve(d, model["schedule"])
        p.sync()
        ref_w, ref_a = ref_w.cpu().numpy(), ref_a.cpu().numpy()
    w = sht.alm_weights(L10)
    for name, dt in MODES:
        with mwf.Plan(N10, L10, model["cl"], model["ninv"], mask=~model["mask"], dtype=dt) as p:
            s, a = p.solve(d.float(), model["schedule"])
            p.sync()
            e_w = rel_l2(s.cpu().numpy(), ref_w)
            e_a = rel_l2(a.cpu().numpy(), ref_a, w)
        _log(f"Nside 1024 lmax 2048 satellite, 80 sweeps, {name} vs FP64: s_WF {e_w:.2e}, alm {e_a:.2e}")
        assert e_w <= SOLVE_TOL[dt] and e_a <= SOLVE_TOL[dt]
