"""GPU tests of the serving loop (wf_server_*): continuous batching of independent
solves, admission by HBM budget, and that each result is the same alone and in
the mix.

A request's map in a lane is one column of the lane's GEMMs and one set of ring
blocks; no sum mixes columns, so the served result should equal a one-map plan
solve of the same dtype. Bars: 1e-6 relative L2 against that alone solve (equal
bits expected and reported), 1e-5 against the FP64 oracle (the reduced-precision
bar).
"""
import sys
import time

import numpy as np
import pytest

from oracle import messenger
from tests.helpers import rel_l2, small_band_inputs

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


def _request(nside, lmax, seed, nsweeps):
    c = small_band_inputs(nside, lmax, seed=seed)
    rs = np.random.default_rng(1000 + seed)
    return dict(nside=nside, lmax=lmax, cl=c["cl"] * rs.uniform(0.5, 2.0), ninv=c["ninv"] * rs.uniform(0.5, 2.0),
                d=c["d"], lam=np.geomspace(rs.uniform(1e2, 1e4), 1.0, nsweeps))


def _random_request(nside, lmax, seed, nsweeps):
    rs = np.random.default_rng(seed)
    npix = 12 * nside * nside
    cl = np.r_[0.0, 0.0, 1.0 / np.arange(2, lmax + 1) ** 2]
    ninv = rs.uniform(0.2, 1.0, npix)
    ninv[rs.random(npix) < 0.2] = 0.0
    return dict(nside=nside, lmax=lmax, cl=cl, ninv=ninv, d=rs.standard_normal(npix),
                lam=np.geomspace(1e3, 1.0, nsweeps))


def _alone(torch, mwf, r, dtype):
    with mwf.Plan(r["nside"], r["lmax"], r["cl"], r["ninv"], dtype=dtype) as p:
        s, _ = p.solve(torch.from_numpy(r["d"].astype(np.float32)).cuda(), r["lam"], want_alm=False)
        p.sync()
        return s.cpu().numpy().astype(np.float64)


def _check_alone(torch, mwf, reqs, results, dtypes):
    for i, (r, (s_wf, lat)) in enumerate(zip(reqs, results)):
        ref = _alone(torch, mwf, r, dtypes[i])
        e = rel_l2(s_wf, ref)
        _log(f"request {i} Nside {r['nside']} lmax {r['lmax']} dtype {dtypes[i]} sweeps {len(r['lam'])}: "
             f"latency {lat * 1e3:.1f} ms, vs alone {e:.2e} (bitwise {np.array_equal(s_wf, ref)})")
        assert e <= 1e-6


def test_server_mix_equals_alone_and_oracle(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    shapes = [(16, 32, 10), (16, 32, 25), (32, 64, 15), (8, 16, 5), (16, 32, 40), (32, 64, 30), (8, 16, 50),
              (64, 128, 20)]
    reqs = [_request(n, l, 7 * i + 1, k) for i, (n, l, k) in enumerate(shapes)]
    with mwf.Server(hbm_budget=4 << 30, max_slots=16) as srv:
        tickets = [srv.submit(r["nside"], r["lmax"], r["cl"], r["ninv"], r["d"], r["lam"]) for r in reqs[:4]]
        time.sleep(0.005)   # the rest arrive while the first ones run
        tickets += [srv.submit(r["nside"], r["lmax"], r["cl"], r["ninv"], r["d"], r["lam"]) for r in reqs[4:]]
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    _log(f"server stats: {st}")
    assert st["completed"] == len(reqs) and st["peak_slots"] >= 2
    _check_alone(torch, mwf, reqs, results, [mwf.WF_F32] * len(reqs))
    for i in (0, 3):
        r = reqs[i]
        ref, _ = messenger.solve(r["d"].astype(np.float32).astype(np.float64), r["ninv"], r["cl"], r["lam"],
                                 r["nside"], r["lmax"])
        e = rel_l2(results[i][0], ref)
        _log(f"request {i} vs oracle {e:.2e}")
        assert e <= 1e-5


def test_server_mixed_dtypes(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    reqs = [_request(16, 32, 100 + i, 12 + 3 * i) for i in range(4)]
    dts = [mwf.WF_F32, mwf.WF_BF16X6, mwf.WF_BF16X3, mwf.WF_BF16X6]
    with mwf.Server(hbm_budget=1 << 30, max_slots=8) as srv:
        tickets = [srv.submit(r["nside"], r["lmax"], r["cl"], r["ninv"], r["d"], r["lam"], dtype=dt)
                   for r, dt in zip(reqs, dts)]
        results = [srv.wait(t) for t in tickets]
        assert srv.stats()["lanes"] == 3
    _check_alone(torch, mwf, reqs, results, dts)


def test_server_evicts_idle_lanes_under_budget(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    # three shapes of roughly 10 MB each (one-slot lane + the shape's tables) under a
    # 16 MiB budget: one lane fits at a time, so each new shape waits until the
    # previous lane is idle and evicted
    reqs = [_random_request(128, l, 50 + i, 6 + i) for i, l in enumerate([256, 255, 254, 256, 255, 254])]
    with mwf.Server(hbm_budget=16 << 20, max_slots=4) as srv:
        tickets = [srv.submit(r["nside"], r["lmax"], r["cl"], r["ninv"], r["d"], r["lam"]) for r in reqs]
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    _log(f"server stats: {st}")
    assert st["lanes_evicted"] >= 1 and st["peak_bytes"] <= 16 << 20
    _check_alone(torch, mwf, reqs, results, [mwf.WF_F32] * len(reqs))


def test_server_stream_of_requests(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    rs = np.random.default_rng(5)
    sizes = [(8, 16), (16, 32), (32, 64), (64, 128)]
    reqs = []
    for i in range(24):
        n, l = sizes[rs.integers(len(sizes))]
        reqs.append(_random_request(n, l, 300 + i, int(rs.integers(4, 30))))
    gaps = rs.exponential(0.002, len(reqs))
    with mwf.Server(hbm_budget=2 << 30, max_slots=12) as srv:
        tickets = []
        for r, g in zip(reqs, gaps):
            tickets.append(srv.submit(r["nside"], r["lmax"], r["cl"], r["ninv"], r["d"], r["lam"]))
            time.sleep(g)
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    _log(f"server stats: {st}")
    assert st["completed"] == len(reqs) and st["map_sweeps"] == sum(len(r["lam"]) for r in reqs)
    pick = [0, 5, 11, 17, 23]
    _check_alone(torch, mwf, [reqs[i] for i in pick], [results[i] for i in pick], [mwf.WF_F32] * len(pick))


def test_server_rejects_bad_requests(torch_dev):
    from paper_1211_0585_amd import mwf
    r = _random_request(8, 16, 1, 3)
    with mwf.Server(hbm_budget=16 << 20, max_slots=2) as srv:
        def code(**kw):
            a = dict(r)
            a.update(kw)
            with pytest.raises(mwf.WFError) as e:
                srv.submit(a["nside"], a["lmax"], a["cl"], a["ninv"], a["d"], a["lam"], dtype=a.get("dtype", 1))
            return e.value.code
        assert code(dtype=mwf.WF_F64) == mwf.WF_EUNSUPPORTED
        assert code(lam=np.array([1.0, -1.0])) == mwf.WF_EINVAL
        assert code(ninv=np.zeros_like(r["ninv"])) == mwf.WF_EINVAL
        d = r["d"].copy()
        d[3] = np.nan
        assert code(d=d) == mwf.WF_EINVAL
        big = _random_request(512, 1024, 2, 1)
        assert code(**big) == mwf.WF_ENOMEM
        srv._npix[12345] = 1        # a ticket the server never issued
        with pytest.raises(mwf.WFError) as e:
            srv.poll(12345)
        assert e.value.code == mwf.WF_EINVAL
        t = srv.submit(r["nside"], r["lmax"], r["cl"], r["ninv"], r["d"], r["lam"])
        s_wf, lat = srv.wait(t)
        assert np.all(np.isfinite(s_wf)) and lat > 0
