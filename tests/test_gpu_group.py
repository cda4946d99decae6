"""GPU parity of task groups: plans of different nside / lmax stepped together,
one launch per phase (wf_group_solve), against the same plans solved one by one
and against the FP64 oracle.

Bars: each group member within 1e-5 relative L2 of the oracle (the reduced-
precision bar); group and separate solves within 1e-6 of each other (they differ
only in the ring-phase launch shape, which may regroup FP32 FFT sums).
"""
import sys

import numpy as np
import pytest

from oracle import messenger
from tests.helpers import alm_rel_l2, rel_l2, small_band_inputs

pytestmark = pytest.mark.gpu

SHAPES = [(16, 32, 3), (32, 64, 2), (64, 128, 1), (8, 16, 4)]
LAMS = np.geomspace(3e3, 1.0, 12)


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


def _cases():
    out = []
    for i, (nside, lmax, nm) in enumerate(SHAPES):
        cs = [small_band_inputs(nside, lmax, seed=10 * i + j) for j in range(nm)]
        d = np.stack([c["d"] for c in cs]).astype(np.float32)
        # the maps of one plan share C_l and N^-1 (those of the first draw)
        out.append(dict(nside=nside, lmax=lmax, nmaps=nm, cl=cs[0]["cl"], ninv=cs[0]["ninv"], d=d))
    return out


@pytest.fixture(scope="module")
def cases():
    return _cases()


def _plans(mwf, cases, dt):
    return [mwf.Plan(c["nside"], c["lmax"], c["cl"], c["ninv"], dtype=dt, max_batch=c["nmaps"]) for c in cases]


@pytest.mark.parametrize("name,dt", [("f32", 1), ("bf16x6", 3)])
def test_group_matches_separate_and_oracle(torch_dev, cases, name, dt):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    plans = _plans(mwf, cases, dt)
    ds = [torch.from_numpy(c["d"]).cuda() for c in cases]
    g = mwf.Group(plans, [c["nmaps"] for c in cases])
    gw, ga = g.solve(ds, LAMS)
    torch.cuda.synchronize()
    for i, (c, p) in enumerate(zip(cases, plans)):
        sw, sa = p.solve(ds[i], LAMS)
        p.sync()
        gwi, gai = gw[i].cpu().numpy(), ga[i].cpu().numpy()
        swi, sai = sw.cpu().numpy(), sa.cpu().numpy()
        e_sep = rel_l2(gwi, swi)
        e_sep_alm = max(alm_rel_l2(gai[k], sai[k], c["lmax"]) for k in range(c["nmaps"]))
        e_or = 0.0
        for k in range(c["nmaps"]):
            ref_map, ref_alm = messenger.solve(c["d"][k].astype(np.float64), c["ninv"], c["cl"], LAMS,
                                               c["nside"], c["lmax"])
            e_or = max(e_or, rel_l2(gwi[k], ref_map), alm_rel_l2(gai[k], ref_alm, c["lmax"]))
        _log(f"group {name} Nside {c['nside']} lmax {c['lmax']} x{c['nmaps']}: vs separate "
             f"{e_sep:.2e}/{e_sep_alm:.2e} (bitwise {np.array_equal(gwi, swi)}), vs oracle {e_or:.2e}")
        assert e_sep <= 1e-6 and e_sep_alm <= 1e-6
        assert e_or <= 1e-5
    g.close()
    for p in plans:
        p.close()


def test_group_autotune_and_resolve(torch_dev, cases):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    plans = _plans(mwf, cases, mwf.WF_F32)
    ds = [torch.from_numpy(c["d"]).cuda() for c in cases]
    g = mwf.Group(plans, [c["nmaps"] for c in cases])
    ct, nct = g.autotune(ds)
    _log(f"group autotune: ana_ct {ct} syn_nct {nct}")
    assert ct in (1, 2) and nct in (1, 2, 4, 8)
    w1, a1 = g.solve(ds, LAMS)
    w2, a2 = g.solve(ds, LAMS)   # a repeated solve reuses the task table
    torch.cuda.synchronize()
    for i in range(len(cases)):
        assert torch.equal(w1[i], w2[i]) and torch.equal(a1[i], a2[i])
    g.close()
    for p in plans:
        p.close()


def test_plan_autotune_keeps_results(torch_dev, cases):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c = cases[1]
    d = torch.from_numpy(c["d"]).cuda()
    with mwf.Plan(c["nside"], c["lmax"], c["cl"], c["ninv"], dtype=mwf.WF_F32, max_batch=c["nmaps"]) as p:
        w0, a0 = p.solve(d, LAMS)
        p.sync()
        w0 = w0.cpu().numpy()
        ct, nct = p.autotune()
        assert ct in (1, 2) and nct in (1, 2, 4, 8)
        w1, a1 = p.solve(d, LAMS)
        p.sync()
        e = rel_l2(w1.cpu().numpy(), w0)
        _log(f"plan autotune ({ct}, {nct}): change vs default shape {e:.2e}")
        assert e <= 1e-6
    with mwf.Plan(c["nside"], c["lmax"], c["cl"], c["ninv"], dtype=mwf.WF_F64) as p:
        assert p.autotune() == (0, 0)


def test_group_rejects_bad_input(torch_dev, cases):
    from paper_1211_0585_amd import mwf
    c = cases[0]
    p64 = mwf.Plan(c["nside"], c["lmax"], c["cl"], c["ninv"], dtype=mwf.WF_F64)
    p32 = mwf.Plan(c["nside"], c["lmax"], c["cl"], c["ninv"], dtype=mwf.WF_F32, max_batch=2)
    pbf = mwf.Plan(c["nside"], c["lmax"], c["cl"], c["ninv"], dtype=mwf.WF_BF16X6)
    with pytest.raises(mwf.WFError) as e:
        mwf.Group([p64], [1])
    assert e.value.code == mwf.WF_EUNSUPPORTED
    with pytest.raises(mwf.WFError) as e:
        mwf.Group([p32, pbf], [1, 1])
    assert e.value.code == mwf.WF_EINVAL
    with pytest.raises(mwf.WFError) as e:
        mwf.Group([p32], [3])
    assert e.value.code == mwf.WF_EINVAL
    for p in (p64, p32, pbf):
        p.close()


def test_group_of_more_tasks_than_one_launch_holds(torch_dev):
    """A group larger than the tasks one launch carries runs each phase in parts;
    every member must still equal its plan solved alone."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    shapes = [(8, 16, 1), (16, 32, 2), (8, 12, 3), (16, 24, 1), (32, 64, 1), (8, 16, 2), (16, 32, 1),
              (8, 10, 1), (16, 20, 2), (8, 16, 1), (32, 40, 1)]
    plans, ds = [], []
    for i, (nside, lmax, nm) in enumerate(shapes):
        c = small_band_inputs(nside, lmax, seed=200 + i)
        plans.append(mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=mwf.WF_F32, max_batch=nm))
        d = np.stack([small_band_inputs(nside, lmax, seed=300 + 10 * i + j)["d"] for j in range(nm)])
        ds.append(torch.from_numpy(d.astype(np.float32)).cuda())
    g = mwf.Group(plans, [s[2] for s in shapes])
    gw, ga = g.solve(ds, LAMS)
    torch.cuda.synchronize()
    worst = 0.0
    for i, p in enumerate(plans):
        sw, sa = p.solve(ds[i], LAMS)
        p.sync()
        e = rel_l2(gw[i].cpu().numpy(), sw.cpu().numpy())
        worst = max(worst, e)
        assert e <= 1e-6, (i, shapes[i], e)
    _log(f"group of {len(shapes)} tasks vs separate: worst {worst:.2e}")
    g.close()
    for p in plans:
        p.close()


def test_uneven_batch_real_shapes_vs_oracle(torch_dev):
    """The uneven batch at its real shapes (32 maps at Nside 128 / lmax 256, 16 at
    256 / 512, 8 at 512 / 1024; satellite recipe at each Nside with N_obs scaled by
    (512 / Nside)^2) as one FP32 task group, two sweeps (lambda = 100, 1): the first
    and last member of each shape against the oracle's solve of the same data
    (<= 1e-5), every member against its plan solved alone (<= 1e-6)."""
    torch = torch_dev
    from paper_1211_0585_amd import mwf, synth
    shapes = [(128, 256, 32), (256, 512, 16), (512, 1024, 8)]
    lams = np.array([100.0, 1.0])
    plans, ds, host, models = [], [], [], []
    for i, (nside, lmax, n) in enumerate(shapes):
        th, ph = mwf.pixel_angles(nside)
        model = synth.satellite_model(th, ph, lmax, nobs_scale=(512.0 / nside) ** 2)
        # data: a seeded noise draw of the model plus a seeded white field (all from the
        # input generator)
        d = np.stack([synth.draw(model, s)["noise"] + 50.0 * synth.rng(500 + 10 * i + s, 3).standard_normal(th.size)
                      for s in range(n)]).astype(np.float32)
        plans.append(mwf.Plan(nside, lmax, model["cl"], model["ninv"], dtype=mwf.WF_F32, max_batch=n))
        ds.append(torch.from_numpy(d).cuda())
        host.append(d)
        models.append(model)
    g = mwf.Group(plans, [n for _, _, n in shapes])
    gw, ga = g.solve(ds, lams)
    torch.cuda.synchronize()
    for i, ((nside, lmax, n), p) in enumerate(zip(shapes, plans)):
        sw, sa = p.solve(ds[i], lams)
        p.sync()
        gwi, gai = gw[i].cpu().numpy(), ga[i].cpu().numpy()
        e_sep = max(rel_l2(gwi[k], sw[k].cpu().numpy()) for k in range(n))
        e_or = 0.0
        for k in (0, n - 1):
            ref_map, ref_alm = messenger.solve(host[i][k].astype(np.float64), models[i]["ninv"], models[i]["cl"],
                                               lams, nside, lmax)
            e_or = max(e_or, rel_l2(gwi[k], ref_map), alm_rel_l2(gai[k], ref_alm, lmax))
        _log(f"uneven batch {n}@({nside},{lmax}): members vs alone {e_sep:.2e}, first/last vs oracle {e_or:.2e}")
        assert e_sep <= 1e-6 and e_or <= 1e-5
    g.close()
    for p in plans:
        p.close()
