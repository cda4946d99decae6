"""Plans driven from several host threads at once, in a fresh process: each thread
builds its own plan (different Nside, so their first launches raise the dynamic-LDS
limits of the same ring kernels concurrently) and solves on its own stream; every
result equals the same solve run alone afterwards, bit for bit."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, threading
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
from paper_1211_0585_amd import mwf
from tests.helpers import small_band_inputs
torch.cuda.init()
shapes = [(16, 32, 1), (32, 64, 1), (64, 128, 1), (128, 256, 1), (32, 64, 0), (64, 128, 0)]
lams = np.concatenate([np.geomspace(1e3, 1.0, 6), np.ones(4)])
cases = [small_band_inputs(n, l, seed=i) for i, (n, l, _) in enumerate(shapes)]
out = [None] * len(shapes)
err = []
def work(i):
    try:
        n, l, dt = shapes[i]
        c = cases[i]
        rt = np.float32 if dt else np.float64
        s = torch.cuda.Stream()
        with mwf.Plan(n, l, c["cl"], c["ninv"], dtype=dt) as p:
            with torch.cuda.stream(s):
                d = torch.from_numpy(c["d"].astype(rt)).cuda()
                w, _ = p.solve(d, lams, stream=s)
                p.sync()
                out[i] = w.cpu().numpy()
    except Exception as e:
        err.append(repr(e))
ts = [threading.Thread(target=work, args=(i,)) for i in range(len(shapes))]
for t in ts: t.start()
for t in ts: t.join()
assert not err, err
for i, (n, l, dt) in enumerate(shapes):
    c = cases[i]
    rt = np.float32 if dt else np.float64
    with mwf.Plan(n, l, c["cl"], c["ninv"], dtype=dt) as p:
        w, _ = p.solve(torch.from_numpy(c["d"].astype(rt)).cuda(), lams)
        p.sync()
        alone = w.cpu().numpy()
    same = np.array_equal(alone, out[i])
    print(f"Nside {n} dtype {dt}: threaded == alone {same}", flush=True)
    assert same
print("ok", flush=True)
"""


def test_plans_from_several_threads():
    r = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], capture_output=True, text=True, timeout=240,
                       cwd=ROOT)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok")
