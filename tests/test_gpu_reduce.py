"""The two-stage reduction of the per-workgroup partial rows (blocks of 256
rows x 32 slots, then the block sums), which the library uses from 1024
workgroup rows on (the large single trial), forced here for every reduction
(HD_RED_TWO_STAGE=1, read once per process, hence a child process) on FP64
trajectories small enough for the oracle's own run: every answer of a Haar
trajectory and of a Gaussian one with Q and Q' alternating within 1e-11 of
the FP64 oracle (Mode A), as for the one-stage form."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, ROOT)
import oracle
import paper_2101_07464_amd as hd
from paper_2101_07464_amd import inputs
out = {}
for ens, n, T, dyn, a, b, pat in ((hd.HAAR, 70001, 14, "tanh", 1.0, 0.5, "Q"),
                                  (hd.GINIBRE, 66000, 12, "tanh", 1.0, 0.5, "alt")):
    sig = 1.0 / np.sqrt(n) if ens == hd.GINIBRE else 1.0
    x1 = inputs.x1_normal(n, seed=5)
    A = hd.LazyMatrix(ens, n, t_max=T, seed=5, sigma=sig,
                      dtype=torch.float64, device="cuda:0")
    X, Y = A.run(torch.from_numpy(x1).to("cuda:0"), T, dyn, a, b, pat)
    torch.cuda.synchronize()
    X, Y = X.cpu().numpy(), Y.cpu().numpy()
    orc = oracle.HDOracle(oracle.HAAR if ens == hd.HAAR else oracle.GINIBRE,
                          n, tmax=T, seed=5, sigma=sig)
    Xo, Yo = oracle.run_trajectory(orc, x1, T, dyn, a, b, pat)
    err = max(float(np.abs(y - yo).max() / np.abs(yo).max())
              for y, yo in zip(Y, Yo))
    out["haar" if ens == hd.HAAR else "ginibre"] = [err, A.status()]
print("RESULT " + json.dumps(out), flush=True)
"""


def test_forced_two_stage_reduction_fp64():
    env = dict(os.environ, HD_RED_TWO_STAGE="1")
    r = subprocess.run([sys.executable, "-c", CHILD.replace("ROOT", repr(ROOT))],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
    res = json.loads(line[len("RESULT "):])
    print("forced two-stage reduction, FP64 Mode A:", res)
    for name, (err, status) in res.items():
        assert status == 0, name
        assert err < 1e-11, (name, err)
