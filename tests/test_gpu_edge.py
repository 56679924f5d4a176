"""Degenerate sizes on the GPU against the oracle: n = 1, 2, 3, 7 (Haar)
and tiny rectangular Gaussian shapes, each run to its full capacity
T = min(m, n) with Q and Q' queries mixed (the last reflectors act on tails
of length one), and a query beyond capacity, which must be refused without
changing the handle.  Tolerances: FP64 1e-11, FP32 1e-4 (max-abs error
over max-abs value)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402
from paper_2101_07464_amd._lib import HDCapacityError  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {torch.float32: 1e-4, torch.float64: 1e-11}


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _full_capacity(ens, m, n, dtype, pattern, sigma=0.7):
    T = min(m, n)
    A = hd.LazyMatrix(ens, n, m=m, t_max=T, seed=4, trial=1, sigma=sigma,
                      dtype=dtype, device=DEV)
    orc = oracle.HDOracle(ens, n, m, tmax=T, seed=4, trial=1, sigma=sigma)
    rng = np.random.default_rng(m * 100 + n)
    worst = 0.0
    for t in range(T):
        tr = pattern[t % len(pattern)] == "T"
        x = rng.standard_normal(m if tr else n)
        xd = torch.from_numpy(x).to(DEV, dtype)
        y = A.rmv(xd) if tr else A.mv(xd)
        ref = orc.query(xd.double().cpu().numpy(), tr)
        worst = max(worst, relerr(y.double().cpu(), ref))
    torch.cuda.synchronize()
    assert A.status() == 0
    assert A.counts()[0] == T
    # one query too many: refused, nothing changes
    with pytest.raises(HDCapacityError):
        A.mv(torch.ones(n, dtype=dtype, device=DEV))
    assert A.counts()[0] == T
    return worst


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 2, 3, 7])
def test_haar_tiny_full_capacity(n, dtype):
    e = _full_capacity(hd.HAAR, n, n, dtype, "QTQ")
    print("haar n=%d %s: %.2e" % (n, dtype, e))
    assert e < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n", [(1, 1), (1, 3), (3, 1), (2, 5), (6, 4)])
def test_gaussian_tiny_full_capacity(m, n, dtype):
    e = _full_capacity(hd.GINIBRE, m, n, dtype, "QTT")
    print("gaussian %dx%d %s: %.2e" % (m, n, dtype, e))
    assert e < TOL[dtype]


def test_haar_run_tiny():
    """hd_run on n = 2, T = 2 (FP64): trajectory against the oracle."""
    n, T = 2, 2
    A = hd.LazyMatrix(hd.HAAR, n, t_max=T, seed=9, dtype=torch.float64,
                      device=DEV)
    x1 = torch.tensor([0.6, -0.8], dtype=torch.float64, device=DEV)
    X, Y = A.run(x1, T, "tanh", 1.0, 0.5, pattern="alt")
    torch.cuda.synchronize()
    orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=9)
    Xo, Yo = oracle.run_trajectory(orc, x1.cpu().numpy(), T, "tanh", 1.0,
                                   0.5, "alt")
    assert relerr(X.cpu(), Xo) < 1e-12 and relerr(Y.cpu(), Yo) < 1e-12


def test_run_zero_steps_is_identity():
    """hd_run with T = 0: no query, x_{T+1} = x_1, counters unchanged."""
    n = 1000
    A = hd.LazyMatrix(hd.HAAR, n, t_max=4, seed=1, device=DEV)
    x1 = torch.randn(n, device=DEV)
    xo, _ = A.run(x1, 0, "tanh", 1.0, 0.5, record=False)
    X, Y = A.run(x1, 0, "tanh", 1.0, 0.5, record=True)
    torch.cuda.synchronize()
    assert torch.equal(xo, x1) and torch.equal(X[0], x1)
    assert Y.shape == (0, n)
    assert A.counts() == (0, 0, 0)
