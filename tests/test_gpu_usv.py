"""Q = U S V (two independent lazy Haar matrices U ~ Haar(m), V ~ Haar(n)
and S = diag(s) in R^{m x n}; section "Other Random Matrix Ensembles") on the
GPU against the oracle, Q and Q' queries mixed, square and rectangular.  Tolerances: FP32 1e-4, FP64 1e-11
(max-abs error over max-abs value)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402
from paper_2101_07464_amd._lib import HDError  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("m,n", [(3001, 3001), (3001, 2200), (1500, 4097)])
@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4),
                                       (torch.float64, 1e-11)])
def test_usv_matches_oracle(dtype, tol, m, n):
    K = 10
    p = min(m, n)
    U = hd.LazyMatrix(hd.HAAR, m, t_max=K, seed=2, trial=1, dtype=dtype,
                      device=DEV)
    V = hd.LazyMatrix(hd.HAAR, n, t_max=K, seed=2, trial=2, dtype=dtype,
                      device=DEV)
    rng = np.random.default_rng(12)
    s = torch.from_numpy(np.linspace(0.1, 3.0, p)).to(DEV, dtype)
    sr = s.double().cpu().numpy()
    ou = oracle.HDOracle(oracle.HAAR, m, tmax=K, seed=2, trial=1)
    ov = oracle.HDOracle(oracle.HAAR, n, tmax=K, seed=2, trial=2)
    worst = 0.0
    for k in range(K):
        tr = bool(rng.random() < 0.5)
        x = torch.from_numpy(rng.standard_normal(m if tr else n)).to(DEV,
                                                                    dtype)
        y = hd.usv_mv(U, V, s, x, transpose=tr)
        assert y.numel() == (n if tr else m)
        ref = oracle.usv_query(ou, ov, sr, x.double().cpu().numpy(), tr)
        worst = max(worst, relerr(y.double().cpu(), ref))
    torch.cuda.synchronize()
    assert U.status() == 0 and V.status() == 0
    assert U.counts()[0] == K and V.counts()[0] == K
    print("USV %dx%d %s: mode B %.2e" % (m, n, dtype, worst))
    assert worst < tol


def test_usv_rejects_mismatched_handles():
    n = 600
    s = torch.ones(n, device=DEV)
    x = torch.ones(n, device=DEV)
    U = hd.LazyMatrix(hd.HAAR, n, t_max=2, device=DEV)
    G = hd.LazyMatrix(hd.GINIBRE, n, t_max=2, device=DEV)
    W = hd.LazyMatrix(hd.HAAR, n, t_max=2, dtype=torch.float64, device=DEV)
    with pytest.raises(HDError):
        hd.usv_mv(U, G, s, x)
    with pytest.raises(ValueError):
        hd.usv_mv(U, W, s, x)
    with pytest.raises(HDError):
        hd.usv_mv(U, U, s, x)
