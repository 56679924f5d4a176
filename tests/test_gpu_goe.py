"""GOE queries (hd_goe_step / LazyGOE) on the GPU against the oracle.

G = (Q + Q') / sqrt(2) for the lazy square Gaussian Q (section "Other
Random Matrix Ensembles"); hd_goe_step forms the sum and the 1/sqrt(2)
itself, so one call answers G x with two queries.  Mode B: the oracle answers the same
inputs.  Tolerances: FP32 1e-4, FP64 1e-11 (max-abs error over max-abs
value).  At the full size of the Gaussian workload the realised G is
checked to be symmetric: a'(G b) = b'(G a).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402
from paper_2101_07464_amd._lib import HDCapacityError, HDError  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4),
                                       (torch.float64, 1e-11)])
def test_goe_matches_oracle(dtype, tol):
    n, K = 3001, 8
    scale = 1 / np.sqrt(n)
    G = hd.LazyGOE(n, t_max=2 * K + 1, seed=6, trial=3, scale=scale,
                   dtype=dtype, device=DEV)
    orc = oracle.HDOracle(oracle.GINIBRE, n, seed=6, trial=3, sigma=scale)
    rng = np.random.default_rng(4)
    worst = 0.0
    for s in range(K):
        x = rng.standard_normal(n)
        y = G.mv(torch.from_numpy(x).to(DEV, dtype))
        xr = torch.from_numpy(x).to(dtype).double().numpy()
        worst = max(worst, relerr(y.double().cpu(), oracle.goe_query(orc, xr)))
        if s == 3:
            # a plain query of the underlying Q in between
            z = rng.standard_normal(n)
            w = hd.LazyMatrix.mv(G, torch.from_numpy(z).to(DEV, dtype))
            zr = torch.from_numpy(z).to(dtype).double().numpy()
            worst = max(worst, relerr(w.double().cpu(), orc.mv(zr)))
    torch.cuda.synchronize()
    assert G.status() == 0 and G.counts()[0] == 2 * K + 1
    print("GOE %s: mode B %.2e" % (dtype, worst))
    assert worst < tol


def test_goe_symmetric_at_full_size():
    """n = 65536, FP32: a'(G b) = b'(G a) for the realised G."""
    n = 65536
    G = hd.LazyGOE(n, t_max=4, seed=1, scale=1 / np.sqrt(n), device=DEV)
    g = torch.Generator().manual_seed(9)
    a = torch.randn(n, generator=g).to(DEV)
    b = torch.randn(n, generator=g).to(DEV)
    gb = G.mv(b)
    ga = G.mv(a)
    torch.cuda.synchronize()
    assert G.status() == 0
    lhs = float(torch.dot(a.double(), gb.double()))
    rhs = float(torch.dot(b.double(), ga.double()))
    scale = float(a.double().norm() * gb.double().norm())
    print("GOE symmetry: %.3e vs %.3e (rel %.2e)" %
          (lhs, rhs, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) / scale < 1e-5


def test_goe_errors():
    n = 500
    G = hd.LazyGOE(n, t_max=3, seed=0, scale=0.1, device=DEV)
    x = torch.ones(n, device=DEV)
    G.mv(x)
    with pytest.raises(HDCapacityError):
        G.mv(x)                       # needs two more queries, one left
    H = hd.LazyMatrix(hd.HAAR, n, t_max=4, device=DEV)
    with pytest.raises(HDError):
        H.goe_mv(x)
    R = hd.LazyMatrix(hd.GINIBRE, n, m=n + 1, t_max=4, device=DEV)
    with pytest.raises(HDError):
        R.goe_mv(x)
