"""Device-side error reporting: a non-finite query makes a reflector norm
non-finite, which sets the handle's sticky flag (hd_status returns
HD_ERR_NONFINITE); hd_reset clears it, and the fresh matrix answers exactly
as the oracle's with the new key."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402
from paper_2101_07464_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("ens", ["haar", "gaussian"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_query_sets_flag_and_reset_clears_it(ens, bad):
    n, T = 5003, 6
    E = hd.HAAR if ens == "haar" else hd.GINIBRE
    EO = oracle.HAAR if ens == "haar" else oracle.GINIBRE
    sig = 1.0 if ens == "haar" else 1.0 / np.sqrt(n)
    A = hd.LazyMatrix(E, n, t_max=T, seed=2, sigma=sig, dtype=torch.float64,
                      device=DEV)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(n)
    A.mv(torch.from_numpy(x).to(DEV))
    assert A.status() == _lib.HD_OK
    xb = rng.standard_normal(n)
    xb[1234] = bad
    A.rmv(torch.from_numpy(xb).to(DEV))
    assert A.status() == _lib.HD_ERR_NONFINITE
    # sticky: a later finite query does not clear it
    A.mv(torch.from_numpy(x).to(DEV))
    assert A.status() == _lib.HD_ERR_NONFINITE
    A.reset(7, 1)
    assert A.status() == _lib.HD_OK
    orc = oracle.HDOracle(EO, n, tmax=T, seed=7, trial=1, sigma=sig)
    for t in range(3):
        xq = rng.standard_normal(n)
        y = (A.rmv if t == 1 else A.mv)(torch.from_numpy(xq).to(DEV))
        assert relerr(y.cpu().numpy(), orc.query(xq, t == 1)) < 1e-11
    assert A.status() == _lib.HD_OK
