"""GPU parity of batched Haar trials (hd_batch_*) against the FP64 oracle and
against separate single-trial handles.

Every trial runs Algorithm 2 with Q-queries only and x_{t+1} = tanh(2 y_t)
(the batched workload's map), x_1 ~ N(0, I/n) keyed by the trial.  Mode B:
the oracle replays each trial's recorded query vectors.  Tolerances: FP64
storage 1e-11, FP32 storage 1e-4 (max-abs error over max-abs value).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402
from paper_2101_07464_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# ragged: sizes below, at and above the 1024-row padding quantum, one T = 1
TRIALS = [(700, 6, 0, 0), (1500, 9, 0, 1), (257, 3, 0, 2), (2048, 12, 0, 3),
          (1025, 1, 0, 4), (3000, 17, 5, 5), (10037, 8, 0, 6),
          (4099, 25, 0, 7)]


def relerr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _x1(dtype):
    return [torch.from_numpy(inputs.x1_normal(n, seed=s, trial=k)).to(DEV, dtype)
            for n, T, s, k in TRIALS]


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11),
                                       (torch.float32, 1e-4)])
def test_batch_matches_oracle(dtype, tol):
    B = hd.HaarBatch(TRIALS, dtype=dtype, device=DEV)
    x1 = _x1(dtype)
    X, Y = B.run(x1, "tanh", 2.0, 0.0, record=True)
    torch.cuda.synchronize()
    assert B.status() == 0
    worst = 0.0
    for (n, T, s, k), Xi, Yi, x in zip(TRIALS, X, Y, x1):
        Xi = Xi.double().cpu().numpy()
        Yi = Yi.double().cpu().numpy()
        assert np.array_equal(Xi[0], x.double().cpu().numpy())
        orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=s, trial=k)
        ref = oracle.replay(orc, Xi[:-1], [False] * T)
        e = max(relerr(y, r) for y, r in zip(Yi, ref))
        worst = max(worst, e)
        # the map itself
        assert relerr(Xi[1:], np.tanh(2.0 * Yi)) < (1e-15 if tol < 1e-6
                                                    else 1e-6)
    print("batch %s Mode B worst %.2e" % (dtype, worst))
    assert worst < tol


def test_batch_equals_single_handles():
    """Each trial's answers equal a separate handle's with the same key."""
    B = hd.HaarBatch(TRIALS, dtype=torch.float64, device=DEV)
    x1 = _x1(torch.float64)
    X, Y = B.run(x1, "tanh", 2.0, 0.0, record=True)
    for (n, T, s, k), Xi, Yi, x in zip(TRIALS, X, Y, x1):
        A = hd.LazyMatrix(hd.HAAR, n, t_max=T, seed=s, trial=k,
                          dtype=torch.float64, device=DEV)
        Xs, Ys = A.run(x, T, "tanh", 2.0, 0.0)
        assert relerr(Yi.cpu().numpy(), Ys.cpu().numpy()) < 1e-12
        assert relerr(Xi.cpu().numpy(), Xs.cpu().numpy()) < 1e-12


def test_batch_final_state_and_rerun():
    """x_{T+1} without recording equals the recorded last row; a second run
    starts over and reproduces it bit for bit."""
    B = hd.HaarBatch(TRIALS, dtype=torch.float32, device=DEV)
    x1 = _x1(torch.float32)
    X, _ = B.run(x1, "tanh", 2.0, 0.0, record=True)
    out1 = B.run(x1, "tanh", 2.0, 0.0)
    out2 = B.run(x1, "tanh", 2.0, 0.0)
    for Xi, a, b in zip(X, out1, out2):
        assert torch.equal(a, Xi[-1])
        assert torch.equal(a, b)


def test_batch_rejects_bad_input():
    with pytest.raises(hd.HDError):
        hd.HaarBatch([(100, 101, 0, 0)], device=DEV)  # T > n
    B = hd.HaarBatch([(300, 4, 0, 0)], device=DEV)
    with pytest.raises(ValueError):
        B.run([torch.zeros(299, device=DEV)], "tanh", 2.0, 0.0)
