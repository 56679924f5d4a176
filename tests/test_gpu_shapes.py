"""Launch shapes and the autotuner on the GPU.

Every launch shape of the panel kernels (workgroups of 1, 2 or 4 chunks of
256 rows) is forced in turn through HD_CPT and checked against the FP64
oracle on the answers to the query vectors the GPU saw (mode B), on ragged
sizes of several workgroups.  The two large workloads run in the shape the
benchmark times (the built-in rule): the Gaussian n = 65536, T = 100
alternating trajectory against the oracle on every step, and the Haar
n = 1e7, T = 200 trajectory against the oracle on its first steps and, on
every step, against the invariant an orthogonal Q fixes at any size:
<Q x_s, Q x_t> = <x_s, x_t>.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402
from paper_2101_07464_amd import inputs  # noqa: E402
from tests.test_gpu_ginibre import replay_following_signs  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {torch.float32: 1e-4, torch.float64: 1e-11}


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _mode_b(A, ens, n, T, X, pattern, seed, trial, sigma=1.0):
    orc = oracle.HDOracle(ens, n, tmax=T, seed=seed, trial=trial,
                          sigma=sigma)
    tr = [pattern == "alt" and t % 2 == 1 for t in range(T)]
    if ens == oracle.HAAR:
        return oracle.replay(orc, X[:T], tr)
    out, _ = replay_following_signs(A, orc, X[:T], tr)
    return out


@pytest.fixture
def clean_shapes(monkeypatch):
    monkeypatch.delenv("HD_CPT", raising=False)
    hd.autotune_clear()
    yield monkeypatch
    hd.autotune_clear()


@pytest.mark.parametrize("cpt", [1, 2, 4])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("ens", ["haar", "ginibre"])
def test_forced_shape_matches_oracle(clean_shapes, ens, dtype, cpt):
    """n = 5000 (ld 5120: 20, 10 or 5 workgroups), T = 16, Q and Q'
    alternating."""
    clean_shapes.setenv("HD_CPT", str(cpt))
    n, T = 5000, 16
    assert hd.shape_rule(hd.HAAR if ens == "haar" else hd.GINIBRE, n,
                         dtype) == cpt
    if ens == "haar":
        A = hd.LazyMatrix(hd.HAAR, n, t_max=T, seed=3, trial=1, dtype=dtype,
                          device=DEV)
        x1 = inputs.x1_normal(n, seed=3, trial=1)
        args = ("tanh", 1.0, 0.5)
        sig = 1.0
    else:
        sig = 1 / np.sqrt(n)
        A = hd.LazyMatrix(hd.GINIBRE, n, t_max=T, seed=3, trial=1, sigma=sig,
                          dtype=dtype, device=DEV)
        x1 = inputs.x1_normal(n, seed=3, trial=1, scale=1.0)
        args = ("soft_hist", 0.1, 0.3)
    X, Y = A.run(torch.from_numpy(x1).to(DEV, dtype), T, *args,
                 pattern="alt")
    torch.cuda.synchronize()
    assert A.status() == 0
    X, Y = X.double().cpu().numpy(), Y.double().cpu().numpy()
    ens_o = oracle.HAAR if ens == "haar" else oracle.GINIBRE
    Yb = _mode_b(A, ens_o, n, T, X, "alt", 3, 1, sig)
    err = max(relerr(y, yb) for y, yb in zip(Y, Yb))
    print("%s %s cpt %d: mode B %.2e" % (ens, dtype, cpt, err))
    assert err < TOL[dtype]


def test_shapes_agree_in_f64(clean_shapes):
    """The three shapes compute the same trajectory (FP64, Haar)."""
    n, T = 3000, 12
    x1 = torch.from_numpy(inputs.x1_normal(n, seed=5)).to(DEV, torch.float64)
    runs = []
    for cpt in (1, 2, 4):
        clean_shapes.setenv("HD_CPT", str(cpt))
        A = hd.LazyMatrix(hd.HAAR, n, t_max=T, seed=5, dtype=torch.float64,
                          device=DEV)
        X, _ = A.run(x1, T, "tanh", 1.0, 0.5)
        runs.append(X.cpu().numpy())
    for r in runs[1:]:
        assert relerr(r, runs[0]) < 1e-12


@pytest.mark.parametrize("ens", ["haar", "ginibre"])
def test_autotune_installs_fastest_shape(clean_shapes, ens):
    n, T = 40000, 10
    E = hd.HAAR if ens == "haar" else hd.GINIBRE
    other = hd.GINIBRE if ens == "haar" else hd.HAAR
    rep = hd.autotune(E, [n], torch.float32, k=6, device=DEV)
    chosen, times = rep[n]
    print("autotune %s n=%d: %s -> %d" % (ens, n, times, chosen))
    assert all(np.isfinite(v) and v > 0 for v in times.values())
    # the fastest shape, unless the built-in one (1 chunk here) is within 3%
    best = min(times, key=times.get)
    assert chosen == (best if times[best] < 0.97 * times[1] else 1)
    # nearest tuned length within a factor of 2, else the built-in rule;
    # other ensembles and storage types keep the built-in rule
    assert hd.shape_rule(E, n + 15000, torch.float32) == chosen
    assert hd.shape_rule(E, 3 * n, torch.float32) == 1
    assert hd.shape_rule(E, n, torch.float64) == 1
    assert hd.shape_rule(other, n, torch.float32) == 1
    # a handle created now runs in the tuned shape and still matches
    sig = 1.0 if ens == "haar" else 1 / np.sqrt(n)
    A = hd.LazyMatrix(E, n, t_max=T, seed=1, sigma=sig, device=DEV)
    x1 = inputs.x1_normal(n, seed=1, scale=None if ens == "haar" else 1.0)
    X, Y = A.run(torch.from_numpy(x1).to(DEV, torch.float32), T, "tanh",
                 1.0, 0.5, pattern="alt")
    torch.cuda.synchronize()
    assert A.status() == 0
    X, Y = X.double().cpu().numpy(), Y.double().cpu().numpy()
    Yb = _mode_b(A, oracle.HAAR if ens == "haar" else oracle.GINIBRE, n, T,
                 X, "alt", 1, 0, sig)
    assert max(relerr(y, yb) for y, yb in zip(Y, Yb)) < 1e-4
    hd.autotune_clear()
    assert hd.shape_rule(E, n, torch.float32) == 1


def test_gaussian_n65536_T100_alternating_full_size(clean_shapes):
    """The Gaussian workload at its full size: n = 65536, T = 100, sigma^2
    = 1/n, Q and Q' alternating, x_{t+1} = soft(y_t, 0.1) + 0.3 x_{t-1},
    FP32 storage; every answer against the oracle (mode B)."""
    n, T = 65536, 100
    sig = 1 / np.sqrt(n)
    A = hd.LazyMatrix(hd.GINIBRE, n, t_max=T, seed=0, sigma=sig, device=DEV)
    x1 = inputs.x1_normal(n, seed=0, scale=1.0)
    X, Y = A.run(torch.from_numpy(x1).to(DEV, torch.float32), T,
                 "soft_hist", 0.1, 0.3, pattern="alt")
    torch.cuda.synchronize()
    assert A.status() == 0 and A.counts() == (T, T // 2, T // 2)
    X, Y = X.double().cpu().numpy(), Y.double().cpu().numpy()
    Yb = _mode_b(A, oracle.GINIBRE, n, T, X, "alt", 0, 0, sig)
    err = [relerr(y, yb) for y, yb in zip(Y, Yb)]
    print("gaussian n=65536 T=100: mode B max %.2e" % max(err))
    assert max(err) < 1e-4
    # Mode A: the free-running trajectory against the oracle's FP64 run,
    # measured against the drift the oracle itself shows with its state
    # rounded to FP32 (these dynamics amplify storage rounding).  The GPU
    # also rounds every stored reflector to FP32, so it injects somewhat
    # more error per step than that state-only run: the whole trajectory
    # must stay within 3x the oracle's largest drift, and every step within
    # 6x that step's drift (or 1e-4 while the drift is below it)
    orc = oracle.HDOracle(oracle.GINIBRE, n, tmax=T, seed=0, sigma=sig)
    Xo, _ = oracle.run_trajectory(orc, X[0], T, "soft_hist", 0.1, 0.3, "alt")
    orc_c = oracle.HDOracle(oracle.GINIBRE, n, tmax=T, seed=0, sigma=sig)
    Xc, _ = oracle.run_trajectory(orc_c, X[0], T, "soft_hist", 0.1, 0.3,
                                  "alt", state_dtype=np.float32)
    ea = [relerr(x, xo) for x, xo in zip(X, Xo)]
    drift = [relerr(xc, xo) for xc, xo in zip(Xc, Xo)]
    print("gaussian n=65536 T=100: mode A max %.2e (FP32-state oracle "
          "drift max %.2e)" % (max(ea), max(drift)))
    ratio = max(e / max(d, 1e-4 / 6) for e, d in zip(ea, drift))
    print("  largest per-step ratio to the drift %.2f" % ratio)
    assert max(ea) <= 3 * max(drift)
    for t, (e, d) in enumerate(zip(ea, drift)):
        assert e <= max(1e-4, 6 * d), (t, e, d)


def test_haar_n1e7_T200_full_size(clean_shapes):
    """The large Haar trial at its full size (n = 1e7, T = 200, FP32, in
    the built-in four-chunk shape), x_{t+1} = tanh(y_t) + 0.1 x_t: the first
    six answers against the oracle (mode B), and the Gram matrix of all 200
    answers against that of the queries."""
    n, T, K = 10_000_000, 200, 6
    assert hd.shape_rule(hd.HAAR, n) == 4
    A = hd.LazyMatrix(hd.HAAR, n, t_max=T, seed=0, device=DEV)
    x1 = torch.from_numpy(inputs.x1_normal(n, seed=0)).to(DEV,
                                                          torch.float32)
    X, Y = A.run(x1, T, "tanh", 1.0, 0.1)
    torch.cuda.synchronize()
    assert A.status() == 0 and A.counts() == (T, T, T)
    # Gram matrices in FP64, 1e6 columns at a time
    GX = torch.zeros((T, T), dtype=torch.float64, device=DEV)
    GY = torch.zeros((T, T), dtype=torch.float64, device=DEV)
    for c in range(0, n, 1_000_000):
        xs = X[:T, c:c + 1_000_000].double()
        ys = Y[:, c:c + 1_000_000].double()
        GX += xs @ xs.T
        GY += ys @ ys.T
    d = torch.sqrt(torch.diagonal(GX))
    gram_err = float(((GY - GX) / torch.outer(d, d)).abs().max())
    Xh = X[:K].double().cpu().numpy()
    Yh = Y[:K].double().cpu().numpy()
    del X, Y
    Yb = _mode_b(A, oracle.HAAR, n, K, Xh, "Q", 0, 0)
    err = max(relerr(y, yb) for y, yb in zip(Yh, Yb))
    print("haar n=1e7 T=200: mode B (first %d) %.2e, Gram %.2e" %
          (K, err, gram_err))
    assert err < 1e-4
    assert gram_err < 1e-4
