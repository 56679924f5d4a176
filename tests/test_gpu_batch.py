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


def test_full_batch_4096_sampled_and_invariants():
    """The batched workload at its full size (4096 Haar trials, n
    log-uniform in [1e3, 1e5], T uniform in [10, 200], FP32, tanh(2y)), as
    the benchmark launches it.  Every trial: the map x_{t+1} = tanh(2 y_t)
    and the isometry ||y_t|| = ||x_t|| at every step; six sampled trials
    (largest n, longest T, smallest n, three seeded picks): every answer
    against the oracle (mode B)."""
    nb, Tb = inputs.ragged_batch(4096)
    trials = [(int(n), int(T), 0, b) for b, (n, T) in enumerate(zip(nb, Tb))]
    B = hd.HaarBatch(trials, dtype=torch.float32, device=DEV)
    x1 = [torch.from_numpy(inputs.x1_normal(n, seed=0, trial=b)).to(
        DEV, torch.float32) for n, T, _, b in trials]
    X, Y = B.run(x1, "tanh", 2.0, 0.0, record=True)
    torch.cuda.synchronize()
    assert B.status() == 0
    del B
    worst_map = worst_iso = 0.0
    for Xi, Yi in zip(X, Y):
        xd, yd = Xi.double(), Yi.double()
        d = (xd[1:] - torch.tanh(2.0 * yd)).abs().max() / \
            xd[1:].abs().max().clamp_min(1e-300)
        worst_map = max(worst_map, float(d))
        nx, ny = xd[:-1].norm(dim=1), yd.norm(dim=1)
        worst_iso = max(worst_iso, float(((ny - nx) / nx).abs().max()))
    n_arr, T_arr = np.array(nb), np.array(Tb)
    pick = {int(n_arr.argmax()), int(T_arr.argmax()), int(n_arr.argmin())}
    pick |= set(int(i) for i in np.random.default_rng(11).choice(
        len(trials), 3, replace=False))
    worst = 0.0
    for i in sorted(pick):
        n, T, s, k = trials[i]
        Xi = X[i].double().cpu().numpy()
        Yi = Y[i].double().cpu().numpy()
        orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=s, trial=k)
        ref = oracle.replay(orc, Xi[:-1], [False] * T)
        worst = max(worst, max(relerr(y, r) for y, r in zip(Yi, ref)))
    print("full batch: map %.2e, isometry %.2e, sampled mode B %.2e (%s)" %
          (worst_map, worst_iso, worst, sorted(pick)))
    assert worst_map < 1e-6
    assert worst_iso < 1e-5
    assert worst < 1e-4


def test_graph_replays_match_direct_runs():
    """hd_batch_set_graph: the first run records the launch sequence into a
    HIP graph, later runs replay it.  Every replay (new inputs included,
    with unrelated eager GPU work and synchronisations in between) must
    equal a direct run bit for bit, in both output modes."""
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B = hd.HaarBatch(TRIALS, dtype=torch.float32, device=DEV)
        D = hd.HaarBatch(TRIALS, dtype=torch.float32, device=DEV)
        B.set_graph(True)
        inputs_sets = [_x1(torch.float32)]
        g = torch.Generator().manual_seed(5)
        inputs_sets.append([torch.randn(n, generator=g).to(DEV) / np.sqrt(n)
                            for n, T, _, _ in TRIALS])
        for rep in range(4):
            x1 = inputs_sets[rep % 2]
            got = [t.clone() for t in B.run(x1, "tanh", 2.0, 0.0)]
            want = D.run(x1, "tanh", 2.0, 0.0)
            s.synchronize()
            for a, b in zip(got, want):
                assert torch.equal(a, b), rep
            # unrelated eager work between replays
            z = torch.randn(512, 512, device=DEV)
            (z @ z).sum().item()
        for rep in range(3):
            x1 = inputs_sets[rep % 2]
            X, Y = B.run(x1, "tanh", 2.0, 0.0, record=True)
            Xd, Yd = D.run(x1, "tanh", 2.0, 0.0, record=True)
            s.synchronize()
            for a, b in zip(X + Y, Xd + Yd):
                assert torch.equal(a, b), rep
        assert B.status() == 0 and D.status() == 0


def test_shapes_and_autotuner():
    """hd_batch_set_shape / hd_batch_autotune: one batch switched between
    1, 2 and 4 chunks per workgroup (and back) answers every query as the
    FP64 oracle does in each shape (Mode B, 1e-11), the shapes agree with
    each other to FP64 rounding, and after the autotuner has timed all
    three and installed one, runs still match the oracle.  With graph
    replay on, a shape change drops the recorded graph: replays after it
    equal direct runs of a second batch in the same shape bit for bit."""
    B = hd.HaarBatch(TRIALS, dtype=torch.float64, device=DEV)
    assert B.shape() == 4
    x1 = _x1(torch.float64)

    def run_and_check():
        X, Y = B.run(x1, "tanh", 2.0, 0.0, record=True)
        torch.cuda.synchronize()
        assert B.status() == 0
        worst = 0.0
        for (n, T, s, k), Xi, Yi in zip(TRIALS, X, Y):
            Xi = Xi.cpu().numpy()
            orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=s, trial=k)
            ref = oracle.replay(orc, Xi[:-1], [False] * T)
            worst = max(worst, max(relerr(y, r) for y, r in
                                   zip(Yi.cpu().numpy(), ref)))
        assert worst < 1e-11, worst
        return [y.cpu().numpy() for y in Y]

    runs = {}
    for c in (1, 2, 4, 1):
        B.set_shape(c)
        assert B.shape() == c
        runs.setdefault(c, []).append(run_and_check())
    for c in (2, 4):
        for a, b in zip(runs[c][0], runs[1][0]):
            assert relerr(a, b) < 1e-12
    for a, b in zip(runs[1][0], runs[1][1]):
        assert np.array_equal(a, b)
    with pytest.raises(hd.HDError):
        B.set_shape(3)
    chosen, ms = B.autotune(x1, "tanh", 2.0, 0.0, reps=1)
    print("batch autotuner: chose %d, ms per run %s" % (chosen, ms))
    assert chosen in (1, 2, 4) and B.shape() == chosen
    assert all(v > 0 for v in ms.values())
    if chosen != 4:
        assert ms[chosen] < 0.97 * ms[4]
    run_and_check()
    # graph replay across a shape change
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        G = hd.HaarBatch(TRIALS, dtype=torch.float32, device=DEV)
        D = hd.HaarBatch(TRIALS, dtype=torch.float32, device=DEV)
        G.set_graph(True)
        xf = _x1(torch.float32)
        for c in (4, 1, 2):
            G.set_shape(c)
            D.set_shape(c)
            for _ in range(2):
                got = [t.clone() for t in G.run(xf, "tanh", 2.0, 0.0)]
                want = D.run(xf, "tanh", 2.0, 0.0)
                s.synchronize()
                for a, b in zip(got, want):
                    assert torch.equal(a, b), c
        assert G.status() == 0 and D.status() == 0
