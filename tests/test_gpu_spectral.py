"""The spectral-method workload of Sec. 2.2 on the GPU against the oracle.

A = [I_n 0] Q with Q Haar of size m (eq. (A_ortho)), measurements
y = tanh|A' xi|, and the power iteration x_{k+1} = scale * m * D x_k with
D = (1/m) A diag(y) A' (eq. (D_mtx)): one query for the measurements and two
per step, the maps fused into the epilogues (hd_spectral_power).  The FP64
oracle runs the same iteration through its own lazy matrix
(oracle.spectral_power).

The power iterates converge, so each new query soon lies in the span of the
earlier ones up to rounding: its reflector is then built from rounding noise
and any two implementations reveal different (equally valid) completions of
Q from there on.  The iterates are compared with the oracle's while the
oracle's own query sequence is well conditioned (the new direction of x_k is
above 1e-3 of its norm); every iterate, at any size, must come from ONE
symmetric D, which makes the Gram matrix of the iterates a Hankel matrix:
x_j' x_{k+1} = x_j' D x_k = x_{j+1}' x_k.  The Rayleigh quotients of the
iterates must not decrease (D is positive semidefinite).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _new_direction(X):
    """Norm of the part of each x_k outside the span of x_1..x_{k-1},
    relative to ||x_k||."""
    out = [1.0]
    for k in range(1, len(X)):
        Qm, _ = np.linalg.qr(X[:k].T)
        r = X[k] - Qm @ (Qm.T @ X[k])
        out.append(float(np.linalg.norm(r) / np.linalg.norm(X[k])))
    return np.array(out)


def _case(m, n, K, dtype, scale, seed):
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    x1 = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    A = hd.LazyMatrix(hd.HAAR, m, t_max=1 + 2 * K, seed=seed, dtype=dtype,
                      device=DEV)
    z, X = A.spectral_power(torch.from_numpy(xi).to(DEV, dtype),
                            torch.from_numpy(x1).to(DEV, dtype), K, scale)
    torch.cuda.synchronize()
    assert A.status() == 0 and A.counts()[0] == 1 + 2 * K
    orc = oracle.HDOracle(oracle.HAAR, m, tmax=1 + 2 * K, seed=seed)
    zo, Xo = oracle.spectral_power(orc, xi, x1, K, scale)
    z, X = z.double().cpu().numpy(), X.double().cpu().numpy()
    ez = relerr(z, zo)
    err = [relerr(a, b) for a, b in zip(X, Xo)]
    eps = _new_direction(Xo)
    kstar = int(np.argmax(np.minimum.accumulate(eps) < 1e-3)) \
        if np.any(eps < 1e-3) else len(eps)
    rq = [X[k] @ X[k + 1] / (X[k] @ X[k]) for k in range(K)]
    nrm = np.linalg.norm(X, axis=1)
    U = X @ X.T
    den = 0.5 * (np.outer(nrm[:-1], nrm[1:]) + np.outer(nrm[1:], nrm[:-1]))
    hank = float(np.max(np.abs(U[:-1, 1:] - U[1:, :-1]) / den))
    return ez, err, kstar, rq, hank


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11),
                                       (torch.float32, 1e-4)])
@pytest.mark.parametrize("scale", [1.0, 1.7])
def test_spectral_power_matches_oracle(dtype, tol, scale):
    ez, err, kstar, rq, hank = _case(3001, 1400, 12, dtype, scale, seed=21)
    print("spectral m=3001 n=1400 %s scale %.1f: z %.2e  X (first %d) %.2e"
          " (all %.2e)  Hankel %.2e" % (dtype, scale, ez, kstar,
                                        max(err[:kstar]), max(err), hank))
    assert ez < tol and max(err[:kstar]) < tol
    assert hank < 10 * tol
    assert all(b >= a * (1 - 10 * tol) for a, b in zip(rq, rq[1:]))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11),
                                       (torch.float32, 1e-4)])
def test_spectral_power_workload_size(dtype, tol):
    """The benchmark's configuration: n = 1e5, m = 2e5, 50 power steps
    (101 queries)."""
    ez, err, kstar, rq, hank = _case(200_000, 100_000, 50, dtype, 1.0,
                                     seed=0)
    print("spectral m=2e5 n=1e5 K=50 %s: z %.2e  X (first %d) %.2e "
          "(all %.2e, per step %s)  Hankel %.2e  rayleigh %.6f" %
          (dtype, ez, kstar, max(err[:kstar]), max(err),
           " ".join("%.1e" % e for e in err[::5]), hank, rq[-1]))
    assert ez < tol and max(err[:kstar]) < tol
    assert hank < 10 * tol
    assert all(b >= a * (1 - 10 * tol) for a, b in zip(rq, rq[1:]))


def test_spectral_power_rejects_bad_arguments():
    A = hd.LazyMatrix(hd.HAAR, 100, t_max=9, dtype=torch.float64, device=DEV)
    xi = torch.ones(40, dtype=torch.float64, device=DEV)
    with pytest.raises(hd.HDCapacityError):
        A.spectral_power(xi, xi.clone(), 5)      # 11 queries > t_max 9
    with pytest.raises(hd.HDError):
        A.spectral_power(torch.ones(100, dtype=torch.float64, device=DEV),
                         torch.ones(100, dtype=torch.float64, device=DEV), 2)
    assert A.counts()[0] == 0
    G = hd.LazyMatrix(hd.GINIBRE, 100, t_max=9, dtype=torch.float64,
                      device=DEV)
    with pytest.raises(hd.HDError):
        G.spectral_power(xi, xi.clone(), 2)
