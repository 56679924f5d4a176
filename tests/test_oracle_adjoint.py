"""Pins of the oracle's LISTA gradient (fixed lazy Q), CPU only.

After the forward and backward passes, a dense matrix reconstructed from
everything the lazy matrix revealed (eq. (Gaussian_t), any W for the part
never revealed) reproduces every answer; dense reverse-mode differentiation
of the same layers with that matrix must then give the same gradient, and a
central finite difference of the dense loss must agree to O(eps^2).
"""
import numpy as np
import pytest

import oracle
from oracle import GINIBRE, HDOracle
from paper_2101_07464_amd import inputs

from dense import ginibre_rec

torch = pytest.importorskip("torch")


def _problem(n, m, L, seed):
    sig = 1.0 / np.sqrt(m)
    orc = HDOracle(GINIBRE, n, m, tmax=min(m, n), seed=seed, sigma=sig)
    xs = inputs.sparse_target(n, 0.1, 2.0, seed=seed)
    noise = inputs.noise(m, 0.01, seed=seed)
    y = orc.query(xs, False) + noise
    rng = np.random.default_rng(seed)
    a = 0.3 + 0.05 * rng.standard_normal(L)
    th = 0.6 + 0.05 * rng.standard_normal(L)
    return orc, sig, xs, y, a, th


def _dense_loss(Q, x1, y, xs, a, th):
    x = x1
    for at, tt in zip(a, th):
        v = x + at * (Q.T @ (y - Q @ x))
        x = torch.sign(v) * torch.clamp(torch.abs(v) - tt, min=0.0)
    return torch.sum((x - xs) ** 2)


@pytest.mark.parametrize("n,m,L", [(64, 32, 8), (90, 60, 5)])
def test_lista_gradient_equals_dense_backprop(n, m, L):
    orc, sig, xs, y, a, th = _problem(n, m, L, seed=n + m)
    x1 = np.zeros(n)
    X, U, V = oracle.lista_forward(orc, x1, y, a, th)
    g = 2.0 * (X[-1] - xs)
    need_x1 = 1 + 4 * L <= min(m, n)  # one query pair more than L - 1
    da, dth, gx1 = oracle.lista_backward(orc, g, a, th, U, V,
                                         need_x1=need_x1)
    t, r, l = orc.counts()
    assert t == 1 + 2 * L + 2 * (L if need_x1 else L - 1)
    rng = np.random.default_rng(1)
    for _ in range(2):
        Q = torch.tensor(ginibre_rec(orc, m, n, sig,
                                     rng.standard_normal((m, n))))
        at = torch.tensor(a, requires_grad=True)
        tt = torch.tensor(th, requires_grad=True)
        x1t = torch.zeros(n, dtype=torch.float64, requires_grad=True)
        loss = _dense_loss(Q, x1t, torch.tensor(y), torch.tensor(xs), at, tt)
        loss.backward()
        assert loss.item() == pytest.approx(float(np.sum(g ** 2) / 4),
                                            rel=1e-12)
        ref = [at.grad.numpy(), tt.grad.numpy()]
        got = [da, dth]
        if need_x1:
            ref.append(x1t.grad.numpy())
            got.append(gx1)
        ref, got = np.concatenate(ref), np.concatenate(got)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_lista_gradient_finite_difference():
    n, m, L = 64, 40, 6
    orc, sig, xs, y, a, th = _problem(n, m, L, seed=5)
    X, U, V = oracle.lista_forward(orc, np.zeros(n), y, a, th)
    da, dth, _ = oracle.lista_backward(orc, 2.0 * (X[-1] - xs), a, th, U, V)
    Q = torch.tensor(ginibre_rec(orc, m, n, sig,
                                 np.random.default_rng(3).standard_normal(
                                     (m, n))))
    yt, xst, z = torch.tensor(y), torch.tensor(xs), torch.zeros(
        n, dtype=torch.float64)
    rng = np.random.default_rng(9)
    for _ in range(3):
        d1, d2 = rng.standard_normal(L), rng.standard_normal(L)
        eps = 1e-6
        lp = _dense_loss(Q, z, yt, xst, torch.tensor(a + eps * d1),
                         torch.tensor(th + eps * d2)).item()
        lm = _dense_loss(Q, z, yt, xst, torch.tensor(a - eps * d1),
                         torch.tensor(th - eps * d2)).item()
        fd = (lp - lm) / (2 * eps)
        an = float(da @ d1 + dth @ d2)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
