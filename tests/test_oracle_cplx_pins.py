"""Pins of the complex FP64 oracle (Sec. 3.4: complex Ginibre, the unitary
group U(n), and the unitary reflector of eq. (Householder_c)) against what
the paper and the mathematics fix, independent of the oracle's own formulas:

* the identities stated below eq. (Householder_c): H(v) v = ||v|| e_1,
  H(v)^H e_1 = v / ||v||, H(v) unitary; and its reduction to the real
  reflector of eq. (Householder) when v is real (checked against the real
  oracle, including v_1 < 0 and v_1 = 0);
* closed forms of the first answers: Q x_1 = ||x_1|| g / ||g|| on U(n) and
  sigma ||x_1|| g on complex Ginibre (g the first complex draw), and the
  second Ginibre answer sigma (p_1 g_1 + nu_2 g_2) with p_1 = x_1^H x_2 /
  ||x_1|| and nu_2 the norm of x_2's component orthogonal to x_1;
* exact reconstruction: one fixed matrix, rebuilt from the exported
  reflectors and basis vectors with an arbitrary completion of the
  unrevealed block, answers every query of a mixed Q / Q^H sequence (this
  fails for a misplaced conjugate or transpose anywhere in the algorithms);
* laws: moments of Haar unitary traces (Diaconis-Shahshahani:
  E|tr U^j|^2 = j for j <= n, E (tr U)^2 = 0, which a real orthogonal matrix
  would fail) and |U_11|^2 ~ Beta(1, n - 1); complex Ginibre entries with
  circular N(0, sigma^2) law; the GUE composition (Q + Q^H) / sqrt(2) is
  Hermitian with E|G_ij|^2 = sigma^2.

The complex-normal mapping (N_2i + i N_2i+1) / sqrt(2) is this project's own
recipe (the paper names no generator): parity unpinned beyond its moments.
"""
import numpy as np
import pytest
from scipy import stats

import oracle


def crand(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def dense_reflector(dim, refl):
    """H_k(p) as a dense dim x dim matrix from exported (w, r, theta)."""
    k = refl["k"]
    M = np.eye(dim, dtype=np.complex128)
    if refl["ident"]:
        return M
    w = refl["w"]
    blk = np.eye(dim - k + 1, dtype=np.complex128) - \
        np.outer(w, w.conj()) / (1.0 + refl["r"])
    M[k - 1:, k - 1:] = -np.exp(-1j * refl["theta"]) * blk
    return M


# --------------------------------------------------------------- reflector --

@pytest.mark.parametrize("n", [1, 2, 7, 64])
def test_reflector_identities(n):
    rng = np.random.default_rng(n)
    v = crand(rng, n)
    nu = np.linalg.norm(v)
    e1 = np.zeros(n, complex)
    e1[0] = 1
    Hv, ident = oracle.capply_householder(v, v)
    assert not ident
    assert np.abs(Hv - nu * e1).max() < 1e-13 * nu
    HHe1, _ = oracle.capply_householder(v, e1, adjoint=True)
    assert np.abs(HHe1 - v / nu).max() < 1e-14
    H = np.array([oracle.capply_householder(v, c)[0]
                  for c in np.eye(n, dtype=complex)]).T
    assert np.abs(H.conj().T @ H - np.eye(n)).max() < 1e-13
    HH = np.array([oracle.capply_householder(v, c, True)[0]
                   for c in np.eye(n, dtype=complex)]).T
    assert np.abs(HH - H.conj().T).max() < 1e-14


@pytest.mark.parametrize("case", ["pos", "neg", "zero_pivot"])
def test_reflector_reduces_to_real(case):
    rng = np.random.default_rng(5)
    v = rng.standard_normal(9)
    v[0] = {"pos": abs(v[0]), "neg": -abs(v[0]), "zero_pivot": 0.0}[case]
    for _ in range(3):
        z = crand(rng, 9)
        got, _ = oracle.capply_householder(v.astype(complex), z)
        re, _ = oracle.apply_householder(v, z.real)
        im, _ = oracle.apply_householder(v, z.imag)
        assert np.abs(got - (re + 1j * im)).max() < 1e-14


def test_reflector_zero_and_pivot_phase():
    z = crand(np.random.default_rng(1), 4)
    out, ident = oracle.capply_householder(np.zeros(4, complex), z)
    assert ident and np.array_equal(out, z)
    # v_1 = 0: theta = 0 by the convention, and still H v = ||v|| e_1
    v = np.array([0, 1 + 2j, -1j, 3], dtype=complex)
    Hv, _ = oracle.capply_householder(v, v)
    assert np.abs(Hv - np.linalg.norm(v) * np.eye(4)[0]).max() < 1e-14


def test_complex_normal_moments():
    g = oracle.cnormals(3, 0, 1, 0, 0, 200_000)
    se = 1 / np.sqrt(g.size)
    assert abs(np.mean(np.abs(g) ** 2) - 1) < 5 * np.sqrt(2) * se
    assert abs(np.mean(g * g)) < 5 * se          # circular: E g^2 = 0
    assert stats.kstest(np.sqrt(2) * g.real, "norm").pvalue > 1e-3
    assert stats.kstest(np.sqrt(2) * g.imag, "norm").pvalue > 1e-3
    # entries are independent of how the stream is sliced
    part = oracle.cnormals(3, 0, 1, 0, 1001, 50)
    assert np.array_equal(part, g[1001:1051])


# ------------------------------------------------------------ closed forms --

def test_haar_first_answers_closed_form():
    n = 40
    rng = np.random.default_rng(2)
    x = crand(rng, n)
    o = oracle.CHDOracle(oracle.HAAR, n, tmax=5, seed=7, trial=3)
    g = oracle.cnormals(7, 3, 1, 0, 0, n)
    y = o.mv(x)
    assert np.abs(y - np.linalg.norm(x) * g / np.linalg.norm(g)).max() < 1e-14
    o2 = oracle.CHDOracle(oracle.HAAR, n, tmax=5, seed=7, trial=3)
    y2 = o2.rmv(x)   # Q^H is Haar too: the same closed form
    assert np.abs(y2 - y).max() < 1e-14


def test_ginibre_first_two_answers_closed_form():
    m, n, sig = 30, 20, 0.7
    rng = np.random.default_rng(4)
    x1, x2 = crand(rng, n), crand(rng, n)
    o = oracle.CHDOracle(oracle.GINIBRE, n, m=m, tmax=5, seed=1, trial=9,
                         sigma=sig)
    g1 = oracle.cnormals(1, 9, 1, 0, 0, m)
    g2 = oracle.cnormals(1, 9, 2, 0, 0, m)
    nu1 = np.linalg.norm(x1)
    assert np.abs(o.mv(x1) - sig * nu1 * g1).max() < 1e-13
    p1 = np.vdot(x1, x2) / nu1
    nu2 = np.linalg.norm(x2 - np.vdot(x1, x2) / nu1 ** 2 * x1)
    assert np.abs(o.mv(x2) - sig * (p1 * g1 + nu2 * g2)).max() < 1e-12
    # the first adjoint query answers sigma ||x|| g (g of length n)
    o2 = oracle.CHDOracle(oracle.GINIBRE, n, m=m, tmax=5, seed=1, trial=9,
                          sigma=sig)
    xa = crand(rng, m)
    gn = oracle.cnormals(1, 9, 1, 0, 0, n)
    assert np.abs(o2.rmv(xa) - sig * np.linalg.norm(xa) * gn).max() < 1e-13


# ---------------------------------------------------------- reconstruction --

def _product(dim, refls, adjoint, order):
    M = np.eye(dim, dtype=np.complex128)
    for R in order(refls):
        D = dense_reflector(dim, R)
        M = M @ (D.conj().T if adjoint else D)
    return M


def test_haar_reconstruction_mixed_queries():
    n, T = 12, 9
    rng = np.random.default_rng(8)
    o = oracle.CHDOracle(oracle.HAAR, n, tmax=T, seed=2, trial=1)
    xs, ys, kinds = [], [], []
    for t in range(T):
        adj = t % 3 == 1
        x = crand(rng, n)
        if t == 5:
            x = 0.3 * xs[0] - 1j * xs[2]   # a query in the span of earlier ones
        xs.append(x)
        kinds.append(adj)
        ys.append(o.query(x, adj))
    Rs = [o.reflector(oracle.SIDE_R, i) for i in range(1, T + 1)]
    Ls = [o.reflector(oracle.SIDE_L, i) for i in range(1, T + 1)]
    # Q = L_1^H .. L_T^H diag(I_T, W) R_T .. R_1 for any unitary W
    Wc, _ = np.linalg.qr(crand(rng, (n - T) * (n - T)).reshape(n - T, n - T))
    D = np.eye(n, dtype=np.complex128)
    D[T:, T:] = Wc
    Lh = _product(n, Ls, True, lambda r: r)               # L_1^H .. L_T^H
    Rp = _product(n, Rs, False, lambda r: r[::-1])        # R_T .. R_1
    Q = Lh @ D @ Rp
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-12
    for x, y, adj in zip(xs, ys, kinds):
        want = Q.conj().T @ x if adj else Q @ x
        assert np.abs(want - y).max() < 1e-12 * np.linalg.norm(x)


def test_ginibre_reconstruction_mixed_queries():
    m, n, sig = 10, 8, 1.3
    rng = np.random.default_rng(9)
    o = oracle.CHDOracle(oracle.GINIBRE, n, m=m, tmax=7, seed=5, trial=2,
                         sigma=sig)
    pattern = [False, True, True, False, False, True, False]
    xs, ys = [], []
    for adj in pattern:
        x = crand(rng, m if adj else n)
        xs.append(x)
        ys.append(o.query(x, adj))
    t, r, l = o.counts()
    assert (t, r, l) == (7, 4, 3)
    S = np.zeros((m, n), dtype=np.complex128)
    for s in range(1, t + 1):
        u, v = o.basis(s)
        S += sig * np.outer(u, v.conj())
    Rs = [o.reflector(oracle.SIDE_R, i) for i in range(1, r + 1)]
    Ls = [o.reflector(oracle.SIDE_L, i) for i in range(1, l + 1)]
    Z = np.zeros((m, n), dtype=np.complex128)
    Z[l:, r:] = crand(rng, (m - l) * (n - r)).reshape(m - l, n - r)
    Lh = _product(m, Ls, True, lambda q: q)
    Rp = _product(n, Rs, False, lambda q: q[::-1])
    Q = S + Lh @ Z @ Rp
    for x, y, adj in zip(xs, ys, pattern):
        want = Q.conj().T @ x if adj else Q @ x
        assert np.abs(want - y).max() < 1e-12 * (1 + np.abs(y).max())


# -------------------------------------------------------------------- laws --

def _haar_dense(n, seed, trial):
    o = oracle.CHDOracle(oracle.HAAR, n, tmax=n, seed=seed, trial=trial)
    return np.array([o.mv(e) for e in np.eye(n, dtype=complex)]).T


def test_haar_unitary_trace_moments_and_entry_law():
    n, N = 5, 3000
    t1, t2, t1sq, u11 = [], [], [], []
    for tr in range(N):
        U = _haar_dense(n, 11, tr)
        if tr < 20:
            assert np.abs(U.conj().T @ U - np.eye(n)).max() < 1e-13
        a = np.trace(U)
        t1.append(abs(a) ** 2)
        t1sq.append(a * a)
        t2.append(abs(np.trace(U @ U)) ** 2)
        u11.append(abs(U[0, 0]) ** 2)
    t1, t2, t1sq = np.array(t1), np.array(t2), np.array(t1sq)
    assert abs(t1.mean() - 1) < 5 * t1.std() / np.sqrt(N)
    assert abs(t2.mean() - 2) < 5 * t2.std() / np.sqrt(N)
    # circular: E (tr U)^2 = 0 (a Haar orthogonal matrix has E (tr O)^2 = 1)
    assert abs(t1sq.mean()) < 5 * np.sqrt(np.mean(np.abs(t1sq) ** 2) / N)
    assert stats.kstest(u11, stats.beta(1, n - 1).cdf).pvalue > 1e-3


def test_complex_ginibre_entry_law_and_gue():
    m, n, sig, N = 4, 3, 0.8, 1500
    re, im, sq, gd, go = [], [], [], [], []
    for tr in range(N):
        o = oracle.CHDOracle(oracle.GINIBRE, n, m=m, tmax=n, seed=4,
                             trial=tr, sigma=sig)
        Q = np.array([o.mv(e) for e in np.eye(n, dtype=complex)]).T
        re.extend(Q.real.ravel())
        im.extend(Q.imag.ravel())
        sq.extend((Q * Q).ravel())
        # GUE: G x = (Q x + Q^H x) / sqrt(2), two queries per x (one
        # column per trial is enough for the law; the symmetry is checked on
        # a full reconstruction below)
        og = oracle.CHDOracle(oracle.GINIBRE, 3, m=3, tmax=2, seed=4,
                              trial=tr, sigma=sig)
        e1 = np.eye(3, dtype=complex)[0]
        col = (og.mv(e1) + og.rmv(e1)) / np.sqrt(2)
        gd.append(col[0])
        go.extend(col[1:])
    s = sig / np.sqrt(2)
    assert stats.kstest(np.array(re) / s, "norm").pvalue > 1e-3
    assert stats.kstest(np.array(im) / s, "norm").pvalue > 1e-3
    sq = np.array(sq)
    assert abs(sq.mean()) < 5 * np.sqrt(np.mean(np.abs(sq) ** 2) / sq.size)
    gd, go = np.array(gd), np.array(go)
    assert np.abs(gd.imag).max() < 1e-14            # real diagonal
    assert stats.kstest(gd.real / sig, "norm").pvalue > 1e-3
    e2 = np.abs(go) ** 2
    assert abs(e2.mean() - sig ** 2) < 5 * e2.std() / np.sqrt(e2.size)


def test_gue_composition_is_hermitian():
    n, sig = 6, 1.1
    o = oracle.CHDOracle(oracle.GINIBRE, n, m=n, tmax=2 * n, seed=3,
                         trial=0, sigma=sig)
    # n Q-queries and n Q^H-queries: r = l = n, within capacity
    G = np.array([(o.mv(e) + o.rmv(e)) / np.sqrt(2)
                  for e in np.eye(n, dtype=complex)]).T
    assert np.abs(G - G.conj().T).max() < 1e-12
