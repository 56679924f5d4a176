"""Pins of the FP64 oracle to facts fixed outside the oracle itself.

Each test checks the oracle against a published known answer, an identity the
paper states, a closed form derived from the paper, a textbook routine
(LAPACK QR), or a distributional fact, chosen so that a dropped term, a wrong
sign, a wrong index or a transposed operand in hd_oracle.c fails one of them.
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import GINIBRE, HAAR, SIDE_L, SIDE_R, HDOracle
from tests.dense import haar_dense, r_factor_positive, reflector_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ---

def test_philox_known_answers():
    """Random123 / SC'11 known-answer vectors for Philox4x32-10."""
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(w, 16) for w in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = oracle.philox4x32_10(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


def test_normals_standard_gaussian():
    """The draws are N(0,1): KS test, first four moments."""
    z = oracle.normals(7, 3, 1, 0, 0, 200000)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert abs(stats.skew(z)) < 5 * np.sqrt(6 / z.size)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / z.size)


def test_normals_streams_independent_and_indexable():
    """Streams for different steps / tags / trials are uncorrelated, and the
    draw for index i does not depend on where a request starts."""
    n = 100000
    a = oracle.normals(0, 0, 1, 0, 0, n)
    for other in [oracle.normals(0, 0, 2, 0, 0, n),
                  oracle.normals(0, 0, 1, 1, 0, n),
                  oracle.normals(0, 1, 1, 0, 0, n),
                  oracle.normals(1, 0, 1, 0, 0, n)]:
        assert abs(np.corrcoef(a, other)[0, 1]) < 5 / np.sqrt(n)
    # neighbouring elements in one stream are uncorrelated too
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 5 / np.sqrt(n)
    part = oracle.normals(0, 0, 1, 0, 12345, 77)
    assert np.array_equal(part, a[12345:12345 + 77])
    # indices beyond 2^34 use the high counter word and still work
    big = oracle.normals(0, 0, 1, 0, (1 << 34) + 5, 3)
    assert np.all(np.isfinite(big)) and not np.array_equal(big, a[5:8])


def test_uniform_words_chi2():
    """Philox output words are uniform (chi-square on 256 bins of the top
    byte over 2^16 blocks)."""
    words = []
    for c in range(1 << 14):
        words.extend(oracle.philox4x32_10([c, 9, 0, 0], [1, 2]))
    top = np.array(words, dtype=np.uint64) >> 24
    counts = np.bincount(top.astype(np.int64), minlength=256)
    assert stats.chisquare(counts).pvalue > 1e-3


# ------------------------------------------------------ Householder (P1) ---

@pytest.mark.parametrize("length", [1, 2, 7, 33])
def test_householder_identities(length):
    """eq. (Householder_property): H(v) v = ||v|| e1, H(v) e1 = v/||v||;
    H symmetric orthogonal with eigenvalues s (once) and -s (length-1 times),
    so trace H = -s (length - 2) with s = sign(v1) (+1 for v1 >= 0)."""
    rng = np.random.default_rng(length)
    for trial in range(5):
        v = rng.standard_normal(length)
        if trial == 4 and length > 1:
            v[0] = 0.0  # sign(0) = +1
        H = np.column_stack([oracle.apply_householder(v, e)[0]
                             for e in np.eye(length)])
        nv = np.linalg.norm(v)
        e1 = np.eye(length)[0]
        assert np.allclose(H @ v, nv * e1, atol=1e-14 * nv)
        assert np.allclose(H @ e1, v / nv, atol=1e-15)
        assert np.allclose(H, H.T, atol=1e-15)
        assert np.allclose(H.T @ H, np.eye(length), atol=1e-14)
        s = 1.0 if v[0] >= 0 else -1.0
        assert np.isclose(np.trace(H), -s * (length - 2), atol=1e-13)


def test_householder_zero_is_identity():
    """H_k(p) = I when p[k:n] = 0 (the convention after eq. (Householder_e))."""
    z = np.arange(5.0)
    out, ident = oracle.apply_householder(np.zeros(5), z)
    assert ident and np.array_equal(out, z)


def test_generalised_reflector_zeroes_tail():
    """eq. (ortho): Z_{1:k} H_k(p) p = 0, via a lazy query whose stored
    reflector is H_k of the transformed query."""
    n = 12
    orc = HDOracle(HAAR, n, seed=4)
    rng = np.random.default_rng(0)
    Rs = []
    for t in range(1, 6):
        x = rng.standard_normal(n)
        orc.mv(x)
        Rs.append(reflector_matrix(n, orc.reflector(SIDE_R, t)))
        p = x.copy()
        for R in Rs[:-1]:
            p = R @ p
        q = Rs[-1] @ p
        assert np.allclose(q[t:], 0, atol=1e-13 * np.linalg.norm(x))
        assert np.allclose(q[:t - 1], p[:t - 1], atol=1e-14)
        assert np.isclose(q[t - 1], np.linalg.norm(p[t - 1:]), rtol=1e-13)


# ------------------------------------------------- first steps (P2) ---

@pytest.mark.parametrize("n", [1, 5, 300])
def test_haar_first_step_closed_form(n):
    """Below eq. (H_1): Q^(1) x_1 = (||x_1|| / ||g_1||) g_1 (and for Q')."""
    rng = np.random.default_rng(n)
    for tr, seed in [(False, 3), (True, 11)]:
        x = rng.standard_normal(n)
        y = HDOracle(HAAR, n, seed=seed, trial=2).query(x, tr)
        g = oracle.normals(seed, 2, 1, 0, 0, n)
        assert np.allclose(y, np.linalg.norm(x) / np.linalg.norm(g) * g,
                           rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("m,n", [(7, 7), (5, 9), (40, 23)])
def test_ginibre_first_step_closed_form(m, n):
    """Below eq. (Gaussian_1): Q^(1) x_1 = ||x_1|| g_1, scaled by sigma."""
    rng = np.random.default_rng(m * n)
    sig = 0.37
    x = rng.standard_normal(n)
    y = HDOracle(GINIBRE, n, m, seed=5, sigma=sig).mv(x)
    g = oracle.normals(5, 0, 1, 0, 0, m)
    assert np.allclose(y, sig * np.linalg.norm(x) * g, rtol=1e-13)
    x = rng.standard_normal(m)
    y = HDOracle(GINIBRE, n, m, seed=5, sigma=sig).rmv(x)
    g = oracle.normals(5, 0, 1, 0, 0, n)
    assert np.allclose(y, sig * np.linalg.norm(x) * g, rtol=1e-13)


def test_ginibre_second_and_third_step_closed_form():
    """Sec. 3.2: Q x_2 = (v_1'x_2) u_1 + (v_2'x_2) u_2 with u_i = g_i and
    v_1, v_2 the Gram-Schmidt basis of (x_1, x_2) (v_1 = R_1 e_1 =
    x_1/||x_1||, v_2 = R_1 R_2 e_2); then Q' x_3 with u_3 = L_1 e_1 =
    x_3/||x_3|| and v_3 = R_1 R_2 Z_{1:2} g_3 orthogonal to v_1, v_2."""
    m, n = 11, 9
    rng = np.random.default_rng(1)
    orc = HDOracle(GINIBRE, n, m, seed=8)
    x1, x2, x3 = rng.standard_normal(n), rng.standard_normal(n), \
        rng.standard_normal(m)
    y1 = orc.mv(x1)
    y2 = orc.mv(x2)
    g1 = oracle.normals(8, 0, 1, 0, 0, m)
    g2 = oracle.normals(8, 0, 2, 0, 0, m)
    v1 = x1 / np.linalg.norm(x1)
    w = x2 - (v1 @ x2) * v1
    v2 = w / np.linalg.norm(w)
    assert np.allclose(y1, np.linalg.norm(x1) * g1, rtol=1e-13)
    assert np.allclose(y2, (v1 @ x2) * g1 + (v2 @ x2) * g2, rtol=1e-12,
                       atol=1e-13)
    y3 = orc.rmv(x3)
    u3, v3 = orc.basis(3)
    assert np.allclose(u3, x3 / np.linalg.norm(x3), atol=1e-14)
    assert abs(v3 @ v1) < 1e-13 and abs(v3 @ v2) < 1e-13
    # v_3 = P_perp g_3 (the part of g_3 outside span{v1, v2}) in law; here
    # check its norm: ||Z_{1:2} g_3[...]|| = ||g_3[3:n]||
    g3 = oracle.normals(8, 0, 3, 0, 0, n)
    assert np.isclose(np.linalg.norm(v3), np.linalg.norm(g3[2:]), rtol=1e-13)
    expect = (g1 @ x3) * v1 + (g2 @ x3) * v2 + (u3 @ x3) * v3
    assert np.allclose(y3, expect, rtol=1e-12, atol=1e-13)


# ----------------------------------------------- reconstruction (P3) ---

def _haar_rec(orc, n, t, W):
    Lm = np.eye(n)
    for i in range(1, t + 1):
        Lm = Lm @ reflector_matrix(n, orc.reflector(SIDE_L, i))
    Rm = np.eye(n)
    for i in range(1, t + 1):
        Rm = reflector_matrix(n, orc.reflector(SIDE_R, i)) @ Rm
    mid = np.eye(n)
    mid[t:, t:] = W
    return Lm @ mid @ Rm


@pytest.mark.parametrize("pattern", ["Q", "QT", "mixed"])
def test_haar_exact_reconstruction(pattern):
    """eq. (H_t) and claim (b) of Theorem 2: for ANY orthogonal W,
    Q_rec = L_1..L_t diag(I_t, W) R_t..R_1 reproduces every past answer
    (Q x_s = y_s or Q' x_s = y_s) and is orthogonal."""
    n, T = 16, 9
    rng = np.random.default_rng(2)
    orc = HDOracle(HAAR, n, seed=21, trial=4)
    hist = []
    for s in range(T):
        tr = {"Q": False, "QT": True, "mixed": bool(rng.random() < 0.5)}[
            pattern]
        x = rng.standard_normal(n)
        hist.append((tr, x, orc.query(x, tr)))
    for _ in range(2):
        Qr = _haar_rec(orc, n, T, haar_dense(n - T, rng))
        assert np.allclose(Qr.T @ Qr, np.eye(n), atol=1e-12)
        for tr, x, y in hist:
            assert np.allclose((Qr.T if tr else Qr) @ x, y, atol=1e-12)


@pytest.mark.parametrize("m,n", [(10, 10), (12, 7), (6, 13)])
def test_ginibre_exact_reconstruction(m, n):
    """eq. (Gaussian_t): for ANY m x n matrix W,
    Q_rec = sum_i u_i v_i' + L_1..L_l Z_{1:l} W Z_{1:r} R_r..R_1 reproduces
    every past answer of the lazy Gaussian matrix."""
    rng = np.random.default_rng(m + 100 * n)
    sig = 1.7
    orc = HDOracle(GINIBRE, n, m, seed=2, trial=9, sigma=sig)
    hist = []
    T = min(m, n) - 1
    for s in range(T):
        tr = bool(rng.random() < 0.5)
        x = rng.standard_normal(m if tr else n)
        hist.append((tr, x, orc.query(x, tr)))
    t, r, l = orc.counts()
    assert t == T and r + l == T
    for _ in range(2):
        Qr = _ginibre_rec(orc, m, n, sig, rng.standard_normal((m, n)))
        for tr, x, y in hist:
            assert np.allclose((Qr.T if tr else Qr) @ x, y, atol=1e-12)


def _ginibre_rec(orc, m, n, sig, W):
    """sigma (sum_i u_i v_i' + L_1..L_l Z_{1:l} W Z_{1:r} R_r..R_1)."""
    t, r, l = orc.counts()
    S = np.zeros((m, n))
    for i in range(1, t + 1):
        u, v = orc.basis(i)
        S += np.outer(u, v)
    Lm = np.eye(m)
    for i in range(1, l + 1):
        Lm = Lm @ reflector_matrix(m, orc.reflector(SIDE_L, i))
    Rm = np.eye(n)
    for i in range(1, r + 1):
        Rm = reflector_matrix(n, orc.reflector(SIDE_R, i)) @ Rm
    Zl = np.diag(np.r_[np.zeros(l), np.ones(m - l)])
    Zr = np.diag(np.r_[np.zeros(r), np.ones(n - r)])
    return sig * (S + Lm @ Zl @ W @ Zr @ Rm)


def test_goe_exact_reconstruction():
    """Section "Other Random Matrix Ensembles": the GOE answers are those of
    the symmetric G = (Q_rec + Q_rec')/sqrt(2), for every completion W of
    the lazy Gaussian Q (mixed with plain queries of Q in between)."""
    n, sig = 11, 1.3
    rng = np.random.default_rng(5)
    orc = HDOracle(GINIBRE, n, seed=4, trial=2, sigma=sig)
    goe, plain = [], []
    for s in range(4):
        x = rng.standard_normal(n)
        goe.append((x, oracle.goe_query(orc, x)))
        if s == 1:
            z = rng.standard_normal(n)
            plain.append((z, orc.mv(z)))
    assert orc.counts()[0] == 9
    for _ in range(2):
        Qr = _ginibre_rec(orc, n, n, sig, rng.standard_normal((n, n)))
        G = (Qr + Qr.T) / np.sqrt(2.0)
        for x, y in goe:
            assert np.allclose(G @ x, y, atol=1e-12)
        for z, y in plain:
            assert np.allclose(Qr @ z, y, atol=1e-12)


def test_goe_entry_variances():
    """G ~ sigma GOE(n): the first answer to x = e_j is column j of G, with
    G_jj ~ N(0, 2 sigma^2) and G_ij ~ N(0, sigma^2) for i != j."""
    n, sig, trials, j = 6, 0.7, 4000, 2
    e = np.zeros(n)
    e[j] = 1.0
    cols = np.array([oracle.goe_query(
        HDOracle(GINIBRE, n, seed=8, trial=k, sigma=sig), e)
        for k in range(trials)])
    sq = cols ** 2
    for i in range(n):
        want = (2.0 if i == j else 1.0) * sig ** 2
        se = sq[:, i].std() / np.sqrt(trials)
        assert abs(sq[:, i].mean() - want) < 5 * se, (i, sq[:, i].mean())
    assert abs(cols.mean(axis=0)).max() < 5 * sig * np.sqrt(2.0 / trials)


@pytest.mark.parametrize("m,n", [(12, 12), (15, 9), (8, 13)])
def test_usv_exact_reconstruction_and_singular_values(m, n):
    """Section "Other Random Matrix Ensembles", Q = U S V with U ~ Haar(m),
    V ~ Haar(n) and S = diag(s) in R^{m x n}: every answer (Q and Q'
    queries, mixed) equals that of U_rec S V_rec for any completions of the
    two lazy Haar matrices, whose singular values are |s|."""
    K = 6
    p = min(m, n)
    rng = np.random.default_rng(8 + m + n)
    s = rng.standard_normal(p) * 2.0
    ou = HDOracle(HAAR, m, seed=3, trial=1)
    ov = HDOracle(HAAR, n, seed=3, trial=2)
    hist = []
    for k in range(K):
        tr = bool(rng.random() < 0.5)
        x = rng.standard_normal(m if tr else n)
        hist.append((tr, x, oracle.usv_query(ou, ov, s, x, tr)))
    assert ou.counts()[0] == K and ov.counts()[0] == K
    S = np.zeros((m, n))
    S[np.arange(p), np.arange(p)] = s
    for _ in range(2):
        Ur = _haar_rec(ou, m, K, haar_dense(m - K, rng))
        Vr = _haar_rec(ov, n, K, haar_dense(n - K, rng))
        Qr = Ur @ S @ Vr
        for tr, x, y in hist:
            assert np.allclose((Qr.T if tr else Qr) @ x, y, atol=1e-12)
        sv = np.linalg.svd(Qr, compute_uv=False)
        assert np.allclose(np.sort(sv), np.sort(np.abs(s)), atol=1e-12)


# ------------------------------------------------------- isometry (P4) ---

def test_haar_isometry_long_mixed():
    """Q orthogonal: ||y_t|| = ||x_t|| for every query of a long mixed run,
    and <Q x_s, Q x_t> = <x_s, x_t> for Q-queries."""
    n, T = 300, 60
    rng = np.random.default_rng(5)
    orc = HDOracle(HAAR, n, seed=1)
    X, Y = [], []
    for s in range(T):
        tr = bool(s % 3 == 2)
        x = rng.standard_normal(n) + (X[-1] if X else 0)
        y = orc.query(x, tr)
        assert np.isclose(np.linalg.norm(y), np.linalg.norm(x), rtol=1e-13)
        if not tr:
            X.append(x)
            Y.append(y)
    X, Y = np.array(X), np.array(Y)
    assert np.allclose(Y @ Y.T, X @ X.T, rtol=1e-12, atol=1e-10)


# -------------------------------------------- textbook reduction (P5) ---

def test_ginibre_q_only_is_gaussian_times_R_factor():
    """Q-queries only: v_i are the Gram-Schmidt vectors of x_1..x_t, so
    Y = sigma * G R_X with G = [g_1..g_t] (the draws) and R_X the
    positive-diagonal R factor of X = [x_1..x_t] (LAPACK QR)."""
    m, n, T = 40, 30, 12
    sig = 0.5
    rng = np.random.default_rng(9)
    orc = HDOracle(GINIBRE, n, m, seed=6, trial=1, sigma=sig)
    X = rng.standard_normal((n, T))
    Y = np.column_stack([orc.mv(X[:, i]) for i in range(T)])
    G = np.column_stack([oracle.normals(6, 1, i + 1, 0, 0, m)
                         for i in range(T)])
    assert np.allclose(Y, sig * G @ r_factor_positive(X), rtol=1e-12,
                       atol=1e-12)


def test_haar_q_only_factorisation():
    """Q-queries only: Y = U R_X with U orthonormal and depending only on the
    draws, not on X (two different X with one seed give the same U);
    U[:, 0] = g_1/||g_1||."""
    n, T = 50, 15
    rng = np.random.default_rng(3)
    Us = []
    for rep in range(2):
        orc = HDOracle(HAAR, n, seed=12, trial=7)
        X = rng.standard_normal((n, T))
        Y = np.column_stack([orc.mv(X[:, i]) for i in range(T)])
        U = Y @ np.linalg.inv(r_factor_positive(X))
        assert np.allclose(U.T @ U, np.eye(T), atol=1e-12)
        Us.append(U)
    assert np.allclose(Us[0], Us[1], atol=1e-11)
    g1 = oracle.normals(12, 7, 1, 0, 0, n)
    assert np.allclose(Us[0][:, 0], g1 / np.linalg.norm(g1), atol=1e-13)


# ---------------------------------------------------- moments (P7) ---

def test_haar_full_reveal_moments():
    """Revealing all n columns (x_t = e_t, T = n) gives a full orthogonal Q;
    over trials E[(tr Q)^2] = 1 and E[Q_ij^2] = 1/n (Haar moments)."""
    n, trials = 6, 3000
    tr2, sq = [], []
    for k in range(trials):
        orc = HDOracle(HAAR, n, seed=100, trial=k)
        Q = np.column_stack([orc.mv(e) for e in np.eye(n)])
        assert np.allclose(Q.T @ Q, np.eye(n), atol=1e-12)
        tr2.append(np.trace(Q) ** 2)
        sq.append(Q[1, 2] ** 2)
    tr2 = np.array(tr2)
    assert abs(tr2.mean() - 1) < 5 * tr2.std() / np.sqrt(trials)
    sq = np.array(sq)
    assert abs(sq.mean() - 1 / n) < 5 * sq.std() / np.sqrt(trials)


def test_ginibre_second_moment():
    """E ||Q' Q x||^2 = sigma^4 m (m + n + 1) ||x||^2 for Q ~ sigma GE(m,n)
    (two queries: Q x, then Q' of the answer)."""
    m, n, trials = 9, 6, 4000
    sig = 0.8
    x = np.random.default_rng(0).standard_normal(n)
    vals = []
    for k in range(trials):
        orc = HDOracle(GINIBRE, n, m, seed=77, trial=k, sigma=sig)
        vals.append(np.sum(orc.rmv(orc.mv(x)) ** 2))
    vals = np.array(vals)
    expect = sig ** 4 * m * (m + n + 1) * (x @ x)
    assert abs(vals.mean() - expect) < 5 * vals.std() / np.sqrt(trials)


# ------------------------------------------------ distribution (P6) ---

def _dense_traj(Q, x1, T, dyn, a, b, pattern):
    f = oracle.DYNAMICS[dyn]
    x, xp = x1.copy(), np.zeros_like(x1)
    for t in range(T):
        M = Q.T if (pattern == "alt" and t % 2 == 1) else Q
        x, xp = f(M @ x, x, xp, a, b), x
    return x


@pytest.mark.parametrize("ens", [HAAR, GINIBRE])
def test_distribution_matches_direct_method(ens):
    """Theorems 1 and 2: the HD trajectory has the law of the direct method.
    Two-sample KS tests (alpha = 1e-3, fixed seeds) on three statistics of
    x_{T+1} against dense-matrix simulations of the same dynamics."""
    n, T, trials = 40, 8, 1500
    rng = np.random.default_rng(ens)
    x1 = rng.standard_normal(n) / np.sqrt(n)
    if ens == HAAR:
        dyn, a, b, pattern = "tanh", 1.0, 0.5, "Q"
    else:
        dyn, a, b, pattern = "soft_hist", 0.1, 0.3, "alt"
    sig = 1 / np.sqrt(n)
    hd, direct = [], []
    for k in range(trials):
        orc = HDOracle(ens, n, seed=31, trial=k, sigma=sig)
        X, _ = oracle.run_trajectory(orc, x1, T, dyn, a, b, pattern)
        hd.append(X[-1])
        Q = haar_dense(n, rng) if ens == HAAR else \
            sig * rng.standard_normal((n, n))
        direct.append(_dense_traj(Q, x1, T, dyn, a, b, pattern))
    hd, direct = np.array(hd), np.array(direct)
    for stat in (lambda X: np.sqrt(n) * X[:, 0],
                 lambda X: np.sum(X ** 2, axis=1) / n,
                 lambda X: X @ x1):
        assert stats.ks_2samp(stat(hd), stat(direct)).pvalue > 1e-3


# ------------------------------------------------ edge cases ---

def test_capacity_and_zero_query():
    """T <= min(m, n) (Alg. 1, Alg. 2 input); a zero query gives the identity
    reflector (convention after eq. (Householder_e)), y = 0, and still counts."""
    orc = HDOracle(HAAR, 4, tmax=3, seed=0)
    y = orc.mv(np.zeros(4))
    assert np.array_equal(y, np.zeros(4))
    assert orc.reflector(SIDE_R, 1)["ident"]
    assert orc.counts() == (1, 1, 1)
    orc.mv(np.ones(4))
    orc.rmv(np.ones(4))
    with pytest.raises(OverflowError):
        orc.mv(np.ones(4))
    assert orc.counts() == (3, 3, 3)
    g = HDOracle(GINIBRE, 2, 5, seed=0)
    g.mv(np.ones(2))
    g.mv(np.ones(2))
    with pytest.raises(OverflowError):  # r would exceed n = 2
        g.mv(np.ones(2))
    with pytest.raises(ValueError):
        HDOracle(HAAR, 4, m=5)


def test_forced_sign_changes_basis_not_law():
    """Forcing the sign of a data reflector flips its orientation (Mode-B
    sign following) while H(v) v = ||v|| e1 still holds."""
    n = 8
    x = np.random.default_rng(0).standard_normal(n)
    a = HDOracle(HAAR, n, seed=3)
    b = HDOracle(HAAR, n, seed=3)
    s = a.mv(x) is not None and a.reflector(SIDE_R, 1)["s"]
    b.force_sign(SIDE_R, 1, -s)
    yb = b.mv(x)
    assert b.reflector(SIDE_R, 1)["s"] == -s
    Hb = reflector_matrix(n, b.reflector(SIDE_R, 1))
    assert np.allclose(Hb @ x, np.linalg.norm(x) * np.eye(n)[0], atol=1e-13)
    assert np.isclose(np.linalg.norm(yb), np.linalg.norm(x), rtol=1e-13)


def test_normalising_map_properties():
    """The map of the large single trial, x_{t+1} = y/||y|| + b x_t
    (eq. (dynamics) with f_t a normalisation plus a memory term): with
    b = 0 the output has unit norm; it is invariant to positive scalings of
    y; and f - b x_t is a positive multiple of y (so neither x_{t-1} nor a
    wrong power of ||y|| enters)."""
    rng = np.random.default_rng(17)
    f = oracle.f_normalize
    for n in (1, 5, 1000):
        y = rng.standard_normal(n) * 3.7
        xt = rng.standard_normal(n)
        xp = rng.standard_normal(n)
        assert abs(np.linalg.norm(f(y, xt, xp, 0.0, 0.0)) - 1.0) < 1e-14
        assert np.allclose(f(y, xt, xp, 0.0, 0.1),
                           f(123.5 * y, xt, xp, 0.0, 0.1), atol=1e-14)
        d = f(y, xt, xp, 0.0, 0.1) - 0.1 * xt
        c = float(d @ y) / float(y @ y)
        assert c > 0 and np.allclose(d, c * y, atol=1e-14)


def test_normalising_trajectory_on_haar_keeps_unit_norm():
    """Along a Haar trajectory with Q-queries only and b = 0, every state
    after the first has unit norm (the lazy Q is an isometry, Theorem 2,
    and the map normalises its answer): ||x_{t+1}|| = 1 and
    ||y_t|| = ||x_t||."""
    n, T = 300, 25
    orc = HDOracle(HAAR, n, seed=8)
    x1 = np.random.default_rng(3).standard_normal(n) * 5.0
    X, Y = oracle.run_trajectory(orc, x1, T, "normalize", 0.0, 0.0)
    assert np.allclose(np.linalg.norm(X[1:], axis=1), 1.0, atol=1e-13)
    assert np.allclose(np.linalg.norm(Y, axis=1),
                       np.linalg.norm(X[:-1], axis=1), rtol=1e-13)


def _spectral_dense(orc, m, n, t, rng):
    """A = [I_n 0] Q_rec (eq. (A_ortho)) for the oracle's lazy Haar Q after
    t queries, completed with a random orthogonal W."""
    Qr = _haar_rec(orc, m, t, haar_dense(m - t, rng))
    return Qr[:n, :]


@pytest.mark.parametrize("scale", [1.0, 2.5])
def test_spectral_power_matches_dense_matrix(scale):
    """Sec. 2.2: the measurements are A' xi, and every power step of the
    oracle's spectral method is x_{k+1} = scale * A diag(y) A' x_k with
    y = tanh|A' xi| (m D of eq. (D_mtx)), for the dense A rebuilt from the
    revealed reflectors (any completion)."""
    m, n, K = 30, 12, 7
    rng = np.random.default_rng(40)
    orc = HDOracle(HAAR, m, seed=3, trial=1)
    xi = rng.standard_normal(n)
    x1 = rng.standard_normal(n)
    z, X = oracle.spectral_power(orc, xi, x1, K, scale)
    assert orc.counts()[0] == 1 + 2 * K
    for _ in range(2):
        A = _spectral_dense(orc, m, n, 1 + 2 * K, rng)
        assert np.allclose(A @ A.T, np.eye(n), atol=1e-12)
        assert np.allclose(z, A.T @ xi, atol=1e-12)
        Dm = A @ np.diag(np.tanh(np.abs(A.T @ xi))) @ A.T
        for k in range(K):
            assert np.allclose(X[k + 1], scale * Dm @ X[k], atol=1e-12)


def test_spectral_power_converges_to_top_eigenvector():
    """Power iteration on D (eq. (D_mtx)) through the lazy matrix ends at
    the leading eigenvector of the dense D built from the revealed
    reflectors, and its Rayleigh quotients never decrease (D is symmetric
    positive semidefinite)."""
    m, n, K = 500, 100, 180
    rng = np.random.default_rng(41)
    orc = HDOracle(HAAR, m, seed=5)
    xi = rng.standard_normal(n)
    z, X = oracle.spectral_power(orc, xi, rng.standard_normal(n), K, 1.0)
    A = _spectral_dense(orc, m, n, 1 + 2 * K, rng)
    ev, U = np.linalg.eigh(A @ np.diag(np.tanh(np.abs(z))) @ A.T)
    x = X[-1] / np.linalg.norm(X[-1])
    assert ev[-1] - ev[-2] > 0.05 * ev[-1]
    assert abs(x @ U[:, -1]) > 1 - 1e-9
    rq = [X[k] @ X[k + 1] / (X[k] @ X[k]) for k in range(K)]
    assert all(b >= a - 1e-12 for a, b in zip(rq, rq[1:]))
    assert abs(rq[-1] - ev[-1]) < 1e-9 * ev[-1]
