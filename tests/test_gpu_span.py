"""Queries in the span of earlier ones, validated through the exported
reflectors.

When a query lies in the span of the earlier data-side queries, p[k:] is
rounding noise: the reflector built from it is one of many valid orthogonal
completions, and which one depends on the order of the sums, so the answers
after it need not match the oracle's.  What is unique is that all answers
come from ONE orthogonal matrix: rebuilding Q from the GPU's own stored
reflectors (hd_export) as Q_rec = L_1..L_t diag(I_t, W) R_t..R_1
(eq. (H_t), claim (b) of Theorem 2, any orthogonal W) must reproduce every
answer, Q_rec x_s = y_s (or Q_rec' x_s = y_s), and Q_rec' Q_rec = I.  For the
Gaussian ensemble the same holds for Q_rec = sigma (sum_i u_i v_i' +
L_1..L_l Z_{1:l} W Z_{1:r} R_r..R_1) (eq. (Gaussian_t)) with any W.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2101_07464_amd as hd  # noqa: E402
from tests.dense import haar_dense  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


class StateHeader(ctypes.Structure):
    """Header of an exported state (the layout hd_export documents)."""
    _fields_ = [("magic", ctypes.c_char * 8), ("ensemble", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("t_max", ctypes.c_int32),
                ("pstride", ctypes.c_int32), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64), ("seed", ctypes.c_uint32),
                ("trial", ctypes.c_uint32), ("sigma", ctypes.c_double),
                ("t", ctypes.c_int32), ("r", ctypes.c_int32),
                ("l", ctypes.c_int32), ("flag", ctypes.c_int32),
                ("pf_step", ctypes.c_int32 * 2),
                ("pending", ctypes.c_int32 * 2),
                ("vcols", ctypes.c_int32 * 2), ("bcols", ctypes.c_int32 * 2),
                ("total_bytes", ctypes.c_uint64)]


def parse_state(buf):
    """Per side: panel columns, tau, nu, sign; per side the explicit basis
    columns (Gaussian)."""
    H = StateHeader.from_buffer_copy(bytes(buf[:ctypes.sizeof(StateHeader)]))
    assert H.magic == b"HDSTATE1" and H.total_bytes == len(buf)
    es = np.float64 if H.storage == 1 else np.float32
    tm = H.t_max
    dims = (H.n, H.m)
    off = ctypes.sizeof(StateHeader)

    def take(count, dt):
        nonlocal off
        nb = np.dtype(dt).itemsize * count
        a = np.frombuffer(bytes(buf[off:off + nb]), dtype=dt).astype(
            np.float64)
        off += nb
        return a

    sides = []
    for s in range(2):
        V = take(dims[s] * H.vcols[s], es).reshape(H.vcols[s], dims[s])
        take(tm * tm, np.float64)  # T factor
        tau = take(tm, np.float64)
        nu = take(tm, np.float64)
        take(tm, np.float64)  # pivots
        sgn = take(tm, np.float64)
        take(tm + 1, np.float64)  # sign prefix
        take(H.pstride, np.float64)  # reduced results of the last pass
        sides.append((V, tau, nu, sgn))
    basis = []
    for s in range(2):
        basis.append(take(dims[s] * H.bcols[s], es).reshape(H.bcols[s],
                                                             dims[s]))
    assert off == len(buf)
    return H, sides, basis


def reflector(dim, V, tau, nu, sgn, j):
    """Dense reflector j (0-based) of a side: identity when its norm is 0,
    else diag(I_j, -s (I - tau u u')) on rows j.. (eq. (Householder_e))."""
    M = np.eye(dim)
    if nu[j] == 0.0:
        return M
    u = V[j, j:]
    M[j:, j:] = -sgn[j] * (np.eye(dim - j) - tau[j] * np.outer(u, u))
    return M


def products(dim, side, count):
    """(P_1 P_2 .. P_count, P_count .. P_1) of the side's reflectors."""
    V, tau, nu, sgn = side
    fwd, rev = np.eye(dim), np.eye(dim)
    for j in range(count):
        Pj = reflector(dim, V, tau, nu, sgn, j)
        fwd = fwd @ Pj
        rev = Pj @ rev
    return fwd, rev


def run_queries(A, xs, flags, dtype):
    ys = []
    for x, tr in zip(xs, flags):
        xt = torch.from_numpy(x).to(DEV, dtype)
        ys.append((A.rmv(xt) if tr else A.mv(xt)).double().cpu().numpy())
    torch.cuda.synchronize()
    assert A.status() == 0
    return ys


FLAGS = [False, False, False, True, True, False, True, False, False, True,
         False, False]


def span_queries(n, m, rng):
    """Query vectors with several in the span of earlier same-side ones:
    x_3 = 0.3 x_1 + 0.7 x_2 (Q), x_5 = -1.5 x_4 (Q'), x_9 = x_1 - x_6 (Q),
    x_12 = 0.3 x_1 (Q); the others random."""
    xs = []
    for q, tr in enumerate(FLAGS, start=1):
        d = m if tr else n
        if q == 3:
            x = 0.3 * xs[0] + 0.7 * xs[1]
        elif q == 5:
            x = -1.5 * xs[3]
        elif q == 9:
            x = xs[0] - xs[5]
        elif q == 12:
            x = 0.3 * xs[0]
        else:
            x = rng.standard_normal(d)
        xs.append(x)
    return xs


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11),
                                       (torch.float32, 1e-4)])
def test_haar_span_queries_one_orthogonal_matrix(dtype, tol):
    n = 40
    rng = np.random.default_rng(31)
    xs = span_queries(n, n, rng)
    if dtype == torch.float32:
        xs = [x.astype(np.float32).astype(np.float64) for x in xs]
    A = hd.LazyMatrix(hd.HAAR, n, t_max=len(FLAGS), seed=5, dtype=dtype,
                      device=DEV)
    ys = run_queries(A, xs, FLAGS, dtype)
    H, sides, _ = parse_state(A.export_state())
    t = H.t
    assert t == len(FLAGS)
    Lf, _ = products(n, sides[1], t)
    _, Rr = products(n, sides[0], t)
    for _ in range(2):
        mid = np.eye(n)
        mid[t:, t:] = haar_dense(n - t, rng)
        Q = Lf @ mid @ Rr
        assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-12
        for x, y, tr in zip(xs, ys, FLAGS):
            yr = (Q.T if tr else Q) @ x
            assert np.abs(yr - y).max() / np.abs(y).max() < tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11),
                                       (torch.float32, 1e-4)])
def test_gaussian_span_queries_one_matrix(dtype, tol):
    n, m = 36, 30
    sig = 0.8
    rng = np.random.default_rng(32)
    xs = span_queries(n, m, rng)
    if dtype == torch.float32:
        xs = [x.astype(np.float32).astype(np.float64) for x in xs]
    A = hd.LazyMatrix(hd.GINIBRE, n, m=m, t_max=len(FLAGS), seed=6,
                      sigma=sig, dtype=dtype, device=DEV)
    ys = run_queries(A, xs, FLAGS, dtype)
    H, sides, basis = parse_state(A.export_state())
    r, l = H.r, H.l
    assert (r, l) == (FLAGS.count(False), FLAGS.count(True))
    Rf, Rr = products(n, sides[0], r)
    Lf, _ = products(m, sides[1], l)
    # basis vectors: u of a Q-query is explicit (basis[1]), its v is
    # R_1..R_r e_r; v of a Q'-query is explicit (basis[0]), its u is
    # L_1..L_l e_l
    S = np.zeros((m, n))
    rq = lq = 0
    for tr in FLAGS:
        if tr:
            lq += 1
            Lp, _ = products(m, sides[1], lq)
            u = Lp[:, lq - 1]
            v = basis[0][lq - 1]
        else:
            rq += 1
            Rp, _ = products(n, sides[0], rq)
            v = Rp[:, rq - 1]
            u = basis[1][rq - 1]
        S += np.outer(u, v)
    for _ in range(2):
        W = np.zeros((m, n))
        W[l:, r:] = rng.standard_normal((m - l, n - r))
        Q = sig * (S + Lf @ W @ Rr)
        for x, y, tr in zip(xs, ys, FLAGS):
            yr = (Q.T if tr else Q) @ x
            assert np.abs(yr - y).max() / np.abs(y).max() < tol
